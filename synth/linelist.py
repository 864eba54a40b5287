"""Counter-based synthetic ExoMol-style line lists.

Every random number is a pure function of (seed, stream, counter) through the
SplitMix64 finaliser (Steele, Lea & Flood 2014), so a line is the same value
whatever the list size or device, and chunks of a large list can be regenerated
independently.  Written with torch integer ops so it runs on the CPU or on a GPU
device; int64 multiplication wraps modulo 2**64 on both.

Distributions (the synthetic stand-ins for the paper's H2O / H2S / CH4 lists):
  * state energies  E = 20000 * u**(1/3)  cm^-1, u ~ U[0,1) (53-bit)
  * J ~ U{0..50},  g = 2J + 1
  * transitions: two uniform state indices, ordered by energy, accepted when
    0 < E_up - E_low <= nu_max (redrawn otherwise; counter-based attempts)
  * log10 A ~ U(-8, 2)  (A stored as float32, as in 12-byte .trans records)
  * gamma_ref ~ U(0.02, 0.1) cm^-1/bar, n ~ U(0.4, 0.8) (float32, per line)
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_STREAM_MUL = 0xD1B54A32D192ED03
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
BASE_SEED = 180109803

# stream ids
STREAM_STATES_E, STREAM_STATES_J = 0, 5
STREAM_PAIRS, STREAM_A, STREAM_BROAD, STREAM_PERTURB = 1, 2, 3, 4


def _s64(v: int) -> int:
    """Two's-complement reinterpretation of a 64-bit pattern."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def splitmix64_ref(z: int) -> int:
    """Pure-Python SplitMix64 finaliser (reference for the tensor version)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def _lsr(z: torch.Tensor, k: int) -> torch.Tensor:
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def _stream_key(seed: int, stream: int) -> int:
    return splitmix64_ref((seed + stream * _STREAM_MUL) & MASK64)


def random_bits(seed: int, stream: int, counter: torch.Tensor) -> torch.Tensor:
    """64-bit random patterns (int64 tensor) for the given int64 counters."""
    key = _stream_key(seed, stream)
    z = counter.to(torch.int64) * _s64(_GOLDEN) + _s64(key + _GOLDEN)
    return _mix(z)


def uniform53(seed: int, stream: int, counter: torch.Tensor) -> torch.Tensor:
    """Doubles in [0, 1) with 53 random bits."""
    return _lsr(random_bits(seed, stream, counter), 11).to(torch.float64) * (2.0 ** -53)


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    index: int
    n_states: int
    n_lines: int
    mass_amu: float
    nu_max: float          # transitions have 0 < nu <= nu_max
    nu_a: float
    nu_b: float
    n_points: int
    temperatures: tuple
    pressures: tuple
    cutoff: float = 25.0
    broadening: str = "per_line"   # or "a0_jlower"

    @property
    def seed(self) -> int:
        return BASE_SEED + 1000 * self.index

    @property
    def dnu(self) -> float:
        return (self.nu_b - self.nu_a) / (self.n_points - 1)


def _c3_T():
    return tuple(100.0 * 30.0 ** (j / 26.0) for j in range(27))


def _c3_P():
    return tuple(10.0 ** (-5.0 + 7.0 * l / 9.0) for l in range(10))


CONFIGS = {
    "C1": WorkloadConfig("C1", 1, 10_000, 100_000, 18.0, 5000.0, 0.0, 5000.0, 50_001,
                         (1000.0,), (1.0,)),
    "C2": WorkloadConfig("C2", 2, 1_000_000, 100_000_000, 34.0, 10000.0, 0.0, 10000.0,
                         1_000_001, (296.0, 2000.0), (1.0,)),
    "C3": WorkloadConfig("C3", 3, 1_000_000, 100_000_000, 34.0, 10000.0, 0.0, 10000.0,
                         1_000_001, _c3_T(), _c3_P()),
    "C4": WorkloadConfig("C4", 4, 100_000, 10_000_000, 34.0, 10000.0, 1000.0, 6000.0,
                         500_001, (1500.0,), (0.1,)),
    "C5": WorkloadConfig("C5", 5, 50_000_000, 4_000_000_000, 16.0, 12000.0, 0.0, 12000.0,
                         1_200_001,
                         tuple(300.0 * 10.0 ** (j / 8.0) for j in range(9)),
                         tuple(10.0 ** (-5.0 + 7.0 * l / 3.0) for l in range(4)),
                         broadening="a0_jlower"),
}


def config_by_name(name: str) -> WorkloadConfig:
    return CONFIGS[name]


def make_states(n_states: int, seed: int, device="cpu"):
    """Energies (float64, cm^-1), total degeneracies g = 2J+1 and J (int32)."""
    idx = torch.arange(n_states, dtype=torch.int64, device=device)
    u = uniform53(seed, STREAM_STATES_E, idx)
    E = 20000.0 * torch.pow(u, 1.0 / 3.0)
    J = torch.floor(uniform53(seed, STREAM_STATES_J, idx) * 51.0).to(torch.int32).clamp_(0, 50)
    g = (2 * J + 1).to(torch.int32)
    return E, g, J


def make_transitions(E: torch.Tensor, n_lines: int, nu_max: float, seed: int,
                     first_line: int = 0, max_attempts: int = 1024):
    """Upper/lower state indices (0-based int32) for lines first_line..first_line+n_lines-1.

    Attempt r of line i draws two state indices from counters 2*(1024*i + r) and
    2*(1024*i + r) + 1; the first accepted attempt wins.
    """
    device = E.device
    line = torch.arange(first_line, first_line + n_lines, dtype=torch.int64, device=device)
    return make_transitions_at(E, line, nu_max, seed, max_attempts)


def make_transitions_at(E: torch.Tensor, line: torch.Tensor, nu_max: float, seed: int, max_attempts: int = 1024):
    """Upper/lower state indices of the lines with the given (int64) indices: the same
    pairs make_transitions gives those lines, so any subset of a large list can be drawn."""
    device = E.device
    line = line.to(device=device, dtype=torch.int64)
    n_lines = line.numel()
    n_states = E.numel()
    upper = torch.full((n_lines,), -1, dtype=torch.int64, device=device)
    lower = torch.full((n_lines,), -1, dtype=torch.int64, device=device)
    todo = torch.arange(n_lines, dtype=torch.int64, device=device)
    for r in range(max_attempts):
        if todo.numel() == 0:
            break
        ctr = (line[todo] * max_attempts + r) * 2
        a = torch.floor(uniform53(seed, STREAM_PAIRS, ctr) * n_states).to(torch.int64).clamp_(0, n_states - 1)
        b = torch.floor(uniform53(seed, STREAM_PAIRS, ctr + 1) * n_states).to(torch.int64).clamp_(0, n_states - 1)
        Ea, Eb = E[a], E[b]
        up = torch.where(Ea >= Eb, a, b)
        lo = torch.where(Ea >= Eb, b, a)
        dE = E[up] - E[lo]
        ok = (dE > 0) & (dE <= nu_max)
        sel = todo[ok]
        upper[sel] = up[ok]
        lower[sel] = lo[ok]
        todo = todo[~ok]
    if todo.numel():
        raise RuntimeError(f"{todo.numel()} lines found no admissible state pair")
    return upper.to(torch.int32), lower.to(torch.int32)


def make_line_params(n_lines: int, seed: int, first_line: int = 0, device="cpu"):
    """Einstein A (float32, s^-1), gamma_ref (float32, cm^-1/bar), n (float32)."""
    line = torch.arange(first_line, first_line + n_lines, dtype=torch.int64, device=device)
    return make_line_params_at(line, seed)


def make_line_params_at(line: torch.Tensor, seed: int):
    """make_line_params for the lines with the given (int64) indices."""
    line = line.to(torch.int64)
    A = torch.pow(10.0, -8.0 + 10.0 * uniform53(seed, STREAM_A, line)).to(torch.float32)
    gref = (0.02 + 0.08 * uniform53(seed, STREAM_BROAD, 2 * line)).to(torch.float32)
    nexp = (0.4 + 0.4 * uniform53(seed, STREAM_BROAD, 2 * line + 1)).to(torch.float32)
    return A, gref, nexp


def make_broadening_table(seed: int, n_j: int = 51, device="cpu"):
    """a0-type table over lower-state J: gamma_ref[J], n[J] (float32)."""
    j = torch.arange(n_j, dtype=torch.int64, device=device) + (1 << 40)
    gref = (0.02 + 0.08 * uniform53(seed, STREAM_BROAD, 2 * j)).to(torch.float32)
    nexp = (0.4 + 0.4 * uniform53(seed, STREAM_BROAD, 2 * j + 1)).to(torch.float32)
    return gref, nexp


def make_vibrational_labels(E: torch.Tensor, band_width: float = 2000.0) -> torch.Tensor:
    """Vibrational (vibronic) manifold label per state, for non-LTE inputs: the synthetic
    states carry no quantum numbers, so states are grouped into energy bands of
    band_width cm^-1, label = floor(E / band_width) (int32)."""
    return torch.floor(E / band_width).to(torch.int32)


def make_linelist(cfg: WorkloadConfig, n_lines: Optional[int] = None, n_states: Optional[int] = None,
                  device="cpu", first_line: int = 0):
    """Full synthetic input for a workload (optionally truncated in size)."""
    ns = cfg.n_states if n_states is None else n_states
    nl = cfg.n_lines if n_lines is None else n_lines
    E, g, J = make_states(ns, cfg.seed, device=device)
    upper, lower = make_transitions(E, nl, cfg.nu_max, cfg.seed, first_line=first_line)
    A, gref, nexp = make_line_params(nl, cfg.seed, first_line=first_line, device=device)
    return dict(E=E, g=g, J=J, upper=upper, lower=lower, A=A, gamma_ref=gref, n_exp=nexp)


def perturbation_normals(n_lines: int, seed: int, device="cpu"):
    """Standard normals (Box-Muller on two counter-based uniforms) for seeded
    perturbations of log A."""
    line = torch.arange(n_lines, dtype=torch.int64, device=device)
    u1 = uniform53(seed, STREAM_PERTURB, 2 * line)
    u2 = uniform53(seed, STREAM_PERTURB, 2 * line + 1)
    u1 = torch.clamp(u1, min=2.0 ** -53)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)
