"""The hot-polyatomic workload's shape through the streaming path, against the oracle:
5e7 states (16 Da), a0 broadening by lower-state J, all 9 x 4 (T, P) points, FP32 Voigt on
0-12000 cm^-1 at 0.01 cm^-1 (1,200,001 points), cut-off 25 cm^-1.  The transitions are a
seeded subsample of the 4e9-transition list drawn by index across its whole range (each
line is the one the full list holds at that index), streamed as device-resident and host
chunks.  Every (T, P) is compared with the oracle on the full grid (1e-5), and at 100 bar,
where every line is resolved (gamma >= 0.3 cm^-1 >> dnu), the integrated cross section
is checked against the sum rule: dnu sum_k sigma_k = sum_i I_i a_i, a_i the area of line
i's Voigt profile over its window on the grid."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import assert_parity, log

pytestmark = pytest.mark.gpu

N_SAMPLE = 8000


def _truncated_voigt_areas(ls, klo, khi, nu_a, dnu):
    """Area of each line's Voigt profile over [nu_klo - dnu/2, nu_khi + dnu/2] (what the
    midpoint sum over its window integrates): the Doppler average of the Lorentz CDF,
    by a 40-node Gauss-Hermite rule (alpha_D << gamma here, so the integrand is smooth)."""
    t, w = np.polynomial.hermite.hermgauss(40)
    a = (nu_a + klo * dnu - 0.5 * dnu) - ls.nu
    b = (nu_a + khi * dnu + 0.5 * dnu) - ls.nu
    shift = ls.alpha_d[:, None] * t[None, :] / math.sqrt(math.log(2.0))
    g = ls.gamma[:, None]
    cdf = (np.arctan((b[:, None] - shift) / g) - np.arctan((a[:, None] - shift) / g)) / math.pi
    return (cdf * w[None, :]).sum(axis=1) / math.sqrt(math.pi)


def test_c5_shaped_stream_matches_oracle_and_sum_rule():
    cfg = synth.CONFIGS["C5"]
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed, device="cuda")
    gt, nt = synth.make_broadening_table(cfg.seed)
    rng = np.random.default_rng(55)
    idx = np.unique(rng.integers(0, cfg.n_lines, N_SAMPLE + 64))[:N_SAMPLE]
    lines = torch.from_numpy(idx.astype(np.int64)).cuda()
    up, lo = synth.linelist.make_transitions_at(E, lines, cfg.nu_max, cfg.seed)
    A = synth.linelist.make_line_params_at(lines, cfg.seed)[0]
    Ts = [t for t in cfg.temperatures for _ in cfg.pressures]
    Ps = [p for _ in cfg.temperatures for p in cfg.pressures]
    from paper_1801_09803_amd import Plan
    plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt",
                precision="fp32", broadening="a0_jlower")
    plan.set_broadening_table(gt.numpy(), nt.numpy())
    plan.set_states(E, g, J)
    log(f"C5 shape: {N_SAMPLE} transitions (indices {idx[0]}..{idx[-1]} of {cfg.n_lines}), {len(Ts)} (T,P)")
    st = plan.stream(Ts, Ps)
    c1, c2 = 3000, 5500
    st.chunk_device(up[:c1], lo[:c1], A[:c1])
    st.chunk(up[c1:c2].cpu().pin_memory(), lo[c1:c2].cpu().pin_memory(), A[c1:c2].cpu().pin_memory())
    st.chunk_device(up[c2:], lo[c2:], A[c2:])
    sig, kept = st.end()
    torch.cuda.synchronize()
    got = sig.double().cpu().numpy()
    Eh, gh, Jh = E.cpu().numpy(), g.cpu().numpy(), J.cpu().numpy()
    uh, lh, Ah = up.cpu().numpy(), lo.cpu().numpy(), A.cpu().numpy()
    Qs = {}
    for i, (T, P) in enumerate(zip(Ts, Ps)):
        if T not in Qs:
            Qs[T] = O.partition_function(Eh, gh, T)
        ls = O.make_lineset(Eh, gh, uh, lh, Ah, T, P, cfg.mass_amu, J=Jh, broad_table=(gt.numpy(), nt.numpy()),
                            Q=Qs[T])
        ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=1)
        assert_parity(got[i], ref, 1e-5, what=f"C5 shape T={T:.0f} P={P:.2e}")
        if P >= 100.0:
            klo, khi = O.window(ls.nu, cfg.nu_a, cfg.dnu, cfg.n_points, cfg.cutoff)
            live = khi >= klo
            assert ls.gamma[live].min() >= 30 * cfg.dnu
            areas = _truncated_voigt_areas(ls, klo[live].astype(np.float64), khi[live].astype(np.float64),
                                           cfg.nu_a, cfg.dnu)
            expect = math.fsum(ls.I[live] * areas)
            area = cfg.dnu * math.fsum(got[i])
            log(f"  sum rule T={T:.0f} P={P:.0f}: dnu sum sigma {area:.9e}, sum I a {expect:.9e}, "
                f"rel {abs(area - expect) / expect:.2e}")
            assert abs(area - expect) <= 1e-5 * expect
    klo, khi = O.window(ls.nu, cfg.nu_a, cfg.dnu, cfg.n_points, cfg.cutoff)
    assert kept == int(np.count_nonzero(khi >= klo))
