"""FP64 CPU oracle: intensities, profiles, sampled cross sections, adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy/SciPy in
double precision; no blocking, fusion or reordering beyond the definitions.

Paper references ("the paper" = ExoCross, arXiv:1801.09803):
  Eq. 1   absorption line intensity            (Sec. "Intensities and partition function")
  Eq. 2   partition function                   (same section)
  Eq. 6-8 cross section = intensity x unit-area profile  (Sec. "Cross sections")
  Eq. 9   equidistant grid, both ends included (Sec. "Grids")
  Eq. 15  Gaussian profile, Eq. 16 Doppler HWHM, Eq. 17 Lorentzian, Eq. 18 its HWHM,
  Eq. 19  Voigt = Doppler (x) Lorentz          (Sec. "Line profiles")
  Sampling method: sigma(nu_k) = I f(nu_k)     (Sec. "Standard line profiles and sampling method")
  Eq. 27-29 binned Lorentzian, Eq. 30-31 Gauss-Hermite binned Voigt (Sec. "Binned Voigt profile")
  Cut-off of the line wings (25 cm^-1 default) (Sec. "Off-set")

Readings where the paper is silent or garbled:
  * Voigt normalisation: Eq. 19/20 as printed carry ln2 where sqrt(ln2) belongs and
    an unscaled gamma; the text says the Voigt is the convolution of the Doppler and
    Lorentz profiles, which (both unit-area) gives
        f_V(D) = sqrt(ln2/pi)/alpha_D * Re w((D + i gamma) sqrt(ln2)/alpha_D).
  * Eq. 29 lacks the minus sign between nu_k and nu_fi; Eq. 30 has alpha_D^2 and
    unshifted nodes; Eq. 31 omits the node shift.  The reading: Gauss-Hermite nodes
    t_j shift the Lorentzian by delta_j = alpha_D t_j / sqrt(ln2), which reproduces
    Eq. 31's prefactor I/(pi^(3/2) dnu) exactly.
  * Window: grid points k with ceil((nu - cut - nu_A)/dnu) <= k <= floor((nu + cut - nu_A)/dnu)
    (inclusive, evaluated in double), clipped to the grid; no pedestal subtraction and
    no renormalisation of the truncated profile; lines centred off-grid whose window
    overlaps the grid are included.
  * Stimulated emission as -expm1(-c2 nu / T).
"""
from __future__ import annotations

import math
import os
from typing import Optional

import numpy as np
from numpy.polynomial.hermite import hermgauss
from scipy.special import wofz

from .constants import AMU_KG, C2, C_LIGHT_CGS, C_LIGHT_SI, K_BOLTZMANN, LN2, P0_REF, T0_REF

__all__ = [
    "grid", "partition_function", "partition_function_dT", "line_centres", "intensities",
    "doppler_hwhm", "lorentz_hwhm", "gauss_profile", "lorentz_profile", "voigt_profile",
    "gh_sampled_profile", "gh_binned_profile", "window", "LineSet", "make_lineset",
    "cross_section", "cross_section_at", "error_metrics", "voigt_adjoint", "faddeeva_derivative",
    "PROFILES",
]

PROFILES = ("doppler", "gauss_fixed", "lorentz", "voigt", "gh_binned", "gh_sampled", "doppler_binned",
            "lorentz_binned")


# ----------------------------------------------------------------------------- grid
def grid(nu_a: float, nu_b: float, n_points: int):
    """Eq. 9: N points including both ends, dnu = (nu_B - nu_A)/(N - 1);
    nu_k = nu_A + k dnu (never accumulated)."""
    if n_points < 2 or not nu_b > nu_a:
        raise ValueError("grid needs n_points >= 2 and nu_b > nu_a")
    dnu = (nu_b - nu_a) / (n_points - 1)
    k = np.arange(n_points, dtype=np.float64)
    return nu_a + k * dnu, dnu


# ------------------------------------------------------------------- states / lines
def partition_function(E, g, T: float) -> float:
    """Eq. 2: Q(T) = sum_n g_n exp(-c2 E_n / T), summed with math.fsum."""
    E = np.asarray(E, np.float64)
    g = np.asarray(g, np.float64)
    return math.fsum(g * np.exp(-C2 * E / T))


def partition_function_dT(E, g, T: float) -> float:
    """dQ/dT = sum_n g_n (c2 E_n / T^2) exp(-c2 E_n / T)  (derivative of Eq. 2)."""
    E = np.asarray(E, np.float64)
    g = np.asarray(g, np.float64)
    return math.fsum(g * (C2 * E / (T * T)) * np.exp(-C2 * E / T))


def line_centres(E, upper, lower, index_base: int = 0):
    """Transition wavenumber nu_fi = E_f - E_i (upper minus lower; Eq. 1 with the
    f <- i convention of the stick-spectrum table)."""
    E = np.asarray(E, np.float64)
    up = np.asarray(upper, np.int64) - index_base
    lo = np.asarray(lower, np.int64) - index_base
    return E[up] - E[lo]


def intensities(E, g, upper, lower, A, T: float, Q: Optional[float] = None, index_base: int = 0):
    """Eq. 1: I = g_f A /(8 pi c nu^2) exp(-c2 E_i/T) (1 - exp(-c2 nu/T)) / Q(T),
    in cm/molecule (c in cm/s, nu in cm^-1)."""
    E = np.asarray(E, np.float64)
    gg = np.asarray(g, np.float64)
    up = np.asarray(upper, np.int64) - index_base
    lo = np.asarray(lower, np.int64) - index_base
    nu = E[up] - E[lo]
    if np.any(nu <= 0):
        raise ValueError("transition with nu <= 0")
    if Q is None:
        Q = partition_function(E, g, T)
    A = np.asarray(A, np.float64)
    stim = -np.expm1(-C2 * nu / T)
    return gg[up] * A / (8.0 * math.pi * C_LIGHT_CGS * nu * nu) * np.exp(-C2 * E[lo] / T) * stim / Q


def doppler_hwhm(nu, T: float, mass_amu: float):
    """Eq. 16: alpha_D = sqrt(2 k_B T ln2 / m) nu / c   (SI inside the root)."""
    return np.sqrt(2.0 * K_BOLTZMANN * T * LN2 / (mass_amu * AMU_KG)) * np.asarray(nu, np.float64) / C_LIGHT_SI


def lorentz_hwhm(gamma_ref, n_exp, T: float, P: float, T0: float = T0_REF, P0: float = P0_REF):
    """Eq. 18: gamma_L = gamma_ref (T0/T)^n P/P0."""
    return np.asarray(gamma_ref, np.float64) * (T0 / T) ** np.asarray(n_exp, np.float64) * (P / P0)


# --------------------------------------------------------------------- profiles
def gauss_profile(delta, alpha):
    """Eq. 15: sqrt(ln2/pi)/alpha exp(-delta^2 ln2/alpha^2), alpha = HWHM."""
    delta = np.asarray(delta, np.float64)
    return math.sqrt(LN2 / math.pi) / alpha * np.exp(-delta * delta * LN2 / (alpha * alpha))


def lorentz_profile(delta, gamma):
    """Eq. 17: gamma / (pi (delta^2 + gamma^2)), gamma = HWHM."""
    delta = np.asarray(delta, np.float64)
    return gamma / (math.pi * (delta * delta + gamma * gamma))


def voigt_profile(delta, alpha_d, gamma):
    """Convolution of Eq. 15 (Doppler HWHM alpha_d) and Eq. 17 (HWHM gamma), via the
    Faddeeva function: sqrt(ln2/pi)/alpha_d Re w((delta + i gamma) sqrt(ln2)/alpha_d)."""
    delta = np.asarray(delta, np.float64)
    s = math.sqrt(LN2) / np.asarray(alpha_d, np.float64)
    z = delta * s + 1j * (np.asarray(gamma, np.float64) * s)
    return math.sqrt(LN2 / math.pi) / np.asarray(alpha_d, np.float64) * wofz(z).real


def _gh_nodes(n_gh: int):
    t, w = hermgauss(n_gh)   # physicists' nodes/weights, sum w = sqrt(pi)
    return t, w


def gh_sampled_profile(delta, alpha_d, gamma, n_gh: int = 30):
    """Gauss-Hermite discretisation of the Voigt convolution (Sec. "Binned Voigt
    profile", Eq. 30 as read): (1/sqrt(pi)) sum_j w_j L(delta - delta_j; gamma),
    delta_j = alpha_d t_j / sqrt(ln2)."""
    delta = np.asarray(delta, np.float64)
    t, w = _gh_nodes(n_gh)
    out = np.zeros(np.broadcast(delta, alpha_d, gamma).shape)
    for tj, wj in zip(t, w):
        dj = np.asarray(alpha_d, np.float64) * tj / math.sqrt(LN2)
        out = out + wj * lorentz_profile(delta - dj, gamma)
    return out / math.sqrt(math.pi)


def gh_binned_profile(delta, alpha_d, gamma, dnu: float, n_gh: int = 30):
    """Bin-averaged Gauss-Hermite Voigt (Eq. 31 as read): per unit intensity
    1/(pi^(3/2) dnu) sum_j w_j [atan(y_j+) - atan(y_j-)],
    y_j+- = (delta - delta_j +- dnu/2)/gamma  (Eq. 29 with the minus sign restored).
    The difference of arctangents is evaluated as atan2(y+ - y-, 1 + y+ y-), equal to it
    for y+ > y-.  gamma == 0 takes the step-function limit (a 30-point histogram)."""
    delta = np.asarray(delta, np.float64)
    t, w = _gh_nodes(n_gh)
    gamma = np.broadcast_to(np.asarray(gamma, np.float64), np.broadcast(delta, alpha_d, gamma).shape)
    alpha_d = np.broadcast_to(np.asarray(alpha_d, np.float64), gamma.shape)
    out = np.zeros(gamma.shape)
    pos = gamma > 0
    for tj, wj in zip(t, w):
        dj = alpha_d * tj / math.sqrt(LN2)
        lo = delta - dj - 0.5 * dnu
        hi = delta - dj + 0.5 * dnu
        g = np.where(pos, gamma, 1.0)
        a, b = hi / g, lo / g
        # atan(a) - atan(b) for a > b, as atan2(a - b, 1 + a b) (an exact identity that
        # avoids cancelling two arctangents near +-pi/2 in the far wings)
        term = np.arctan2(dnu / g, 1.0 + a * b)
        # gamma -> 0: atan(+-inf) steps; half weight when an edge sits on the node
        step = (np.sign(hi) - np.sign(lo)) * (math.pi / 2.0)
        out = out + wj * np.where(pos, term, step)
    return out / (math.pi ** 1.5 * dnu)


# ----------------------------------------------------------------------- windows
def window(nu, nu_a: float, dnu: float, n_points: int, cutoff: float):
    """Grid indices covered by each line's cut-off window (Sec. "Off-set", reading:
    inclusive bounds computed in double), clipped to [0, n_points-1].  Empty windows
    come back with k_lo > k_hi."""
    nu = np.asarray(nu, np.float64)
    klo = np.ceil((nu - cutoff - nu_a) / dnu)
    khi = np.floor((nu + cutoff - nu_a) / dnu)
    klo = np.maximum(klo, 0.0)
    khi = np.minimum(khi, float(n_points - 1))
    return klo.astype(np.int64), khi.astype(np.int64)


# ------------------------------------------------------------------ line sets
class LineSet:
    """Per-line quantities at one (T, P): centre, intensity, widths."""

    def __init__(self, nu, I, alpha_d, gamma, E_low=None, gamma_ref=None, n_exp=None):
        self.nu = np.asarray(nu, np.float64)
        self.I = np.asarray(I, np.float64)
        self.alpha_d = np.asarray(alpha_d, np.float64)
        self.gamma = np.asarray(gamma, np.float64)
        self.E_low = E_low
        self.gamma_ref = gamma_ref
        self.n_exp = n_exp

    def __len__(self):
        return self.nu.size


def make_lineset(E, g, upper, lower, A, T: float, P: float, mass_amu: float,
                 gamma_ref=None, n_exp=None, J=None, broad_table=None,
                 T0: float = T0_REF, P0: float = P0_REF, Q: Optional[float] = None,
                 index_base: int = 0, gamma_const=None, n_const=None) -> LineSet:
    """Evaluate Eq. 1, 16 and 18 for every transition.

    Broadening: per-line arrays (gamma_ref, n_exp), or an a0 table indexed by the
    lower state's J (Sec. "Broadening parameters"), or constants."""
    E = np.asarray(E, np.float64)
    up = np.asarray(upper, np.int64) - index_base
    lo = np.asarray(lower, np.int64) - index_base
    nu = E[up] - E[lo]
    I = intensities(E, g, upper, lower, A, T, Q=Q, index_base=index_base)
    aD = doppler_hwhm(nu, T, mass_amu)
    if broad_table is not None:
        gt, nt = (np.asarray(a, np.float64) for a in broad_table)
        jl = np.asarray(J, np.int64)[lo]
        jl = np.minimum(jl, gt.size - 1)
        gref, nex = gt[jl], nt[jl]
    elif gamma_ref is not None:
        gref = np.asarray(gamma_ref, np.float64)
        nex = np.asarray(n_exp, np.float64)
    else:
        gref = np.full(nu.shape, float(gamma_const))
        nex = np.full(nu.shape, float(n_const))
    gam = lorentz_hwhm(gref, nex, T, P, T0, P0)
    return LineSet(nu, I, aD, gam, E_low=E[lo], gamma_ref=gref, n_exp=nex)


def _profile_values(kind, delta, aD, gam, dnu, alpha_fixed, n_gh):
    if kind == "voigt":
        return voigt_profile(delta, aD, gam)
    if kind == "doppler":
        return gauss_profile(delta, aD)
    if kind == "gauss_fixed":
        return gauss_profile(delta, alpha_fixed)
    if kind == "lorentz":
        return lorentz_profile(delta, gam)
    if kind == "gh_sampled":
        return gh_sampled_profile(delta, aD, gam, n_gh)
    if kind == "gh_binned":
        return gh_binned_profile(delta, aD, gam, dnu, n_gh)
    if kind == "doppler_binned":
        from .binned import gauss_binned_profile
        return gauss_binned_profile(delta, aD, dnu)
    if kind == "lorentz_binned":
        from .binned import lorentz_binned_profile
        return lorentz_binned_profile(delta, gam, dnu)
    raise ValueError(kind)


# Workers get the line arrays through fork (module globals), not pickling.
_WORK = {}


def _block_sigma(args):
    i0, i1 = args
    w = _WORK
    ls, nu_a, dnu, n_points, cut, kind = w["ls"], w["nu_a"], w["dnu"], w["n"], w["cut"], w["kind"]
    sig = np.zeros(n_points)
    step = w["block"]
    for b0 in range(i0, i1, step):
        b1 = min(b0 + step, i1)
        nu = ls.nu[b0:b1]
        klo, khi = window(nu, nu_a, dnu, n_points, cut)
        cnt = np.maximum(khi - klo + 1, 0)
        tot = int(cnt.sum())
        if tot == 0:
            continue
        owner = np.repeat(np.arange(b1 - b0), cnt)
        first = np.cumsum(cnt) - cnt
        k = klo[owner] + (np.arange(tot) - first[owner])
        delta = (nu_a + k.astype(np.float64) * dnu) - nu[owner]
        f = _profile_values(kind, delta, ls.alpha_d[b0:b1][owner], ls.gamma[b0:b1][owner],
                            dnu, w["alpha_fixed"], w["n_gh"])
        sig += np.bincount(k, weights=ls.I[b0:b1][owner] * f, minlength=n_points)
    return sig


def _default_workers():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def cross_section(ls: LineSet, nu_a: float, nu_b: float, n_points: int, cutoff: float = 25.0,
                  profile: str = "voigt", alpha_fixed: float = 0.0, n_gh: int = 30,
                  workers: Optional[int] = None, block: Optional[int] = None):
    """Sampled cross section sigma_k = sum_lines I f(nu_k - nu) over each line's
    window (Eq. 7 and the sampling method; the Gauss-Hermite binned variant is the
    bin average of Eq. 31).  Lines are split over worker processes, each with its
    own grid; the grids are added at the end."""
    _, dnu = grid(nu_a, nu_b, n_points)
    n = len(ls)
    if block is None:
        per_line = 2.0 * cutoff / dnu + 1.0
        mult = n_gh if profile in ("gh_binned", "gh_sampled") else 1
        block = max(1, int(4e6 / (per_line * mult)))
    _WORK.clear()
    _WORK.update(ls=ls, nu_a=nu_a, dnu=dnu, n=n_points, cut=cutoff, kind=profile,
                 alpha_fixed=alpha_fixed, n_gh=n_gh, block=block)
    nw = _default_workers() if workers is None else workers
    nw = max(1, min(nw, (n + block - 1) // block))
    if nw == 1:
        return _block_sigma((0, n))
    import multiprocessing as mp
    bounds = np.linspace(0, n, nw + 1).astype(np.int64)
    ctx = mp.get_context("fork")
    with ctx.Pool(nw) as pool:
        parts = pool.map(_block_sigma, [(int(bounds[i]), int(bounds[i + 1])) for i in range(nw)])
    out = np.zeros(n_points)
    for p in parts:
        out += p
    return out


def cross_section_at(ls: LineSet, k_points, nu_a: float, nu_b: float, n_points: int,
                     cutoff: float = 25.0, profile: str = "voigt", alpha_fixed: float = 0.0,
                     n_gh: int = 30):
    """sigma at selected grid indices only, summing every line whose window holds
    the point (same window rule as ``cross_section``)."""
    _, dnu = grid(nu_a, nu_b, n_points)
    klo, khi = window(ls.nu, nu_a, dnu, n_points, cutoff)
    out = np.zeros(len(k_points))
    for i, k in enumerate(np.asarray(k_points, np.int64)):
        m = (klo <= k) & (k <= khi)
        if not np.any(m):
            continue
        delta = (nu_a + float(k) * dnu) - ls.nu[m]
        f = _profile_values(profile, delta, ls.alpha_d[m], ls.gamma[m], dnu, alpha_fixed, n_gh)
        out[i] = math.fsum(ls.I[m] * f)
    return out


# ----------------------------------------------------------------- error metrics
def error_metrics(sig_hat, sig, rel_floor: float = 1e-6):
    """Max relative error over points with sigma > rel_floor * max(sigma), and the
    relative error of the integrated area (sum times dnu; dnu cancels)."""
    sig_hat = np.asarray(sig_hat, np.float64)
    sig = np.asarray(sig, np.float64)
    if sig.size == 0 or not np.any(sig > 0):
        return dict(max_rel=float(np.max(np.abs(sig_hat))) if sig_hat.size else 0.0, area_rel=0.0, n_checked=0)
    m = sig > rel_floor * sig.max()
    rel = np.abs(sig_hat[m] - sig[m]) / sig[m]
    a_ref = math.fsum(sig)
    area = abs(math.fsum(sig_hat) - a_ref) / a_ref
    return dict(max_rel=float(rel.max()), area_rel=float(area), n_checked=int(m.sum()))


# ------------------------------------------------------------------------ adjoint
def faddeeva_derivative(z):
    """w'(z) for Im z >= 0.  |z| < 30: the identity w' = -2 z w + 2i/sqrt(pi) (loses at
    most ~3.3 digits to cancellation there); |z| >= 30: the asymptotic series
    w'(z) = -(i/sqrt(pi)) sum_k (2k+1)!! / (2^k z^(2k+2)), k = 0..14 (Abramowitz & Stegun
    7.1.23 differentiated; the omitted terms are below 1e-22 relative), where the identity
    would cancel ~log10|z|^2 digits."""
    z = np.asarray(z, complex)
    out = np.empty(z.shape, complex)
    big = np.abs(z) >= 30.0
    zs = z[~big]
    out[~big] = -2.0 * zs * wofz(zs) + 2j / math.sqrt(math.pi)
    zb = z[big]
    if zb.size:
        inv2 = 1.0 / (zb * zb)
        term = inv2.copy()          # k = 0: 1/z^2
        acc = term.copy()
        for k in range(1, 15):
            term = term * (2 * k + 1) / 2.0 * inv2
            acc = acc + term
        out[big] = -1j / math.sqrt(math.pi) * acc
    return out


def voigt_adjoint(E, g, upper, lower, A, gamma_ref, n_exp, T: float, P: float, mass_amu: float,
                  nu_a: float, nu_b: float, n_points: int, gbar, cutoff: float = 25.0,
                  T0: float = T0_REF, P0: float = P0_REF, index_base: int = 0):
    """Gradients of L(sigma) given gbar = dL/dsigma on the grid, for the sampled
    Voigt cross section (this extension has no counterpart in the paper; it follows
    from differentiating Eq. 1, 2, 16, 18 and the Voigt profile).

    With z = x + iy, x = sqrt(ln2) D/alpha_D, y = sqrt(ln2) gamma/alpha_D,
    W = w(z), W' = dw/dz (faddeeva_derivative), N = sqrt(ln2/pi)/alpha_D, phi = N Re W:
        dphi/dgamma   = -N (sqrt(ln2)/alpha_D) Im W'
        dphi/dalpha_D = -(N/alpha_D) (Re W + Re(z W'))
    Per line: R0 = sum gbar phi, Rg = sum gbar dphi/dgamma, Ra = sum gbar dphi/dalpha.
    Returns dict with dL/dT, dL/dP and per-line dL/dlnA, dL/dgamma_ref, dL/dn.
    """
    E = np.asarray(E, np.float64)
    Q = partition_function(E, g, T)
    dQ = partition_function_dT(E, g, T)
    ls = make_lineset(E, g, upper, lower, A, T, P, mass_amu, gamma_ref=gamma_ref, n_exp=n_exp,
                      T0=T0, P0=P0, Q=Q, index_base=index_base)
    _, dnu = grid(nu_a, nu_b, n_points)
    gbar = np.asarray(gbar, np.float64)
    klo, khi = window(ls.nu, nu_a, dnu, n_points, cutoff)
    n = len(ls)
    R0 = np.zeros(n)
    Rg = np.zeros(n)
    Ra = np.zeros(n)
    sq = math.sqrt(LN2)
    for i in range(n):
        if klo[i] > khi[i]:
            continue
        k = np.arange(klo[i], khi[i] + 1)
        D = (nu_a + k.astype(np.float64) * dnu) - ls.nu[i]
        aD = ls.alpha_d[i]
        s = sq / aD
        z = D * s + 1j * ls.gamma[i] * s
        W = wofz(z)
        Wp = faddeeva_derivative(z)
        Nrm = math.sqrt(LN2 / math.pi) / aD
        phi = Nrm * W.real
        dphi_dg = -Nrm * s * Wp.imag
        dphi_da = -(Nrm / aD) * (W.real + (z * Wp).real)
        gb = gbar[k]
        R0[i] = math.fsum(gb * phi)
        Rg[i] = math.fsum(gb * dphi_dg)
        Ra[i] = math.fsum(gb * dphi_da)
    S = ls.I
    up = np.asarray(upper, np.int64) - index_base
    lo = np.asarray(lower, np.int64) - index_base
    El = E[lo]
    nu = ls.nu
    xnu = C2 * nu / T
    tau = C2 * El / (T * T) - (C2 * nu / (T * T)) / np.expm1(xnu) - dQ / Q
    gam = ls.gamma
    d_lnA = S * R0
    d_gref = S * Rg * gam / ls.gamma_ref
    d_n = S * Rg * gam * math.log(T0 / T)
    d_P = math.fsum(S * Rg * gam / P) if P > 0 else math.fsum(S * Rg * ls.gamma_ref * (T0 / T) ** ls.n_exp / P0)
    d_T = math.fsum(S * (tau * R0 + Ra * ls.alpha_d / (2.0 * T) - Rg * ls.n_exp * gam / T))
    return dict(dT=d_T, dP=d_P, dlnA=d_lnA, dgamma_ref=d_gref, dn=d_n, R0=R0, Rg=Rg, Ra=Ra)
