"""Vectorized Voigt (V-V) and its area-normalised form (VVN): FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy/SciPy in double
precision; it reuses the pinned grid, window and profile functions of ``xsec``.

Paper references ("the paper" = ExoCross, arXiv:1801.09803):
  Sec. "Vectorized Voigt approximation": the profile is the Voigt profile within a
      radius R (4 cm^-1) of the line centre and, beyond it, a reference Voigt profile
      f_ref (the profile of a line centred at 1 cm^-1) times a continuity factor beta
      (Eq. for f^{V-V} and Eq. for beta); beta is usually set to 1.
  Sec. "Binned Vectorized Voigt with the line area preserved" (VVN): the line's
      profile values are summed and the intensity divided by that sum.

Readings where the paper is silent or ambiguous:
  * f_ref has the Doppler HWHM of Eq. 16 at nu = 1 cm^-1 (same T and mass) and the
    line's own Lorentz HWHM (the paper keeps one reference per set of broadening
    parameters; with per-line parameters every line forms its own set).  It is taken
    at the same offset from the line centre: the wing value at nu_k is
    beta f_ref(nu_k - nu_fi).
  * Core region: grid points with ceil((nu - R - nu_A)/dnu) <= k <= floor((nu + R -
    nu_A)/dnu), the inclusive double-precision rule of the cut-off window.
  * beta = f_V(R)/f_ref(R) when requested, else 1; beta = 1 where f_ref(R) = 0
    (gamma = 0: the wings are zero).
  * VVN: the profile values (core and beta-scaled wings) are summed over the whole
    cut-off window on the extended grid nu_A + k dnu (not clipped to the grid's ends,
    so the factor is a property of the line alone), and the intensity is divided by
    dnu times that sum: dnu sum_k sigma_k = I for a line whose window lies on the grid.
    A line whose sum is zero contributes nothing.
"""
from __future__ import annotations

import math
import os
from typing import Optional

import numpy as np

from .xsec import LineSet, doppler_hwhm, grid, voigt_profile

__all__ = [
    "vv_reference_hwhm", "vv_core_bounds", "window_unclipped", "vv_beta", "vv_profile_values",
    "vv_line_norm", "cross_section_vv", "cross_section_vv_at", "VV_RADIUS",
]

VV_RADIUS = 4.0   # cm^-1, the paper's distance from the centre beyond which f_ref is used


def vv_reference_hwhm(T: float, mass_amu: float) -> float:
    """Doppler HWHM of the reference line: Eq. 16 at nu = 1 cm^-1."""
    return float(doppler_hwhm(1.0, T, mass_amu))


def window_unclipped(nu, nu_a: float, dnu: float, cutoff: float):
    """Cut-off window of each line on the extended grid nu_A + k dnu (k any integer):
    ceil((nu - cut - nu_A)/dnu) <= k <= floor((nu + cut - nu_A)/dnu)."""
    nu = np.asarray(nu, np.float64)
    return (np.ceil((nu - cutoff - nu_a) / dnu).astype(np.int64),
            np.floor((nu + cutoff - nu_a) / dnu).astype(np.int64))


def vv_core_bounds(nu, nu_a: float, dnu: float, radius: float):
    """Grid indices within the V-V radius of each line (same rule as the window)."""
    return window_unclipped(nu, nu_a, dnu, radius)


def vv_beta(alpha_d, gamma, alpha_ref: float, radius: float, use_beta: bool):
    """Continuity factor (Eq. for beta): f_V(R; alpha_d, gamma) / f_ref(R; gamma),
    or 1 when not requested or when f_ref(R) = 0."""
    alpha_d = np.asarray(alpha_d, np.float64)
    gamma = np.asarray(gamma, np.float64)
    if not use_beta:
        return np.ones(np.broadcast(alpha_d, gamma).shape)
    num = voigt_profile(np.full(gamma.shape, radius), alpha_d, gamma)
    den = voigt_profile(np.full(gamma.shape, radius), alpha_ref, gamma)
    out = np.ones(gamma.shape)
    pos = den > 0
    out[pos] = num[pos] / den[pos]
    return out


def vv_profile_values(delta, core, alpha_d, gamma, alpha_ref: float, beta):
    """V-V profile (Eq. for f^{V-V}): the Voigt profile at core points, beta f_ref at
    the others.  All arguments are per point."""
    delta = np.asarray(delta, np.float64)
    core = np.asarray(core, bool)
    out = np.empty(delta.shape)
    out[core] = voigt_profile(delta[core], np.asarray(alpha_d)[core], np.asarray(gamma)[core])
    w = ~core
    out[w] = np.asarray(beta)[w] * voigt_profile(delta[w], alpha_ref, np.asarray(gamma)[w])
    return out


def _line_points(nu, klo, khi):
    cnt = np.maximum(khi - klo + 1, 0)
    tot = int(cnt.sum())
    owner = np.repeat(np.arange(nu.size), cnt)
    first = np.cumsum(cnt) - cnt
    k = klo[owner] + (np.arange(tot) - first[owner])
    return owner, k


def _vv_lines(ls: LineSet, i0: int, i1: int, nu_a: float, dnu: float, cutoff: float, radius: float,
              alpha_ref: float, use_beta: bool, normalise: bool, k_clip: Optional[tuple]):
    """Profile values of lines [i0, i1) over their windows, with the per-line intensity
    scale: returns (owner, k, f, scale)."""
    nu = ls.nu[i0:i1]
    aD = ls.alpha_d[i0:i1]
    gam = ls.gamma[i0:i1]
    klo, khi = window_unclipped(nu, nu_a, dnu, cutoff)
    if not normalise and k_clip is not None:
        klo = np.maximum(klo, k_clip[0])
        khi = np.minimum(khi, k_clip[1])
    owner, k = _line_points(nu, klo, khi)
    delta = (nu_a + k.astype(np.float64) * dnu) - nu[owner]
    kvlo, kvhi = vv_core_bounds(nu, nu_a, dnu, radius)
    core = (k >= kvlo[owner]) & (k <= kvhi[owner])
    beta = vv_beta(aD, gam, alpha_ref, radius, use_beta)
    f = vv_profile_values(delta, core, aD[owner], gam[owner], alpha_ref, beta[owner])
    scale = np.ones(nu.size)
    if normalise:
        tot = np.bincount(owner, weights=f, minlength=nu.size)
        scale = np.zeros(nu.size)
        pos = tot > 0
        scale[pos] = 1.0 / (dnu * tot[pos])
    return owner, k, f, scale


def vv_line_norm(ls: LineSet, nu_a: float, dnu: float, cutoff: float, T: float, mass_amu: float,
                 radius: float = VV_RADIUS, use_beta: bool = False):
    """Per-line VVN factor 1/(dnu sum_k f^{V-V}_k) over the unclipped window."""
    aref = vv_reference_hwhm(T, mass_amu)
    out = np.zeros(len(ls))
    step = 2000
    for b0 in range(0, len(ls), step):
        b1 = min(b0 + step, len(ls))
        out[b0:b1] = _vv_lines(ls, b0, b1, nu_a, dnu, cutoff, radius, aref, use_beta, True, None)[3]
    return out


_WORK = {}


def _vv_block(args):
    i0, i1 = args
    w = _WORK
    ls, n = w["ls"], w["n"]
    sig = np.zeros(n)
    for b0 in range(i0, i1, w["block"]):
        b1 = min(b0 + w["block"], i1)
        owner, k, f, scale = _vv_lines(ls, b0, b1, w["nu_a"], w["dnu"], w["cut"], w["R"], w["aref"],
                                       w["beta"], w["norm"], (0, n - 1))
        on = (k >= 0) & (k < n)
        if not np.any(on):
            continue
        wts = (ls.I[b0:b1] * scale)[owner[on]] * f[on]
        sig += np.bincount(k[on], weights=wts, minlength=n)
    return sig


def cross_section_vv(ls: LineSet, nu_a: float, nu_b: float, n_points: int, T: float, mass_amu: float,
                     cutoff: float = 25.0, radius: float = VV_RADIUS, use_beta: bool = False,
                     normalise: bool = False, workers: Optional[int] = None, block: Optional[int] = None):
    """Sampled V-V (normalise=False) or VVN (normalise=True) cross section:
    sigma_k = sum_lines I' f^{V-V}(nu_k - nu) over each line's window clipped to the
    grid, I' = I (V-V) or I / (dnu sum_window f^{V-V}) (VVN)."""
    _, dnu = grid(nu_a, nu_b, n_points)
    n = len(ls)
    if block is None:
        block = max(1, int(4e6 / (2.0 * cutoff / dnu + 1.0)))
    _WORK.clear()
    _WORK.update(ls=ls, nu_a=nu_a, dnu=dnu, n=n_points, cut=cutoff, R=radius,
                 aref=vv_reference_hwhm(T, mass_amu), beta=use_beta, norm=normalise, block=block)
    try:
        nw = len(os.sched_getaffinity(0)) if workers is None else workers
    except AttributeError:
        nw = os.cpu_count() or 1
    nw = max(1, min(nw, (n + block - 1) // block))
    if nw == 1:
        return _vv_block((0, n))
    import multiprocessing as mp
    bounds = np.linspace(0, n, nw + 1).astype(np.int64)
    with mp.get_context("fork").Pool(nw) as pool:
        parts = pool.map(_vv_block, [(int(bounds[i]), int(bounds[i + 1])) for i in range(nw)])
    out = np.zeros(n_points)
    for p in parts:
        out += p
    return out


def cross_section_vv_at(ls: LineSet, k_points, nu_a: float, nu_b: float, n_points: int, T: float,
                        mass_amu: float, cutoff: float = 25.0, radius: float = VV_RADIUS,
                        use_beta: bool = False):
    """V-V sigma (not normalised) at selected grid indices, summing every line whose
    window holds the point."""
    _, dnu = grid(nu_a, nu_b, n_points)
    aref = vv_reference_hwhm(T, mass_amu)
    klo, khi = window_unclipped(ls.nu, nu_a, dnu, cutoff)
    kvlo, kvhi = vv_core_bounds(ls.nu, nu_a, dnu, radius)
    out = np.zeros(len(k_points))
    for i, k in enumerate(np.asarray(k_points, np.int64)):
        m = (klo <= k) & (k <= khi)
        if not np.any(m):
            continue
        delta = (nu_a + float(k) * dnu) - ls.nu[m]
        core = (kvlo[m] <= k) & (k <= kvhi[m])
        beta = vv_beta(ls.alpha_d[m], ls.gamma[m], aref, radius, use_beta)
        f = vv_profile_values(delta, core, ls.alpha_d[m], ls.gamma[m], aref, beta)
        out[i] = math.fsum(ls.I[m] * f)
    return out
