"""Bin-averaged Gaussian and Lorentzian profiles and super-line histograms: FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references ("the paper" = ExoCross, arXiv:1801.09803):
  Sec. "Binned Gaussian profile with analytical integrals": the cross section averaged
      over the bin [nu_k - dnu/2, nu_k + dnu/2] of a Gaussian line, I/(2 dnu) times the
      difference of error functions at the scaled bin edges.
  Sec. "Binned Lorentzian profile with analytical integrals": the same average of a
      Lorentzian line, I/(pi dnu) times the difference of arctangents (Eq. 27-28; its
      definition of the scaled edges is printed without the minus sign between nu_k and
      nu_fi, restored here as for the Gauss-Hermite profiles).
  Sec. "Super-lines": per grid point the sum of the intensities of the lines falling
      into its bin (the "Bin" option).

Readings of the paper:
  * The binned profiles use the same cut-off windows as the sampled ones (bins whose
    centre lies within the cut-off of the line).
  * A difference of error functions is evaluated without cancellation in the tails as a
    difference of complementary error functions of same-signed arguments (an identity).
  * gamma = 0 in the binned Lorentzian takes the step-function limit: 1/dnu inside the
    bin, 1/(2 dnu) when the line sits on an edge.
  * Super-line bins are half-open, [nu_k - dnu/2, nu_k + dnu/2): the bin index of a line
    is floor((nu - nu_A)/dnu + 0.5) in double; lines whose bin is off the grid are not
    counted.  The histogram is returned as a cross section, the intensity sum divided by
    dnu, so that dnu sum_k sigma_k is the total intensity on the grid (multiply by dnu for
    the super-line intensities I_k).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

from .xsec import LineSet, grid

__all__ = ["erf_difference", "gauss_binned_profile", "lorentz_binned_profile", "stick_bins",
           "super_line_histogram"]


def erf_difference(a, b):
    """erf(b) - erf(a) for a <= b: erfc(a) - erfc(b) when both are >= 0, erfc(-b) -
    erfc(-a) when both are <= 0, erf(b) - erf(a) when the interval holds 0."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    pos = a >= 0.0
    neg = b <= 0.0
    out = erf(b) - erf(a)
    out = np.where(pos, erfc(a) - erfc(b), out)
    out = np.where(neg, erfc(-b) - erfc(-a), out)
    return out


def gauss_binned_profile(delta, alpha, dnu: float):
    """Per unit intensity: (1/(2 dnu)) [erf(x+) - erf(x-)], x+- = sqrt(ln2) (delta +- dnu/2)/alpha
    (Sec. "Binned Gaussian profile with analytical integrals"; alpha = HWHM)."""
    delta = np.asarray(delta, np.float64)
    s = math.sqrt(math.log(2.0)) / np.asarray(alpha, np.float64)
    return erf_difference(s * (delta - 0.5 * dnu), s * (delta + 0.5 * dnu)) / (2.0 * dnu)


def lorentz_binned_profile(delta, gamma, dnu: float):
    """Per unit intensity: (1/(pi dnu)) [atan(y+) - atan(y-)], y+- = (delta +- dnu/2)/gamma
    (Eq. 27-28 with the minus sign restored).  The difference of arctangents is taken as
    atan2(y+ - y-, 1 + y+ y-) (equal for y+ > y-); gamma = 0 gives the step limit."""
    delta = np.asarray(delta, np.float64)
    gamma = np.broadcast_to(np.asarray(gamma, np.float64), delta.shape)
    pos = gamma > 0
    g = np.where(pos, gamma, 1.0)
    hi = (delta + 0.5 * dnu) / g
    lo = (delta - 0.5 * dnu) / g
    term = np.arctan2(dnu / g, 1.0 + hi * lo)
    step = (np.sign(delta + 0.5 * dnu) - np.sign(delta - 0.5 * dnu)) * (math.pi / 2.0)
    return np.where(pos, term, step) / (math.pi * dnu)


def stick_bins(nu, nu_a: float, dnu: float):
    """Bin index of each line: floor((nu - nu_A)/dnu + 0.5) (half-open bins)."""
    return np.floor((np.asarray(nu, np.float64) - nu_a) / dnu + 0.5).astype(np.int64)


def super_line_histogram(ls: LineSet, nu_a: float, nu_b: float, n_points: int):
    """Sec. "Super-lines": sigma_k = (sum of I over the lines in bin k) / dnu."""
    _, dnu = grid(nu_a, nu_b, n_points)
    k = stick_bins(ls.nu, nu_a, dnu)
    on = (k >= 0) & (k < n_points)
    out = np.zeros(n_points)
    # per bin, a correctly rounded sum of its intensities
    order = np.argsort(k[on], kind="stable")
    kk = k[on][order]
    II = np.asarray(ls.I, np.float64)[on][order]
    if kk.size:
        starts = np.flatnonzero(np.r_[True, kk[1:] != kk[:-1]])
        ends = np.r_[starts[1:], kk.size]
        for s0, e0 in zip(starts, ends):
            out[kk[s0]] = math.fsum(II[s0:e0])
    return out / dnu
