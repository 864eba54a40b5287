"""Intensity thresholds: FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper reference ("the paper" = ExoCross, arXiv:1801.09803), Sec. "Intensity thresholds":
a constant threshold in cm/molecule, or the dynamic HITRAN cut-off
    I_cut(nu) = I_crit (nu/nu_crit) tanh(c2 nu / (2 T))   for nu <= nu_crit,
    I_cut(nu) = I_crit                                     for nu >  nu_crit,
with nu_crit = 2000 cm^-1 and I_crit = 1e-29 cm/molecule by default.

Readings of the paper:
  * A line is kept when its intensity (Eq. 1 at the call's T) is >= the threshold at its
    own wavenumber; dropped lines contribute nothing.
  * The formula is used as printed (its two branches meet only to tanh(c2 nu_crit/(2T))).
"""
from __future__ import annotations

import numpy as np

from .constants import C2
from .xsec import LineSet

__all__ = ["intensity_cutoff", "apply_threshold", "NU_CRIT_HITRAN", "I_CRIT_HITRAN"]

NU_CRIT_HITRAN = 2000.0    # cm^-1
I_CRIT_HITRAN = 1e-29      # cm/molecule


def intensity_cutoff(nu, T: float, mode: str, i_crit: float = I_CRIT_HITRAN, nu_crit: float = NU_CRIT_HITRAN):
    """Threshold at each line's wavenumber: mode "constant" (i_crit everywhere) or "hitran"."""
    nu = np.asarray(nu, np.float64)
    if mode == "constant":
        return np.full(nu.shape, float(i_crit))
    if mode != "hitran":
        raise ValueError(mode)
    low = i_crit * (nu / nu_crit) * np.tanh(C2 * nu / (2.0 * T))
    return np.where(nu <= nu_crit, low, i_crit)


def apply_threshold(ls: LineSet, T: float, mode: str, i_crit: float = I_CRIT_HITRAN,
                    nu_crit: float = NU_CRIT_HITRAN) -> LineSet:
    """The lines whose intensity reaches the threshold (I >= I_cut(nu))."""
    keep = ls.I >= intensity_cutoff(ls.nu, T, mode, i_crit, nu_crit)
    return LineSet(ls.nu[keep], ls.I[keep], ls.alpha_d[keep], ls.gamma[keep])
