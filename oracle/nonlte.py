"""Two-temperature (vibrational / rotational) non-LTE populations: FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper reference ("the paper" = ExoCross, arXiv:1801.09803): Sec. "Treating non-local
thermodynamic equilibrium (non-LTE)", the energy split E = E_vib + E_rot and the
population F(T_vib, T_rot) = exp(-c2 E_vib/T_vib) exp(-c2 E_rot/T_rot) used in place of
the Boltzmann factor in intensities and partition functions.

Readings of the paper:
  * E_vib of a state is the energy of the lowest state of its vibrational (vibronic)
    manifold (the paper's J = 0 / lowest allowed J state; along a rotational ladder that
    is the manifold's lowest energy), found from a per-state manifold label;
    E_rot = E - E_vib >= 0.
  * Absorption intensity: Eq. 1 with the populations per degeneracy replaced by F,
        I = g_up A / (8 pi c nu^2) (F_low - F_up) / Q(T_vib, T_rot),
    the population difference that Eq. 1's exp(-c2 E_low/T)(1 - exp(-c2 nu/T)) is in
    LTE (so T_vib = T_rot = T gives Eq. 1).  It is negative for an inverted transition.
  * Emissivity: h c g_up A nu F_up / (4 pi Q(T_vib, T_rot)).
  * Q(T_vib, T_rot) = sum g F.  Doppler and pressure widths use T_rot (the kinetic
    temperature taken equal to the rotational one).
"""
from __future__ import annotations

import math

import numpy as np

from .constants import C2, C_LIGHT_CGS
from .emission import H_PLANCK_CGS
from .xsec import LineSet, doppler_hwhm, lorentz_hwhm, T0_REF, P0_REF

__all__ = ["vibrational_energies", "nlte_populations", "partition_function_nlte", "intensities_nlte",
           "emissivities_nlte", "make_lineset_nlte"]


def vibrational_energies(E, labels):
    """E_vib per state: the lowest energy among the states with the same manifold label."""
    E = np.asarray(E, np.float64)
    lab = np.asarray(labels, np.int64)
    lowest = {}
    for e, l in zip(E.tolist(), lab.tolist()):
        if l not in lowest or e < lowest[l]:
            lowest[l] = e
    return np.array([lowest[l] for l in lab.tolist()], np.float64)


def nlte_populations(E, E_vib, T_vib: float, T_rot: float):
    """F = exp(-c2 E_vib/T_vib) exp(-c2 (E - E_vib)/T_rot) per state."""
    E = np.asarray(E, np.float64)
    Ev = np.asarray(E_vib, np.float64)
    return np.exp(-C2 * Ev / T_vib) * np.exp(-C2 * (E - Ev) / T_rot)


def partition_function_nlte(E, g, E_vib, T_vib: float, T_rot: float) -> float:
    """Q(T_vib, T_rot) = sum g F (correctly rounded sum)."""
    return math.fsum(np.asarray(g, np.float64) * nlte_populations(E, E_vib, T_vib, T_rot))


def _indices(upper, lower, index_base):
    return np.asarray(upper, np.int64) - index_base, np.asarray(lower, np.int64) - index_base


def intensities_nlte(E, g, E_vib, upper, lower, A, T_vib: float, T_rot: float, Q=None, index_base: int = 0):
    """I = g_up A/(8 pi c nu^2) (F_low - F_up)/Q, with F_low - F_up = F_low (1 - F_up/F_low)
    formed through expm1 of the log ratio (no cancellation for small nu)."""
    E = np.asarray(E, np.float64)
    Ev = np.asarray(E_vib, np.float64)
    up, lo = _indices(upper, lower, index_base)
    nu = E[up] - E[lo]
    if np.any(nu <= 0):
        raise ValueError("transition with nu <= 0")
    if Q is None:
        Q = partition_function_nlte(E, g, Ev, T_vib, T_rot)
    F_low = nlte_populations(E[lo], Ev[lo], T_vib, T_rot)
    # ln F_low - ln F_up = c2 [(Ev_up - Ev_low)/T_vib + (Er_up - Er_low)/T_rot]
    dEv = Ev[up] - Ev[lo]
    d = C2 * (dEv / T_vib + (nu - dEv) / T_rot)
    gg = np.asarray(g, np.float64)
    A = np.asarray(A, np.float64)
    return gg[up] * A / (8.0 * math.pi * C_LIGHT_CGS * nu * nu) * F_low * (-np.expm1(-d)) / Q


def emissivities_nlte(E, g, E_vib, upper, lower, A, T_vib: float, T_rot: float, Q=None, index_base: int = 0):
    """eps = h c g_up A nu F_up / (4 pi Q(T_vib, T_rot)) (erg/s/sr/molecule)."""
    E = np.asarray(E, np.float64)
    Ev = np.asarray(E_vib, np.float64)
    up, lo = _indices(upper, lower, index_base)
    nu = E[up] - E[lo]
    if Q is None:
        Q = partition_function_nlte(E, g, Ev, T_vib, T_rot)
    F_up = nlte_populations(E[up], Ev[up], T_vib, T_rot)
    gg = np.asarray(g, np.float64)
    return H_PLANCK_CGS * C_LIGHT_CGS * gg[up] * np.asarray(A, np.float64) * nu * F_up / (4.0 * math.pi * Q)


def make_lineset_nlte(E, g, E_vib, upper, lower, A, T_vib: float, T_rot: float, P: float, mass_amu: float,
                      gamma_ref, n_exp, T0: float = T0_REF, P0: float = P0_REF, emission: bool = False,
                      index_base: int = 0) -> LineSet:
    """Per-line centre, non-LTE intensity (or emissivity) and widths at T_rot."""
    E = np.asarray(E, np.float64)
    up, lo = _indices(upper, lower, index_base)
    nu = E[up] - E[lo]
    f = emissivities_nlte if emission else intensities_nlte
    I = f(E, g, E_vib, upper, lower, A, T_vib, T_rot, index_base=index_base)
    return LineSet(nu, I, doppler_hwhm(nu, T_rot, mass_amu), lorentz_hwhm(gamma_ref, n_exp, T_rot, P, T0, P0))
