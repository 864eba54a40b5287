"""Emission and state reductions: FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references ("the paper" = ExoCross, arXiv:1801.09803):
  Eq. for the emissivity (Sec. "Intensities and partition function"), Sec. "Radiative
  lifetime", Sec. "Cooling function", and the specific heat from the moments of the
  partition function (Sec. "Partition function", Eq. for C_p).

Readings of the paper:
  * Emissivity: the emitting state is the transition's upper state (the printed formula
    labels it i with A_fi), and the stated unit (erg/s/sr/molecule) needs the factor hc:
        eps = h c g_up A nu exp(-c2 E_up/T) / (4 pi Q(T)).
    Emission cross sections are sum eps f(nu_k - nu) with the absorption profiles.
  * Cooling function: W(T) = sum over transitions of eps (as printed: 1/(4 pi Q) sum A hc
    nu g_up exp(-c2 E_up/T)), erg/s/sr/molecule.
  * Lifetime: tau = 1 / sum of A over the transitions leaving a state; a state with none
    has an infinite lifetime.
  * Specific heat: Q' = T dQ/dT = sum g x e^-x and the second moment Q'' = sum g x^2 e^-x
    (x = c2 E/T; the printed "T^2 d^2Q/dT^2" is this moment minus 2Q'), and
        C_p = R [Q''/Q - (Q'/Q)^2] + 5R/2
    (the printed formula lacks the square; the internal-state heat capacity plus the
    ideal gas's translational 3R/2 and R), J/K/mol.
"""
from __future__ import annotations

import math

import numpy as np

from .constants import C2, C_LIGHT_CGS, H_PLANCK, K_BOLTZMANN
from .xsec import partition_function

__all__ = ["emissivities", "cooling_function", "lifetimes", "partition_moments", "heat_capacity",
           "H_PLANCK_CGS", "R_GAS"]

H_PLANCK_CGS = H_PLANCK * 1e7                  # erg s
R_GAS = K_BOLTZMANN * 6.02214076e23             # J/(K mol), exact SI


def emissivities(E, g, upper, lower, A, T: float, Q=None, index_base: int = 0):
    """eps = h c g_up A nu exp(-c2 E_up/T) / (4 pi Q(T)) (erg/s/sr/molecule)."""
    E = np.asarray(E, np.float64)
    gg = np.asarray(g, np.float64)
    up = np.asarray(upper, np.int64) - index_base
    lo = np.asarray(lower, np.int64) - index_base
    nu = E[up] - E[lo]
    if Q is None:
        Q = partition_function(E, g, T)
    A = np.asarray(A, np.float64)
    return H_PLANCK_CGS * C_LIGHT_CGS * gg[up] * A * nu * np.exp(-C2 * E[up] / T) / (4.0 * math.pi * Q)


def cooling_function(E, g, upper, lower, A, T: float, index_base: int = 0) -> float:
    """W(T): the sum of the emissivities of all transitions (correctly rounded sum)."""
    return math.fsum(emissivities(E, g, upper, lower, A, T, index_base=index_base))


def lifetimes(n_states: int, upper, A, index_base: int = 0):
    """tau_i = 1 / sum_f A (s); states without transitions get inf."""
    up = np.asarray(upper, np.int64) - index_base
    tot = np.zeros(n_states)
    order = np.argsort(up, kind="stable")
    su, sa = up[order], np.asarray(A, np.float64)[order]
    if su.size:
        starts = np.flatnonzero(np.r_[True, su[1:] != su[:-1]])
        ends = np.r_[starts[1:], su.size]
        for s0, e0 in zip(starts, ends):
            tot[su[s0]] = math.fsum(sa[s0:e0])
    with np.errstate(divide="ignore"):
        return np.where(tot > 0, 1.0 / np.where(tot > 0, tot, 1.0), np.inf)


def partition_moments(E, g, T: float):
    """(Q, Q' = sum g x e^-x, Q'' = sum g x^2 e^-x), x = c2 E/T, each correctly rounded."""
    E = np.asarray(E, np.float64)
    gg = np.asarray(g, np.float64)
    x = C2 * E / T
    w = gg * np.exp(-x)
    return math.fsum(w), math.fsum(w * x), math.fsum(w * x * x)


def heat_capacity(E, g, T: float) -> float:
    """C_p = R [Q''/Q - (Q'/Q)^2] + 5R/2 (J/K/mol)."""
    Q, Q1, Q2 = partition_moments(E, g, T)
    return R_GAS * (Q2 / Q - (Q1 / Q) ** 2) + 2.5 * R_GAS
