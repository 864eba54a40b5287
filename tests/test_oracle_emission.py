"""Pins of the emission and state-reduction oracle (CPU only): Kirchhoff's law, two-level
and many-level closed forms of the cooling function and of the heat capacity (Schottky,
Einstein, rigid rotor), and brute-force lifetimes."""
import math

import numpy as np
import pytest

import oracle as O


def _planck_wavenumber(nu, T):
    # spectral radiance per unit wavenumber, erg s^-1 sr^-1 cm^-2 (cm^-1)^-1:
    # B = 2 h c^2 nu^3 / (exp(h c nu / k T) - 1), with h c / k = c2
    h = 6.62607015e-27
    c = 2.99792458e10
    return 2 * h * c * c * nu ** 3 / math.expm1(1.438776877503933802 * nu / T)


def test_emissivity_over_intensity_is_the_planck_function():
    # Kirchhoff's law for a line in LTE: eps / I = B_nu(T) (independent of A, g, E, Q)
    rng = np.random.default_rng(1)
    E = np.concatenate([[0.0], rng.uniform(100, 8000, 30)])
    g = rng.integers(1, 20, E.size)
    up = np.arange(1, E.size)
    lo = np.zeros(E.size - 1, np.int64)
    A = 10 ** rng.uniform(-3, 2, up.size)
    for T in (296.0, 1500.0, 5000.0):
        eps = O.emissivities(E, g, up, lo, A, T)
        I = O.intensities(E, g, up, lo, A, T)
        nu = E[up] - E[lo]
        ratio = eps / I
        ref = np.array([_planck_wavenumber(v, T) for v in nu])
        assert np.max(np.abs(ratio / ref - 1)) < 1e-12


def test_cooling_function_of_a_two_level_system():
    # W = h c nu A g_u exp(-c2 E_u/T) / (4 pi (g_l + g_u exp(-c2 E_u/T))); high-T limit
    # h c nu A g_u / (4 pi (g_l + g_u))
    Eu, gl, gu, A = 1234.5, 3, 5, 17.0
    hc = 6.62607015e-27 * 2.99792458e10
    for T in (100.0, 1000.0, 1e7):
        b = math.exp(-O.C2 * Eu / T)
        ref = hc * Eu * A * gu * b / (4 * math.pi * (gl + gu * b))
        got = O.cooling_function([0.0, Eu], [gl, gu], [1], [0], [A], T)
        assert abs(got - ref) < 1e-13 * ref
    assert abs(O.cooling_function([0.0, Eu], [gl, gu], [1], [0], [A], 1e9) / (hc * Eu * A * gu / (4 * math.pi * 8)) - 1) < 1e-5


def test_lifetimes_are_inverse_decay_rate_sums():
    rng = np.random.default_rng(3)
    n = 40
    up = rng.integers(0, n, 300)
    A = 10 ** rng.uniform(-2, 3, 300)
    tau = O.lifetimes(n, up, A)
    for i in range(n):
        s = sum(A[k] for k in range(300) if up[k] == i)
        if s == 0:
            assert math.isinf(tau[i])
        else:
            assert abs(tau[i] * s - 1) < 1e-14
    assert O.lifetimes(3, [1, 3], [2.0, 4.0], index_base=1)[0] == 0.5


def test_heat_capacity_closed_forms():
    R = O.R_GAS
    # two levels (Schottky anomaly): C_int = R x^2 g e^-x / (1 + g e^-x)^2 with g = g_u/g_l
    E1, T = 800.0, 600.0
    x = O.C2 * E1 / T
    gr = 3.0
    schottky = R * x * x * gr * math.exp(-x) / (1 + gr * math.exp(-x)) ** 2
    assert abs(O.heat_capacity([0.0, E1], [1, 3], T) - (schottky + 2.5 * R)) < 1e-12 * R
    # harmonic oscillator (Einstein function): C_int = R x^2 e^x / (e^x - 1)^2
    w = 1500.0
    E = w * np.arange(0, 400)
    for T in (300.0, 2000.0):
        x = O.C2 * w / T
        einstein = R * x * x * math.exp(x) / math.expm1(x) ** 2
        assert abs(O.heat_capacity(E, np.ones(E.size), T) - (einstein + 2.5 * R)) < 1e-10 * R
    # linear rigid rotor at high T: C_rot -> R (so C_p -> 7R/2)
    J = np.arange(0, 3000)
    E = 1.0 * J * (J + 1)
    cp = O.heat_capacity(E, 2 * J + 1, 3000.0)
    assert abs(cp / R - 3.5) < 1e-3
    # the moments are T dQ/dT and sum g x^2 e^-x: check the first against a finite difference
    Q, Q1, Q2 = O.partition_moments(E, 2 * J + 1, 500.0)
    h = 1e-3
    fd = 500.0 * (O.partition_function(E, 2 * J + 1, 500.0 + h) - O.partition_function(E, 2 * J + 1, 500.0 - h)) / (2 * h)
    assert abs(Q1 - fd) < 1e-7 * Q1
