"""Pins of the two-temperature non-LTE oracle (CPU only): the manifold energies by brute
force, the factorisation Q(T_vib, T_rot) = Q_vib(T_vib) Q_rot(T_rot) of a separable
vibration-rotation spectrum (harmonic oscillator in closed form), a two-level vibrational
band in closed form, the LTE limit, the sign of inverted transitions, and emission over
absorption as the Planck function at the transition's excitation temperature."""
import math

import numpy as np

import oracle as O

H_CGS = 6.62607015e-27
C_CGS = 2.99792458e10


def _planck(nu, T):
    return 2 * H_CGS * C_CGS * C_CGS * nu ** 3 / math.expm1(1.438776877503933802 * nu / T)


def test_vibrational_energies_are_manifold_minima():
    E = [5.0, 1.0, 7.0, 3.0, 2.0, 9.0]
    lab = [0, 0, 1, 1, 2, 1]
    assert list(O.vibrational_energies(E, lab)) == [1.0, 1.0, 3.0, 3.0, 2.0, 3.0]


def _ladder(omega=1000.0, B=2.0, n_v=60, n_J=120):
    v, J = np.meshgrid(np.arange(n_v), np.arange(n_J), indexing="ij")
    E = (omega * v + B * J * (J + 1)).ravel().astype(np.float64)
    return E, (2 * J + 1).ravel(), v.ravel(), J.ravel()


def test_separable_spectrum_factorises():
    omega, B = 1000.0, 2.0
    E, g, v, J = _ladder(omega, B)
    Ev = O.vibrational_energies(E, v)
    assert np.array_equal(Ev, omega * v)
    Jr = np.arange(120)
    for Tv, Tr in [(3000.0, 300.0), (300.0, 3000.0), (1500.0, 1500.0)]:
        q_vib = 1.0 / -math.expm1(-O.C2 * omega / Tv)         # harmonic oscillator, closed form
        q_rot = math.fsum((2 * Jr + 1) * np.exp(-O.C2 * B * Jr * (Jr + 1) / Tr))
        q = O.partition_function_nlte(E, g, Ev, Tv, Tr)
        assert abs(q / (q_vib * q_rot) - 1) < 1e-12, (Tv, Tr)


def test_two_level_vibrational_band():
    # ground (g = 1) and one excited vibrational state (g = 3), both at J = 0 of their
    # manifolds: I = g_1 A/(8 pi c w^2) (1 - e^-u)/(1 + 3 e^-u), u = c2 w/T_vib, for any T_rot
    w, A = 2143.0, 33.0
    for Tv in (500.0, 3000.0):
        u = O.C2 * w / Tv
        ref = 3 * A / (8 * math.pi * C_CGS * w * w) * (-math.expm1(-u)) / (1 + 3 * math.exp(-u))
        for Tr in (100.0, 1000.0, 5000.0):
            got = O.intensities_nlte([0.0, w], [1, 3], [0.0, w], [1], [0], [A], Tv, Tr)[0]
            assert abs(got / ref - 1) < 1e-13


def test_lte_limit_is_eq1():
    rng = np.random.default_rng(2)
    E = np.sort(rng.uniform(0, 10000, 300))
    lab = (E // 1500).astype(int)
    Ev = O.vibrational_energies(E, lab)
    g = rng.integers(1, 30, E.size)
    up = rng.integers(150, 300, 500)
    lo = rng.integers(0, 150, 500)
    A = 10 ** rng.uniform(-3, 2, 500)
    for T in (296.0, 2500.0):
        a = O.intensities_nlte(E, g, Ev, up, lo, A, T, T)
        b = O.intensities(E, g, up, lo, A, T)
        assert np.max(np.abs(a / b - 1)) < 1e-12
        e1 = O.emissivities_nlte(E, g, Ev, up, lo, A, T, T)
        e2 = O.emissivities(E, g, up, lo, A, T)
        assert np.max(np.abs(e1 / e2 - 1)) < 1e-12


def test_inverted_transitions_are_negative():
    # T_vib > T_rot: a band transition whose rotational energy falls can be inverted;
    # the sign follows c2 [dE_vib/T_vib + dE_rot/T_rot] (brute force per line)
    E, g, v, J = _ladder(1000.0, 2.0, n_v=4, n_J=40)
    Ev = O.vibrational_energies(E, v)
    pairs = [(i, j) for i in range(E.size) for j in range(E.size) if E[i] > E[j] and abs(v[i] - v[j]) == 1]
    up = np.array([p[0] for p in pairs])
    lo = np.array([p[1] for p in pairs])
    Tv, Tr = 6000.0, 150.0
    I = O.intensities_nlte(E, g, Ev, up, lo, np.ones(up.size), Tv, Tr)
    n_neg = 0
    for k in range(up.size):
        dEv = Ev[up[k]] - Ev[lo[k]]
        dEr = (E[up[k]] - Ev[up[k]]) - (E[lo[k]] - Ev[lo[k]])
        s = dEv / Tv + dEr / Tr
        assert (I[k] < 0) == (s < 0)
        n_neg += s < 0
    assert n_neg > 0


def test_emission_over_absorption_at_the_excitation_temperature():
    rng = np.random.default_rng(4)
    E = np.sort(rng.uniform(0, 12000, 200))
    lab = (E // 2000).astype(int)
    Ev = O.vibrational_energies(E, lab)
    g = rng.integers(1, 20, E.size)
    up = rng.integers(100, 200, 300)
    lo = rng.integers(0, 100, 300)
    A = 10 ** rng.uniform(-2, 2, 300)
    Tv, Tr = 2500.0, 800.0
    eps = O.emissivities_nlte(E, g, Ev, up, lo, A, Tv, Tr)
    I = O.intensities_nlte(E, g, Ev, up, lo, A, Tv, Tr)
    for k in range(up.size):
        nu = E[up[k]] - E[lo[k]]
        # F_low/F_up = exp(c2 nu / T_ex) defines the excitation temperature
        ln_ratio = (Ev[up[k]] - Ev[lo[k]]) / Tv + ((E[up[k]] - Ev[up[k]]) - (E[lo[k]] - Ev[lo[k]])) / Tr
        T_ex = nu / ln_ratio
        if T_ex <= 0:
            continue
        assert abs(eps[k] / I[k] / _planck(nu, T_ex) - 1) < 1e-10
