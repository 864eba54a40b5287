"""Pins of the FP64 oracle against facts the paper or mathematics fix (CPU only).

Each test checks the oracle against something other than itself: printed values,
closed forms, textbook identities, independent library routines (mpmath, SciPy
quadrature, scipy.special.voigt_profile), or brute force on tiny inputs.
"""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


# ---------------------------------------------------------------- grid (Eq. 9)
def test_grid_includes_both_ends():
    nu, dnu = O.grid(0.0, 5000.0, 50001)
    assert dnu == 0.1
    assert nu[0] == 0.0 and nu[-1] == 5000.0 and nu.size == 50001
    nu, dnu = O.grid(1000.0, 6000.0, 500001)
    assert abs(dnu - 0.01) < 1e-15 and abs(nu[-1] - 6000.0) < 1e-9


# ------------------------------------------------------------ Q(T) (Eq. 2)
def test_partition_single_and_two_level():
    assert O.partition_function([0.0], [7], 300.0) == 7.0
    E1, T = 1000.0, 750.0
    expect = 3.0 + 5.0 * math.exp(-(6.62607015e-34 * 299792458.0 / 1.380649e-23 * 100) * E1 / T)
    assert abs(O.partition_function([0.0, E1], [3, 5], T) - expect) < 1e-15 * expect


def test_partition_rigid_rotor_high_T():
    # E_J = B J(J+1), g = 2J+1; classical expansion Q = t (1 + 1/(3t) + 1/(15 t^2) + 4/(315 t^3))
    # with t = T/(c2 B) (McDowell 1988 series; truncation error O(t^-4)).
    B = 2.0
    J = np.arange(0, 2000)
    E = B * J * (J + 1)
    for T in (500.0, 2000.0):
        t = T / (O.C2 * B)
        expect = t * (1 + 1 / (3 * t) + 1 / (15 * t * t) + 4 / (315 * t ** 3))
        got = O.partition_function(E, 2 * J + 1, T)
        assert abs(got - expect) / expect < 5.0 / t ** 4 + 1e-14


def test_partition_derivative_matches_finite_difference():
    rng = np.random.default_rng(0)
    E = rng.uniform(0, 5000, 300)
    g = rng.integers(1, 40, 300)
    T = 900.0
    h = 1e-3
    fd = (O.partition_function(E, g, T + h) - O.partition_function(E, g, T - h)) / (2 * h)
    assert abs(O.partition_function_dT(E, g, T) - fd) / abs(fd) < 1e-8


# --------------------------------------------- nu convention (stick table)
def test_transition_wavenumber_is_upper_minus_lower(golden_dir):
    rows = np.loadtxt(os.path.join(golden_dir, "kcl_stick_extract.txt"))
    nu_printed, E_up, E_low = rows[:, 0], rows[:, 3], rows[:, 5]
    E = np.concatenate([E_up, E_low])
    n = rows.shape[0]
    nu = O.line_centres(E, np.arange(n), np.arange(n) + n)
    # energies are printed to 4 decimals: difference good to 1e-4
    assert np.all(np.abs(nu - nu_printed) <= 1.01e-4)


# ----------------------------------------------------- intensities (Eq. 1)
def _one_line_I(Eup, Elow, gup, A, T, Q):
    return O.intensities([Elow, Eup], [1, gup], [1], [0], [A], T, Q=Q)[0]


def test_intensity_is_boltzmann_population_difference():
    # g_f A/(8 pi c nu^2) (exp(-c2 E_i/T) - exp(-c2 E_f/T)) / Q: Eq. 1 with the
    # stimulated-emission factor written as a difference of two Boltzmann factors.
    T, Q = 1234.0, 321.0
    for Elow, Eup in ((0.0, 1.0), (300.0, 2300.0), (5000.0, 9999.0)):
        nu = Eup - Elow
        I = _one_line_I(Eup, Elow, 13, 2.5, T, Q)
        c = 2.99792458e10
        expect = 13 * 2.5 / (8 * math.pi * c * nu * nu) * (
            float(mpmath.exp(-O.C2 * Elow / T)) - float(mpmath.exp(-O.C2 * Eup / T))) / Q
        assert abs(I - expect) / expect < 2e-13


def test_intensity_small_nu_uses_expm1():
    # nu -> 0: 1 - exp(-x) = x - x^2/2 + x^3/6, x = c2 nu/T; a naive 1-exp form
    # loses all digits here.
    T, nu = 3000.0, 1e-6
    I = _one_line_I(nu, 0.0, 1, 1.0, T, 1.0)
    x = O.C2 * nu / T
    c = 2.99792458e10
    expect = 1.0 / (8 * math.pi * c * nu * nu) * (x - x * x / 2 + x ** 3 / 6)
    assert abs(I - expect) / expect < 1e-14


def test_intensity_linear_in_A_and_inverse_in_Q():
    a = _one_line_I(2000.0, 100.0, 5, 1.0, 800.0, 10.0)
    b = _one_line_I(2000.0, 100.0, 5, 3.0, 800.0, 10.0)
    c = _one_line_I(2000.0, 100.0, 5, 1.0, 800.0, 40.0)
    assert abs(b / a - 3.0) < 1e-15 and abs(a / c - 4.0) < 1e-15


# ------------------------------------------------------------ Doppler (Eq. 16)
def test_doppler_width_from_maxwell_velocity_variance():
    # 1D Maxwell-Boltzmann: <v^2> = k_B T / m.  The Doppler-shifted profile's second
    # moment must be (nu/c)^2 k_B T / m; this pins Eq. 16 together with Eq. 15.
    nu, T, m = 3000.0, 700.0, 18.0
    aD = O.doppler_hwhm(nu, T, m)
    var = integrate.quad(lambda d: d * d * O.gauss_profile(d, aD), -50 * aD, 50 * aD, limit=200)[0]
    expect = (nu / 299792458.0) ** 2 * 1.380649e-23 * T / (m * 1.66053906660e-27)
    assert abs(var - expect) / expect < 1e-9


# ----------------------------------------------------------------- profiles
@pytest.mark.parametrize("alpha,gamma", [(0.01, 0.05), (0.05, 0.001), (0.02, 0.02)])
def test_profiles_unit_area_and_hwhm(alpha, gamma):
    G = integrate.quad(lambda d: O.gauss_profile(d, alpha), -np.inf, np.inf)[0]
    L = integrate.quad(lambda d: O.lorentz_profile(d, gamma), -np.inf, np.inf)[0]
    V = integrate.quad(lambda d: O.voigt_profile(d, alpha, gamma), -np.inf, np.inf, limit=500)[0]
    assert abs(G - 1) < 1e-10 and abs(L - 1) < 1e-8 and abs(V - 1) < 1e-7
    assert abs(O.gauss_profile(alpha, alpha) / O.gauss_profile(0.0, alpha) - 0.5) < 1e-15
    assert abs(O.lorentz_profile(gamma, gamma) / O.lorentz_profile(0.0, gamma) - 0.5) < 1e-15


def test_truncated_areas_closed_forms():
    cut, alpha, gamma = 25.0, 0.8, 0.3
    G = integrate.quad(lambda d: O.gauss_profile(d, alpha), -cut, cut)[0]
    L = integrate.quad(lambda d: O.lorentz_profile(d, gamma), -cut, cut, limit=200)[0]
    assert abs(G - math.erf(cut * math.sqrt(math.log(2)) / alpha)) < 1e-12
    assert abs(L - 2 / math.pi * math.atan(cut / gamma)) < 1e-12


@pytest.mark.parametrize("alpha,gamma,delta", [
    (0.01, 0.05, 0.0), (0.01, 0.05, 0.3), (0.05, 0.001, 0.02), (0.05, 0.001, 0.2),
    (0.02, 0.02, 1.0), (0.003, 0.0004, 0.004)])
def test_voigt_equals_brute_force_convolution(alpha, gamma, delta):
    conv = integrate.quad(lambda t: O.gauss_profile(t, alpha) * O.lorentz_profile(delta - t, gamma),
                          -40 * alpha, 40 * alpha, points=[delta] if abs(delta) < 40 * alpha else None,
                          limit=1000, epsabs=0, epsrel=1e-12)[0]
    # tails of the Gaussian beyond 40 alpha are below 1e-300
    assert abs(O.voigt_profile(delta, alpha, gamma) - conv) / conv < 1e-9


def test_voigt_matches_scipy_voigt_profile_and_limits():
    d = np.linspace(-2, 2, 41)
    alpha, gamma = 0.07, 0.03
    ref = special.voigt_profile(d, alpha / math.sqrt(2 * math.log(2)), gamma)
    assert np.max(np.abs(O.voigt_profile(d, alpha, gamma) - ref) / ref) < 1e-12
    # gamma -> 0: Gaussian; alpha -> 0: Lorentzian
    assert np.allclose(O.voigt_profile(d[:30], alpha, 0.0), O.gauss_profile(d[:30], alpha), rtol=1e-13)
    lo = O.voigt_profile(d, 1e-7, gamma)
    assert np.max(np.abs(lo - O.lorentz_profile(d, gamma)) / O.lorentz_profile(d, gamma)) < 1e-6


def test_faddeeva_against_mpmath():
    # w(z) = exp(-z^2) erfc(-i z); real part on the imaginary axis = exp(y^2) erfc(y)
    for z in (0.3 + 0.01j, 4.0 + 1e-6j, 12.0 + 0.5j, 1e-3 + 2.0j, 30.0 + 3.0j):
        ref = mpmath.exp(-mpmath.mpc(z) ** 2) * mpmath.erfc(-1j * mpmath.mpc(z))
        got = special.wofz(z)
        assert abs(got.real - float(ref.real)) / abs(float(ref.real)) < 1e-12


# -------------------------------------------------------------- window rule
def test_window_is_inclusive_and_clipped():
    nu_a, nu_b, n = 0.0, 100.0, 201   # dnu = 0.5
    k_lo, k_hi = O.window(np.array([30.0, 30.25, 2.0, 120.0, 130.5]), nu_a, 0.5, n, 25.0)
    assert (k_lo[0], k_hi[0]) == (10, 110)          # both ends exactly on grid points
    assert (k_lo[1], k_hi[1]) == (11, 110)
    assert (k_lo[2], k_hi[2]) == (0, 54)            # clipped at the start
    assert (k_lo[3], k_hi[3]) == (190, 200)         # centre off-grid, window overlaps
    assert k_lo[4] > k_hi[4]                        # window misses the grid


# ---------------------------------------------------------- full sigma
def _tiny_lines(seed=1, n=40):
    rng = np.random.default_rng(seed)
    nu = rng.uniform(5.0, 45.0, n)
    I = 10 ** rng.uniform(-22, -19, n)
    aD = rng.uniform(0.01, 0.2, n)
    gam = rng.uniform(0.005, 0.3, n)
    return O.LineSet(nu, I, aD, gam)


@pytest.mark.parametrize("profile", ["voigt", "doppler", "lorentz"])
def test_cross_section_equals_double_loop(profile):
    ls = _tiny_lines()
    nu_a, nu_b, n, cut = 0.0, 50.0, 2001, 3.0
    sig = O.cross_section(ls, nu_a, nu_b, n, cut, profile=profile, workers=1)
    dnu = (nu_b - nu_a) / (n - 1)
    ref = np.zeros(n)
    s2 = math.sqrt(2 * math.log(2))
    for i in range(len(ls)):
        for k in range(n):
            d = (nu_a + k * dnu) - ls.nu[i]
            if abs(d) > cut + 1e-9:
                continue
            if profile == "voigt":
                f = special.voigt_profile(d, ls.alpha_d[i] / s2, ls.gamma[i])
            elif profile == "doppler":
                f = special.voigt_profile(d, ls.alpha_d[i] / s2, 0.0)
            else:
                f = ls.gamma[i] / math.pi / (d * d + ls.gamma[i] ** 2)
            ref[k] += ls.I[i] * f
    m = ref > 0
    assert np.max(np.abs(sig[m] - ref[m]) / ref[m]) < 1e-12
    assert np.all(sig[~m] == 0)


def test_cross_section_workers_agree():
    ls = _tiny_lines(n=300)
    a = O.cross_section(ls, 0.0, 50.0, 2001, 3.0, workers=1)
    b = O.cross_section(ls, 0.0, 50.0, 2001, 3.0, workers=3, block=17)
    assert np.max(np.abs(a - b) / np.maximum(a, 1e-300)) < 1e-13


def test_sum_rule_resolved_lines():
    # All lines resolved (gamma >= 2 dnu, alpha_D >= dnu) and far from the grid ends:
    # dnu * sum_k sigma_k = sum_i I_i a_i(cut), a = truncated Voigt area, to within the
    # Poisson-aliasing bound of the sampled sum.
    rng = np.random.default_rng(3)
    n = 20
    ls = O.LineSet(rng.uniform(20, 30, n), 10 ** rng.uniform(-21, -19, n),
                   rng.uniform(0.02, 0.05, n), rng.uniform(0.04, 0.08, n))
    dnu = 0.01
    sig = O.cross_section(ls, 0.0, 50.0, 5001, 5.0, workers=1)
    area = dnu * sig.sum()
    trunc = [integrate.quad(lambda d: O.voigt_profile(d, ls.alpha_d[i], ls.gamma[i]), -5.0, 5.0,
                            points=[0.0], limit=400, epsrel=1e-12)[0] for i in range(n)]
    expect = float(np.sum(ls.I * np.array(trunc)))
    assert abs(area - expect) / expect < 1e-6


def test_cross_section_at_matches_full_grid():
    ls = _tiny_lines(seed=5, n=60)
    sig = O.cross_section(ls, 0.0, 50.0, 2001, 3.0, workers=1)
    ks = np.array([0, 7, 400, 1000, 1999, 2000])
    got = O.cross_section_at(ls, ks, 0.0, 50.0, 2001, 3.0)
    assert np.allclose(got, sig[ks], rtol=1e-13, atol=0)


# ---------------------------------------------------- Gauss-Hermite variants
def test_gh_binned_area_telescopes():
    # Eq. 31 (as read): dnu * sum_k sigma_k = I (1/sqrt(pi)) sum_j w_j (1/pi)
    #   [atan(y_j at the last bin's upper edge) - atan(y_j at the first bin's lower edge)]
    t, w = np.polynomial.hermite.hermgauss(30)
    nu0, aD, gam, I = 12.3456, 0.08, 0.02, 2.0
    ls = O.LineSet([nu0], [I], [aD], [gam])
    n, nu_a, nu_b = 1001, 10.0, 15.0
    dnu = (nu_b - nu_a) / (n - 1)
    sig = O.cross_section(ls, nu_a, nu_b, n, 100.0, profile="gh_binned", workers=1)
    lo_edge = nu_a - dnu / 2 - nu0
    hi_edge = nu_b + dnu / 2 - nu0
    dj = aD * t / math.sqrt(math.log(2))
    expect = I / math.sqrt(math.pi) * np.sum(w * (np.arctan((hi_edge - dj) / gam)
                                               - np.arctan((lo_edge - dj) / gam))) / math.pi
    assert abs(dnu * sig.sum() - expect) / expect < 1e-12


def test_gh_binned_lorentz_limit():
    # alpha_D -> 0: every node collapses onto the centre; Eq. 31 becomes Eq. 28.
    d = np.linspace(-1, 1, 81)
    gam, dnu = 0.03, 0.025
    binned_lor = (np.arctan((d + dnu / 2) / gam) - np.arctan((d - dnu / 2) / gam)) / (math.pi * dnu)
    got = O.gh_binned_profile(d, 1e-12, gam, dnu)
    assert np.max(np.abs(got - binned_lor) / binned_lor) < 1e-9


def test_gh_sampled_close_to_voigt_when_lorentz_dominates():
    d = np.linspace(-0.5, 0.5, 51)
    aD, gam = 0.01, 0.05      # y ~ 4: 30 nodes resolve the convolution
    rel = np.abs(O.gh_sampled_profile(d, aD, gam) - O.voigt_profile(d, aD, gam)) / O.voigt_profile(d, aD, gam)
    assert rel.max() < 1e-8


# ------------------------------------------------------------ a0 broadening
def test_a0_table_selects_by_lower_J(golden_dir):
    rows = [ln.split() for ln in open(os.path.join(golden_dir, "cs_air_broad_a0.txt")) if ln[0] != "#"]
    J = np.array([int(r[3]) for r in rows])
    table_g = np.zeros(J.max() + 1)
    table_n = np.zeros(J.max() + 1)
    table_g[J] = [float(r[1]) for r in rows]
    table_n[J] = [float(r[2]) for r in rows]
    # states: 0 (J=2, lower), 1 (J=3, upper), 2 (J=35, lower), 3 (J=36, upper)
    E = np.array([0.0, 10.0, 100.0, 130.0])
    Js = np.array([2, 3, 35, 36])
    ls = O.make_lineset(E, 2 * Js + 1, [1, 3], [0, 2], [1.0, 1.0], 296.0, 1.0, 40.0,
                        J=Js, broad_table=(table_g, table_n))
    assert np.allclose(ls.gamma, [0.0840, 0.0720], rtol=1e-15)
    ls2 = O.make_lineset(E, 2 * Js + 1, [1, 3], [0, 2], [1.0, 1.0], 600.0, 2.0, 40.0,
                         J=Js, broad_table=(table_g, table_n))
    assert np.allclose(ls2.gamma, [0.0840 * 2 * (296 / 600) ** 0.091, 0.0720 * 2 * (296 / 600) ** 0.067])


# ------------------------------------------------------------ error metric
def test_error_metrics():
    ref = np.array([1.0, 1e-3, 1e-8, 0.0])
    m = O.error_metrics(ref * (1 + np.array([1e-6, -2e-6, 0.5, 0.0])), ref)
    assert abs(m["max_rel"] - 2e-6) < 1e-12 and m["n_checked"] == 2


def test_gh_binned_arctangent_difference_identity():
    # the oracle's atan2 form equals atan(y+) - atan(y-) evaluated in 50-digit arithmetic,
    # including far wings where the two arctangents nearly cancel
    mpmath.mp.dps = 50
    t, w = np.polynomial.hermite.hermgauss(30)
    for delta, aD, gam, dnu in ((3e-4, 0.02, 0.03, 0.01), (24.9, 0.03, 0.002, 0.01), (-7.3, 0.5, 0.1, 1.0),
                                (0.0, 1e-4, 1e-5, 0.01)):
        ref = mpmath.mpf(0)
        for tj, wj in zip(t, w):
            dj = mpmath.mpf(aD) * tj / mpmath.sqrt(mpmath.log(2))
            hi = (mpmath.mpf(delta) - dj + mpmath.mpf(dnu) / 2) / gam
            lo = (mpmath.mpf(delta) - dj - mpmath.mpf(dnu) / 2) / gam
            ref += wj * (mpmath.atan(hi) - mpmath.atan(lo))
        ref = ref / (mpmath.pi ** 1.5 * dnu)
        got = O.gh_binned_profile(np.array([delta]), aD, gam, dnu)[0]
        assert abs(got - float(ref)) <= 1e-12 * abs(float(ref))
    mpmath.mp.dps = 15


def test_faddeeva_derivative_against_mpmath():
    # w'(z) = -2 z w(z) + 2i/sqrt(pi) evaluated in 60-digit arithmetic
    mpmath.mp.dps = 60
    for z in (0.5 + 0.1j, 5.0 + 1e-6j, 29.0 + 3.0j, 31.0 + 0.01j, 800.0 + 2.0j, 3e5 + 10.0j, 1e-3 + 45.0j,
              -40.0 + 1e-3j):
        zm = mpmath.mpc(z)
        w = mpmath.exp(-zm * zm) * mpmath.erfc(-1j * zm)
        ref = complex(-2 * zm * w + 2j / mpmath.sqrt(mpmath.pi))
        got = O.faddeeva_derivative(np.array([z]))[0]
        assert abs(got - ref) <= 1e-12 * abs(ref), (z, got, ref)
    mpmath.mp.dps = 15
