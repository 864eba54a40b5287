"""Pins of the bin-averaged Gaussian / Lorentzian profiles and the super-line histogram
(CPU only): numerical quadrature of the sampled profiles over a bin, telescoping areas,
limits, and a brute-force histogram with explicit edge comparisons."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


@pytest.mark.parametrize("alpha,dnu", [(0.05, 0.01), (0.01, 0.1), (0.3, 1.0), (2e-3, 1e-3)])
def test_gauss_binned_is_the_bin_average(alpha, dnu):
    # Sec. "Binned Gaussian profile with analytical integrals": the bin average of Eq. 15
    for delta in (0.0, 0.3 * dnu, 0.5 * dnu, 2.0 * alpha, 5.0 * alpha, 9.0 * alpha):
        ref = integrate.quad(lambda x: float(O.gauss_profile(x, alpha)), delta - dnu / 2, delta + dnu / 2,
                             epsabs=0.0, epsrel=1e-13, limit=200)[0] / dnu
        got = float(O.gauss_binned_profile(delta, alpha, dnu))
        assert abs(got - ref) <= 1e-11 * ref + 1e-300, (delta, got, ref)


@pytest.mark.parametrize("gamma,dnu", [(0.05, 0.01), (0.01, 0.1), (0.5, 1.0), (1e-4, 0.01)])
def test_lorentz_binned_is_the_bin_average(gamma, dnu):
    # Eq. 27-28 (minus sign restored): the bin average of Eq. 17
    for delta in (0.0, 0.3 * dnu, 0.5 * dnu, 3.0 * gamma, 20.0 * dnu, 25.0):
        ref = integrate.quad(lambda x: float(O.lorentz_profile(x, gamma)), delta - dnu / 2, delta + dnu / 2,
                             epsabs=0.0, epsrel=1e-13, limit=400, points=[0.0] if abs(delta) < dnu else None)[0] / dnu
        got = float(O.lorentz_binned_profile(delta, gamma, dnu))
        assert abs(got - ref) <= 1e-11 * ref, (delta, got, ref)


def test_binned_areas_telescope_to_the_closed_forms():
    # summing the bin averages over consecutive bins gives the integral over their union
    alpha, gamma, dnu = 0.07, 0.03, 0.02
    k = np.arange(-200, 201)
    d = k * dnu + 0.0037
    lo, hi = d[0] - dnu / 2, d[-1] + dnu / 2
    g = dnu * math.fsum(O.gauss_binned_profile(d, alpha, dnu))
    s = math.sqrt(math.log(2)) / alpha
    assert abs(g - 0.5 * (math.erf(s * hi) - math.erf(s * lo))) < 1e-13
    lz = dnu * math.fsum(O.lorentz_binned_profile(d, gamma, dnu))
    assert abs(lz - (math.atan(hi / gamma) - math.atan(lo / gamma)) / math.pi) < 1e-13


def test_binned_profiles_tend_to_the_sampled_ones_on_fine_bins():
    delta = np.array([0.0, 0.02, 0.08])
    for dnu in (1e-3, 1e-4):
        rg = O.gauss_binned_profile(delta, 0.05, dnu) / O.gauss_profile(delta, 0.05)
        rl = O.lorentz_binned_profile(delta, 0.03, dnu) / O.lorentz_profile(delta, 0.03)
        # second-order midpoint error: f''/(24 f) dnu^2
        assert np.max(np.abs(rg - 1)) < 2e3 * dnu ** 2 and np.max(np.abs(rl - 1)) < 2e3 * dnu ** 2


def test_lorentz_binned_pure_doppler_limit_is_a_step():
    dnu = 0.5
    d = np.array([0.0, 0.2, 0.25, 0.3, -0.25, 1.0])
    got = O.lorentz_binned_profile(d, 0.0, dnu)
    assert np.allclose(got, np.array([1, 1, 0.5, 0, 0.5, 0]) / dnu)


def test_erf_difference_matches_mpmath_in_the_tails():
    import mpmath
    mpmath.mp.dps = 40
    for a, b in ((6.0, 6.001), (-8.2, -8.0), (-0.001, 0.002), (3.0, 30.0), (0.5, 0.5000001)):
        ref = float(mpmath.erf(b) - mpmath.erf(a))
        # SciPy's erfc keeps ~1e-12 relative accuracy in the far tail; a close pair (a, b)
        # loses a further factor ~1/(b - a) to the subtraction
        assert abs(float(O.erf_difference(a, b)) - ref) <= 1e-12 * abs(ref) / min(1.0, (b - a)) + 1e-300


def _brute_bins(nu, nu_a, dnu, n):
    out = [[] for _ in range(n)]
    for i, v in enumerate(nu):
        for k in range(n):
            c = nu_a + k * dnu
            if c - dnu / 2 <= v < c + dnu / 2:
                out[k].append(i)
    return out


def test_super_line_histogram_equals_brute_force_bins():
    # Sec. "Super-lines": bin sums of intensities (half-open bins; dnu = 0.5 so that the
    # edges are exact and lines placed on them go to the upper bin)
    rng = np.random.default_rng(4)
    nu_a, nu_b, n = 10.0, 30.0, 41
    dnu = 0.5
    nu = np.concatenate([rng.uniform(9.0, 31.0, 300), [10.25, 12.75, 29.75, 30.25, 9.75, 9.7499]])
    I = 10 ** rng.uniform(-3, 0, nu.size)
    ls = O.LineSet(nu, I, np.full(nu.size, 0.01), np.full(nu.size, 0.01))
    got = O.super_line_histogram(ls, nu_a, nu_b, n)
    bins = _brute_bins(nu, nu_a, dnu, n)
    ref = np.array([math.fsum(I[b]) for b in bins]) / dnu
    assert np.array_equal(got, ref)
    # every line whose bin is on the grid is counted exactly once
    inside = (nu >= nu_a - dnu / 2) & (nu < nu_b + dnu / 2)
    assert abs(dnu * math.fsum(got) - math.fsum(I[inside])) < 1e-13 * math.fsum(I)


@pytest.mark.parametrize("profile", ["doppler_binned", "lorentz_binned"])
def test_binned_cross_section_equals_double_loop(profile):
    rng = np.random.default_rng(8)
    n_l = 25
    ls = O.LineSet(rng.uniform(-1.0, 51.0, n_l), 10 ** rng.uniform(-2, 0, n_l), rng.uniform(0.01, 0.2, n_l),
                   rng.uniform(0.005, 0.3, n_l))
    import mpmath
    mpmath.mp.dps = 30
    nu_a, nu_b, n, cut = 0.0, 50.0, 501, 3.0
    sig = O.cross_section(ls, nu_a, nu_b, n, cut, profile=profile, workers=1)
    dnu = (nu_b - nu_a) / (n - 1)
    ref = np.zeros(n)
    for i in range(n_l):
        for k in range(n):
            d = (nu_a + k * dnu) - ls.nu[i]
            if abs(d) > cut:
                continue
            if profile == "doppler_binned":
                # 30-digit error functions: the tails are a difference of nearly equal numbers
                s = mpmath.sqrt(mpmath.log(2)) / ls.alpha_d[i]
                v = float((mpmath.erf(s * (d + dnu / 2)) - mpmath.erf(s * (d - dnu / 2))) / (2 * dnu))
            else:
                g = ls.gamma[i]
                v = (math.atan((d + dnu / 2) / g) - math.atan((d - dnu / 2) / g)) / (math.pi * dnu)
            ref[k] += ls.I[i] * v
    m = ref > 1e-9 * ref.max()
    assert np.max(np.abs(sig[m] - ref[m]) / ref[m]) < 1e-10
