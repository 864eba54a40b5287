"""Pins of the Vectorized Voigt oracle (V-V and VVN) against facts the paper and the
mathematics fix (CPU only): the paper's stated wing-error bound, reduction to the
pinned Voigt cross section, continuity, area conservation and a brute-force double
loop written independently of the vectorised oracle."""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O
from oracle import vvoigt as V


def _voigt_scalar(delta, alpha, gamma):
    # scipy.special.voigt_profile takes the Gaussian standard deviation, not the HWHM
    return float(special.voigt_profile(delta, alpha / math.sqrt(2.0 * math.log(2.0)), gamma))


def test_reference_width_is_doppler_width_of_a_line_at_one_wavenumber():
    # Eq. 16 is linear in nu: the reference HWHM is alpha_D(nu)/nu for any nu
    for T, m in ((296.0, 34.0), (5000.0, 18.0)):
        aref = V.vv_reference_hwhm(T, m)
        for nu in (0.5, 1.0, 2500.0, 30000.0):
            assert abs(float(O.doppler_hwhm(nu, T, m)) / nu - aref) < 1e-15 * aref
        # thermal speed: alpha/nu = sqrt(2 ln2 k T / m) / c (independent evaluation in mpmath)
        import mpmath
        mpmath.mp.dps = 30
        v = mpmath.sqrt(2 * mpmath.log(2) * mpmath.mpf("1.380649e-23") * T / (m * mpmath.mpf("1.66053906660e-27")))
        assert abs(float(v / mpmath.mpf(299792458)) - aref) < 1e-14 * aref


def test_wing_error_bound_of_the_paper_figure():
    # Sec. "Vectorized Voigt approximation", figure of the relative error at 4 cm^-1:
    # H2O, T = 5000 K, gamma_L from Eq. 18 with gamma0 = 0.0709, T0 = 296 K, n = 0.5,
    # P0 = 1 bar; over 0-30000 cm^-1 the error never exceeds 1 % and grows with nu;
    # at 1 bar it is almost the same as at 1e-20 bar.
    T, m = 5000.0, 18.0
    aref = V.vv_reference_hwhm(T, m)
    nu = np.linspace(1.0, 30000.0, 1200)
    aD = O.doppler_hwhm(nu, T, m)
    errs = {}
    for P in (1e-20, 1.0, 10.0):
        g = O.lorentz_hwhm(np.full(nu.shape, 0.0709), np.full(nu.shape, 0.5), T, P)
        f_line = np.array([_voigt_scalar(4.0, a, gg) for a, gg in zip(aD, g)])
        f_ref = np.array([_voigt_scalar(4.0, aref, gg) for gg in g])
        err = np.abs(f_ref - f_line) / f_line
        assert err.max() < 0.01
        assert np.all(np.diff(err) > 0)
        # the oracle's beta is exactly f_line / f_ref
        b = V.vv_beta(aD, g, aref, 4.0, True)
        assert np.max(np.abs(b * f_ref - f_line) / f_line) < 1e-12
        errs[P] = err
    assert np.max(np.abs(errs[1.0] - errs[1e-20]) / errs[1e-20][-1]) < 0.01


def test_radius_beyond_cutoff_is_the_voigt_cross_section():
    rng = np.random.default_rng(3)
    n = 300
    ls = O.LineSet(rng.uniform(-1.0, 101.0, n), 10 ** rng.uniform(-3, 0, n), rng.uniform(0.005, 0.05, n),
                   rng.uniform(0.001, 0.1, n))
    ref = O.cross_section(ls, 0.0, 100.0, 2001, cutoff=5.0, profile="voigt", workers=1)
    got = V.cross_section_vv(ls, 0.0, 100.0, 2001, 296.0, 34.0, cutoff=5.0, radius=6.0, workers=1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * ref.max()


def test_beta_makes_the_profile_continuous_at_the_radius():
    aref = V.vv_reference_hwhm(2000.0, 34.0)
    aD = np.array([0.001, 0.02, 0.08])
    g = np.array([0.0005, 0.05, 0.2])
    b = V.vv_beta(aD, g, aref, 4.0, True)
    d = np.full(3, 4.0)
    inner = V.vv_profile_values(d, np.ones(3, bool), aD, g, aref, b)
    outer = V.vv_profile_values(d, np.zeros(3, bool), aD, g, aref, b)
    assert np.max(np.abs(inner - outer) / inner) < 1e-14
    # beta defaults to 1 (the paper's usual choice) and is 1 for gamma = 0
    assert np.all(V.vv_beta(aD, g, aref, 4.0, False) == 1.0)
    assert V.vv_beta(np.array([0.02]), np.array([0.0]), aref, 4.0, True)[0] == 1.0
    # wings beyond R follow the Lorentzian: the reference Doppler width is ~1e-6 cm^-1
    dd = np.array([4.0, 10.0, 25.0])
    lor = g[1] / (math.pi * (dd * dd + g[1] ** 2))
    ref = V.vv_profile_values(dd, np.zeros(3, bool), np.full(3, aD[1]), np.full(3, g[1]), aref, np.ones(3))
    assert np.max(np.abs(ref - lor) / lor) < 1e-9


def _brute_force(nu, I, aD, g, nu_a, dnu, n, cut, R, aref, use_beta, normalise):
    """Double loop over lines and grid points; every decision is an explicit distance test."""
    sig = [0.0] * n
    for i in range(len(nu)):
        beta = 1.0
        if use_beta and g[i] > 0:
            beta = _voigt_scalar(R, aD[i], g[i]) / _voigt_scalar(R, aref, g[i])
        vals = {}
        k = int(math.floor((nu[i] - cut - nu_a) / dnu)) - 2
        while nu_a + k * dnu <= nu[i] + cut + 2 * dnu:
            d = (nu_a + k * dnu) - nu[i]
            if abs(d) <= cut:
                if abs(d) <= R:
                    vals[k] = _voigt_scalar(d, aD[i], g[i])
                else:
                    vals[k] = beta * _voigt_scalar(d, aref, g[i])
            k += 1
        scale = 1.0
        if normalise:
            tot = math.fsum(vals.values())
            scale = 1.0 / (dnu * tot) if tot > 0 else 0.0
        for k, v in vals.items():
            if 0 <= k < n:
                sig[k] += I[i] * scale * v
    return np.array(sig)


@pytest.mark.parametrize("use_beta,normalise", [(False, False), (True, False), (False, True), (True, True)])
def test_vv_equals_brute_force_double_loop(use_beta, normalise):
    rng = np.random.default_rng(11)
    nu_a, nu_b, n, cut, R = 10.0, 40.0, 301, 3.0, 1.0
    nu = np.concatenate([rng.uniform(nu_a - 2.5, nu_b + 2.5, 12), [nu_a + 0.05, nu_b - 0.07]])
    I = 10 ** rng.uniform(-2, 0, nu.size)
    aD = rng.uniform(0.02, 0.2, nu.size)
    g = rng.uniform(0.0, 0.3, nu.size)
    g[0] = 0.0
    T, m = 1500.0, 18.0
    aref = V.vv_reference_hwhm(T, m)
    ls = O.LineSet(nu, I, aD, g)
    got = V.cross_section_vv(ls, nu_a, nu_b, n, T, m, cutoff=cut, radius=R, use_beta=use_beta,
                             normalise=normalise, workers=1)
    _, dnu = O.grid(nu_a, nu_b, n)
    ref = _brute_force(nu, I, aD, g, nu_a, dnu, n, cut, R, aref, use_beta, normalise)
    assert np.max(np.abs(got - ref)) <= 1e-12 * ref.max()
    if not normalise:
        at = V.cross_section_vv_at(ls, [0, 17, 150, 299, 300], nu_a, nu_b, n, T, m, cutoff=cut, radius=R,
                                   use_beta=use_beta)
        assert np.max(np.abs(at - ref[[0, 17, 150, 299, 300]])) <= 1e-12 * ref.max()


def test_vvn_preserves_the_line_area():
    # Sec. "Binned Vectorized Voigt with the line area preserved": dnu sum_k sigma_k = I for
    # lines whose window lies on the grid, whatever the grid step and the profile widths.
    rng = np.random.default_rng(5)
    for dnu_target, n_lines in ((0.01, 40), (1.0, 40)):
        nu_a, nu_b = 0.0, 200.0
        n = int(round((nu_b - nu_a) / dnu_target)) + 1
        nu = rng.uniform(40.0, 160.0, n_lines)
        I = 10 ** rng.uniform(-3, 0, n_lines)
        ls = O.LineSet(nu, I, rng.uniform(0.001, 0.1, n_lines), rng.uniform(0.001, 0.2, n_lines))
        sig = V.cross_section_vv(ls, nu_a, nu_b, n, 2000.0, 34.0, cutoff=25.0, normalise=True, workers=1)
        _, dnu = O.grid(nu_a, nu_b, n)
        assert abs(dnu * math.fsum(sig) - math.fsum(I)) < 1e-12 * math.fsum(I)
        # not normalised, the truncated Voigt area on a fine grid falls short of I (Lorentz
        # wings beyond the cut-off), so the renormalisation is not a no-op
        raw = V.cross_section_vv(ls, nu_a, nu_b, n, 2000.0, 34.0, cutoff=25.0, normalise=False, workers=1)
        assert dnu * math.fsum(raw) < (1 - 1e-3) * math.fsum(I)
    # a line whose window leaves the grid keeps only its on-grid share of I
    ls = O.LineSet(np.array([1.0]), np.array([1.0]), np.array([0.01]), np.array([0.05]))
    n = 2001
    sig = V.cross_section_vv(ls, 0.0, 20.0, n, 296.0, 34.0, cutoff=5.0, normalise=True, workers=1)
    _, dnu = O.grid(0.0, 20.0, n)
    share = dnu * math.fsum(sig)
    assert 0.5 < share < 0.999
    norm = V.vv_line_norm(ls, 0.0, dnu, 5.0, 296.0, 34.0)
    klo, khi = V.window_unclipped(ls.nu, 0.0, dnu, 5.0)
    ks = np.arange(klo[0], khi[0] + 1)
    f = np.array([_voigt_scalar((k * dnu) - 1.0, 0.01, 0.05) if abs(k * dnu - 1.0) <= 4.0
                  else _voigt_scalar(k * dnu - 1.0, V.vv_reference_hwhm(296.0, 34.0), 0.05) for k in ks])
    assert abs(norm[0] * dnu * math.fsum(f) - 1.0) < 1e-12
    assert abs(share - dnu * math.fsum(f[ks >= 0]) / (dnu * math.fsum(f))) < 1e-12
