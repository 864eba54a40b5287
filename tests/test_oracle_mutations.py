"""Planted-mistake checks: each plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) must make at least one pin fail.
Mistakes are planted in the oracle on the CPU via monkeypatch."""
import math

import numpy as np
import pytest
from scipy.special import wofz

import oracle as O
import oracle.xsec as X
from tests import test_oracle_pins as pins


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(X, name, fn)
    monkeypatch.setattr(O, name, fn)


def _bad_intensity(variant):
    def f(E, g, upper, lower, A, T, Q=None, index_base=0):
        E = np.asarray(E, np.float64); gg = np.asarray(g, np.float64)
        up = np.asarray(upper, np.int64) - index_base; lo = np.asarray(lower, np.int64) - index_base
        nu = E[up] - E[lo]
        if Q is None:
            Q = X.partition_function(E, g, T)
        A = np.asarray(A, np.float64)
        stim = -np.expm1(-O.C2 * nu / T)
        boltz = np.exp(-O.C2 * E[lo] / T)
        pref = gg[up] * A / (8.0 * math.pi * O.C_LIGHT_CGS * nu * nu)
        if variant == "no_stim":
            stim = 1.0
        elif variant == "naive_stim":
            stim = 1.0 - np.exp(-O.C2 * nu / T)
        elif variant == "upper_boltz":
            boltz = np.exp(-O.C2 * E[up] / T)
        elif variant == "lower_g":
            pref = gg[lo] * A / (8.0 * math.pi * O.C_LIGHT_CGS * nu * nu)
        elif variant == "no_8pi":
            pref = gg[up] * A / (O.C_LIGHT_CGS * nu * nu)
        return pref * boltz * stim / Q
    return f


@pytest.mark.parametrize("variant,pin", [
    ("no_stim", pins.test_intensity_is_boltzmann_population_difference),
    ("naive_stim", pins.test_intensity_small_nu_uses_expm1),
    ("upper_boltz", pins.test_intensity_is_boltzmann_population_difference),
    ("lower_g", pins.test_intensity_is_boltzmann_population_difference),
    ("no_8pi", pins.test_intensity_is_boltzmann_population_difference),
])
def test_intensity_mistakes_are_caught(monkeypatch, variant, pin):
    _patch(monkeypatch, "intensities", _bad_intensity(variant))
    with pytest.raises(AssertionError):
        pin()


def test_doppler_without_ln2_is_caught(monkeypatch):
    _patch(monkeypatch, "doppler_hwhm",
           lambda nu, T, m: np.sqrt(2.0 * O.K_BOLTZMANN * T / (m * O.AMU_KG)) * np.asarray(nu) / O.C_LIGHT_SI)
    with pytest.raises(AssertionError):
        pins.test_doppler_width_from_maxwell_velocity_variance()


def _bad_voigt(variant):
    def f(delta, alpha_d, gamma):
        delta = np.asarray(delta, np.float64)
        s = (math.log(2) if variant == "ln2" else math.sqrt(math.log(2))) / np.asarray(alpha_d)
        y = np.asarray(gamma) * (1.0 if variant == "unscaled_gamma" else s)
        return math.sqrt(math.log(2) / math.pi) / np.asarray(alpha_d) * wofz(delta * s + 1j * y).real
    return f


@pytest.mark.parametrize("variant", ["ln2", "unscaled_gamma"])
def test_voigt_mistakes_are_caught(monkeypatch, variant):
    _patch(monkeypatch, "voigt_profile", _bad_voigt(variant))
    with pytest.raises(AssertionError):
        pins.test_voigt_equals_brute_force_convolution(0.01, 0.05, 0.3)


def test_exclusive_window_is_caught(monkeypatch):
    def bad(nu, nu_a, dnu, n_points, cutoff):
        nu = np.asarray(nu, np.float64)
        klo = np.floor((nu - cutoff - nu_a) / dnu) + 1
        khi = np.ceil((nu + cutoff - nu_a) / dnu) - 1
        return np.maximum(klo, 0).astype(np.int64), np.minimum(khi, n_points - 1).astype(np.int64)
    _patch(monkeypatch, "window", bad)
    with pytest.raises(AssertionError):
        pins.test_window_is_inclusive_and_clipped()


def test_reversed_centre_is_caught(monkeypatch, golden_dir):
    _patch(monkeypatch, "line_centres",
           lambda E, upper, lower, index_base=0: np.asarray(E)[np.asarray(lower)] - np.asarray(E)[np.asarray(upper)])
    with pytest.raises(AssertionError):
        pins.test_transition_wavenumber_is_upper_minus_lower(golden_dir)


def test_partition_without_degeneracy_is_caught(monkeypatch):
    _patch(monkeypatch, "partition_function",
           lambda E, g, T: math.fsum(np.exp(-O.C2 * np.asarray(E, np.float64) / T)))
    with pytest.raises(AssertionError):
        pins.test_partition_single_and_two_level()


def test_gh_without_node_shift_is_caught(monkeypatch):
    def bad(delta, alpha_d, gamma, dnu, n_gh=30):
        t, w = np.polynomial.hermite.hermgauss(n_gh)
        delta = np.asarray(delta, np.float64)
        out = 0.0
        for tj, wj in zip(t, w):
            out = out + wj * (np.arctan((delta + dnu / 2) / gamma) - np.arctan((delta - dnu / 2) / gamma))
        return out / (math.pi ** 1.5 * dnu)
    _patch(monkeypatch, "gh_binned_profile", bad)
    with pytest.raises(AssertionError):
        pins.test_gh_binned_area_telescopes()


def test_inverted_temperature_exponent_is_caught(monkeypatch, golden_dir):
    _patch(monkeypatch, "lorentz_hwhm",
           lambda gref, n, T, P, T0=296.0, P0=1.0: np.asarray(gref) * (T / T0) ** np.asarray(n) * (P / P0))
    with pytest.raises(AssertionError):
        pins.test_a0_table_selects_by_lower_J(golden_dir)


def test_wrong_adjoint_sign_is_caught(monkeypatch):
    real = X.voigt_adjoint

    def bad(*a, **k):
        r = real(*a, **k)
        r["dT"] = -r["dT"]
        return r
    _patch(monkeypatch, "voigt_adjoint", bad)
    from tests import test_oracle_adjoint as adj
    with pytest.raises(AssertionError):
        adj.test_adjoint_matches_central_differences(1500.0, 0.1)


# ------------------------------------------------------------ Vectorized Voigt
import oracle.vvoigt as VV  # noqa: E402
from tests import test_oracle_vvoigt as vpins  # noqa: E402


def test_vv_wrong_reference_width_is_caught(monkeypatch):
    monkeypatch.setattr(VV, "vv_reference_hwhm", lambda T, m: float(O.doppler_hwhm(1.0, T, m)) * 10.0)
    with pytest.raises(AssertionError):
        vpins.test_reference_width_is_doppler_width_of_a_line_at_one_wavenumber()


def test_vv_inverted_beta_is_caught(monkeypatch):
    good = VV.vv_beta

    def bad(alpha_d, gamma, alpha_ref, radius, use_beta):
        b = good(alpha_d, gamma, alpha_ref, radius, use_beta)
        return 1.0 / b
    monkeypatch.setattr(VV, "vv_beta", bad)
    with pytest.raises(AssertionError):
        vpins.test_beta_makes_the_profile_continuous_at_the_radius()


def test_vv_core_bound_off_by_one_is_caught(monkeypatch):
    def bad(nu, nu_a, dnu, radius):
        nu = np.asarray(nu, np.float64)
        return (np.floor((nu - radius - nu_a) / dnu).astype(np.int64),
                np.floor((nu + radius - nu_a) / dnu).astype(np.int64))
    monkeypatch.setattr(VV, "vv_core_bounds", bad)
    with pytest.raises(AssertionError):
        vpins.test_vv_equals_brute_force_double_loop(False, False)


@pytest.mark.parametrize("variant", ["no_dnu", "clipped"])
def test_vvn_normalisation_mistakes_are_caught(monkeypatch, variant):
    good = VV._vv_lines

    def bad(ls, i0, i1, nu_a, dnu, cutoff, radius, alpha_ref, use_beta, normalise, k_clip):
        if variant == "clipped" and normalise:
            # sum over the on-grid part of the window only
            owner, k, f, _ = good(ls, i0, i1, nu_a, dnu, cutoff, radius, alpha_ref, use_beta, False, None)
            n = ls.nu[i0:i1].size
            on = (k >= 0) & (k <= (k_clip[1] if k_clip else 10 ** 9))
            tot = np.bincount(owner[on], weights=f[on], minlength=n)
            return owner, k, f, np.where(tot > 0, 1.0 / (dnu * np.where(tot > 0, tot, 1.0)), 0.0)
        owner, k, f, scale = good(ls, i0, i1, nu_a, dnu, cutoff, radius, alpha_ref, use_beta, normalise, k_clip)
        if variant == "no_dnu" and normalise:
            scale = scale * dnu
        return owner, k, f, scale
    monkeypatch.setattr(VV, "_vv_lines", bad)
    with pytest.raises(AssertionError):
        vpins.test_vvn_preserves_the_line_area()


# ------------------------------------------------------------ binned profiles, super-lines
import oracle.binned as BN  # noqa: E402
from tests import test_oracle_binned as bpins  # noqa: E402


def test_gauss_binned_without_the_half_is_caught(monkeypatch):
    good = BN.gauss_binned_profile
    monkeypatch.setattr(BN, "gauss_binned_profile", lambda d, a, dnu: 2.0 * good(d, a, dnu))
    monkeypatch.setattr(O, "gauss_binned_profile", lambda d, a, dnu: 2.0 * good(d, a, dnu))
    with pytest.raises(AssertionError):
        bpins.test_binned_areas_telescope_to_the_closed_forms()


def test_lorentz_binned_with_full_width_edges_is_caught(monkeypatch):
    good = BN.lorentz_binned_profile
    monkeypatch.setattr(O, "lorentz_binned_profile", lambda d, g, dnu: good(d, g, 2.0 * dnu) * 2.0)
    with pytest.raises(AssertionError):
        bpins.test_lorentz_binned_is_the_bin_average(0.05, 0.01)


def test_super_line_bins_by_truncation_are_caught(monkeypatch):
    monkeypatch.setattr(BN, "stick_bins",
                        lambda nu, nu_a, dnu: np.floor((np.asarray(nu) - nu_a) / dnu).astype(np.int64))
    with pytest.raises(AssertionError):
        bpins.test_super_line_histogram_equals_brute_force_bins()


# ------------------------------------------------------------ intensity thresholds
import oracle.threshold as TH  # noqa: E402
from tests import test_oracle_threshold as tpins  # noqa: E402


def test_threshold_without_the_half_in_tanh_is_caught(monkeypatch):
    def bad(nu, T, mode, i_crit=1e-29, nu_crit=2000.0):
        nu = np.asarray(nu, np.float64)
        if mode == "constant":
            return np.full(nu.shape, float(i_crit))
        return np.where(nu <= nu_crit, i_crit * (nu / nu_crit) * np.tanh(O.C2 * nu / T), i_crit)
    monkeypatch.setattr(TH, "intensity_cutoff", bad)
    monkeypatch.setattr(O, "intensity_cutoff", bad)
    with pytest.raises(AssertionError):
        tpins.test_hitran_cutoff_limits()


def test_strict_threshold_is_caught(monkeypatch):
    def bad(ls, T, mode, i_crit=1e-29, nu_crit=2000.0):
        keep = ls.I > TH.intensity_cutoff(ls.nu, T, mode, i_crit, nu_crit)
        return O.LineSet(ls.nu[keep], ls.I[keep], ls.alpha_d[keep], ls.gamma[keep])
    monkeypatch.setattr(TH, "apply_threshold", bad)
    monkeypatch.setattr(O, "apply_threshold", bad)
    with pytest.raises(AssertionError):
        tpins.test_threshold_keeps_exactly_the_lines_at_or_above_it()


# ------------------------------------------------------------ emission and state reductions
import oracle.emission as EM  # noqa: E402
from tests import test_oracle_emission as epins  # noqa: E402


def test_emissivity_from_the_lower_state_is_caught(monkeypatch):
    def bad(E, g, upper, lower, A, T, Q=None, index_base=0):
        E = np.asarray(E, np.float64); gg = np.asarray(g, np.float64)
        up = np.asarray(upper, np.int64) - index_base; lo = np.asarray(lower, np.int64) - index_base
        nu = E[up] - E[lo]
        Q = X.partition_function(E, g, T) if Q is None else Q
        return EM.H_PLANCK_CGS * O.C_LIGHT_CGS * gg[lo] * np.asarray(A) * nu * np.exp(-O.C2 * E[lo] / T) / (4 * math.pi * Q)
    monkeypatch.setattr(EM, "emissivities", bad)
    monkeypatch.setattr(O, "emissivities", bad)
    with pytest.raises(AssertionError):
        epins.test_emissivity_over_intensity_is_the_planck_function()


def test_heat_capacity_without_the_square_is_caught(monkeypatch):
    def bad(E, g, T):
        Q, Q1, Q2 = EM.partition_moments(E, g, T)
        return EM.R_GAS * (Q2 / Q - Q1 / Q) + 2.5 * EM.R_GAS
    monkeypatch.setattr(EM, "heat_capacity", bad)
    monkeypatch.setattr(O, "heat_capacity", bad)
    with pytest.raises(AssertionError):
        epins.test_heat_capacity_closed_forms()


# ------------------------------------------------------------ non-LTE populations
import oracle.nonlte as NL  # noqa: E402
from tests import test_oracle_nonlte as npins  # noqa: E402


def test_swapped_vibrational_and_rotational_temperatures_are_caught(monkeypatch):
    def swapped(E, E_vib, T_vib, T_rot):
        E = np.asarray(E, np.float64); Ev = np.asarray(E_vib, np.float64)
        return np.exp(-O.C2 * Ev / T_rot) * np.exp(-O.C2 * (E - Ev) / T_vib)
    monkeypatch.setattr(NL, "nlte_populations", swapped)
    with pytest.raises(AssertionError):
        npins.test_separable_spectrum_factorises()


def test_manifold_energy_from_the_highest_state_is_caught(monkeypatch):
    def highest(E, labels):
        E = np.asarray(E, np.float64); lab = np.asarray(labels, np.int64)
        top = {}
        for e, l in zip(E.tolist(), lab.tolist()):
            top[l] = max(top.get(l, e), e)
        return np.array([top[l] for l in lab.tolist()])
    monkeypatch.setattr(NL, "vibrational_energies", highest)
    monkeypatch.setattr(O, "vibrational_energies", highest)
    with pytest.raises(AssertionError):
        npins.test_separable_spectrum_factorises()


def test_non_lte_intensity_without_stimulated_emission_is_caught(monkeypatch):
    def no_stim(E, g, E_vib, upper, lower, A, T_vib, T_rot, Q=None, index_base=0):
        E = np.asarray(E, np.float64); Ev = np.asarray(E_vib, np.float64)
        up = np.asarray(upper, np.int64) - index_base; lo = np.asarray(lower, np.int64) - index_base
        nu = E[up] - E[lo]
        if Q is None:
            Q = NL.partition_function_nlte(E, g, Ev, T_vib, T_rot)
        F_low = NL.nlte_populations(E[lo], Ev[lo], T_vib, T_rot)
        gg = np.asarray(g, np.float64)
        return gg[up] * np.asarray(A, np.float64) / (8 * math.pi * O.C_LIGHT_CGS * nu * nu) * F_low / Q
    monkeypatch.setattr(NL, "intensities_nlte", no_stim)
    monkeypatch.setattr(O, "intensities_nlte", no_stim)
    with pytest.raises(AssertionError):
        npins.test_two_level_vibrational_band()
