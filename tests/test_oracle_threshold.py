"""Pins of the intensity-threshold oracle (CPU only): the HITRAN cut-off's limits and a
brute-force selection with explicit comparisons."""
import math

import numpy as np

import oracle as O


def test_hitran_cutoff_limits():
    # Sec. "Intensity thresholds": I_crit above nu_crit; below it I_crit (nu/nu_crit)
    # tanh(c2 nu/(2T)), which for c2 nu << T is quadratic in nu and for c2 nu >> T linear
    T = 296.0
    assert np.all(O.intensity_cutoff([2000.0001, 5000.0, 12000.0], T, "hitran") == 1e-29)
    small = np.array([0.01, 0.02, 0.04])
    c = O.intensity_cutoff(small, T, "hitran")
    assert np.allclose(c[1:] / c[:-1], 4.0, rtol=1e-8)
    k = O.C2 / (2 * T)   # c2 / (2T), c2 = hc/k_B in cm K
    x = 0.01 * k
    assert abs(c[0] - 1e-29 * (0.01 / 2000.0) * x * (1 - x * x / 3)) < 1e-12 * c[0]   # tanh x = x - x^3/3 + ...
    big = O.intensity_cutoff(np.array([1000.0, 1500.0]), 50.0, "hitran")
    assert abs(big[1] / big[0] - 1.5) < 1e-11                      # tanh saturated at 50 K
    # at 296 K the two branches nearly meet at nu_crit (tanh(4.86) = 0.99988)
    edge = O.intensity_cutoff(np.array([2000.0]), 296.0, "hitran")[0]
    assert 0.9998 < edge / 1e-29 < 1.0


def test_threshold_keeps_exactly_the_lines_at_or_above_it():
    rng = np.random.default_rng(2)
    n = 400
    nu = rng.uniform(1.0, 6000.0, n)
    I = 10 ** rng.uniform(-34, -24, n)
    ls = O.LineSet(nu, I, np.full(n, 0.01), np.full(n, 0.02))
    for mode, ic in (("constant", 1e-29), ("hitran", 1e-29), ("hitran", 1e-27)):
        kept = O.apply_threshold(ls, 500.0, mode, ic, 2000.0)
        ref = []
        for i in range(n):
            if mode == "constant":
                cut = ic
            elif nu[i] <= 2000.0:
                cut = ic * (nu[i] / 2000.0) * math.tanh(O.C2 * nu[i] / (2 * 500.0))
            else:
                cut = ic
            if I[i] >= cut:
                ref.append(i)
        assert np.array_equal(kept.nu, nu[ref]) and np.array_equal(kept.I, I[ref])
    # a line exactly at the threshold is kept
    one = O.LineSet(np.array([3000.0]), np.array([1e-29]), np.array([0.01]), np.array([0.01]))
    assert len(O.apply_threshold(one, 300.0, "constant", 1e-29)) == 1
