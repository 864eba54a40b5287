"""Interpolation error of the node-sampled Voigt far wing (FP32 path, CPU check of the design).

The FP32 Voigt sweep samples each far line (centre at least R = max(0.57 (WW - 1), the
|z| < 8 radius) grid steps from every point of a wavefront of WW points) at the 16
Chebyshev points of the first kind across the wavefront (positions rounded to float, as
the kernel computes them) and takes the degree-15 polynomial through the node sums at
each point (barycentric form).  The wing it samples is the 2-node Gauss-Hermite rational
in x where |z| >= 40, the 4-node one where 8 <= |z| < 40.  This checks, in FP64, that the
interpolation error of such wings stays below 3e-8 relative over the widths and distances
they meet, and that the rationals agree with Re w (SciPy's wofz) there; the profile rules
themselves are pinned elsewhere.
"""
import math

import numpy as np
import pytest
from scipy.special import roots_hermite, wofz

N_NODES = 16


def reach(ww):
    return (57 * (ww - 1) + 99) // 100


def node_positions(ww):
    m = np.arange(N_NODES)
    u = (1.0 - np.cos(np.pi * (2 * m + 1) / (2 * N_NODES))) / 2.0
    return ((ww - 1) * u).astype(np.float32).astype(np.float64)


def weights(ww):
    """Rows of the interpolation weights, one per point of the wavefront."""
    p = node_positions(ww)
    c = np.array([1.0 / np.prod([p[m] - p[k] for k in range(N_NODES) if k != m]) for m in range(N_NODES)])
    o = np.arange(ww, dtype=float)[:, None]
    t = c / (o - p)
    return t / t.sum(axis=1, keepdims=True)


def gh_rule(x, y, n):
    t, w = roots_hermite(n)
    return (y / math.pi) * sum(wj / ((x - tj) ** 2 + y * y) for tj, wj in zip(t, w))


def worst_error(ww, rule, distances, widths, ys, zone):
    wt = weights(ww)
    nodes = node_positions(ww)
    pts = np.arange(ww, dtype=float)
    worst, cases = 0.0, 0
    for a_d in widths:                                       # Doppler HWHM in grid steps
        s = math.sqrt(math.log(2.0)) / a_d
        for dist in distances:
            for y in ys:
                for side in (-1.0, 1.0):                     # line left or right of the wavefront
                    c = -dist if side < 0 else (ww - 1) + dist
                    z_near = math.hypot(s * dist, y)
                    if not zone(s * dist, z_near):
                        continue
                    f_pts = gh_rule(s * (pts - c), y, rule)
                    f_nod = gh_rule(s * (nodes - c), y, rule)
                    worst = max(worst, float(np.max(np.abs(wt @ f_nod - f_pts) / f_pts)))
                    cases += 1
    return worst, cases


@pytest.mark.parametrize("ww", [64, 128, 256, 512])
def test_two_node_far_wing_interpolation_error(ww):
    r = reach(ww)
    worst, cases = worst_error(ww, 2, (r, r + 0.5, 2 * r, 6 * r), (0.002, 0.05, 0.5, 2.0, 5.0),
                               (1e-4, 0.1, 1.0, 10.0, 100.0, 1e3, 1e4), lambda x, z: z >= 40.0)
    assert cases > 20
    assert worst < 3e-8, worst


@pytest.mark.parametrize("ww", [64, 128, 256, 512])
def test_four_node_far_wing_interpolation_error(ww):
    # lines inside the |z| < 40 radius but beyond R: every point at |x| >= 8
    r = reach(ww)
    widths = [r / 8.0 * f for f in (0.1, 0.5, 1.0)] + [r / 30.0]
    worst, cases = worst_error(ww, 4, (r, r + 0.5, 1.5 * r, 3 * r), widths, (1e-4, 0.1, 1.0, 5.0, 20.0),
                               lambda x, z: x >= 8.0 and z < 40.0)
    assert cases > 10
    assert worst < 3e-8, worst


def test_interpolation_reproduces_degree_15_polynomials():
    # the weights are those of the interpolating polynomial at the rounded node positions
    rng = np.random.default_rng(7)
    for ww in (64, 512):
        coef = rng.standard_normal(16)
        f = lambda v: np.polynomial.polynomial.polyval(v / (ww - 1), coef)
        got = weights(ww) @ f(node_positions(ww))
        assert np.max(np.abs(got - f(np.arange(ww, dtype=float)))) < 1e-9 * np.max(np.abs(coef)) * 16


def test_gh_rules_are_the_far_wing():
    # beyond |z| = 40 the 2-node rule, for 8 <= |z| < 40 the 4-node rule, match Re w to well
    # inside the 1e-6 wing budget
    x = np.array([40.0, 200.0, 5e3, 1e6])
    for y in (1e-4, 1.0, 30.0):
        ref = wofz(x + 1j * y).real
        assert np.max(np.abs(gh_rule(x, y, 2) - ref) / ref) < 1e-6
    for x in (8.0, 12.0, 30.0):
        for y in (1e-4, 0.5, 3.0):
            ref = wofz(x + 1j * y).real
            assert abs(gh_rule(x, y, 4) - ref) / ref < 1e-6
