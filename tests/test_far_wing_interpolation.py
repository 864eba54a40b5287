"""Interpolation error of the node-sampled Voigt far wing (FP32 path, CPU check of the design).

The FP32 Voigt sweep samples each far line (centre at least 24 node spacings from every
point of a wavefront of WW grid points) at 16 equispaced nodes across the wavefront and
interpolates the node sums to the points with an 8-point Lagrange stencil.  The wing it
samples is the 2-node Gauss-Hermite rational in x (|z| >= 40 there).  This checks, in
FP64, that the interpolation error of such a wing stays below 3e-8 relative over the
widths and distances it meets, and that the rational agrees with Re w (SciPy's wofz)
there; the profile rules themselves are pinned elsewhere.
"""
import math

import numpy as np
import pytest
from scipy.special import wofz

N_NODES, STENCIL, SPACINGS = 16, 8, 24


def reach(ww):
    return (SPACINGS * (ww - 1) + N_NODES - 2) // (N_NODES - 1)


def lagrange_rows(ww):
    """Per point o of the wavefront: stencil start and the 8 weights (nodes at m (ww-1)/15)."""
    rows = []
    for o in range(ww):
        u = o * (N_NODES - 1) / (ww - 1)
        i0 = min(max(int(math.floor(u)) - 3, 0), N_NODES - STENCIL)
        t = u - i0
        w = np.ones(STENCIL)
        for a in range(STENCIL):
            for b in range(STENCIL):
                if b != a:
                    w[a] *= (t - b) / (a - b)
        rows.append((i0, w))
    return rows


def two_node(x, y):
    q = x * x + y * y
    return y / math.sqrt(math.pi) * (q + 0.5) / ((q - 0.5) ** 2 + 2.0 * y * y)


@pytest.mark.parametrize("ww", [64, 128, 256])
def test_far_wing_interpolation_error(ww):
    rows = lagrange_rows(ww)
    nodes = np.arange(N_NODES) * (ww - 1) / (N_NODES - 1)
    pts = np.arange(ww, dtype=float)
    worst = 0.0
    for a_d in (0.002, 0.05, 0.5, 2.0, 5.0):                # Doppler HWHM in grid steps
        s = math.sqrt(math.log(2.0)) / a_d
        for dist in (reach(ww), reach(ww) + 0.5, 3 * reach(ww)):
            if dist * s < 40.0:                              # not a 2-node wing there
                continue
            for y in (1e-4, 0.1, 1.0, 10.0, 100.0, 1e3, 1e4):
                for side in (-1.0, 1.0):                     # line left or right of the wavefront
                    c = -dist if side < 0 else (ww - 1) + dist
                    f_pts = two_node(s * (pts - c), y)
                    f_nod = two_node(s * (nodes - c), y)
                    approx = np.array([np.dot(w, f_nod[i0:i0 + STENCIL]) for i0, w in rows])
                    worst = max(worst, float(np.max(np.abs(approx - f_pts) / f_pts)))
    assert worst < 3e-8, worst


def test_two_node_rational_is_the_far_wing():
    # beyond |z| = 40 the 2-node rule matches Re w to well inside the 1e-6 wing budget
    x = np.array([40.0, 200.0, 5e3, 1e6])
    for y in (1e-4, 1.0, 30.0):
        ref = wofz(x + 1j * y).real
        assert np.max(np.abs(two_node(x, y) - ref) / ref) < 1e-6
