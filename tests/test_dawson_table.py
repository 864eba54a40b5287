"""The core pre-pass's table of Dawson's function D(x) (Im w on the real axis is
(2/sqrt(pi)) D(x)), as the library's host code builds it at plan creation, against SciPy's
dawsn, an independent implementation: one polynomial per half-unit interval of |x| < 8.5
in u = 4 (x - (i/2 + 1/4)), evaluated as the kernel does (Horner in u).  CPU only: the host
routine is compiled into a small driver."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.special import dawsn

from tests.conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1801_09803_amd", "csrc")


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    out = tmp_path_factory.mktemp("dawson")
    exe = str(out / "dawson_table_host")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-x", "hip", "-I", CSRC,
                        "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host", "dawson_table_host.cpp"),
                        os.path.join(CSRC, "xs_quadrature.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = subprocess.run([exe], capture_output=True, text=True, check=True, timeout=60).stdout.split()
    n_iv, n_c = int(lines[0]), int(lines[1])
    return np.array([float(v) for v in lines[2:]]).reshape(n_iv, n_c)


def evaluate(t, x):
    ax = np.abs(x)
    iv = np.minimum((ax * 2.0).astype(int), t.shape[0] - 1)
    u = (ax - (0.5 * iv + 0.25)) * 4.0
    p = np.zeros_like(x)
    for j in range(t.shape[1] - 1, -1, -1):
        p = p * u + t[iv, j]
    return np.copysign(p, x)


def test_dawson_table_matches_scipy(table):
    x = np.linspace(-8.49, 8.49, 170001)
    got, ref = evaluate(table, x), dawsn(x)
    assert np.max(np.abs(got - ref)) < 5e-15
    big = np.abs(x) > 0.5
    assert np.max(np.abs(got[big] - ref[big]) / np.abs(ref[big])) < 1e-13


def test_dawson_table_is_continuous_across_intervals(table):
    # the two polynomials meeting at each interval boundary agree there
    for i in range(table.shape[0] - 1):
        left = sum(table[i, j] * 1.0 ** j for j in range(table.shape[1]))      # u = +1 of interval i
        right = sum(table[i + 1, j] * (-1.0) ** j for j in range(table.shape[1]))   # u = -1 of interval i+1
        assert abs(left - right) < 1e-14, i


def test_dawson_table_small_x_limit(table):
    # D(x) = x - 2x^3/3 + 4x^5/15 - ... near 0, and D(0) = 0; the table's error there is
    # absolute (its interval 0 is centred on x = 1/4), so the tolerance is too
    x = np.array([0.0, 1e-8, 1e-6, 1e-4, 1e-2])
    series = x - 2.0 * x ** 3 / 3.0 + 4.0 * x ** 5 / 15.0
    assert np.max(np.abs(evaluate(table, x) - series)) < 2e-15
    assert np.max(np.abs(evaluate(table, -x) + series)) < 2e-15
