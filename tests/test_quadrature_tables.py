"""The quadrature tables the library's host code builds at plan creation, against
independent implementations: the Gauss-Hermite rules against NumPy's hermgauss, Weideman's
coefficients (SIAM J. Numer. Anal. 31, 1497 (1994)) through his rational form against
SciPy's wofz, and the core pre-pass's table of Dawson's function D(x) (Im w on the real
axis is (2/sqrt(pi)) D(x)) against SciPy's dawsn.  CPU only: the host routines are
compiled into a small driver, tests/host/quadrature_tables_host.cpp."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.special import dawsn, wofz

from tests.conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1801_09803_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("quadrature") / "quadrature_tables_host")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-x", "hip", "-I", CSRC,
                        "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host", "quadrature_tables_host.cpp"),
                        os.path.join(CSRC, "xs_quadrature.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    def run(*args):
        out = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, check=True, timeout=120)
        return out.stdout.split("\n")

    return run


# ---------------------------------------------------------------- Gauss-Hermite rules

@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 12, 24, 30, 31, 40, 64])
def test_gauss_hermite_rule_matches_numpy(driver, n):
    lines = driver("gh", n)
    assert int(lines[0]) == n
    tw = np.array([[float(v) for v in ln.split()] for ln in lines[1:n + 1]])
    t_ref, w_ref = np.polynomial.hermite.hermgauss(n)
    assert np.all(np.diff(tw[:, 0]) > 0)                        # ascending nodes
    assert np.max(np.abs(tw[:, 0] - t_ref)) < 1e-12 * max(1.0, np.max(np.abs(t_ref)))
    assert np.max(np.abs(tw[:, 1] - w_ref) / w_ref) < 1e-12
    assert abs(np.sum(tw[:, 1]) - np.sqrt(np.pi)) < 1e-13      # integral of exp(-t^2)


# ---------------------------------------------------------------- Weideman's w(z)

def weideman(lines, z):
    n, L = int(lines[0].split()[0]), float(lines[0].split()[1])
    a = np.array([float(v) for v in lines[1:n + 1]])
    Z = (L + 1j * z) / (L - 1j * z)
    p = np.zeros_like(z)
    for c in a[::-1]:                        # p(Z) = sum_m a_m Z^(m-1)
        p = p * Z + c
    return 2.0 * p / (L - 1j * z) ** 2 + 1.0 / (np.sqrt(np.pi) * (L - 1j * z))


def core_points():
    # the region where the library evaluates Weideman's form: |z| < 8, y >= 0.2, and the
    # real axis (whose imaginary part starts the small-y series in the FP64 path)
    x, y = np.meshgrid(np.linspace(-8.0, 8.0, 321), np.concatenate([[0.0], np.geomspace(0.2, 8.0, 60)]))
    z = (x + 1j * y).ravel()
    return z[np.abs(z) < 8.0]


# N = 24 serves the FP32 path (profile target 1e-5 relative), N = 40 the FP64 path (1e-10);
# measured: 8e-11 absolute and 7e-9 relative in Re w (N = 24), 1e-15 and 2e-14 (N = 40)
@pytest.mark.parametrize("n,abs_tol,rel_tol", [(24, 2e-10, 2e-8), (40, 1e-14, 2e-13)])
def test_weideman_coefficients_reproduce_wofz(driver, n, abs_tol, rel_tol):
    z = core_points()
    got, ref = weideman(driver("weideman", n), z), wofz(z)
    assert np.max(np.abs(got - ref)) < abs_tol
    off = z.imag >= 0.2                       # relative accuracy of Re w where it is used
    assert np.max(np.abs(got[off].real - ref[off].real) / ref[off].real) < rel_tol


def test_weideman_L_is_the_published_choice(driver):
    for n in (24, 40):
        L = float(driver("weideman", n)[0].split()[1])
        assert L == pytest.approx(np.sqrt(n / np.sqrt(2.0)), rel=1e-15)


# ---------------------------------------------------------------- Dawson's function

@pytest.fixture(scope="module")
def table(driver):
    lines = driver("dawson")
    n_iv, n_c = map(int, lines[0].split())
    return np.array([float(v) for v in lines[1:1 + n_iv * n_c]]).reshape(n_iv, n_c)


def evaluate(t, x):
    # one polynomial per half-unit interval of |x| < 8.5, in u = 4 (x - (i/2 + 1/4)),
    # Horner in u, odd extension
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
        left = np.sum(table[i])                                            # u = +1 of interval i
        right = np.sum(table[i + 1] * (-1.0) ** np.arange(table.shape[1]))   # u = -1 of interval i+1
        assert abs(left - right) < 1e-14, i


def test_dawson_table_small_x_limit(table):
    # D(x) = x - 2x^3/3 + 4x^5/15 - ... near 0, and D(0) = 0; the table's error there is
    # absolute (its interval 0 is centred on x = 1/4), so the tolerance is too
    x = np.array([0.0, 1e-8, 1e-6, 1e-4, 1e-2])
    series = x - 2.0 * x ** 3 / 3.0 + 4.0 * x ** 5 / 15.0
    assert np.max(np.abs(evaluate(table, x) - series)) < 2e-15
    assert np.max(np.abs(evaluate(table, -x) + series)) < 2e-15
