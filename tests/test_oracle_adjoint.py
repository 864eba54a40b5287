"""The oracle's analytic adjoint against central finite differences of the oracle's
own forward cross section (a different computation: no derivative formulas)."""
import math

import numpy as np
import pytest

import oracle as O


def _case(seed=11, n_states=60, n_lines=25):
    rng = np.random.default_rng(seed)
    E = np.sort(rng.uniform(0, 3000, n_states))
    g = rng.integers(1, 30, n_states)
    up, lo = [], []
    while len(up) < n_lines:
        a, b = rng.integers(0, n_states, 2)
        if E[a] - E[b] > 10 and E[a] - E[b] < 60:
            up.append(a); lo.append(b)
    A = 10 ** rng.uniform(-2, 1, n_lines)
    gref = rng.uniform(0.02, 0.1, n_lines)
    nexp = rng.uniform(0.4, 0.8, n_lines)
    return E, g, np.array(up), np.array(lo), A, gref, nexp


GRID = (5.0, 70.0, 3251)
MASS, CUT = 34.0, 4.0


def _sigma(E, g, up, lo, A, gref, nexp, T, P):
    ls = O.make_lineset(E, g, up, lo, A, T, P, MASS, gamma_ref=gref, n_exp=nexp)
    return O.cross_section(ls, *GRID, CUT, workers=1)


def _loss(sig, ref):
    return float(np.sum((sig - ref) ** 2))


@pytest.mark.parametrize("T,P", [(1500.0, 0.1), (400.0, 1.0)])
def test_adjoint_matches_central_differences(T, P):
    E, g, up, lo, A, gref, nexp = _case()
    sig = _sigma(E, g, up, lo, A, gref, nexp, T, P)
    ref = _sigma(E, g, up, lo, A * 1.3, gref * 1.1, nexp, T * 1.05, P)
    gbar = 2.0 * (sig - ref)
    adj = O.voigt_adjoint(E, g, up, lo, A, gref, nexp, T, P, MASS, *GRID, gbar, cutoff=CUT)

    def L(**kw):
        args = dict(E=E, g=g, up=up, lo=lo, A=A, gref=gref, nexp=nexp, T=T, P=P)
        args.update(kw)
        return _loss(_sigma(**args), ref)

    def cd(fp, fm, h):
        return (fp - fm) / (2 * h)

    scale = abs(L()) + 1e-300
    h = 1e-6 * T
    assert abs(cd(L(T=T + h), L(T=T - h), h) - adj["dT"]) <= 1e-6 * abs(adj["dT"]) + 1e-9 * scale / T
    h = 1e-6 * P
    assert abs(cd(L(P=P + h), L(P=P - h), h) - adj["dP"]) <= 1e-6 * abs(adj["dP"]) + 1e-9 * scale / P
    for i in (0, 7, 13, 24):
        e = np.zeros_like(A); e[i] = 1.0
        hA = 1e-6
        d = cd(L(A=A * np.exp(hA * e)), L(A=A * np.exp(-hA * e)), hA)
        assert abs(d - adj["dlnA"][i]) <= 1e-6 * abs(d) + 1e-10 * scale
        hg = 1e-6 * gref[i]
        d = cd(L(gref=gref + hg * e), L(gref=gref - hg * e), hg)
        assert abs(d - adj["dgamma_ref"][i]) <= 1e-6 * abs(d) + 1e-10 * scale / gref[i]
        hn = 1e-6 * nexp[i]
        d = cd(L(nexp=nexp + hn * e), L(nexp=nexp - hn * e), hn)
        assert abs(d - adj["dn"][i]) <= 1e-6 * abs(d) + 1e-10 * scale / nexp[i]
