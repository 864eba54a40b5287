"""GPU parity of the bin-averaged Gaussian / Lorentzian profiles and the super-line
histograms against the FP64 oracle, through the C ABI (1e-5 for the FP32 path, 1e-10
for the FP64 path; super-line sums 1e-12 (FP64) and float rounding (FP32))."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import assert_parity, host, log, make_plan, oracle_lineset

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-10


def _case(seed, n_lines=3000, numax=300.0, nu_a=0.0, nu_b=200.0, n_points=20001, mass=28.0, n_states=400):
    cfg = synth.WorkloadConfig("binned", 50 + seed, n_states, n_lines, mass, numax, nu_a, nu_b, n_points,
                               (800.0,), (0.5,), cutoff=25.0)
    return cfg, synth.make_linelist(cfg, device="cuda")


def _run(plan, d, Ts, Ps):
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    out = plan.cross_section(Ts, Ps)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("profile", ["doppler_binned", "lorentz_binned"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("grid", ["fine", "coarse"])
def test_binned_profiles(profile, precision, grid):
    # fine: dnu = 0.01 (bins much narrower than the lines); coarse: dnu = 1 (bins wider
    # than the Doppler widths, the case the paper recommends them for)
    if grid == "fine":
        cfg, d = _case(1)
        T, P = 800.0, 0.5
    else:
        cfg, d = _case(2, n_lines=20000, numax=2100.0, nu_a=0.0, nu_b=2000.0, n_points=2001, n_states=2000)
        T, P = 1500.0, 0.05
    h = host(d)
    log(f"{profile} {precision} {grid}")
    got = _run(make_plan(cfg, precision, profile=profile), d, [T], [P])[0]
    ls = oracle_lineset(h, cfg, T, P)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile=profile)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"{profile} {precision} {grid}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_lorentz_binned_pure_doppler_limit(precision):
    # P = 0: each line's intensity lands in its own bin (the step limit)
    cfg, d = _case(3, n_lines=1500, n_points=2001)
    h = host(d)
    got = _run(make_plan(cfg, precision, profile="lorentz_binned"), d, [600.0], [0.0])[0]
    ls = oracle_lineset(h, cfg, 600.0, 0.0)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile="lorentz_binned")
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"lorentz_binned P=0 {precision}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_super_lines_match_the_oracle_histogram(precision):
    cfg, d = _case(4, n_lines=200000, numax=260.0, nu_a=10.0, nu_b=250.0, n_points=4801, n_states=5000)
    h = host(d)
    Ts, Ps = [296.0, 2000.0], [1.0, 1.0]
    got = _run(make_plan(cfg, precision, profile="superlines"), d, Ts, Ps)
    for i, T in enumerate(Ts):
        ls = oracle_lineset(h, cfg, T, 1.0)
        ref = O.super_line_histogram(ls, cfg.nu_a, cfg.nu_b, cfg.n_points)
        if precision == "fp64":
            assert np.array_equal(got[i] == 0.0, ref == 0.0)   # the same bins are occupied
            m = ref > 0
        else:
            m = ref > 1e-6 * ref.max()   # float output: the usual parity floor
        rel = np.abs(got[i][m] - ref[m]) / ref[m]
        log(f"  super-lines {precision} T={T}: max rel {rel.max():.2e} over {m.sum()} bins")
        assert rel.max() <= (1e-12 if precision == "fp64" else 1e-6)


def test_super_lines_graph_replay_equals_direct_call():
    cfg, d = _case(5, n_lines=50000, n_points=2001)
    plan = make_plan(cfg, "fp32", profile="superlines")
    Ts, Ps = [300.0, 1200.0], [1.0, 1.0]
    ref = _run(plan, d, Ts, Ps)
    g = plan.graph(Ts, Ps)
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.double().cpu().numpy(), ref), rep
        plan.cross_section([Ts[0]], [Ps[0]])
        torch.cuda.synchronize()
