"""GPU parity of the HIP path against the FP64 CPU oracle (through the C ABI).

Tolerances: the FP32 path must match the oracle within 1e-5 relative (max over grid
points above 1e-6 of the maximum, and integrated area); the FP64 path within 1e-10.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import assert_parity, device_linelist, host, log, make_plan, oracle_lineset

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-10


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["C1"]
    d = device_linelist(cfg)
    h = host(d)
    return cfg, d, h


def _run(plan, d, T, P, with_broad=True):
    plan.set_states(d["E"], d["g"], d["J"])
    if with_broad:
        plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    else:
        plan.set_lines(d["upper"], d["lower"], d["A"])
    out = plan.cross_section(T, P)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def test_partition_function_matches_fsum(c1):
    cfg, d, h = c1
    plan = make_plan(cfg)
    plan.set_states(d["E"], d["g"], d["J"])
    Ts = [100.0, 296.0, 1000.0, 3000.0]
    Q, dQ = plan.partition_function(Ts)
    Q, dQ = Q.cpu().numpy(), dQ.cpu().numpy()
    for i, T in enumerate(Ts):
        q = O.partition_function(h["E"], h["g"], T)
        dq = O.partition_function_dT(h["E"], h["g"], T)
        log(f"  Q({T}) rel err {abs(Q[i]-q)/q:.2e}  dQ/dT rel err {abs(dQ[i]-dq)/abs(dq):.2e}")
        assert abs(Q[i] - q) <= 1e-13 * q
        assert abs(dQ[i] - dq) <= 1e-13 * abs(dq)


@pytest.fixture(scope="module")
def c1_oracle(c1):
    cfg, d, h = c1
    T, P = cfg.temperatures[0], cfg.pressures[0]
    ls = oracle_lineset(h, cfg, T, P)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile="voigt", workers=1)
    return ref


@pytest.mark.parametrize("spw", [1, 2, 4])
def test_c1_voigt_fp32(c1, c1_oracle, spw):
    cfg, d, h = c1
    log(f"C1 voigt fp32 slices_per_wave={spw}")
    plan = make_plan(cfg, "fp32", slices_per_wave=spw)
    got = _run(plan, d, [cfg.temperatures[0]], [cfg.pressures[0]])[0]
    assert_parity(got, c1_oracle, TOL32, what=f"C1 voigt fp32 P={spw}")
    assert plan.lines_kept() == cfg.n_lines


def test_c1_voigt_fp64(c1, c1_oracle):
    cfg, d, h = c1
    log("C1 voigt fp64")
    plan = make_plan(cfg, "fp64")
    got = _run(plan, d, [cfg.temperatures[0]], [cfg.pressures[0]])[0]
    assert_parity(got, c1_oracle, TOL64, what="C1 voigt fp64")


@pytest.mark.parametrize("profile", ["doppler", "lorentz", "gauss_fixed"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c1_other_profiles(c1, profile, precision):
    cfg, d, h = c1
    log(f"C1 {profile} {precision}")
    n = 20000
    sub = {k: (v[:n] if k in ("upper", "lower", "A", "gamma_ref", "n_exp") else v) for k, v in d.items()}
    hs = {k: (v[:n] if k in ("upper", "lower", "A", "gamma_ref", "n_exp") else v) for k, v in h.items()}
    T, P = 700.0, 3.0
    kw = dict(alpha_fixed=0.3) if profile == "gauss_fixed" else {}
    plan = make_plan(cfg, precision, profile=profile, **kw)
    got = _run(plan, sub, [T], [P])[0]
    ls = oracle_lineset(hs, cfg, T, P)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile=profile,
                          alpha_fixed=kw.get("alpha_fixed", 0.0), workers=1)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"{profile} {precision}")


def _small_case(seed, n_states=400, n_lines=3000, numax=300.0):
    cfg = synth.WorkloadConfig("tiny", 90 + seed, n_states, n_lines, 28.0, numax, 0.0, 200.0, 20001,
                               (800.0,), (0.5,), cutoff=25.0)
    return cfg, synth.make_linelist(cfg, device="cuda")


@pytest.mark.parametrize("T,P", [(100.0, 1e-5), (300.0, 0.0), (3000.0, 100.0), (1500.0, 0.1)])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_voigt_extreme_widths(T, P, precision):
    # narrow Doppler lines at low T and P, pure Doppler at P = 0, broad lines at 100 bar;
    # the grid (20001 points, dnu = 0.01) spans several tiles with a ragged last tile, and
    # lines centred beyond the grid end overlap it through their windows
    cfg, d = _small_case(1)
    log(f"voigt extremes T={T} P={P} {precision}")
    h = host(d)
    plan = make_plan(cfg, precision)
    got = _run(plan, d, [T], [P])[0]
    ls = oracle_lineset(h, cfg, T, P)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=1)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"T={T} P={P} {precision}")


def test_batched_tp_equals_single_calls():
    cfg, d = _small_case(2)
    plan = make_plan(cfg, "fp32")
    Ts, Ps = [200.0, 900.0, 2500.0], [0.01, 1.0, 30.0]
    allr = _run(plan, d, Ts, Ps)
    for i in range(3):
        one = plan.cross_section([Ts[i]], [Ps[i]])
        torch.cuda.synchronize()
        assert np.array_equal(one.double().cpu().numpy()[0], allr[i])


def test_deterministic_bitwise():
    cfg, d = _small_case(3)
    plan = make_plan(cfg, "fp32")
    a = _run(plan, d, [1000.0], [1.0])
    b = plan.cross_section([1000.0], [1.0]).double().cpu().numpy()
    assert np.array_equal(a, b)


def test_tile_shapes_agree():
    cfg, d = _small_case(4)
    outs = []
    for spw in (1, 2, 4, 8):
        plan = make_plan(cfg, "fp32", slices_per_wave=spw)
        outs.append(_run(plan, d, [1000.0], [1.0])[0])
    for o in outs[1:]:
        m = O.error_metrics(o, outs[0])
        assert m["max_rel"] < 2e-6


def test_index_base_and_a0_broadening():
    cfg, d = _small_case(5)
    h = host(d)
    gt, nt = synth.make_broadening_table(cfg.seed)
    gt, nt = gt.numpy(), nt.numpy()
    plan = make_plan(cfg, "fp64", broadening="a0_jlower", index_base=1)
    plan.set_broadening_table(gt, nt)
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"] + 1, d["lower"] + 1, d["A"])
    got = plan.cross_section([1200.0], [2.0]).cpu().numpy()[0]
    ls = O.make_lineset(h["E"], h["g"], h["upper"], h["lower"], h["A"], 1200.0, 2.0, cfg.mass_amu,
                        J=h["J"], broad_table=(gt, nt))
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=1)
    assert_parity(got, ref, TOL64, what="a0 + index_base 1")


def test_const_broadening():
    cfg, d = _small_case(6)
    h = host(d)
    plan = make_plan(cfg, "fp32", broadening="const", gamma_const=0.07, n_const=0.5)
    got = _run(plan, d, [500.0], [1.0], with_broad=False)[0]
    ls = O.make_lineset(h["E"], h["g"], h["upper"], h["lower"], h["A"], 500.0, 1.0, cfg.mass_amu,
                        gamma_const=0.07, n_const=0.5)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=1)
    assert_parity(got, ref, TOL32, what="const broadening")


def test_empty_and_dropped_lines():
    cfg, d = _small_case(7)
    plan = make_plan(cfg, "fp32")
    plan.set_states(d["E"], d["g"], d["J"])
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    plan.set_lines(e, e, torch.empty(0, dtype=torch.float32, device="cuda"),
                   torch.empty(0, dtype=torch.float32, device="cuda"),
                   torch.empty(0, dtype=torch.float32, device="cuda"))
    assert plan.lines_kept() == 0
    out = plan.cross_section([300.0], [1.0])
    assert torch.count_nonzero(out).item() == 0
    # every line far beyond the grid: all dropped
    plan2 = make_plan(synth.WorkloadConfig("far", 0, 1, 1, 28.0, 1.0, 0.0, 10.0, 1001, (1.0,), (1.0,)), "fp32")
    E = torch.tensor([0.0, 500.0, 900.0], dtype=torch.float64, device="cuda")
    g = torch.ones(3, dtype=torch.int32, device="cuda")
    plan2.set_states(E, g)
    up = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    lo = torch.tensor([0, 0], dtype=torch.int32, device="cuda")
    one = torch.ones(2, dtype=torch.float32, device="cuda")
    plan2.set_lines(up, lo, one, one * 0.05, one * 0.5)
    assert plan2.lines_kept() == 0
    assert torch.count_nonzero(plan2.cross_section([300.0], [1.0])).item() == 0


def test_invalid_transitions_report_errors():
    from paper_1801_09803_amd import XsecError
    cfg, d = _small_case(8, n_lines=100)
    plan = make_plan(cfg, "fp32")
    plan.set_states(d["E"], d["g"], d["J"])
    bad = d["upper"].clone()
    bad[17] = cfg.n_states + 5
    with pytest.raises(XsecError) as ei:
        plan.set_lines(bad, d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    assert ei.value.name == "XS_ERR_INDEX"
    with pytest.raises(XsecError) as ei:
        plan.set_lines(d["lower"], d["upper"], d["A"], d["gamma_ref"], d["n_exp"])   # nu < 0
    assert ei.value.name == "XS_ERR_NU_NONPOS"
    with pytest.raises(XsecError) as ei:
        plan.cross_section([300.0], [1.0])      # no valid line set after the failures
    assert ei.value.name == "XS_ERR_STATE"
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    with pytest.raises(XsecError) as ei:
        plan.cross_section([-5.0], [1.0])
    assert ei.value.name == "XS_ERR_ARG"


@pytest.mark.parametrize("profile", ["gh_sampled", "gh_binned"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("T,P", [(800.0, 0.5), (2500.0, 0.02)])
def test_gauss_hermite_profiles(profile, precision, T, P):
    cfg, d = _small_case(9, n_lines=1500)
    h = host(d)
    plan = make_plan(cfg, precision, profile=profile)
    got = _run(plan, d, [T], [P])[0]
    ls = oracle_lineset(h, cfg, T, P)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile=profile, workers=1)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"{profile} {precision} T={T}")


@pytest.mark.parametrize("profile", ["gh_sampled", "gh_binned"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n_gh", [1, 2, 20, 31, 64])
def test_gauss_hermite_rule_size(profile, precision, n_gh):
    # gh_nodes: the Gauss-Hermite rule of Eq. 30-31 with n_gh nodes (odd rules hold a node
    # at zero; one node is the Lorentzian itself) against the oracle's rule of that size
    cfg, d = _small_case(11, n_lines=1200)
    h = host(d)
    plan = make_plan(cfg, precision, profile=profile, gh_nodes=n_gh)
    got = _run(plan, d, [1200.0], [0.3])[0]
    ls = oracle_lineset(h, cfg, 1200.0, 0.3)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile=profile, n_gh=n_gh, workers=1)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"{profile} {precision} n_gh={n_gh}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_gh_binned_pure_doppler_limit(precision):
    # P = 0: each node becomes a delta function; the binned profile is a 30-point
    # histogram of the Gaussian (the oracle's step-function limit)
    cfg, d = _small_case(10, n_lines=1500)
    h = host(d)
    plan = make_plan(cfg, precision, profile="gh_binned")
    got = _run(plan, d, [1000.0], [0.0])[0]
    ls = oracle_lineset(h, cfg, 1000.0, 0.0)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile="gh_binned", workers=1)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"gh_binned P=0 {precision}")


@pytest.mark.parametrize("T", [1000.0, 3000.0])
def test_far_wing_zone_accuracy(T):
    # sparse lines on a fine grid: between lines the cross section is made of far wings,
    # most of them in the one-pole zone (|x| >= 1000, relative error <= 1e-6) of the FP32
    # path; the whole result stays within a few 1e-6 of the oracle
    cfg = synth.WorkloadConfig("far", 77, 2000, 300, 34.0, 2100.0, 0.0, 2000.0, 200001, (T,), (1.0,))
    d = device_linelist(cfg)
    h = host(d)
    got = _run(make_plan(cfg, "fp32"), d, [T], [1.0])[0]
    ls = oracle_lineset(h, cfg, T, 1.0)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff)
    assert_parity(got, ref, 3e-6, what=f"far-wing zone T={T}")
    # the gaps, far below the usual floor of 1e-6 of the maximum, point by point
    m = ref > 1e-12 * ref.max()
    rel = np.abs(got[m] - ref[m]) / ref[m]
    log(f"  far-wing zone T={T}: max rel {rel.max():.3e} over {m.sum()} points above 1e-12 of the maximum")
    assert m.sum() > 100000
    assert rel.max() <= 3e-6


def test_far_wing_inside_the_mid_zone_radius():
    # a fine grid (0.001 cm^-1) at 3000 K: Doppler widths of ~17 grid steps put the
    # |z| < 40 radius (~800 steps) far beyond the far-wing reach (146 steps for 256-point
    # wavefronts) and the |z| < 8 radius (~160 steps) beyond it too: the node-sampled
    # lines start at the |z| < 8 radius, and those inside the |z| < 40 radius take the
    # 4-node rule at the nodes
    cfg = synth.WorkloadConfig("fine", 78, 3000, 200000, 34.0, 10000.0, 4995.0, 5005.0, 10001,
                               (3000.0,), (1.0,), cutoff=5.0)
    d = device_linelist(cfg)
    h = host(d)
    plan = make_plan(cfg, "fp32")
    plan.set_timing(True)
    got = _run(plan, d, [3000.0], [1.0])[0]
    t = plan.kernel_times()
    assert t["far_launches"] > 0
    ls = oracle_lineset(h, cfg, 3000.0, 1.0)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff)
    assert_parity(got, ref, TOL32, what="fine grid, 3000 K")


@pytest.mark.parametrize("waves,slices", [(1, 4), (2, 2), (1, 1), (4, 2), (1, 8), (2, 8)])
def test_window_ends_at_the_grid_edges(waves, slices):
    # lines centred within 40 cm^-1 of either end of a fine grid (0.01 cm^-1, cut-off 25):
    # their windows start or end inside wavefronts all along both edges, many clipped at the
    # grid's first or last point, with and without a ragged last wavefront (20001 points);
    # broad lines (30 bar) make the wings count.  The far-wing kernel node-samples these
    # window ends; the whole grid is checked against the oracle.
    cfg = synth.WorkloadConfig("edges", 515, 3000, 60000, 28.0, 260.0, 0.0, 200.0, 20001, (1500.0,), (30.0,))
    d = device_linelist(cfg)
    E = d["E"]
    nu = E[d["upper"].long()] - E[d["lower"].long()]
    keep = ((nu < 40.0) | ((nu > 160.0) & (nu < 240.0))).nonzero().squeeze(1)
    d = dict(d, **{k: d[k][keep].contiguous() for k in ("upper", "lower", "A", "gamma_ref", "n_exp")})
    h = host(d)
    log(f"edges: {keep.numel()} lines, tile {waves} x {slices}")
    plan = make_plan(cfg, "fp32", waves_per_block=waves, slices_per_wave=slices, n_split=4)
    got = _run(plan, d, [1500.0], [30.0])[0]
    ls = oracle_lineset(h, cfg, 1500.0, 30.0)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=1)
    assert_parity(got, ref, TOL32, what=f"grid edges {waves}x{slices}")


@pytest.mark.parametrize("waves,slices", [(1, 4), (2, 2)])
def test_narrow_lines_centred_past_the_grid_end(waves, slices):
    # Doppler-narrow lines (300 K, 1e-3 bar: cores of a few grid steps) centred up to 40
    # cm^-1 beyond the last point of a grid whose last wavefront is ragged (20001 points):
    # their core ranges, clipped to the grid, are empty, while the last 64-point slice runs
    # past the grid's end over their centres; such lines must take the 4-node rule there,
    # never stored core values.  The whole grid is checked against the oracle.
    cfg = synth.WorkloadConfig("past_end", 516, 3000, 60000, 28.0, 260.0, 0.0, 200.0, 20001, (300.0,), (1e-3,))
    d = device_linelist(cfg)
    E = d["E"]
    nu = E[d["upper"].long()] - E[d["lower"].long()]
    keep = ((nu > 150.0) & (nu < 240.0)).nonzero().squeeze(1)
    d = dict(d, **{k: d[k][keep].contiguous() for k in ("upper", "lower", "A", "gamma_ref", "n_exp")})
    h = host(d)
    n_past = int((nu[keep] > 200.0).sum().item())
    log(f"past end: {keep.numel()} lines ({n_past} centred past the grid), tile {waves} x {slices}")
    assert n_past > 100
    plan = make_plan(cfg, "fp32", waves_per_block=waves, slices_per_wave=slices, n_split=4)
    got = _run(plan, d, [300.0], [1e-3])[0]
    ls = oracle_lineset(h, cfg, 300.0, 1e-3)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=1)
    assert_parity(got, ref, TOL32, what=f"past grid end {waves}x{slices}")
