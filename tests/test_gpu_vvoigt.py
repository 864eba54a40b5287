"""GPU parity of the Vectorized Voigt profiles (V-V, and the area-normalised VVN) against
the FP64 oracle, through the C ABI.  Tolerances as for the Voigt profile: 1e-5 for the
FP32 path, 1e-10 for the FP64 path."""
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
    cfg = synth.WorkloadConfig("vv", 70 + seed, n_states, n_lines, mass, numax, nu_a, nu_b, n_points,
                               (800.0,), (0.5,), cutoff=25.0)
    return cfg, synth.make_linelist(cfg, device="cuda")


def _run(plan, d, Ts, Ps):
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    out = plan.cross_section(Ts, Ps)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def _near_grid(ls, cfg):
    """The oracle's lines restricted to those whose window can reach the grid (the others
    add nothing; the normalised form would otherwise sum their whole windows)."""
    m = (ls.nu >= cfg.nu_a - cfg.cutoff - 1.0) & (ls.nu <= cfg.nu_b + cfg.cutoff + 1.0)
    return O.LineSet(ls.nu[m], ls.I[m], ls.alpha_d[m], ls.gamma[m])


def _oracle_vv(h, cfg, T, P, radius, beta, norm):
    ls = _near_grid(oracle_lineset(h, cfg, T, P), cfg)
    return O.cross_section_vv(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, T, cfg.mass_amu, cutoff=cfg.cutoff,
                              radius=radius, use_beta=beta, normalise=norm)


@pytest.mark.parametrize("profile", ["vvoigt", "vvoigt_norm"])
@pytest.mark.parametrize("beta", [False, True])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("T,P", [(296.0, 1.0), (2500.0, 0.05)])
def test_vv_fine_grid(profile, beta, precision, T, P):
    # dnu = 0.01: 5001-point windows, the FP32 path's segmented sweep with the wing runs
    # split at R; lines centred beyond the grid end reach it through their windows
    cfg, d = _case(1)
    h = host(d)
    log(f"{profile} beta={beta} {precision} T={T} P={P}")
    plan = make_plan(cfg, precision, profile=profile, vv_beta=beta)
    got = _run(plan, d, [T], [P])[0]
    ref = _oracle_vv(h, cfg, T, P, 4.0, beta, profile == "vvoigt_norm")
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"{profile} {precision} T={T}")


@pytest.mark.parametrize("spw", [2, 4])
@pytest.mark.parametrize("profile", ["vvoigt", "vvoigt_norm"])
def test_vv_coarse_grid(spw, profile):
    # dnu = 0.1 (501-point windows); 4 slices per wavefront leave no room for the
    # segmented sweep, so every line carries per-slice codes
    cfg, d = _case(2, n_lines=20000, numax=2100.0, nu_a=0.0, nu_b=2000.0, n_points=20001, mass=18.0,
                   n_states=2000)
    h = host(d)
    log(f"{profile} coarse spw={spw}")
    plan = make_plan(cfg, "fp32", profile=profile, vv_beta=True, slices_per_wave=spw)
    got = _run(plan, d, [1000.0], [1.0])[0]
    ref = _oracle_vv(h, cfg, 1000.0, 1.0, 4.0, True, profile == "vvoigt_norm")
    assert_parity(got, ref, TOL32, what=f"{profile} coarse spw={spw}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_vv_radius_inside_the_centre_near_zone(precision):
    # R = 0.5 cm^-1 for hot, light, high-wavenumber lines: the radius of the |z| < 40
    # zones (~120 grid steps) exceeds R (50 steps), so lines centred near a wavefront
    # switch to the reference wing inside their zone-by-zone evaluation
    cfg, d = _case(3, n_lines=60000, numax=5150.0, nu_a=5000.0, nu_b=5100.0, n_points=10001, mass=16.0,
                   n_states=3000)
    h = host(d)
    plan = make_plan(cfg, precision, profile="vvoigt", vv_beta=True, vv_radius=0.5)
    got = _run(plan, d, [3000.0], [0.2])[0]
    ref = _oracle_vv(h, cfg, 3000.0, 0.2, 0.5, True, False)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"R=0.5 {precision}")


def test_vv_radius_beyond_cutoff_is_the_voigt_profile():
    cfg, d = _case(4)
    h = host(d)
    got = _run(make_plan(cfg, "fp32", profile="vvoigt", vv_radius=30.0), d, [800.0], [0.5])[0]
    voigt = _run(make_plan(cfg, "fp32", profile="voigt"), d, [800.0], [0.5])[0]
    ls = oracle_lineset(h, cfg, 800.0, 0.5)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile="voigt")
    assert_parity(got, ref, TOL32, what="R > cutoff")
    m = voigt > 1e-6 * voigt.max()
    assert np.max(np.abs(got[m] - voigt[m]) / voigt[m]) < 2e-6


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_vvn_preserves_line_areas(precision):
    # lines whose windows lie on the grid: dnu sum_k sigma_k = sum_i I_i (Sec. "Binned
    # Vectorized Voigt with the line area preserved"), on a coarse and a fine grid
    for n_points, T in ((2151, 1500.0), (43001, 296.0)):
        # (the grid starts below zero so that every window, nu in (0, 300], lies on it)
        cfg, d = _case(5, n_lines=4000, numax=300.0, nu_a=-30.0, nu_b=400.0, n_points=n_points)
        plan = make_plan(cfg, precision, profile="vvoigt_norm", vv_beta=True)
        sig = _run(plan, d, [T], [1.0])[0]
        h = host(d)
        ls = oracle_lineset(h, cfg, T, 1.0)
        inside = (ls.nu - cfg.cutoff >= cfg.nu_a + cfg.dnu) & (ls.nu + cfg.cutoff <= cfg.nu_b - cfg.dnu)
        assert inside.all()
        area = cfg.dnu * math.fsum(sig)
        tot = math.fsum(ls.I)
        log(f"  VVN area {precision} N={n_points}: rel {abs(area - tot) / tot:.2e}")
        assert abs(area - tot) <= (1e-6 if precision == "fp32" else 1e-11) * tot


def test_vv_batch_and_graph_replay_equal_direct_calls():
    cfg, d = _case(6, n_lines=2000)
    plan = make_plan(cfg, "fp32", profile="vvoigt_norm", vv_beta=True)
    Ts, Ps = [250.0, 900.0, 2500.0], [0.01, 1.0, 30.0]
    allr = _run(plan, d, Ts, Ps)
    for i in range(3):
        one = plan.cross_section([Ts[i]], [Ps[i]])
        torch.cuda.synchronize()
        assert np.array_equal(one.double().cpu().numpy()[0], allr[i])
    g = plan.graph(Ts, Ps)
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.double().cpu().numpy(), allr), rep
        plan.cross_section([Ts[0]], [Ps[0]])   # eager work between replays
        torch.cuda.synchronize()


def test_vv_rejects_a_radius_too_small_for_the_reference_wing():
    from paper_1801_09803_amd.binding import XsecError
    cfg, d = _case(7, n_lines=500, mass=1.0)
    plan = make_plan(cfg, "fp32", profile="vvoigt", vv_radius=0.1)
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    with pytest.raises(XsecError) as ei:
        plan.cross_section([5000.0], [1.0])
    assert ei.value.name == "XS_ERR_ARG"
    plan.cross_section([50.0], [1.0])        # x_ref = sqrt(ln2) R / alpha_ref grows as T falls
    torch.cuda.synchronize()
