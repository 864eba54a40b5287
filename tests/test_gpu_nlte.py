"""GPU parity of two-temperature non-LTE populations against the FP64 oracle, through the
C ABI: Q(T_vib, T_rot) (1e-12), cross sections for absorption and emission (1e-5 FP32,
1e-10 FP64), inverted transitions (normwise), the LTE limit, batches of different T_vib,
and the state errors."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import assert_parity, host, log, make_plan

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-10


def _case(seed, n_lines=4000, n_states=400, numax=300.0, nu_a=0.0, nu_b=200.0, n_points=20001):
    cfg = synth.WorkloadConfig("nlte", 90 + seed, n_states, n_lines, 28.0, numax, nu_a, nu_b, n_points,
                               (800.0,), (0.5,), cutoff=25.0)
    d = synth.make_linelist(cfg, device="cuda")
    d["v"] = synth.make_vibrational_labels(d["E"])
    return cfg, d


def _plan(cfg, d, precision="fp32", profile="voigt", labels=True, **kw):
    plan = make_plan(cfg, precision, profile=profile, **kw)
    plan.set_states(d["E"], d["g"], d["J"])
    if labels:
        plan.set_vibrational_labels(d["v"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    return plan


def _oracle(h, cfg, Tr, Tv, P, emission=False):
    Ev = O.vibrational_energies(h["E"], h["v"])
    ls = O.make_lineset_nlte(h["E"], h["g"], Ev, h["upper"], h["lower"], h["A"], Tv, Tr, P, cfg.mass_amu,
                             h["gamma_ref"], h["n_exp"], emission=emission)
    return O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff), ls


@pytest.mark.parametrize("which", ["C1", "C2"])
def test_nlte_partition_function(which):
    cfg = synth.CONFIGS[which]
    E, g, _ = synth.make_states(cfg.n_states, cfg.seed, device="cuda")
    v = synth.make_vibrational_labels(E)
    plan = make_plan(cfg, "fp32")
    plan.set_states(E, g)
    plan.set_vibrational_labels(v)
    pts = [(296.0, 296.0), (300.0, 3000.0), (3000.0, 300.0), (1000.0, 5000.0)]
    Q = plan.partition_function_nlte([p[0] for p in pts], [p[1] for p in pts]).cpu().numpy()
    Eh, gh, vh = E.cpu().numpy(), g.cpu().numpy(), v.cpu().numpy()
    Ev = O.vibrational_energies(Eh, vh)
    for i, (Tr, Tv) in enumerate(pts):
        ref = O.partition_function_nlte(Eh, gh, Ev, Tv, Tr)
        log(f"  {which} Q(T_rot={Tr}, T_vib={Tv}) rel {abs(Q[i] / ref - 1):.1e}")
        assert abs(Q[i] / ref - 1) <= 1e-12
    # equal temperatures: the LTE partition function
    Ql, _ = plan.partition_function([296.0])
    assert abs(Q[0] / Ql[0].item() - 1) <= 1e-13


@pytest.mark.parametrize("precision,profile,emission", [("fp32", "voigt", False), ("fp64", "voigt", False),
                                                        ("fp64", "voigt", True), ("fp32", "doppler", True),
                                                        ("fp64", "lorentz_binned", False)])
def test_nlte_cross_sections(precision, profile, emission):
    cfg, d = _case(1)
    h = host(d)
    Tr, Tv, P = 1500.0, 600.0, 0.5     # T_vib < T_rot: no inversion
    plan = _plan(cfg, d, precision, profile)
    if emission:
        plan.set_intensity_kind("emission")
    got = plan.cross_section_nlte([Tr], [Tv], [P])[0].double().cpu().numpy()
    Ev = O.vibrational_energies(h["E"], h["v"])
    ls = O.make_lineset_nlte(h["E"], h["g"], Ev, h["upper"], h["lower"], h["A"], Tv, Tr, P, cfg.mass_amu,
                             h["gamma_ref"], h["n_exp"], emission=emission)
    assert np.all(ls.I > 0)
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile=profile)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64,
                  what=f"non-LTE {profile} {precision} emission={emission}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_inverted_transitions(precision):
    cfg, d = _case(2)
    h = host(d)
    Tr, Tv, P = 300.0, 4000.0, 0.5     # hot vibrations, cold rotations: inverted band lines
    plan = _plan(cfg, d, precision)
    got = plan.cross_section_nlte([Tr], [Tv], [P])[0].double().cpu().numpy()
    ref, ls = _oracle(h, cfg, Tr, Tv, P)
    near = (ls.nu > cfg.nu_a - cfg.cutoff) & (ls.nu < cfg.nu_b + cfg.cutoff)
    n_inv = int(np.sum(ls.I[near] < 0))
    log(f"  inverted lines near the grid: {n_inv} of {int(near.sum())}; min sigma {ref.min():.3e}")
    assert n_inv > 0 and ref.min() < 0
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    log(f"  inverted {precision}: normwise error {err:.2e}")
    assert err <= (TOL32 if precision == "fp32" else TOL64)


def test_lte_limit_and_batch_of_vibrational_temperatures():
    cfg, d = _case(3)
    lte = _plan(cfg, d, "fp64", labels=False)
    nl = _plan(cfg, d, "fp64")
    T = 900.0
    a = lte.cross_section([T], [1.0])[0].cpu().numpy()
    b = nl.cross_section_nlte([T], [T], [1.0])[0].cpu().numpy()
    c = nl.cross_section([T], [1.0])[0].cpu().numpy()          # T_vib = T_rot on a non-LTE line set
    assert_parity(b, a, 1e-12, what="non-LTE at T_vib = T_rot vs LTE")
    assert np.array_equal(b, c)
    # a batch of different vibrational temperatures equals one call per point
    f32 = _plan(cfg, d, "fp32")
    Tv = [300.0, 900.0, 2700.0]
    allr = f32.cross_section_nlte([T] * 3, Tv, [1.0] * 3).double().cpu().numpy()
    h = host(d)
    for i, tv in enumerate(Tv):
        one = f32.cross_section_nlte([T], [tv], [1.0])[0].double().cpu().numpy()
        assert np.array_equal(one, allr[i])
        if tv <= T:
            ref, _ = _oracle(h, cfg, T, tv, 1.0)
            assert_parity(allr[i], ref, TOL32, what=f"batch T_vib={tv}")


def test_nlte_threshold_and_graph():
    cfg, d = _case(4)
    h = host(d)
    Tr, Tv, P = 1200.0, 500.0, 0.5
    plan = _plan(cfg, d, "fp32")
    ref_all, ls = _oracle(h, cfg, Tr, Tv, P)
    near = (ls.nu > cfg.nu_a - cfg.cutoff) & (ls.nu < cfg.nu_b + cfg.cutoff)
    vals = np.unique(ls.I[near])
    cut = float(np.sqrt(vals[vals.size // 2 - 1] * vals[vals.size // 2]))
    plan.set_intensity_threshold("constant", cut)
    got = plan.cross_section_nlte([Tr], [Tv], [P])[0].double().cpu().numpy()
    keep = ls.I >= cut
    kept = O.LineSet(ls.nu[keep], ls.I[keep], ls.alpha_d[keep], ls.gamma[keep])
    assert_parity(got, O.cross_section(kept, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff), TOL32,
                  what="non-LTE + threshold")
    # graphs replay the T_vib = T_rot values
    plan.set_intensity_threshold("none")
    direct = plan.cross_section([Tr], [P])[0].double().cpu().numpy()
    g = plan.graph([Tr], [P])
    for rep in range(2):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out[0].double().cpu().numpy(), direct), rep


def test_nlte_state_errors():
    from paper_1801_09803_amd.binding import XsecError
    cfg, d = _case(5, n_lines=500)
    plan = _plan(cfg, d, "fp32", labels=False)
    with pytest.raises(XsecError) as ei:
        plan.cross_section_nlte([800.0], [800.0], [1.0])
    assert ei.value.name == "XS_ERR_STATE"
    with pytest.raises(XsecError) as ei:
        plan.partition_function_nlte([800.0], [800.0])
    assert ei.value.name == "XS_ERR_STATE"
    bad = d["v"].clone()
    bad[3] = 10
    with pytest.raises(XsecError) as ei:
        plan.set_vibrational_labels(bad, n_labels=10)
    assert ei.value.name == "XS_ERR_INDEX"
    plan.set_vibrational_labels(d["v"])
    with pytest.raises(XsecError) as ei:      # labels invalidate the line set
        plan.cross_section_nlte([800.0], [800.0], [1.0])
    assert ei.value.name == "XS_ERR_STATE"
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    with pytest.raises(XsecError) as ei:
        plan.cross_section_nlte([800.0], [0.0], [1.0])
    assert ei.value.name == "XS_ERR_ARG"
    gbar = torch.ones(cfg.n_points, dtype=torch.float32, device="cuda")
    with pytest.raises(XsecError) as ei:
        plan.cross_section_adjoint(800.0, 1.0, gbar, cfg.n_lines)
    assert ei.value.name == "XS_ERR_UNSUPPORTED"
    plan.set_vibrational_labels(None)                 # back to LTE
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    plan.cross_section_adjoint(800.0, 1.0, gbar, cfg.n_lines)


def test_nlte_line_set_streamed_in_chunks():
    # a stream rebuilds the line set per chunk: each chunk carries its states' vibrational
    # energies, and the streamed sums match one call over the whole list (T_vib = T_rot
    # there, as for every stream) and the oracle's non-LTE cross section at T_vib = T_rot
    cfg, d = _case(6, n_lines=6000)
    h = host(d)
    T, P = 1100.0, 0.3
    plan = _plan(cfg, d, "fp32")
    direct = plan.cross_section([T], [P])[0].double().cpu().numpy()
    st = plan.stream([T], [P])
    hd = {k: v.cpu() for k, v in d.items()}
    for a, b in ((0, 2500), (2500, 4000), (4000, 6000)):
        st.chunk(hd["upper"][a:b].contiguous(), hd["lower"][a:b].contiguous(), hd["A"][a:b].contiguous(),
                 hd["gamma_ref"][a:b].contiguous(), hd["n_exp"][a:b].contiguous())
    sig, kept = st.end()
    got = sig[0].double().cpu().numpy()
    assert 0 < kept <= 6000
    m = O.error_metrics(got, direct)
    log(f"  non-LTE stream vs one call: max rel {m['max_rel']:.2e}")
    assert m["max_rel"] <= 2e-6 and m["area_rel"] <= 2e-6
    ref, _ = _oracle(h, cfg, T, T, P)
    assert_parity(got, ref, TOL32, what="non-LTE stream vs oracle")
