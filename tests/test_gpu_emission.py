"""GPU parity of the emission and state reductions against the FP64 oracle, through the
C ABI: partition-function moments and C_p (1e-12 / 1e-10), radiative lifetimes and the
cooling function (1e-12 / 1e-11: FP64 sums in another order), and emission cross sections
(1e-5 FP32, 1e-10 FP64), with Kirchhoff's law for one line as a property check."""
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


def _case(seed, n_lines=4000, n_states=400, numax=300.0, nu_a=0.0, nu_b=200.0, n_points=20001):
    cfg = synth.WorkloadConfig("emis", 70 + seed, n_states, n_lines, 28.0, numax, nu_a, nu_b, n_points,
                               (800.0,), (0.5,), cutoff=25.0)
    return cfg, synth.make_linelist(cfg, device="cuda")


def _set(plan, d):
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])


def _emission_lineset(h, cfg, T, P):
    ls = oracle_lineset(h, cfg, T, P)
    eps = O.emissivities(h["E"], h["g"], h["upper"], h["lower"], h["A"], T)
    return O.LineSet(ls.nu, eps, ls.alpha_d, ls.gamma)


@pytest.mark.parametrize("which", ["C1", "C2"])
def test_partition_moments_and_heat_capacity(which):
    cfg = synth.CONFIGS[which]
    E, g, _ = synth.make_states(cfg.n_states, cfg.seed, device="cuda")
    plan = make_plan(cfg, "fp32")
    plan.set_states(E, g)
    Ts = [50.0, 296.0, 1000.0, 3000.0, 10000.0]
    Q, Q1, Q2, Cp = (x.cpu().numpy() for x in plan.partition_moments(Ts))
    Qf, _ = plan.partition_function(Ts)
    Eh, gh = E.cpu().numpy(), g.cpu().numpy()
    for i, T in enumerate(Ts):
        q, q1, q2 = O.partition_moments(Eh, gh, T)
        cp = O.heat_capacity(Eh, gh, T)
        r = [abs(Q[i] / q - 1), abs(Q1[i] / q1 - 1), abs(Q2[i] / q2 - 1)]
        log(f"  {which} T={T}: Q {r[0]:.1e} Q' {r[1]:.1e} Q'' {r[2]:.1e} C_p {Cp[i]:.6f} vs {cp:.6f}")
        assert max(r) <= 1e-12
        assert abs(Cp[i] - cp) <= 1e-10 * cp
        assert abs(Qf[i].item() / Q[i] - 1) <= 1e-13   # the partition-function call agrees


def test_lifetimes_match_the_oracle():
    cfg, d = _case(1, n_lines=100000, n_states=10000)
    h = host(d)
    plan = make_plan(cfg, "fp32")
    plan.set_states(d["E"], d["g"], d["J"])
    tau = plan.lifetimes(d["upper"], d["A"]).cpu().numpy()
    ref = O.lifetimes(h["E"].size, h["upper"], h["A"])
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(tau), fin)
    assert 0 < fin.sum() < fin.size        # both kinds of states occur
    rel = np.abs(tau[fin] / ref[fin] - 1)
    log(f"  lifetimes: max rel {rel.max():.2e} over {fin.sum()} states")
    assert rel.max() <= 1e-12


def test_lifetimes_index_base_and_log_A():
    cfg, d = _case(2, n_lines=20000, n_states=2000)
    h = host(d)
    plan = make_plan(cfg, "fp32", index_base=1, a_is_log=True)
    plan.set_states(d["E"], d["g"], d["J"])
    lnA = torch.log(d["A"])
    tau = plan.lifetimes(d["upper"] + 1, lnA).cpu().numpy()
    A_used = np.exp(lnA.cpu().numpy().astype(np.float64))    # the library exponentiates in double
    ref = O.lifetimes(h["E"].size, h["upper"] + 1, A_used, index_base=1)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(tau), fin)
    assert np.max(np.abs(tau[fin] / ref[fin] - 1)) <= 1e-12


def test_cooling_function_matches_the_oracle():
    cfg, d = _case(3, n_lines=100000, n_states=10000, numax=5000.0)
    h = host(d)
    plan = make_plan(cfg, "fp32")
    plan.set_states(d["E"], d["g"], d["J"])
    Ts = [100.0, 296.0, 1000.0, 3000.0, 5000.0]
    W = plan.cooling_function(d["upper"], d["lower"], d["A"], Ts).cpu().numpy()
    for i, T in enumerate(Ts):
        ref = O.cooling_function(h["E"], h["g"], h["upper"], h["lower"], h["A"], T)
        log(f"  W({T}) = {W[i]:.6e} (oracle {ref:.6e})")
        assert abs(W[i] / ref - 1) <= 1e-11


def test_state_reductions_reject_bad_transitions_and_handle_empty_lists():
    from paper_1801_09803_amd.binding import XsecError
    cfg, d = _case(4, n_lines=1000, n_states=200)
    plan = make_plan(cfg, "fp32")
    plan.set_states(d["E"], d["g"], d["J"])
    bad = d["upper"].clone()
    bad[17] = 200                                    # one past the last state
    with pytest.raises(XsecError) as ei:
        plan.lifetimes(bad, d["A"])
    assert ei.value.name == "XS_ERR_INDEX"
    with pytest.raises(XsecError) as ei:
        plan.cooling_function(d["upper"], d["upper"], d["A"], [300.0])   # nu = 0
    assert ei.value.name == "XS_ERR_NU_NONPOS"
    with pytest.raises(XsecError) as ei:
        plan.cooling_function(d["upper"], d["lower"], d["A"], [0.0])
    assert ei.value.name == "XS_ERR_ARG"
    empty_i = torch.empty(0, dtype=torch.int32, device="cuda")
    empty_a = torch.empty(0, dtype=torch.float32, device="cuda")
    assert torch.isinf(plan.lifetimes(empty_i, empty_a)).all()
    assert plan.cooling_function(empty_i, empty_i, empty_a, [300.0, 900.0]).eq(0).all()
    # the plan still works after the failures
    tau = plan.lifetimes(d["upper"], d["A"]).cpu().numpy()
    ref = O.lifetimes(200, d["upper"].cpu().numpy(), d["A"].cpu().numpy())
    fin = np.isfinite(ref)
    assert np.max(np.abs(tau[fin] / ref[fin] - 1)) <= 1e-12


@pytest.mark.parametrize("profile,precision", [("voigt", "fp32"), ("voigt", "fp64"), ("doppler", "fp32"),
                                               ("lorentz_binned", "fp64"), ("superlines", "fp64")])
def test_emission_cross_sections(profile, precision):
    cfg, d = _case(5)
    h = host(d)
    T, P = 1500.0, 0.5
    plan = make_plan(cfg, precision, profile=profile)
    _set(plan, d)
    plan.set_intensity_kind("emission")
    got = plan.cross_section([T], [P])[0].double().cpu().numpy()
    ls = _emission_lineset(h, cfg, T, P)
    if profile == "superlines":
        ref = O.super_line_histogram(ls, cfg.nu_a, cfg.nu_b, cfg.n_points)
        m = ref > 0
        assert np.array_equal(got > 0, m)
        assert np.max(np.abs(got[m] / ref[m] - 1)) <= 1e-12
        return
    ref = O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, profile=profile)
    assert_parity(got, ref, TOL32 if precision == "fp32" else TOL64, what=f"emission {profile} {precision}")


def test_emission_over_absorption_of_one_line_is_the_planck_function():
    # Kirchhoff's law holds line by line: both cross sections share the profile, so their
    # ratio is B_nu(T) at the line's wavenumber at every grid point
    cfg, d = _case(6, n_lines=1, n_states=50, numax=180.0, n_points=4001)
    plan = make_plan(cfg, "fp64")
    _set(plan, d)
    T = 2500.0
    ab = plan.cross_section([T], [1.0])[0].cpu().numpy()
    plan.set_intensity_kind("emission")
    em = plan.cross_section([T], [1.0])[0].cpu().numpy()
    nu = (d["E"][d["upper"].long()] - d["E"][d["lower"].long()]).item()
    h, c = 6.62607015e-27, 2.99792458e10
    B = 2 * h * c * c * nu ** 3 / math.expm1(O.C2 * nu / T)
    m = ab > 1e-6 * ab.max()
    assert m.sum() > 10
    assert np.max(np.abs(em[m] / ab[m] / B - 1)) <= 1e-12


def test_emission_with_threshold_graph_and_stream():
    from paper_1801_09803_amd.binding import XsecError
    cfg, d = _case(7)
    h = host(d)
    T, P = 1200.0, 0.5
    plan = make_plan(cfg, "fp32")
    _set(plan, d)
    stale = plan.graph([T], [P])
    plan.set_intensity_kind("emission")
    with pytest.raises(XsecError) as ei:
        stale.launch()
    assert ei.value.name == "XS_ERR_STATE"
    # a threshold on the emissivity: keep about half of the lines near the grid
    ls = _emission_lineset(h, cfg, T, P)
    near = (ls.nu > cfg.nu_a - cfg.cutoff) & (ls.nu < cfg.nu_b + cfg.cutoff)
    v = np.unique(ls.I[near])
    cut = float(np.sqrt(v[v.size // 2 - 1] * v[v.size // 2]))
    plan.set_intensity_threshold("constant", cut)
    direct = plan.cross_section([T], [P])[0].double().cpu().numpy()
    keep = ls.I >= cut
    kept = O.LineSet(ls.nu[keep], ls.I[keep], ls.alpha_d[keep], ls.gamma[keep])
    assert_parity(direct, O.cross_section(kept, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff), TOL32,
                  what="emission + threshold")
    g = plan.graph([T], [P])
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out[0].double().cpu().numpy(), direct), rep
        plan.cross_section([300.0], [1.0])
        torch.cuda.synchronize()
    # the adjoint is for absorption only
    plan.set_intensity_threshold("none")
    gbar = torch.ones(cfg.n_points, dtype=torch.float32, device="cuda")
    with pytest.raises(XsecError) as ei:
        plan.cross_section_adjoint(T, P, gbar, cfg.n_lines)
    assert ei.value.name == "XS_ERR_UNSUPPORTED"
    # a stream keeps the kind it began with
    st = plan.stream([T], [P])
    hd = {k: v.cpu() for k, v in d.items()}
    half = cfg.n_lines // 2
    st.chunk(hd["upper"][:half], hd["lower"][:half], hd["A"][:half], hd["gamma_ref"][:half], hd["n_exp"][:half])
    plan.set_intensity_kind("absorption")
    with pytest.raises(XsecError) as ei:
        st.chunk(hd["upper"][half:], hd["lower"][half:], hd["A"][half:], hd["gamma_ref"][half:],
                 hd["n_exp"][half:])
    assert ei.value.name == "XS_ERR_STATE"
    st.end()


def test_lifetimes_and_cooling_beyond_the_bucketed_range():
    # more states than the bucketed pass takes (8192 buckets of 4096): the global-atomic
    # pass; a few transitions among 3.4e7 states
    n_states = 8192 * 4096 + 5
    g = torch.full((n_states,), 3, dtype=torch.int32, device="cuda")
    E = torch.linspace(0.0, 30000.0, n_states, dtype=torch.float64, device="cuda")
    cfg = synth.WorkloadConfig("big", 9, n_states, 1, 28.0, 300.0, 0.0, 200.0, 2001, (800.0,), (0.5,))
    rng = np.random.default_rng(8)
    lo = rng.integers(0, n_states - 1, 20000)
    up = np.minimum(lo + rng.integers(1, 5000, lo.size), n_states - 1)
    A = (10 ** rng.uniform(-3, 2, lo.size)).astype(np.float32)
    plan = make_plan(cfg, "fp32")
    plan.set_states(E, g)
    tau = plan.lifetimes(torch.tensor(up, dtype=torch.int32, device="cuda"),
                         torch.tensor(A, device="cuda")).cpu().numpy()
    s = {}
    for u, a in zip(up.tolist(), A.astype(np.float64).tolist()):
        s.setdefault(u, []).append(a)
    for u, vals in list(s.items())[:2000]:
        assert abs(tau[u] * math.fsum(vals) - 1) <= 1e-12
    assert np.isinf(tau[[0, n_states - 1]]).all() or (n_states - 1) in s
    Eh = E.cpu().numpy()
    W = plan.cooling_function(torch.tensor(up, dtype=torch.int32, device="cuda"),
                              torch.tensor(lo, dtype=torch.int32, device="cuda"),
                              torch.tensor(A, device="cuda"), [2000.0]).item()
    ref = O.cooling_function(Eh, np.full(n_states, 3), up, lo, A, 2000.0)
    log(f"  W(2000 K) over {n_states} states: {W:.6e} (oracle {ref:.6e})")
    assert abs(W / ref - 1) <= 1e-11
