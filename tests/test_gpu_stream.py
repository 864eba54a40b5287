"""Line-list streaming on the GPU (through the C ABI): chunks of transitions from pinned
host memory, copied while the previous chunk computes, summed on the device.

Inputs follow the hot-polyatomic workload's recipe at a reduced size: 16 Da, states
with E = 20000 u^(1/3), a0 broadening by lower-state J, 3 (T, P) points spanning
300-3000 K and 1e-5-100 bar, grid 0-3000 cm^-1 at 0.01 (300001 points), chunks of
60000, 60000, 0 and 37123 transitions (ragged and empty chunks)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import log, make_plan

pytestmark = pytest.mark.gpu

TS = [300.0, 1000.0, 3000.0]
PS = [1e-5, 0.4642, 100.0]
CHUNKS = [60000, 60000, 0, 37123]


@pytest.fixture(scope="module")
def case():
    cfg = synth.WorkloadConfig("stream", 7777, 20000, sum(CHUNKS), 16.0, 3000.0, 0.0, 3000.0, 300001,
                               tuple(TS), tuple(PS), cutoff=25.0, broadening="a0_jlower")
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed, device="cuda")
    gt, nt = synth.make_broadening_table(cfg.seed)
    chunks, first = [], 0
    for n in CHUNKS:
        up, lo = synth.linelist.make_transitions(E, n, cfg.nu_max, cfg.seed, first_line=first)
        A, gr, ne = synth.linelist.make_line_params(n, cfg.seed, first_line=first, device="cuda")
        chunks.append({k: v.cpu().pin_memory() for k, v in
                       dict(upper=up, lower=lo, A=A, gamma_ref=gr, n_exp=ne).items()})
        first += n
    allv = {k: torch.cat([c[k] for c in chunks]) for k in chunks[0]}
    return cfg, dict(E=E, g=g, J=J), (gt.numpy(), nt.numpy()), chunks, allv


def _plan(cfg, states, table, precision, broadening="a0_jlower"):
    plan = make_plan(cfg, precision, broadening=broadening)
    if broadening == "a0_jlower":
        plan.set_broadening_table(*table)
    plan.set_states(states["E"], states["g"], states["J"])
    return plan


def _stream(plan, chunks, per_line=False, upto=None):
    st = plan.stream(TS, PS)
    for c in chunks[:upto]:
        if per_line:
            st.chunk(c["upper"], c["lower"], c["A"], c["gamma_ref"], c["n_exp"])
        else:
            st.chunk(c["upper"], c["lower"], c["A"])
    return st


def _single(plan, allv, per_line=False):
    dev = {k: v.cuda() for k, v in allv.items()}
    if per_line:
        plan.set_lines(dev["upper"], dev["lower"], dev["A"], dev["gamma_ref"], dev["n_exp"])
    else:
        plan.set_lines(dev["upper"], dev["lower"], dev["A"])
    out = plan.cross_section(TS, PS)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), plan.lines_kept()


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("fp64", 1e-12)])
def test_stream_matches_one_call_over_all_lines(case, precision, tol):
    cfg, states, table, chunks, allv = case
    log(f"stream vs single call, {precision}")
    st = _stream(_plan(cfg, states, table, precision), chunks)
    assert st.stats()["chunks"] == len(CHUNKS)
    sig, kept = st.end()
    got = sig.double().cpu().numpy()
    ref, kept1 = _single(_plan(cfg, states, table, precision), allv)
    assert kept == kept1 > 0
    for i in range(len(TS)):
        m = O.error_metrics(got[i], ref[i])
        log(f"  T={TS[i]} P={PS[i]}: max rel {m['max_rel']:.2e} area {m['area_rel']:.2e}")
        assert m["max_rel"] <= tol and m["area_rel"] <= tol


def test_stream_matches_oracle_at_sampled_points(case):
    cfg, states, table, chunks, allv = case
    st = _stream(_plan(cfg, states, table, "fp32"), chunks)
    got = st.end()[0].double().cpu().numpy()
    E, g, J = (states[k].cpu().numpy() for k in ("E", "g", "J"))
    h = {k: v.numpy() for k, v in allv.items()}
    ks = np.unique(np.concatenate([np.linspace(0, cfg.n_points - 1, 601).astype(np.int64), [1, cfg.n_points - 2]]))
    for i, (T, P) in enumerate(zip(TS, PS)):
        ls = O.make_lineset(E, g, h["upper"], h["lower"], h["A"], T, P, cfg.mass_amu, J=J, broad_table=table)
        _, dnu = O.grid(cfg.nu_a, cfg.nu_b, cfg.n_points)
        top = np.argsort(-ls.I)[:40]
        kc = np.clip(np.rint((ls.nu[top] - cfg.nu_a) / dnu).astype(np.int64), 0, cfg.n_points - 1)
        kk = np.unique(np.concatenate([ks, kc]))
        ref = O.cross_section_at(ls, kk, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff)
        m = ref > 1e-6 * ref.max()
        rel = np.abs(got[i][kk][m] - ref[m]) / ref[m]
        log(f"  oracle T={T} P={P}: max rel {rel.max():.2e} over {m.sum()} points")
        assert m.sum() >= 8 and rel.max() <= 1e-5


def test_stream_checkpoint_and_resume(case, tmp_path):
    cfg, states, table, chunks, allv = case
    ref = _stream(_plan(cfg, states, table, "fp32"), chunks).end()[0].cpu().numpy()
    st = _stream(_plan(cfg, states, table, "fp32"), chunks, upto=2)
    path = str(tmp_path / "stream.ckpt")
    st.checkpoint(path)
    st.end()                                    # the interrupted run
    from paper_1801_09803_amd import Stream
    st2 = Stream.resume(_plan(cfg, states, table, "fp32"), path, n_tp=len(TS))
    s = st2.stats()
    assert s["chunks"] == 2 and s["lines"] == sum(CHUNKS[:2]) and 0 < s["kept"] <= s["lines"]
    for c in chunks[2:]:
        st2.chunk(c["upper"], c["lower"], c["A"])
    got = st2.end()[0].cpu().numpy()
    assert np.array_equal(got, ref)


def test_stream_per_line_broadening(case):
    cfg, states, table, chunks, allv = case
    st = _stream(_plan(cfg, states, table, "fp32", "per_line"), chunks, per_line=True)
    got = st.end()[0].double().cpu().numpy()
    ref, _ = _single(_plan(cfg, states, table, "fp32", "per_line"), allv, per_line=True)
    for i in range(len(TS)):
        assert O.error_metrics(got[i], ref[i])["max_rel"] <= 2e-6


def test_stream_reports_invalid_transitions(case):
    cfg, states, table, chunks, allv = case
    st = _plan(cfg, states, table, "fp32").stream(TS, PS)
    bad = chunks[0]["upper"].clone()
    bad[5] = cfg.n_states + 3                   # out of range: rejected by the prep kernel's check
    st.chunk(bad, chunks[0]["lower"], chunks[0]["A"])
    with pytest.raises(Exception) as e:
        st.chunk(chunks[1]["upper"], chunks[1]["lower"], chunks[1]["A"])    # the bad chunk computes here
    assert "XS_ERR_INDEX" in str(e.value)
    st.end()


def test_stream_injected_fault_then_resume_is_bitwise(case, tmp_path, monkeypatch):
    # checkpoint after two chunks, an injected fault at the third (XS_FAULT_INJECT=chunk:2:
    # refused before any copy or device work), then a resumed stream finishes the list;
    # its sums equal the uninterrupted run's bit for bit
    cfg, states, table, chunks, allv = case
    ref = _stream(_plan(cfg, states, table, "fp32"), chunks).end()[0].cpu().numpy()
    st = _stream(_plan(cfg, states, table, "fp32"), chunks, upto=2)
    path = str(tmp_path / "inject.ckpt")
    st.checkpoint(path)
    monkeypatch.setenv("XS_FAULT_INJECT", "chunk:2")
    c = chunks[2]
    with pytest.raises(Exception) as e:
        st.chunk(c["upper"], c["lower"], c["A"])
    assert "XS_ERR_INJECTED" in str(e.value)
    assert st.stats()["chunks"] == 2                 # the refused chunk left no trace
    st.end()                                         # the interrupted run ends here
    monkeypatch.delenv("XS_FAULT_INJECT")
    from paper_1801_09803_amd import Stream
    st2 = Stream.resume(_plan(cfg, states, table, "fp32"), path, n_tp=len(TS))
    for c in chunks[2:]:
        st2.chunk(c["upper"], c["lower"], c["A"])
    got = st2.end()[0].cpu().numpy()
    assert np.array_equal(got, ref)


def test_stream_resume_refuses_another_geometry(case, tmp_path):
    cfg, states, table, chunks, allv = case
    st = _stream(_plan(cfg, states, table, "fp32"), chunks, upto=1)
    path = str(tmp_path / "geo.ckpt")
    st.checkpoint(path)
    st.end()
    from paper_1801_09803_amd import Plan, Stream
    for kw, what in ((dict(cutoff=20.0), "cut-off"), (dict(mass_da=17.0), "mass"),
                     (dict(profile="lorentz"), "profile")):
        args = dict(cutoff=cfg.cutoff, profile="voigt", precision="fp32", broadening="a0_jlower")
        mass = kw.pop("mass_da", cfg.mass_amu)
        args.update(kw)
        plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, mass, **args)
        plan.set_broadening_table(*table)
        plan.set_states(states["E"], states["g"], states["J"])
        with pytest.raises(Exception) as e:
            Stream.resume(plan, path, n_tp=len(TS))
        assert "XS_ERR_ARG" in str(e.value) and what in str(e.value), str(e.value)
    # the same grid points over another range
    plan = Plan(cfg.nu_a + 1.0, cfg.nu_b + 1.0, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt",
                precision="fp32", broadening="a0_jlower")
    plan.set_broadening_table(*table)
    plan.set_states(states["E"], states["g"], states["J"])
    with pytest.raises(Exception) as e:
        Stream.resume(plan, path, n_tp=len(TS))
    assert "grid range" in str(e.value)


def test_stream_device_chunks_equal_host_chunks(case):
    # chunks already in device memory (no copy) give the host-chunk stream's sums bit for
    # bit, also when the two kinds alternate
    cfg, states, table, chunks, allv = case
    ref = _stream(_plan(cfg, states, table, "fp32"), chunks).end()
    st = _plan(cfg, states, table, "fp32").stream(TS, PS)
    for i, c in enumerate(chunks):
        if i % 2 == 0:
            st.chunk_device(c["upper"].cuda(), c["lower"].cuda(), c["A"].cuda())
        else:
            st.chunk(c["upper"], c["lower"], c["A"])
    assert st.stats()["chunks"] == len(CHUNKS)
    got = st.end()
    assert got[1] == ref[1]
    assert torch.equal(got[0], ref[0])
