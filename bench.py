"""Benchmark: Voigt line-profiles/s at a 25 cm^-1 cut-off on one MI355X.

Headline (default): the hot-polyatomic workload.  4e9 synthetic transitions (int32 upper,
int32 lower, float A) among 5e7 states (16 Da) are generated on the device and kept in
HBM (48 GB); cross sections at 9 temperatures (300-3000 K) x 4 pressures (1e-5-100 bar)
with a0 broadening by lower-state J, Voigt profile sampled on 0-12000 cm^-1 at
0.01 cm^-1 (1,200,001 points), FP32 profile arithmetic with FP64 line setup.  One step =
one chunk of 2^28 transitions (15 chunks hold the list) through the whole path for all
36 (T, P), accumulated on the device (xs_stream_chunk_device); step i takes chunk
i mod 15, so 15 steps cover the list once.  The CPU oracle is timed on a bounded sample
of the same list before the GPU is touched.

Sub-entries: the single-cross-section workload (1e8 transitions, 296 K and 2000 K at
1 bar: timed steps of line preparation + batched call, the plain FP64 path, a graph
replay, and the 270-point (T, P) grid on the same list); the retrieval workload (1e7
transitions, forward + adjoint, FP32 against FP64, one shared dL/dsigma); the first
chunks of the 4e9-transition list streamed from pinned host memory (host-to-device copies
included); the paper's single-core timings as context.  --workload C2 makes the
single-cross-section workload the headline; --all-legs adds the Vectorized Voigt, binned,
threshold and emission legs.

Prints one JSON line (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Tile-kernel flops per grid-point evaluation by the zone the point falls in, as the
# kernel's formulas are written (FMA = 2, reciprocal = 1): one pole at |x| >= 1000 (x, den,
# accumulate FMA + rcp) 7; 2-node rule at |z| >= 40 (x, p, den, num, accumulate FMA + rcp)
# 11; 4-node rule at 8 <= |z| < 40 (x + two node pairs of three FMA and a rcp + two
# accumulate FMA) 20; a core value precomputed by the FP64 pre-pass, added: 1.
ZONE_FLOPS = {"one_pole": 7, "two_node": 11, "four_node": 20, "core": 1, "far_node": 11, "far_node4": 20,
              "far_exact": 11}
FAR_NODES = 16        # far-wing nodes per wavefront of the FP32 Voigt sweep
FAR_ZONES = ("far_node", "far_node4", "far_exact")   # evaluations of the node-sampled kernels


def far_reach(ww):
    """Grid steps between a wavefront of ww points and the nearest node-sampled line centre
    (0.57 (ww - 1), rounded up: 16 Chebyshev nodes across the wavefront)."""
    return (57 * (ww - 1) + 99) // 100


def zone_counts(cfg, d, T, P, waves=None, slices=None, chunk=1 << 24):
    """zone_counts_multi for one (T, P)."""
    return zone_counts_multi(cfg, d, [(T, P)], waves, slices, chunk)[0]


def zone_counts_multi(cfg, d, tps, waves=None, slices=None, chunk=1 << 24):
    """Window points of every line per zone at each (T, P) of tps (x = sqrt(ln2)(nu_k - nu)/alpha_D,
    |z|^2 = x^2 + y^2, y = sqrt(ln2) gamma/alpha_D), counted from index ranges.  d holds E,
    upper, lower and the per-line gamma_ref, n_exp.

    With the tile shape (waves, slices) of the FP32 Voigt sweep, the tile kernel evaluates
    only the (line, wavefront) pairs whose centre lies within R grid steps of the wavefront
    of 64 * slices points, R = max(far reach, the wavefront's |z| < 8 radius: the Doppler
    width at the largest wavenumber near it); their points are counted per zone.  Every
    other pair the window overlaps goes to the node-sampled kernels: FAR_NODES node
    evaluations each, by the 4-node rule (far_node4) when the centre lies within the
    wavefront's |z| < 40 radius rm, else the 2-node rule (far_node), plus, where the window
    starts or ends inside the wavefront, the points of that end's block evaluated one by one
    (far_exact).  R and rm vary by at most a grid step between neighbouring wavefronts; they
    are taken at the centre's."""
    import torch
    kB, amu, c_si, ln2 = 1.380649e-23, 1.66053906660e-27, 299792458.0, math.log(2.0)
    betas = {T: math.sqrt(2.0 * kB * T * ln2 / (cfg.mass_amu * amu)) / c_si for T, _ in tps}
    E = d["E"]
    tots = [{k: 0 for k in ZONE_FLOPS} for _ in tps]
    n = d["upper"].numel()
    far = waves is not None
    dnu = (cfg.nu_b - cfg.nu_a) / (cfg.n_points - 1)
    R_of, rm_of = {}, {}
    if far:
        ww = 64 * slices
        bw = 4 if slices == 1 else 8          # points per window-end block of the far kernel
        reach = far_reach(ww)
        hmin = math.floor(cfg.cutoff / dnu) - 2
        n_waves = -(-cfg.n_points // (waves * ww)) * waves
        numax = max(abs(cfg.nu_a), abs(cfg.nu_b)) + cfg.cutoff
        for T in betas:
            # the library's per-wavefront radii: rm of the |z| < 40 zone and R (node-sampled
            # lines beyond it) = max(reach, the |z| < 8 radius)
            rm = math.ceil(40.0 * betas[T] * numax / (math.sqrt(ln2) * dnu) + 2.0)
            scale = 40.0 * betas[T] / (math.sqrt(ln2) * dnu)
            w = torch.arange(n_waves, dtype=torch.float64, device=E.device)
            nlo = cfg.nu_a + (w * ww - rm - 1) * dnu
            nhi = cfg.nu_a + (w * ww + ww - 1 + rm + 1) * dnu
            rw = torch.ceil(scale * torch.maximum(nlo.abs(), nhi.abs())) + 2.0
            rm_of[T] = torch.minimum(rw, torch.full_like(rw, rm))
            span = max(reach, rm) + 1
            nlo = cfg.nu_a + (w * ww - span) * dnu
            nhi = cfg.nu_a + (w * ww + ww - 1 + span) * dnu
            r8 = torch.ceil(0.2 * scale * torch.maximum(nlo.abs(), nhi.abs())) + 2.0
            R_of[T] = torch.clamp(torch.minimum(r8, torch.full_like(r8, rm)), min=reach)
            # the window ends are node-sampled only beyond both radii (the library's condition)
            assert hmin - ww + 2 >= max(reach, rm), "window ends not node-sampled here: counts would not match"
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        nu = E[d["upper"][a:b].long()] - E[d["lower"][a:b].long()]
        gref, nexp = d["gamma_ref"][a:b].double(), d["n_exp"][a:b].double()
        klo_raw = torch.ceil(((nu - cfg.cutoff) - cfg.nu_a) / cfg.dnu)
        klo = torch.clamp(klo_raw, min=0)
        khi = torch.clamp(torch.floor(((nu + cfg.cutoff) - cfg.nu_a) / cfg.dnu), max=cfg.n_points - 1)
        live = khi >= klo
        if far:
            kc = torch.floor((nu - cfg.nu_a) / cfg.dnu + 0.5)
            wl, wr = torch.floor(klo / ww), torch.floor(khi / ww)
            wc = torch.clamp(torch.floor(kc / ww), 0, n_waves - 1).long()
        cache = {}
        for i, (T, P) in enumerate(tps):
            s = math.sqrt(ln2) / (betas[T] * nu)
            if T not in cache:
                if far:
                    # the tile kernel's part of the window: wavefronts within R of the centre
                    R = R_of[T][wc]
                    na = torch.maximum(torch.ceil((kc - R - ww + 1) / ww), wl)
                    nb = torch.minimum(torch.floor((kc + R) / ww), wr)
                    near_w = torch.clamp(nb - na + 1, min=0)
                    lo_k = torch.where(near_w > 0, torch.maximum(klo, na * ww), khi + 1)
                    hi_k = torch.minimum(khi, nb * ww + ww - 1)
                    far_w = torch.where(live, (wr - wl + 1) - near_w, torch.zeros_like(wl))
                    # of the far wavefronts, those within rm of the centre take the 4-node rule
                    rmc = rm_of[T][wc]
                    ma = torch.maximum(torch.ceil((kc - rmc - ww + 1) / ww), wl)
                    mb = torch.minimum(torch.floor((kc + rmc) / ww), wr)
                    mid_w = torch.where(live, torch.clamp(torch.clamp(mb - ma + 1, min=0) - near_w, min=0),
                                        torch.zeros_like(wl))
                    # (a window cut by the grid's start has no left end on it)
                    left_far = live & (klo_raw >= 0) & ((wl < na) | (near_w == 0))
                    right_far = live & ((wr > nb) | (near_w == 0))
                    ex_l = torch.where(left_far, bw - torch.remainder(klo - wl * ww, bw), torch.zeros_like(klo))
                    ex_r = torch.where(right_far, torch.remainder(khi - wr * ww, bw) + 1, torch.zeros_like(khi))
                    far4 = FAR_NODES * int(mid_w.sum().item())
                    far_pairs = FAR_NODES * int(far_w.sum().item()) - far4
                    far_ex = int((ex_l + ex_r).sum().item())
                else:
                    lo_k, hi_k, far_pairs, far4, far_ex = klo, khi, 0, 0, 0
                n_all = int(torch.clamp(hi_k - lo_k + 1, min=0).sum().item())
                cache[T] = (lo_k, hi_k, far_pairs, far4, far_ex, n_all, None)

            lo_k, hi_k, far_pairs, far4, far_ex, n_all, n_x = cache[T]

            def inside(X):   # points of [lo_k, hi_k] with |x| < X
                R_ = X / s
                lo = torch.maximum(torch.floor((nu - R_ - cfg.nu_a) / cfg.dnu) + 1, lo_k)
                hi = torch.minimum(torch.ceil((nu + R_ - cfg.nu_a) / cfg.dnu) - 1, hi_k)
                return int(torch.where(X > 0, torch.clamp(hi - lo + 1, min=0), torch.zeros_like(X)).sum().item())

            if n_x is None:
                n_x = inside(torch.full_like(nu, 1000.0))
                cache[T] = (lo_k, hi_k, far_pairs, far4, far_ex, n_all, n_x)
            y2 = (gref * torch.pow(296.0 / T, nexp) * P * s) ** 2
            n_40 = inside(torch.sqrt(torch.clamp(1600.0 - y2, min=0.0)))
            n_8 = inside(torch.sqrt(torch.clamp(64.0 - y2, min=0.0)))
            t = tots[i]
            t["one_pole"] += n_all - n_x
            t["two_node"] += n_x - n_40
            t["four_node"] += n_40 - n_8
            t["core"] += n_8
            t["far_node"] += far_pairs
            t["far_node4"] += far4
            t["far_exact"] += far_ex
        del cache
    return tots

# HBM traffic of the dominant kernel (the tile kernel) from two rocprofv3 --pmc runs of this
# script with the tile configuration fixed (1 wave, 4 slices, 32 shares): FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, scaled by the same counters on a 1 GiB device copy
# (FETCH_SIZE reads 0.5 GiB -> x2, WRITE_SIZE 1 GiB -> x1).  C5: one (T, P) per dispatch,
# averaged over the 36 of one 2^28-line chunk; C2: both (T, P) in one dispatch.  Valid only
# for the kernel sources they were taken with (hash below).
TRAFFIC = {
    "kernel_sources": ['xs_forward_f32.hip', 'xs_records.hpp', 'xs_far.hpp', 'xs_forward_common.hpp', 'xs_voigt.hpp',
                       'xs_forward.hpp', 'xs_internal.hpp'],
    "sha256": "cd5f2811b759394ae8df0630c8dd02bf45741bacc90008f83895f041a61f2f66",
    "fetch_scale": 2.0,
    "write_scale": 1.0,
    "C5": {"fetch_kib": 38084300.0, "write_kib": 378624.0, "tp_per_dispatch": 1},
    "C2": {"fetch_kib": 24000800.0, "write_kib": 631665.0, "tp_per_dispatch": 2},
}


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC["kernel_sources"]:
        with open(os.path.join(ROOT, "paper_1801_09803_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes_per_launch(workload, tp_per_launch):
    """HBM bytes per tile-kernel launch of tp_per_launch (T, P) on the workload (C5 or C2),
    or None when the kernel sources changed since the counters were taken."""
    if TRAFFIC["sha256"] is None or TRAFFIC["sha256"] != kernel_sources_sha() or workload not in TRAFFIC:
        return None
    t = TRAFFIC[workload]
    per_tp = (t["fetch_kib"] * TRAFFIC["fetch_scale"] + t["write_kib"] * TRAFFIC["write_scale"]) * 1024.0 \
        / t["tp_per_dispatch"]
    return per_tp * tp_per_launch


PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (published, packed)
PEAK_FP32_UNPACKED = 78.6    # 256 CU x 64 lanes x 2 flop x 2.4 GHz without packed FP32


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(cfg, n_sample_lines, temps, pressures):
    """Time the FP64 oracle (as it stands) on the first n_sample_lines lines."""
    import numpy as np
    import oracle as O
    import synth
    d = synth.make_linelist(cfg, n_lines=n_sample_lines, device="cpu")
    h = {k: v.numpy() for k, v in d.items()}
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    profiles = 0
    for T, P in zip(temps, pressures):
        ls = O.make_lineset(h["E"], h["g"], h["upper"], h["lower"], h["A"], T, P, cfg.mass_amu,
                            gamma_ref=h["gamma_ref"], n_exp=h["n_exp"])
        O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=cores)
        klo, khi = O.window(ls.nu, cfg.nu_a, cfg.dnu, cfg.n_points, cfg.cutoff)
        profiles += int(np.count_nonzero(khi >= klo))
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=profiles / dt, unit="line-profiles/s", cores=cores, kind="oracle",
                sample=f"first {n_sample_lines} lines of the same list x {len(temps)} (T,P), full grid; "
                       f"{dt:.1f} s wall on {cores} processes ({cpu})")


# The paper's own single-core timings of its cross-section hot path (its Table of total
# times: BT2 water, 5e8 transitions, 0-30000 cm^-1 at 0.1 cm^-1, I/O excluded, one core of
# an Intel Core i5-2500 at 3.30 GHz): context only, another machine, list and grid.
PAPER_CONTEXT = {
    "hardware": "1 core, Intel Core i5-2500 @ 3.30 GHz",
    "workload": "BT2 H2O, 5e8 transitions, 0-30000 cm^-1 at 0.1 cm^-1, I/O excluded",
    "humlicek_voigt_s": 2775.6,
    "vectorized_voigt_s": 251.2,
    "humlicek_threshold_1e-30_s": 832.6,
    "vectorized_voigt_threshold_1e-30_s": 70.0,
    "humlicek_line_profiles_per_s": 5e8 / 2775.6,
    "vectorized_voigt_line_profiles_per_s": 5e8 / 251.2,
    "note": "context, not the target: the paper prints no GPU figure",
}


def cpu_baseline_c5(cfg, n_lines, tps):
    """The FP64 oracle (as it stands) on the first n_lines transitions of the hot-polyatomic
    list at the given (T, P) points (a0 broadening), full grid."""
    import numpy as np
    import oracle as O
    import synth
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed, device="cpu")
    up, lo = synth.linelist.make_transitions(E, n_lines, cfg.nu_max, cfg.seed)
    A = synth.linelist.make_line_params(n_lines, cfg.seed)[0]
    gt, nt = synth.make_broadening_table(cfg.seed)
    Eh, gh, Jh = E.numpy(), g.numpy(), J.numpy()
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    profiles = 0
    Qs = {}
    for T, P in tps:
        if T not in Qs:
            Qs[T] = O.partition_function(Eh, gh, T)
        ls = O.make_lineset(Eh, gh, up.numpy(), lo.numpy(), A.numpy(), T, P, cfg.mass_amu, J=Jh,
                            broad_table=(gt.numpy(), nt.numpy()), Q=Qs[T])
        O.cross_section(ls, cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.cutoff, workers=cores)
        klo, khi = O.window(ls.nu, cfg.nu_a, cfg.dnu, cfg.n_points, cfg.cutoff)
        profiles += int(np.count_nonzero(khi >= klo))
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=profiles / dt, unit="line-profiles/s", cores=cores, kind="oracle",
                sample=f"first {n_lines} transitions of the 4e9-transition list x {len(tps)} (T,P) "
                       f"{[(round(T, 1), P) for T, P in tps]}, full 1,200,001-point grid, Q(T) over the 5e7 "
                       f"states included; {dt:.1f} s wall on {cores} processes ({cpu})")


def c5_run(args):
    """Headline: the hot-polyatomic workload.  4e9 transitions (int32 upper, int32 lower,
    float A: 48 GB) among 5e7 states (16 Da), generated on the device and kept in HBM; 9 T
    (300-3000 K) x 4 P (1e-5-100 bar); a0 broadening by lower-state J; FP32 Voigt on
    0-12000 cm^-1 at 0.01 cm^-1 (1,200,001 points), cut-off 25 cm^-1.

    One step = one chunk of chunk_lines transitions (2^28: 15 chunks hold the list) through
    the whole path for all 36 (T, P): xs_stream_chunk_device (line preparation and sort,
    Q(T), core pre-passes, tile and far-wing kernels, share combine) and the compensated
    accumulation into the stream's sums.  Step i takes chunk i mod 15, so 15 steps cover
    the list once.  Warm-up steps run on a stream that is discarded."""
    import torch
    import synth
    from paper_1801_09803_amd import Plan
    cfg = synth.CONFIGS["C5"]
    dev = torch.device("cuda:0")
    temps = [t for t in cfg.temperatures for _ in cfg.pressures]
    press = [p for _ in cfg.temperatures for p in cfg.pressures]
    n_tp = len(temps)
    n_total = args.lines or cfg.n_lines
    chunk = min(args.chunk_lines, n_total)
    n_chunks = -(-n_total // chunk)

    base = None
    if not args.no_cpu_baseline:
        cores = len(os.sched_getaffinity(0))
        n_s = args.cpu_lines_per_core // 2 * cores
        tps_s = [(temps[i], press[i]) for i in range(16, 20)]   # 1000 K at the four pressures
        log(f"cpu baseline: oracle on {n_s} C5 lines x {len(tps_s)} (T,P), {cores} processes")
        base = cpu_baseline_c5(cfg, n_s, tps_s)
        log(f"cpu baseline: {base['value']:.3e} line-profiles/s")

    log(f"C5: generating {cfg.n_states} states and {n_total} transitions on {torch.cuda.get_device_name(0)}")
    t_gen = time.perf_counter()
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed, device=dev)
    gt, nt = synth.make_broadening_table(cfg.seed)
    upper = torch.empty(n_total, dtype=torch.int32, device=dev)
    lower = torch.empty(n_total, dtype=torch.int32, device=dev)
    A = torch.empty(n_total, dtype=torch.float32, device=dev)
    gen = 1 << 27
    for a in range(0, n_total, gen):
        b = min(n_total, a + gen)
        up, lo = synth.linelist.make_transitions(E, b - a, cfg.nu_max, cfg.seed, first_line=a)
        upper[a:b], lower[a:b] = up, lo
        A[a:b] = synth.linelist.make_line_params(b - a, cfg.seed, first_line=a, device=dev)[0]
        del up, lo
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    log(f"C5: list generated in {t_gen:.1f} s ({n_total * 12 / 1e9:.1f} GB resident)")

    def part(i):
        a = i * chunk
        b = min(n_total, a + chunk)
        return upper[a:b], lower[a:b], A[a:b]

    plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt",
                precision="fp32", broadening="a0_jlower")
    plan.set_broadening_table(gt.numpy(), nt.numpy())
    plan.set_states(E, g, J)
    tune = None
    if args.tile:
        w, sl, sp, tb = (int(v) for v in args.tile.split(","))
        plan.set_tile_config(w, sl, sp, tb)
    elif args.autotune_ms > 0:
        # tuned on the first chunk at the four pressures of 1000 K
        plan.set_lines(*part(0))
        t_tune = time.perf_counter()
        chosen = plan.autotune(temps[16:20], press[16:20], budget_ms=args.autotune_ms)
        tune = dict(chosen=chosen, wall_s=time.perf_counter() - t_tune, budget_ms=args.autotune_ms,
                    tuned_on="chunk 0 at 1000 K and the four pressures")
        log(f"C5 autotune: {chosen} in {tune['wall_s']:.1f} s")
    stream = torch.cuda.current_stream()
    if args.warmup > 0:
        st = plan.stream(temps, press)
        for i in range(args.warmup):
            log(f"C5 warm-up step {i}")
            st.chunk_device(*part(i % n_chunks))
        st.end()
        del st
    out = torch.empty((n_tp, cfg.n_points), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    plan.set_timing(True)
    log(f"C5: timing {args.steps} steps of {chunk} transitions x {n_tp} (T,P)")
    t0 = time.perf_counter()
    st = plan.stream(temps, press, out=out)
    for i in range(args.steps):
        st.chunk_device(*part(i % n_chunks))
        log(f"C5 step {i} (chunk {i % n_chunks}) handed over at {time.perf_counter() - t0:.1f} s")
    _, kept = st.end()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = plan.kernel_times()
    plan.set_timing(False)
    tile = plan.tile_config()
    log(f"C5: {elapsed:.1f} s, {kept * n_tp / elapsed:.3e} line-profiles/s")
    del st, plan
    torch.cuda.empty_cache()

    # algorithmic work of the timed steps: zone points of the tile kernel, node and
    # window-end evaluations of the far kernel, window points (every chunk a step used,
    # times the steps that used it)
    log("C5: counting zone points of the timed chunks")
    uses = [0] * n_chunks
    for i in range(args.steps):
        uses[i % n_chunks] += 1
    zone_tot = {k: 0 for k in ZONE_FLOPS}
    window_points = 0
    jl_max = gt.numel() - 1
    gt_d, nt_d = gt.to(dev), nt.to(dev)
    for c in range(n_chunks):
        if uses[c] == 0:
            continue
        up, lo, _ = part(c)
        jl = torch.clamp(J[lo.long()].long(), max=jl_max)
        dc = dict(E=E, upper=up, lower=lo, gamma_ref=gt_d[jl], n_exp=nt_d[jl])
        zs = zone_counts_multi(cfg, dc, list(zip(temps, press)), tile["waves"], tile["slices"], chunk=1 << 27)
        for z in zs:
            for k, v in z.items():
                zone_tot[k] += uses[c] * v
        nu = E[up.long()] - E[lo.long()]
        klo = torch.clamp(torch.ceil(((nu - cfg.cutoff) - cfg.nu_a) / cfg.dnu), min=0)
        khi = torch.clamp(torch.floor(((nu + cfg.cutoff) - cfg.nu_a) / cfg.dnu), max=cfg.n_points - 1)
        window_points += uses[c] * n_tp * int(torch.clamp(khi - klo + 1, min=0).sum().item())
        del dc, jl, nu, klo, khi
    del upper, lower, A
    torch.cuda.empty_cache()

    tile_zones = [k for k in ZONE_FLOPS if k not in FAR_ZONES]
    flops = sum(ZONE_FLOPS[k] * zone_tot[k] for k in tile_zones)
    tile_pts = sum(zone_tot[k] for k in tile_zones)
    avg_launch_s = kt["forward_ms"] / kt["forward_launches"] / 1e3
    achieved = flops / kt["forward_launches"] / avg_launch_s / 1e12
    far_s = kt["far_ms"] / 1e3
    value = kept * n_tp / elapsed
    return {
        "metric": "Voigt line-profiles/s at 25 cm^-1 cutoff",
        "value": value,
        "unit": "line-profiles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"C5 hot polyatomic: {n_total} transitions (int32 upper, int32 lower, float A) resident "
                        f"in HBM, {cfg.n_states} states, {cfg.mass_amu} Da, 9 T x 4 P = {n_tp} (T,P) "
                        f"(T {cfg.temperatures[0]:.0f}-{cfg.temperatures[-1]:.0f} K log, P 1e-5-100 bar log), a0 "
                        f"broadening, Voigt FP32, {cfg.nu_a}-{cfg.nu_b} cm^-1 ({cfg.n_points} points, dnu 0.01), "
                        f"cutoff {cfg.cutoff}",
            "step": f"one chunk of {chunk} transitions through all {n_tp} (T,P): line preparation and sort, Q(T), "
                    f"pre-passes, tile and far-wing kernels, compensated accumulation; step i takes chunk "
                    f"i mod {n_chunks}",
            "chunks_in_list": n_chunks,
            "full_list_passes_timed": args.steps / n_chunks,
            "lines_kept_timed": kept,
            "n_tp": n_tp,
            "point_evaluations_timed": window_points,
            "tile": {"waves": tile["waves"], "slices_per_wave": tile["slices"], "n_split": tile["last_split"],
                     "tp_block": tile["last_block"]},
            "autotune": tune,
            "list_generation_s": t_gen,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic_bytes_per_launch("C5", kt["forward_tp"] / kt["forward_launches"]),
            "kernel": "fwd_f32_kernel<Voigt> (tile kernel, one launch per block of (T,P) per chunk)",
            "avg_launch_ms": avg_launch_s * 1e3,
            "launches": kt["forward_launches"],
            "tp_per_launch": kt["forward_tp"] / kt["forward_launches"],
            "algorithmic_flops_per_launch": flops / kt["forward_launches"],
            "flops_per_eval": flops / max(tile_pts, 1),
            "zone_flops": ZONE_FLOPS,
            "zone_points_timed": zone_tot,
            "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED,
        },
        "far_wing_kernel": {
            "avg_launch_ms": kt["far_ms"] / max(kt["far_launches"], 1),
            "node_evaluations_timed": zone_tot["far_node"] + zone_tot["far_node4"],
            "four_node_rule_node_evaluations_timed": zone_tot["far_node4"],
            "window_end_point_evaluations_timed": zone_tot["far_exact"],
            "achieved_tflops": sum(ZONE_FLOPS[k] * zone_tot[k] for k in FAR_ZONES) / far_s / 1e12
            if far_s > 0 else None,
        },
        "step_breakdown_ms": {
            "line_prep_and_sort": kt["prep_ms"] / args.steps,
            "pre_passes": kt["core_ms"] / args.steps,
            "tile_kernel": kt["forward_ms"] / args.steps,
            "far_wing_kernel": kt["far_ms"] / args.steps,
            "split_combine": kt["combine_ms"] / args.steps,
        },
        "point_evaluations_per_s": window_points / elapsed,
        "cpu_baseline": base,
    }


def c2_run(args, workload="C2", with_baseline=False, steps=3, warmup=1):
    """The single-cross-section workload (1e8 lines, 296 K and 2000 K at 1 bar): timed
    steps of line preparation + Q(T) + one batched FP32 call over both (T, P), the plain
    FP64 path, a graph replay, the 270-point (T, P) grid on the same list, and the
    Vectorized Voigt, binned, threshold and emission legs when asked for."""
    import synth
    cfg = synth.CONFIGS[workload]
    n_lines = args.lines or cfg.n_lines
    temps, pressures = list(cfg.temperatures), list(cfg.pressures) * (len(cfg.temperatures) // len(cfg.pressures) or 1)
    if len(pressures) != len(temps):
        pressures = [cfg.pressures[0]] * len(temps)

    base = None
    if with_baseline:
        cores = len(os.sched_getaffinity(0))
        n_s = min(n_lines, args.cpu_lines_per_core * cores)
        log(f"cpu baseline: oracle on {n_s} lines, {cores} processes")
        base = cpu_baseline(cfg, n_s, temps, pressures)
        log(f"cpu baseline: {base['value']:.3e} line-profiles/s")

    import torch
    from paper_1801_09803_amd import Plan

    dev = torch.device("cuda:0")
    log(f"generating {n_lines} lines / {cfg.n_states} states on {torch.cuda.get_device_name(0)}")
    d = synth.make_linelist(cfg, n_lines=n_lines, device=dev)
    torch.cuda.synchronize()

    # algorithmic units: grid points inside every kept line's window (same for each (T,P))
    E = d["E"]
    nu = E[d["upper"].long()] - E[d["lower"].long()]
    klo = torch.clamp(torch.ceil(((nu - cfg.cutoff) - cfg.nu_a) / cfg.dnu), min=0)
    khi = torch.clamp(torch.floor(((nu + cfg.cutoff) - cfg.nu_a) / cfg.dnu), max=cfg.n_points - 1)
    evals_per_tp = int(torch.clamp(khi - klo + 1, min=0).sum().item())
    del nu, klo, khi

    def make(precision):
        return Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff,
                    profile="voigt", precision=precision, slices_per_wave=args.slices_per_wave)

    plan = make("fp32")
    plan.set_states(d["E"], d["g"], d["J"])
    stream = torch.cuda.current_stream()
    tune = None
    if args.tile:
        w, sl, sp, tb = (int(v) for v in args.tile.split(","))
        plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
        plan.set_tile_config(w, sl, sp, tb)
    elif args.autotune_ms > 0:
        plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
        t_tune = time.perf_counter()
        chosen = plan.autotune(temps, pressures, budget_ms=args.autotune_ms)
        tune = dict(chosen=chosen, wall_s=time.perf_counter() - t_tune, budget_ms=args.autotune_ms)
        log(f"autotune: {chosen} in {tune['wall_s']:.1f} s")
    out = torch.empty((len(temps), cfg.n_points), dtype=torch.float32, device=dev)

    def step():
        plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
        ev0.record(stream)
        plan.cross_section(temps, pressures, out=out)
        ev1.record(stream)

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(warmup):
        log(f"warmup step {i}")
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)   # hipEvents around each library kernel launch, on this stream
    kern_ms = []
    log(f"timing {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
        torch.cuda.synchronize()
        kern_ms.append(ev0.elapsed_time(ev1))
        log(f"step {i}: forward {kern_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = plan.kernel_times()
    plan.set_timing(False)
    n_kept = plan.lines_kept()
    n_tp = len(temps)
    value = n_kept * n_tp * steps / elapsed
    ms_step = 1e3 * elapsed / steps
    avg_launch_s = kt["forward_ms"] / kt["forward_launches"] / 1e3
    tp_per_launch = kt["forward_tp"] / kt["forward_launches"]
    # forward time per (T, P): tile kernel + node-sampled far-wing kernel
    fwd_s_per_tp = (kt["forward_ms"] + kt["far_ms"]) / kt["forward_tp"] / 1e3
    # region-weighted algorithmic flops of the timed launches (every step covers all (T, P))
    tile = plan.tile_config()
    zones = [zone_counts(cfg, d, T, P, tile["waves"], tile["slices"]) for T, P in zip(temps, pressures)]
    # the tile kernel evaluates the window points outside the node-sampled far wing
    tile_zones = [k for k in ZONE_FLOPS if k not in FAR_ZONES]
    flops_step = sum(sum(ZONE_FLOPS[k] * z[k] for k in tile_zones) for z in zones)
    tile_points_step = sum(sum(z[k] for k in tile_zones) for z in zones)
    launches_per_step = kt["forward_launches"] / steps
    flops_per_launch = flops_step / launches_per_step
    achieved = flops_per_launch / avg_launch_s / 1e12
    flops_per_eval = flops_step / tile_points_step
    # far-wing kernel: FAR_NODES evaluations per (line, wavefront) it samples; it reads 28 B
    # of line data (hot record words and kc) per 2-node pair
    far_nodes_step = sum(z["far_node"] + z["far_node4"] for z in zones)
    far_exact_step = sum(z["far_exact"] for z in zones)
    far_flops_step = sum(sum(ZONE_FLOPS[k] * z[k] for k in FAR_ZONES) for z in zones)
    far_s_step = kt["far_ms"] / 1e3 / steps
    far_obj = None
    if kt["far_launches"] > 0 and far_nodes_step > 0:
        far_obj = {
            "avg_launch_ms": kt["far_ms"] / kt["far_launches"],
            "node_evaluations_per_tp": far_nodes_step / len(temps),
            "window_end_point_evaluations_per_tp": far_exact_step / len(temps),
            "four_node_rule_node_evaluations_per_tp": sum(z["far_node4"] for z in zones) / len(temps),
            "achieved_tflops": far_flops_step / far_s_step / 1e12,
            "line_data_GBps": 28.0 * far_nodes_step / FAR_NODES / far_s_step / 1e9,
            "note": "node-sampled wings (every (line, wavefront) pair whose centre lies beyond max(far reach, "
                    "|z| < 8 radius)): 16 evaluations per pair by the 2-node rule (11 flops) or, inside the "
                    "|z| < 40 radius, the 4-node rule (20 flops), and the points of a window end's block one "
                    "by one; one 16-node barycentric interpolation per point; line data from L2/MALL",
        }

    result = {
        "metric": "Voigt line-profiles/s at 25 cm^-1 cutoff",
        "value": value,
        "unit": "line-profiles/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {n_lines} transitions, {cfg.n_states} states, {cfg.mass_amu} Da, "
                        f"T={temps} K, P={pressures} bar, Voigt, {cfg.nu_a}-{cfg.nu_b} cm^-1 "
                        f"({cfg.n_points} points, dnu={cfg.dnu}), cutoff {cfg.cutoff}",
            "lines_kept": n_kept,
            "n_tp": n_tp,
            "point_evaluations_per_tp": evals_per_tp,
            "precision": "fp32 profiles, fp64 line setup, compensated fp32 sums",
            "step": "xs_set_lines (prep + sort) + Q(T) + batched forward",
            "tile": {"waves": tile["waves"], "slices_per_wave": tile["slices"],
                     "n_split": tile["last_split"], "tp_block": tile["last_block"]},
            "autotune": tune,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic_bytes_per_launch(workload, tp_per_launch),
            "kernel": "fwd_f32_kernel<Voigt> (tile kernel, one launch per block of (T,P))",
            "avg_launch_ms": avg_launch_s * 1e3,
            "tp_per_launch": tp_per_launch,
            "algorithmic_flops_per_launch": flops_per_launch,
            "flops_per_eval": flops_per_eval,
            "zone_flops": ZONE_FLOPS,
            "zone_points_per_tp": {f"T={T}": z for T, z in zip(temps, zones)},
            "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED,
        },
        "far_wing_kernel": far_obj,
        "step_breakdown_ms": {
            "line_prep_and_sort": kt["prep_ms"] / steps,
            "voigt_core_prepass": kt["core_ms"] / steps,
            "tile_kernel": kt["forward_ms"] / steps,
            "far_wing_kernel": kt["far_ms"] / steps,
            "split_combine": kt["combine_ms"] / steps,
        },
        "forward_line_profiles_per_s": n_kept / fwd_s_per_tp,
        "point_evaluations_per_s": evals_per_tp / fwd_s_per_tp,
        "cpu_baseline": base,
    }

    if not args.no_fp64:
        plan64 = make("fp64")
        plan64.set_states(d["E"], d["g"], d["J"])
        plan64.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
        out64 = torch.empty((1, cfg.n_points), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        log("timing the plain FP64 path (one call per (T,P))")
        ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev2.record(stream)
        for T, P in zip(temps, pressures):
            plan64.cross_section([T], [P], out=out64)
        ev3.record(stream)
        torch.cuda.synchronize()
        t64 = ev2.elapsed_time(ev3) / 1e3
        result["fp64_plain_forward_line_profiles_per_s"] = n_kept * n_tp / t64
        result["fp32_vs_fp64_forward_speedup"] = t64 / (fwd_s_per_tp * n_tp)
        # agreement of the two paths on the last (T, P)
        ref = out64[0]
        got = out[-1].double()
        mask = ref > 1e-6 * ref.max()
        result["fp32_vs_fp64_max_rel"] = float(((got - ref).abs()[mask] / ref[mask]).max().item())
        result["fp32_vs_fp64_area_rel"] = float(abs(got.sum().item() - ref.sum().item()) / ref.sum().item())
        del plan64, out64

    if not args.no_graph:
        # the batched call captured once and replayed (no host work, no waits)
        graph = plan.graph(temps, pressures)
        graph.launch()
        torch.cuda.synchronize()
        ev4, ev5 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        ev4.record(stream)
        for _ in range(reps):
            graph.launch()
        ev5.record(stream)
        torch.cuda.synchronize()
        tg = ev4.elapsed_time(ev5) / 1e3 / reps
        result["graph_replay"] = {"ms": tg * 1e3, "line_profiles_per_s": n_kept * n_tp / tg,
                                  "equal_to_direct_call": bool(torch.equal(graph.sigma, out))}
        log(f"graph replay {tg * 1e3:.1f} ms")
        graph.close()

    if args.all_legs and not args.no_vv:
        result["vectorized_voigt"] = vv_leg(cfg, d, temps, pressures, tile, out, n_kept, stream, log)
    if args.all_legs and not args.no_binned:
        result["binned_profiles"] = binned_leg(cfg, d, temps, pressures, n_kept, stream, log)
    if args.all_legs and not args.no_threshold:
        result["intensity_threshold"] = threshold_leg(cfg, d, temps, pressures, tile, n_kept, stream, log)
    if not args.no_c3 and cfg.name == "C2":
        result["c3_grid"] = c3_leg(synth.CONFIGS["C3"], d, tile, n_kept, stream, log)
    if args.all_legs and not args.no_emission:
        result["emission_and_state_reductions"] = emission_leg(cfg, d, temps, pressures, tile, n_kept, stream,
                                                                log)

    del plan, out, d
    torch.cuda.empty_cache()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15,
                    help="timed steps (C5: one 2^28-transition chunk through all 36 (T, P) each; 15 cover "
                         "the 4e9-transition list once)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C5", help="headline workload: C5 (default) or C2")
    ap.add_argument("--chunk-lines", type=int, default=1 << 28, help="C5: transitions per step")
    ap.add_argument("--no-c2", action="store_true", help="C5 headline: skip the C2 / C3 sub-entries")
    ap.add_argument("--c2-steps", type=int, default=5, help="timed steps of the C2 sub-entry")
    ap.add_argument("--all-legs", action="store_true",
                    help="also run the Vectorized Voigt, binned, threshold and emission legs on C2")
    ap.add_argument("--lines", type=int, default=0, help="truncate the line list (profiling runs)")
    ap.add_argument("--slices-per-wave", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-vv", action="store_true", help="skip the Vectorized Voigt leg")
    ap.add_argument("--no-binned", action="store_true", help="skip the binned-profile / super-line leg")
    ap.add_argument("--no-threshold", action="store_true", help="skip the intensity-threshold leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 270-point (T, P) grid leg")
    ap.add_argument("--no-emission", action="store_true",
                    help="skip the emission cross-section and state-reduction leg")
    ap.add_argument("--stream-chunks", type=int, default=4)
    ap.add_argument("--stream-chunk-lines", type=int, default=1 << 24)
    ap.add_argument("--autotune-ms", type=float, default=6000.0,
                    help="autotuner budget (0: keep the library's default tile shape)")
    ap.add_argument("--tile", default="", help="fixed tile config waves,slices,n_split,tp_block")
    ap.add_argument("--cpu-lines-per-core", type=int, default=40000)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--valu-probe", type=int, default=0,
                    help="only run the library's FMA-loop kernel with this many iterations per "
                         "thread (VALU counter calibration)")
    args = ap.parse_args()

    if args.valu_probe:
        import torch
        from paper_1801_09803_amd import binding
        n_threads = 256 * 256 * 64     # 64 workgroups of 256 per CU
        out = torch.empty(n_threads, dtype=torch.float32, device="cuda")
        binding.valu_probe(out, args.valu_probe)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.valu_probe(out, args.valu_probe)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fma = n_threads * 16 * args.valu_probe
        print(json.dumps({"valu_probe_threads": n_threads, "iters": args.valu_probe,
                          "v_fma_f32_per_launch": fma, "wall_s": dt,
                          "fp32_tflops": 2.0 * fma / dt / 1e12}), flush=True)
        return

    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe * 2**18, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 4}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    result = {}
    if args.workload == "C5":
        result = c5_run(args)
        if not args.no_c2:
            result["c2"] = c2_run(args, steps=args.c2_steps, warmup=1)
    else:
        result = c2_run(args, args.workload, with_baseline=not args.no_cpu_baseline, steps=args.steps,
                        warmup=args.warmup)
    import synth
    import torch
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        result["fwd_adj"] = fwd_adj(synth.CONFIGS["C4"], torch.device("cuda:0"), torch.cuda.current_stream(), log)
    if not args.no_stream:
        result["streaming_from_host"] = stream_run(synth.CONFIGS["C5"], torch.device("cuda:0"), log,
                                                   args.stream_chunks, args.stream_chunk_lines)
    result["paper_cpu_context"] = PAPER_CONTEXT
    print(json.dumps(result), flush=True)


def vv_leg(cfg, d, temps, pressures, tile, voigt_out, n_kept, stream, log):
    """The Vectorized Voigt (beta = 1) and its area-normalised form (with beta) on the same
    list and tile shape: one call over all (T, P), pre-passes included, and how far each
    departs from the Voigt result of the timed steps (an approximation, not an error)."""
    import torch
    from paper_1801_09803_amd import Plan
    legs = {}
    for prof, beta in (("vvoigt", False), ("vvoigt_norm", True)):
        plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile=prof,
                    precision="fp32", vv_beta=beta)
        plan.set_states(d["E"], d["g"], d["J"])
        plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
        plan.set_tile_config(tile["waves"], tile["slices"], tile["last_split"], 1)
        out = torch.empty((len(temps), cfg.n_points), dtype=torch.float32, device="cuda")
        plan.cross_section(temps, pressures, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 2
        plan.set_timing(True)
        e0.record(stream)
        for _ in range(reps):
            plan.cross_section(temps, pressures, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        kt = plan.kernel_times()
        plan.set_timing(False)
        t_call = e0.elapsed_time(e1) / 1e3 / reps
        ntp = len(temps)
        ref, got = voigt_out.double(), out.double()
        mask = ref > 1e-6 * ref.max()
        legs[prof] = {
            "vv_beta": beta,
            "line_profiles_per_s": n_kept * ntp / t_call,
            "call_ms": t_call * 1e3,
            "tile_kernel_ms_per_tp": kt["forward_ms"] / kt["forward_tp"],
            "pre_passes_ms_per_tp": kt["core_ms"] / (reps * ntp),
            "max_rel_vs_voigt": float(((got - ref).abs()[mask] / ref[mask]).max().item()),
            "area_rel_vs_voigt": float(((got.sum(dim=1) - ref.sum(dim=1)) / ref.sum(dim=1)).abs().max().item()),
        }
        log(f"{prof}: {t_call * 1e3:.1f} ms per call ({legs[prof]['tile_kernel_ms_per_tp']:.1f} ms tile kernel per (T,P))")
        del plan, out
    legs["note"] = ("same list, grid and tile shape as the headline; radius 4 cm^-1; call = Q(T) + "
                    "pre-passes + tile kernel for all (T,P), line preparation excluded")
    return legs


def threshold_leg(cfg, d, temps, pressures, tile, n_kept, stream, log):
    """The headline workload with HITRAN's dynamic intensity cut-off at its defaults
    (I_crit = 1e-29 cm/molecule, nu_crit = 2000 cm^-1): one call over both (T, P), the
    share of lines kept at each (computed here from the same arrays, for the report)."""
    import torch
    from paper_1801_09803_amd import Plan
    plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt")
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    plan.set_tile_config(tile["waves"], tile["slices"], tile["last_split"], 1)
    plan.set_intensity_threshold("hitran", 1e-29, 2000.0)
    out = torch.empty((len(temps), cfg.n_points), dtype=torch.float32, device="cuda")
    plan.cross_section(temps, pressures, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    plan.set_timing(True)
    e0.record(stream)
    for _ in range(reps):
        plan.cross_section(temps, pressures, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.set_timing(False)
    t = e0.elapsed_time(e1) / 1e3 / reps
    # kept shares (Eq. 1 in double on the same arrays; the library does this per (T, P))
    c2 = 1.4387768775039338
    E = d["E"]
    up, lo = d["upper"].long(), d["lower"].long()
    nu = E[up] - E[lo]
    A = d["A"].double()
    gup = d["g"].double()[up]
    cA = gup * A / (8.0 * math.pi * 2.99792458e10 * nu * nu)
    shares = []
    for T in temps:
        Q = float((d["g"].double() * torch.exp(-c2 * E / T)).sum().item())
        S = cA * torch.exp(-c2 * E[lo] / T) * (-torch.expm1(-c2 * nu / T)) / Q
        cut = torch.where(nu <= 2000.0, 1e-29 * (nu / 2000.0) * torch.tanh(c2 * nu / (2.0 * T)),
                          torch.full_like(nu, 1e-29))
        shares.append(float((S >= cut).double().mean().item()))
    del plan, out
    log(f"threshold: {t * 1e3:.1f} ms per call, kept {shares}")
    return {"mode": "hitran", "i_crit": 1e-29, "nu_crit": 2000.0, "call_ms": t * 1e3,
            "line_profiles_per_s_of_the_list": n_kept * len(temps) / t,
            "tile_kernel_ms_per_tp": kt["forward_ms"] / kt["forward_tp"],
            "far_kernel_ms_per_tp": kt["far_ms"] / kt["forward_tp"],
            "pre_passes_ms_per_tp": kt["core_ms"] / (reps * len(temps)),
            "kept_share_per_tp": shares,
            "note": "throughput counts every line of the list (kept or dropped), as the headline does; "
                    "call = Q(T) + threshold compaction + pre-passes + tile kernel"}


def c3_leg(cfg3, d, tile, n_kept, stream, log):
    """The C3 grid on C2's list: all 27 x 10 (T, P) cross sections from one batched FP32
    call (Q, pre-passes and tile kernels, in the headline's tile shape), against the plain
    FP64 path timed on three of the points (one call each) and scaled to 270."""
    import torch
    from paper_1801_09803_amd import Plan
    Ts = [T for T in cfg3.temperatures for _ in cfg3.pressures]
    Ps = [P for _ in cfg3.temperatures for P in cfg3.pressures]
    plan = Plan(cfg3.nu_a, cfg3.nu_b, cfg3.n_points, cfg3.mass_amu, cutoff=cfg3.cutoff, profile="voigt")
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    plan.set_tile_config(tile["waves"], tile["slices"], tile["last_split"], 0)
    out = torch.empty((len(Ts), cfg3.n_points), dtype=torch.float32, device="cuda")
    log(f"C3: {len(Ts)} (T, P) in one call")
    plan.cross_section(Ts[:4], Ps[:4], out=out[:4])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.set_timing(True)
    e0.record(stream)
    plan.cross_section(Ts, Ps, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.set_timing(False)
    t = e0.elapsed_time(e1) / 1e3
    del plan
    # plain FP64 path: one call per (T, P) on three points of the grid
    p64 = Plan(cfg3.nu_a, cfg3.nu_b, cfg3.n_points, cfg3.mass_amu, cutoff=cfg3.cutoff, profile="voigt",
               precision="fp64")
    p64.set_states(d["E"], d["g"], d["J"])
    p64.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    o64 = torch.empty((1, cfg3.n_points), dtype=torch.float64, device="cuda")
    pick = [0, 135, 269]
    p64.cross_section([Ts[0]], [Ps[0]], out=o64)
    torch.cuda.synchronize()
    t64, dev64 = 0.0, 0.0
    for i in pick:
        e0.record(stream)
        p64.cross_section([Ts[i]], [Ps[i]], out=o64)
        e1.record(stream)
        torch.cuda.synchronize()
        t64 += e0.elapsed_time(e1) / 1e3
        ref, got = o64[0], out[i].double()
        m = ref > 1e-6 * ref.max()
        dev64 = max(dev64, float(((got - ref).abs()[m] / ref[m]).max().item()))
    del p64, o64, out
    t64_all = t64 / len(pick) * len(Ts)
    log(f"C3: {t:.2f} s for 270 (T, P) ({n_kept * len(Ts) / t:.3e} line-profiles/s); plain FP64 "
        f"~{t64_all:.0f} s (from 3 points)")
    return {"n_tp": len(Ts), "call_s": t, "line_profiles_per_s": n_kept * len(Ts) / t,
            "tile_kernel_ms_per_tp": kt["forward_ms"] / kt["forward_tp"],
            "far_kernel_ms_per_tp": kt["far_ms"] / kt["forward_tp"],
            "pre_passes_ms_per_tp": kt["core_ms"] / len(Ts),
            "tp_block": 0,
            "fp64_plain_s_per_tp": t64 / len(pick), "fp64_plain_s_extrapolated": t64_all,
            "fp32_batched_vs_fp64_plain_speedup": t64_all / t,
            "fp32_vs_fp64_max_rel_at_sampled_tp": dev64,
            "note": "C3 = C2's 1e8 lines at 27 T (100-3000 K, log) x 10 P (1e-5-100 bar, log); one FP32 "
                    "call over all 270 (Q, pre-passes, tile kernels; line preparation excluded); the FP64 "
                    "plain time is 3 single-(T,P) calls scaled to 270"}


def emission_leg(cfg, d, temps, pressures, tile, n_kept, stream, log):
    """Emission cross sections of the headline workload (same list, grid and tile shape),
    and the state reductions over the same list: radiative lifetimes, the cooling function
    at 27 temperatures (100-3000 K, log-spaced) and the partition-function moments with C_p
    at the same temperatures."""
    import time
    import torch
    import synth
    from paper_1801_09803_amd import Plan
    plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt")
    plan.set_states(d["E"], d["g"], d["J"])
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    plan.set_tile_config(tile["waves"], tile["slices"], tile["last_split"], 1)
    plan.set_intensity_kind("emission")
    out = torch.empty((len(temps), cfg.n_points), dtype=torch.float32, device="cuda")
    plan.cross_section(temps, pressures, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 2
    plan.set_timing(True)
    e0.record(stream)
    for _ in range(reps):
        plan.cross_section(temps, pressures, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.set_timing(False)
    t_em = e0.elapsed_time(e1) / 1e3 / reps
    n_lines, n_states = d["upper"].numel(), d["E"].numel()
    Ts = [100.0 * 30.0 ** (j / 26.0) for j in range(27)]

    def wall(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # non-LTE populations: manifold labels (2000 cm^-1 energy bands of the synthetic states),
    # the line set rebuilt with its vibrational energies, then one call over both points with
    # T_vib = 1000 K
    plan.set_intensity_kind("absorption")
    plan.set_vibrational_labels(synth.make_vibrational_labels(d["E"]))
    plan.set_lines(d["upper"], d["lower"], d["A"], d["gamma_ref"], d["n_exp"])
    t_vib = [1000.0] * len(temps)
    plan.cross_section_nlte(temps, t_vib, pressures, out=out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        plan.cross_section_nlte(temps, t_vib, pressures, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    t_nlte = e0.elapsed_time(e1) / 1e3 / reps
    plan.set_vibrational_labels(None)
    t_tau = wall(lambda: plan.lifetimes(d["upper"], d["A"]))
    t_w = wall(lambda: plan.cooling_function(d["upper"], d["lower"], d["A"], Ts))
    t_m = wall(lambda: plan.partition_moments(Ts))
    # algorithmic bytes: lifetimes read upper + A (8 B per transition) and read-modify-write
    # 8 B per state twice (sum, tau); the cooling function reads upper, lower, A and two
    # energies (24 B per transition, the energies mostly from cache)
    tau_bytes = 8.0 * n_lines + 24.0 * n_states
    del plan, out
    log(f"emission: {t_em * 1e3:.1f} ms per call; non-LTE {t_nlte * 1e3:.1f} ms per call; lifetimes {t_tau * 1e3:.2f} ms, cooling (27 T) "
        f"{t_w * 1e3:.2f} ms, moments (27 T) {t_m * 1e3:.3f} ms")
    return {"emission_call_ms": t_em * 1e3, "emission_line_profiles_per_s": n_kept * len(temps) / t_em,
            "emission_tile_kernel_ms_per_tp": kt["forward_ms"] / kt["forward_tp"],
            "emission_far_kernel_ms_per_tp": kt["far_ms"] / kt["forward_tp"],
            "nlte_call_ms": t_nlte * 1e3, "nlte_line_profiles_per_s": n_kept * len(temps) / t_nlte,
            "nlte_T_vib": t_vib,
            "lifetimes_ms": t_tau * 1e3, "lifetimes_transitions_per_s": n_lines / t_tau,
            "lifetimes_algorithmic_GBps": tau_bytes / t_tau / 1e9,
            "cooling_27T_ms": t_w * 1e3, "cooling_transitions_per_s": n_lines / t_w,
            "moments_cp_27T_ms": t_m * 1e3, "moments_state_temperatures_per_s": n_states * len(Ts) / t_m,
            "note": "state reductions: whole synchronous calls (argument checks, device work, the wait for "
                    "the index flags), wall clock; emission call = Q(T) + pre-passes + tile kernel"}


def binned_leg(cfg2, d2, temps, pressures, n_kept2, stream, log):
    """Bin-averaged profiles on the coarse C1 grid they are meant for (0.1 cm^-1; the
    sampled Voigt profile timed alongside), and super-line histograms of the C2 list."""
    import torch
    import synth
    from paper_1801_09803_amd import Plan

    def timed(plan, Ts, Ps, out, reps=5):
        plan.cross_section(Ts, Ps, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.cross_section(Ts, Ps, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    res = {}
    cfg1 = synth.CONFIGS["C1"]
    d1 = synth.make_linelist(cfg1, device="cuda")
    out1 = torch.empty((1, cfg1.n_points), dtype=torch.float32, device="cuda")
    T1, P1 = [cfg1.temperatures[0]], [cfg1.pressures[0]]
    for prof in ("voigt", "doppler_binned", "lorentz_binned"):
        plan = Plan(cfg1.nu_a, cfg1.nu_b, cfg1.n_points, cfg1.mass_amu, cutoff=cfg1.cutoff, profile=prof)
        plan.set_states(d1["E"], d1["g"], d1["J"])
        plan.set_lines(d1["upper"], d1["lower"], d1["A"], d1["gamma_ref"], d1["n_exp"])
        t = timed(plan, T1, P1, out1)
        res[f"C1_{prof}"] = {"call_ms": t * 1e3, "line_profiles_per_s": plan.lines_kept() / t}
        log(f"C1 {prof}: {t * 1e3:.2f} ms per call")
        del plan
    plan = Plan(cfg2.nu_a, cfg2.nu_b, cfg2.n_points, cfg2.mass_amu, cutoff=cfg2.cutoff, profile="superlines")
    plan.set_states(d2["E"], d2["g"], d2["J"])
    plan.set_lines(d2["upper"], d2["lower"], d2["A"], d2["gamma_ref"], d2["n_exp"])
    out2 = torch.empty((len(temps), cfg2.n_points), dtype=torch.float32, device="cuda")
    t = timed(plan, temps, pressures, out2, reps=3)
    res["C2_superlines"] = {"call_ms": t * 1e3, "lines_per_s": n_kept2 * len(temps) / t,
                            "note": "per-bin intensity sums of the 1e8 sorted lines for both (T,P); "
                                    "line preparation excluded"}
    log(f"C2 super-lines: {t * 1e3:.2f} ms per call")
    res["note"] = ("C1: 1e5 lines, 0-5000 cm^-1 at 0.1, 1000 K, 1 bar, FP32; call = Q(T) + pre-passes + "
                   "tile kernel, line preparation excluded")
    return res


def stream_run(cfg, dev, log, n_chunks, chunk):
    """Hot-polyatomic workload streamed from pinned host memory: the first n_chunks
    chunks of `chunk` transitions (of the 4e9-line list), 5e7 states, 9 T x 4 P, a0
    broadening, FP32 Voigt on 0-12000 cm^-1 at 0.01.  Timed from xs_stream_begin to the
    end of xs_stream_end: host-to-device copies, line preparation, core pre-pass, tile
    kernels and accumulation."""
    import torch
    import synth
    from paper_1801_09803_amd import Plan
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed, device=dev)
    gt, nt = synth.make_broadening_table(cfg.seed)
    T = [t for t in cfg.temperatures for _ in cfg.pressures]
    P = [p for _ in cfg.temperatures for p in cfg.pressures]
    host, evals = [], 0
    for c in range(n_chunks):
        up, lo = synth.linelist.make_transitions(E, chunk, cfg.nu_max, cfg.seed, first_line=c * chunk)
        A = synth.linelist.make_line_params(chunk, cfg.seed, first_line=c * chunk, device=dev)[0]
        nu = E[up.long()] - E[lo.long()]
        klo = torch.clamp(torch.ceil(((nu - cfg.cutoff) - cfg.nu_a) / cfg.dnu), min=0)
        khi = torch.clamp(torch.floor(((nu + cfg.cutoff) - cfg.nu_a) / cfg.dnu), max=cfg.n_points - 1)
        evals += int(torch.clamp(khi - klo + 1, min=0).sum().item())
        host.append([t.cpu().pin_memory() for t in (up, lo, A)])
        del up, lo, A, nu, klo, khi
        if n_chunks > 4:
            log(f"  generated chunk {c + 1}/{n_chunks}")
    plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt",
                precision="fp32", broadening="a0_jlower")
    plan.set_broadening_table(gt.numpy(), nt.numpy())
    plan.set_states(E, g, J)
    out = torch.empty((len(T), cfg.n_points), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log(f"streaming {n_chunks} chunks of {chunk} lines x {len(T)} (T,P)")
    t0 = time.perf_counter()
    st = plan.stream(T, P, out=out)
    for c, h in enumerate(host):
        st.chunk(*h)
        if n_chunks > 4:
            log(f"  chunk {c + 1}/{n_chunks} handed over")
    _, kept = st.end()
    dt = time.perf_counter() - t0
    n_lines = n_chunks * chunk
    res = {
        "workload": f"{cfg.name}: first {n_lines} of {cfg.n_lines} transitions in {n_chunks} chunks of {chunk}, "
                    f"{cfg.n_states} states, {cfg.mass_amu} Da, {len(T)} (T,P) (9 T x 4 P), a0 broadening, "
                    f"{cfg.nu_a}-{cfg.nu_b} cm^-1 ({cfg.n_points} points), Voigt FP32",
        "wall_s": dt,
        "lines_kept": kept,
        "line_profiles_per_s": kept * len(T) / dt,
        "point_evaluations_per_s": evals * len(T) / dt,
        "h2d_bytes": n_lines * 12,
        "full_list_extrapolated_s": dt * cfg.n_lines / n_lines,
        "note": "timed from stream begin to end, host-to-device copies included; the full-list time is a "
                "linear extrapolation unless the chunks cover the whole list",
    }
    log(f"streaming: {dt:.2f} s, {res['line_profiles_per_s']:.3e} line-profiles/s")
    del plan, out, st, host
    return res


def fwd_adj(cfg, dev, stream, log):
    """Retrieval step (forward + adjoint) on the retrieval workload: batched FP32 path
    against the plain FP64 path; dL/dsigma = 2 (sigma - sigma*) with sigma* from the
    seeded perturbation (T x 1.05, gamma_ref x 1.1, ln A + N(0, 0.05)).  Each timed step
    runs its own forward and adjoint; the gradient comparison feeds both precisions'
    adjoints one dL/dsigma, from the FP64 forward (rounded to float for the FP32 path)."""
    import torch
    import synth
    from paper_1801_09803_amd import Plan
    d = synth.make_linelist(cfg, device=dev)
    T, P = cfg.temperatures[0], cfg.pressures[0]
    logA = torch.log(d["A"].double()).float()
    pert = synth.linelist.perturbation_normals(cfg.n_lines, cfg.seed).to(dev)
    res = {"workload": f"{cfg.name}: {cfg.n_lines} transitions, {cfg.n_states} states, T={T} K, P={P} bar, "
                       f"{cfg.nu_a}-{cfg.nu_b} cm^-1 ({cfg.n_points} points), Voigt"}
    plans, targets = {}, {}
    for prec in ("fp64", "fp32"):
        plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff, profile="voigt",
                    precision=prec, a_is_log=True)
        plan.set_states(d["E"], d["g"], d["J"])
        plan.set_lines(d["upper"], d["lower"], (logA.double() + 0.05 * pert).float(), d["gamma_ref"] * 1.1,
                       d["n_exp"])
        targets[prec] = plan.cross_section([1.05 * T], [P]).clone()
        plan.set_lines(d["upper"], d["lower"], logA, d["gamma_ref"], d["n_exp"])
        plans[prec] = plan
    kept = plans["fp32"].lines_kept()
    for prec in ("fp32", "fp64"):
        plan, target = plans[prec], targets[prec]

        def once():
            sig = plan.cross_section([T], [P])[0]
            g = 2.0 * (sig - target[0])
            return plan.cross_section_adjoint(T, P, g)

        once()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3 if prec == "fp32" else 1
        e0.record(stream)
        for _ in range(reps):
            once()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"{prec}_fwd_adj_ms"] = ms
        res[f"{prec}_line_profiles_per_s"] = 2 * kept / (ms / 1e3)
        log(f"fwd+adj {prec}: {ms:.1f} ms")
    res["lines_kept"] = kept
    res["fp32_vs_fp64_speedup"] = res["fp64_fwd_adj_ms"] / res["fp32_fwd_adj_ms"]
    # one dL/dsigma for both adjoints
    gbar = 2.0 * (plans["fp64"].cross_section([T], [P])[0] - targets["fp64"][0])
    g64 = [t.double() if t.numel() > 1 else t.item() for t in plans["fp64"].cross_section_adjoint(T, P, gbar)]
    g32 = [t.double() if t.numel() > 1 else t.item()
           for t in plans["fp32"].cross_section_adjoint(T, P, gbar.float().contiguous())]
    torch.cuda.synchronize()
    res["fp32_vs_fp64_dT_rel"] = abs(g32[0] - g64[0]) / abs(g64[0])
    res["fp32_vs_fp64_dP_rel"] = abs(g32[1] - g64[1]) / abs(g64[1])
    for name, i in (("dlnA", 2), ("dgamma_ref", 3), ("dn", 4)):
        a, b = g32[i], g64[i]
        m = b.abs() > 1e-6 * b.abs().max()
        res[f"fp32_vs_fp64_{name}_max_rel"] = float(((a - b).abs()[m] / b.abs()[m]).max().item())
    res["gradient_comparison"] = ("one dL/dsigma (from the FP64 forward) into both adjoints; per-line maxima over "
                                  "lines whose FP64 gradient exceeds 1e-6 of the largest")
    res["note"] = "one line-profile = one (line, T, P) forward evaluation or its adjoint; the step counts both"
    del plans
    return res


if __name__ == "__main__":
    main()
