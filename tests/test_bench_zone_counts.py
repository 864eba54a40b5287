"""The tile kernel's algorithmic flops, which the bench line's roofline divides by the
kernel's time, come from bench.zone_counts_multi: window points per evaluation zone,
counted from index ranges over whole lines, with the node-sampling radii of the centre's
wavefront.  Here the same counts are enumerated one (line, wavefront, grid point) at a time
with each wavefront's own radii (the library's rule for the FP32 Voigt sweep: lines centred
more than R = max(far reach, |z| < 8 radius) grid steps from a wavefront are node-sampled
at 16 nodes, by the 4-node rule inside the |z| < 40 radius, and the blocks holding their
window ends are evaluated point by point).  CPU only."""
import math

import numpy as np
import pytest
import torch

import bench
import synth
from synth.linelist import WorkloadConfig

CFG = WorkloadConfig("zones", 9, 20_000, 300, 2.0, 3000.0, 0.0, 3000.0, 300_001,
                     (296.0, 3000.0), (1.0, 1e-3))


def enumerate_zones(cfg, d, T, P, waves, slices):
    kB, amu, c_si, ln2 = 1.380649e-23, 1.66053906660e-27, 299792458.0, math.log(2.0)
    beta = math.sqrt(2.0 * kB * T * ln2 / (cfg.mass_amu * amu)) / c_si     # alpha_D / nu
    dnu, n_pts = cfg.dnu, cfg.n_points
    ww = 64 * slices
    bw = 4 if slices == 1 else 8
    reach = (57 * (ww - 1) + 99) // 100
    n_waves = -(-n_pts // (waves * ww)) * waves
    numax = max(abs(cfg.nu_a), abs(cfg.nu_b)) + cfg.cutoff
    scale = 40.0 * beta / (math.sqrt(ln2) * dnu)          # |z| < 40 radius per cm^-1
    rm_all = math.ceil(scale * numax + 2.0)

    def edges(w, span):
        return (abs(cfg.nu_a + (w * ww - span) * dnu), abs(cfg.nu_a + (w * ww + ww - 1 + span) * dnu))

    def rm_of(w):        # |z| < 40 radius of the lines that can lie near wavefront w
        return min(math.ceil(scale * max(edges(w, rm_all + 1))) + 2, rm_all)

    def r_of(w):         # node-sampling radius of wavefront w
        r8 = min(math.ceil(0.2 * scale * max(edges(w, max(reach, rm_all) + 1))) + 2, rm_all)
        return max(r8, reach)

    R = [r_of(w) for w in range(n_waves)]
    RM = [rm_of(w) for w in range(n_waves)]
    out = dict.fromkeys(bench.ZONE_FLOPS, 0)
    E = d["E"].numpy()
    up, lo = d["upper"].numpy().astype(np.int64), d["lower"].numpy().astype(np.int64)
    gref, nexp = d["gamma_ref"].double().numpy(), d["n_exp"].double().numpy()
    for i in range(up.size):
        nu = E[up[i]] - E[lo[i]]
        klo_raw = math.ceil(((nu - cfg.cutoff) - cfg.nu_a) / dnu)
        klo, khi = max(klo_raw, 0), min(math.floor(((nu + cfg.cutoff) - cfg.nu_a) / dnu), n_pts - 1)
        if khi < klo:
            continue
        kc = math.floor((nu - cfg.nu_a) / dnu + 0.5)
        s = math.sqrt(ln2) / (beta * nu)
        y = gref[i] * (296.0 / T) ** nexp[i] * P * s
        for w in range(klo // ww, khi // ww + 1):
            w0, w1 = w * ww, w * ww + ww - 1
            dist = max(w0 - kc, kc - w1, 0)                # grid steps from the centre to the wavefront
            if dist <= R[w]:
                k = np.arange(max(klo, w0), min(khi, w1) + 1)
                x = np.abs(s * ((cfg.nu_a + k * dnu) - nu))
                z2 = x * x + y * y
                out["one_pole"] += int(np.sum(x >= 1000.0))
                near = x < 1000.0
                out["two_node"] += int(np.sum(near & (z2 >= 1600.0)))
                out["four_node"] += int(np.sum(near & (z2 < 1600.0) & (z2 >= 64.0)))
                out["core"] += int(np.sum(z2 < 64.0))
                continue
            out["far_node4" if dist <= RM[w] else "far_node"] += bench.FAR_NODES
            if w == klo // ww and klo_raw >= 0:            # the window starts in this wavefront
                out["far_exact"] += bw - (klo - w0) % bw
            if w == khi // ww:                             # ... or ends in it
                out["far_exact"] += (khi - w0) % bw + 1
    return out


@pytest.fixture(scope="module")
def lines():
    return synth.make_linelist(CFG)


@pytest.mark.parametrize("waves,slices", [(1, 4), (1, 1), (2, 2)])
def test_zone_counts_equal_a_point_by_point_enumeration(lines, waves, slices):
    tps = [(T, P) for T in CFG.temperatures for P in CFG.pressures]
    got = bench.zone_counts_multi(CFG, lines, tps, waves, slices)
    far4 = 0
    for (T, P), g in zip(tps, got):
        ref = enumerate_zones(CFG, lines, T, P, waves, slices)
        # the tile kernel's zones (the roofline's flops) and the node-sampled pairs agree
        # exactly; which far pairs take the 4-node rule may differ by a pair or two, since the
        # bench takes the |z| < 40 radius at the centre's wavefront (it grows by under a
        # grid step from one wavefront to the next)
        for k in ("one_pole", "two_node", "four_node", "core", "far_exact"):
            assert g[k] == ref[k], (T, P, k, g, ref)
        assert g["far_node"] + g["far_node4"] == ref["far_node"] + ref["far_node4"], (T, P, g, ref)
        assert abs(g["far_node4"] - ref["far_node4"]) <= 2 * bench.FAR_NODES, (T, P, g, ref)
        assert min(ref["one_pole"], ref["two_node"], ref["four_node"], ref["core"], ref["far_node"],
                   ref["far_exact"]) > 0
        far4 += ref["far_node4"]
    assert far4 > 0       # at 3000 K (2 Da) the |z| < 40 radius reaches past the sampling radius


def test_zone_counts_without_the_far_split_cover_every_window_point(lines):
    # no tile shape: every window point is the tile kernel's, each in exactly one zone
    g = bench.zone_counts(CFG, lines, 2000.0, 1.0)
    E = lines["E"]
    nu = (E[lines["upper"].long()] - E[lines["lower"].long()]).numpy()
    klo = np.maximum(np.ceil(((nu - CFG.cutoff) - CFG.nu_a) / CFG.dnu), 0)
    khi = np.minimum(np.floor(((nu + CFG.cutoff) - CFG.nu_a) / CFG.dnu), CFG.n_points - 1)
    total = int(np.clip(khi - klo + 1, 0, None).sum())
    assert g["one_pole"] + g["two_node"] + g["four_node"] + g["core"] == total
    assert g["far_node"] == g["far_node4"] == g["far_exact"] == 0
