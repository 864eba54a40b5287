"""The seeded input generators (shared by the oracle and the GPU runs as input data only):
counter-based, so a line is the same whatever the list size, chunking or device."""
import torch

import synth
from synth.linelist import splitmix64_ref, random_bits


def test_splitmix64_tensor_matches_reference():
    ctr = torch.arange(0, 50, dtype=torch.int64)
    got = random_bits(180109803, 2, ctr).tolist()
    key = splitmix64_ref((180109803 + 2 * 0xD1B54A32D192ED03) & ((1 << 64) - 1))
    for c, v in zip(range(50), got):
        ref = splitmix64_ref((c * 0x9E3779B97F4A7C15 + key + 0x9E3779B97F4A7C15) & ((1 << 64) - 1))
        assert (v & ((1 << 64) - 1)) == ref


def test_lines_by_index_equal_lines_by_range():
    cfg = synth.CONFIGS["C1"]
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed)
    up, lo = synth.linelist.make_transitions(E, 300, cfg.nu_max, cfg.seed, first_line=1000)
    A, gr, ne = synth.linelist.make_line_params(300, cfg.seed, first_line=1000)
    idx = torch.tensor([1000, 1001, 1137, 1299], dtype=torch.int64)
    up2, lo2 = synth.linelist.make_transitions_at(E, idx, cfg.nu_max, cfg.seed)
    A2, gr2, ne2 = synth.linelist.make_line_params_at(idx, cfg.seed)
    sel = idx - 1000
    assert torch.equal(up[sel], up2) and torch.equal(lo[sel], lo2)
    assert torch.equal(A[sel], A2) and torch.equal(gr[sel], gr2) and torch.equal(ne[sel], ne2)
    # every pair is admissible: 0 < E_up - E_low <= nu_max
    dE = E[up2.long()] - E[lo2.long()]
    assert bool(((dE > 0) & (dE <= cfg.nu_max)).all())
