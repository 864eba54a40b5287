"""xs_partition_function_noalloc (the entry point for callers that cannot allocate)
against xs_partition_function, through the C ABI: two calls in a row, the second with
fewer temperatures, each bitwise equal to the allocating call and within 1e-13 of the
oracle's correctly rounded sum; plus the refusal of too many temperatures."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

P = ctypes.c_void_p


def _lib():
    from paper_1801_09803_amd.binding import load_library
    lib = load_library()
    lib.xs_partition_function_noalloc.restype = ctypes.c_int32
    lib.xs_partition_function_noalloc.argtypes = [P, ctypes.c_int32, P, P, P, P]
    return lib


def _doubles(vals):
    return (ctypes.c_double * len(vals))(*vals)


def test_noalloc_partition_function_matches_the_allocating_call():
    from paper_1801_09803_amd import Plan
    lib = _lib()
    cfg = synth.WorkloadConfig("noalloc", 31, 30000, 10, 18.0, 5000.0, 0.0, 5000.0, 101, (1000.0,), (1.0,))
    E, g, J = synth.linelist.make_states(cfg.n_states, cfg.seed, device="cuda")
    plan = Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu)
    plan.set_states(E, g, J)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    Eh, gh = E.cpu().numpy(), g.cpu().numpy()
    for n in (200, 7):                       # the second call is smaller
        T = list(np.geomspace(80.0, 5000.0, n))
        Q0 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        D0 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        st = lib.xs_partition_function_noalloc(plan._h, n, _doubles(T), Q0.data_ptr(), D0.data_ptr(), s)
        assert st == 0, lib.xs_last_error()
        Q1, D1 = plan.partition_function(T)
        torch.cuda.synchronize()
        assert torch.equal(Q0, Q1) and torch.equal(D0, D1), n
        for i in (0, n // 2, n - 1):
            ref = O.partition_function(Eh, gh, T[i])
            assert abs(Q0[i].item() / ref - 1.0) <= 1e-13, (n, T[i])
        log(f"  noalloc n_T={n}: bitwise equal to xs_partition_function, oracle 1e-13")
    # one temperature, NULL derivative output
    Q0 = torch.empty(1, dtype=torch.float64, device="cuda")
    assert lib.xs_partition_function_noalloc(plan._h, 1, _doubles([296.0]), Q0.data_ptr(), None, s) == 0
    Q1, _ = plan.partition_function([296.0])
    torch.cuda.synchronize()
    assert torch.equal(Q0, Q1)
    plan.close()


def test_noalloc_partition_function_refuses_too_many_temperatures():
    lib = _lib()
    T = _doubles([300.0] * 257)
    assert lib.xs_partition_function_noalloc(None, 257, T, None, None, None) == 1
    assert b"256" in lib.xs_last_error()
    assert lib.xs_partition_function_noalloc(None, 0, T, None, None, None) == 1
