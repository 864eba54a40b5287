"""The C-ABI library loads and exports every entry point include/xsec.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "xsec.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xs_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("xs_plan_create", "xs_plan_destroy", "xs_set_states", "xs_set_lines",
              "xs_partition_function", "xs_cross_section", "xs_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1801_09803_amd import lib_path
    if not os.path.exists(lib_path()):
        pytest.fail("libxsec.so is not built (run python -m paper_1801_09803_amd.build)")
    lib = ctypes.CDLL(lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_defaults_without_gpu():
    from paper_1801_09803_amd.binding import XsOpts, load_library
    lib = load_library()
    assert lib.xs_version() == 6
    o = XsOpts()
    assert lib.xs_opts_default(ctypes.byref(o)) == 0
    assert o.cutoff == 25.0 and o.T0 == 296.0 and o.P0 == 1.0 and o.profile == 3


@pytest.mark.parametrize("field,value", [("n_points", 1), ("cutoff", 0.0), ("mass_da", -1.0),
                                         ("profile", 11), ("index_base", 2), ("slices_per_wave", 3),
                                         ("slices_per_wave", 16),
                                         ("n_split", 65), ("n_split", -1), ("tp_block", 257),
                                         ("vv_beta", 2), ("vv_radius", -1.0), ("vv_radius", float("nan")),
                                         ("gh_nodes", -1), ("gh_nodes", 65)])
def test_plan_create_rejects_bad_options_on_host(field, value):
    # option validation happens before any device call
    from paper_1801_09803_amd.binding import XsOpts, load_library
    lib = load_library()
    o = XsOpts()
    lib.xs_opts_default(ctypes.byref(o))
    o.nu_a, o.nu_b, o.n_points, o.mass_da = 0.0, 10.0, 101, 18.0
    setattr(o, field, value)
    h = ctypes.c_void_p()
    st = lib.xs_plan_create(ctypes.byref(o), ctypes.byref(h))
    assert st in (1, 7) and not h.value
    assert lib.xs_last_error()


def test_null_arguments_are_rejected_without_gpu():
    from paper_1801_09803_amd.binding import load_library
    lib = load_library()
    assert lib.xs_plan_destroy(None) == 0
    assert lib.xs_set_states(None, 10, None, None, None, None) == 1
    assert lib.xs_cross_section(None, 1, None, None, None, None) == 1


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, printed by a C program compiled against it."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "xsec.h"\nint main(void) {\n'
                   f'  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct,mirror", [("xs_opts", "XsOpts"), ("xs_timings", "XsKernelTimes")])
def test_struct_layouts_match_the_header(struct, mirror, tmp_path):
    # the binding's ctypes mirrors keep the C sizes and every field offset
    from paper_1801_09803_amd import binding
    cls = getattr(binding, mirror)
    fields = [f for f, _ in cls._fields_]
    size, offs = _c_layout(struct, fields, tmp_path)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs


def test_graph_and_tuning_calls_reject_null_plans_on_host():
    from paper_1801_09803_amd.binding import load_library
    lib = load_library()
    h = ctypes.c_void_p()
    T = (ctypes.c_double * 1)(296.0)
    P = (ctypes.c_double * 1)(1.0)
    assert lib.xs_graph_create(None, 1, T, P, None, ctypes.byref(h)) == 1 and not h.value
    assert lib.xs_graph_launch(None, None) == 1
    assert lib.xs_graph_set_tp(None, T, P, None) == 1
    assert lib.xs_graph_destroy(None) == 0
    assert lib.xs_set_tile_config(None, 4, 2, 0, 0) == 1
    assert lib.xs_autotune(None, 1, T, P, 10.0, None, None) == 1


def test_stream_calls_reject_null_arguments_on_host():
    from paper_1801_09803_amd.binding import load_library
    lib = load_library()
    h = ctypes.c_void_p()
    T = (ctypes.c_double * 1)(296.0)
    P = (ctypes.c_double * 1)(1.0)
    assert lib.xs_stream_begin(None, 1, T, P, None, None, ctypes.byref(h)) == 1 and not h.value
    assert lib.xs_stream_chunk(None, 0, None, None, None, None, None) == 1
    assert lib.xs_stream_end(None, None) == 1
    assert lib.xs_stream_checkpoint(None, b"x") == 1
    assert lib.xs_stream_resume(None, b"x", None, None, ctypes.byref(h)) == 1 and not h.value
    assert lib.xs_stream_stats(None, None) == 1


def test_state_reduction_and_emission_calls_reject_null_plans_on_host():
    from paper_1801_09803_amd.binding import load_library
    lib = load_library()
    T = (ctypes.c_double * 1)(296.0)
    assert lib.xs_set_intensity_kind(None, 1) == 1
    assert lib.xs_partition_moments(None, 1, T, None, None, None, None, None) == 1
    assert lib.xs_lifetimes(None, 0, None, None, None, None) == 1
    assert lib.xs_cooling_function(None, 0, None, None, None, 1, T, None, None) == 1
    assert lib.xs_set_vibrational_labels(None, 1, None, None) == 1
    assert lib.xs_cross_section_nlte(None, 1, T, T, T, None, None) == 1
    assert lib.xs_partition_function_nlte(None, 1, T, T, None, None) == 1


def test_binding_handles_skip_the_library_in_forked_processes():
    # objects inherited by a forked worker (the oracle's process pool) must not call into
    # the HIP runtime from their destructors
    import os
    from paper_1801_09803_amd import binding as B

    class Fake:
        pass
    f = Fake()
    f._pid = os.getpid()
    assert B._owner(f)
    f._pid = os.getpid() + 1
    assert not B._owner(f)
    assert not B._owner(Fake())


@pytest.mark.parametrize("precision,waves", [(0, 0), (1, 4), (1, 8)])
def test_eight_slices_need_fp32_and_narrow_workgroups(precision, waves):
    # 512-point wavefronts exist for the FP32 kernels with 1 or 2 wavefronts per workgroup
    from paper_1801_09803_amd.binding import XsOpts, load_library
    lib = load_library()
    o = XsOpts()
    lib.xs_opts_default(ctypes.byref(o))
    o.nu_a, o.nu_b, o.n_points, o.mass_da = 0.0, 10.0, 101, 18.0
    o.slices_per_wave, o.precision, o.waves_per_block = 8, precision, waves
    h = ctypes.c_void_p()
    assert lib.xs_plan_create(ctypes.byref(o), ctypes.byref(h)) == 1 and not h.value
    assert b"8 slices" in lib.xs_last_error()
