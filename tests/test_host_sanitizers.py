"""Host-side argument validation of the library under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU (no GPU needed).

The library's sources are compiled with the sanitizers on their host code only (the device
code is compiled as usual and never runs here), linked into a separate shared library, and
driven by tests/host/validate_host.c through the C ABI: every bad option, NULL handle and
out-of-range size must return its documented status, a valid plan without a device must
fail cleanly with XS_ERR_HIP (or XS_ERR_OOM), and the sanitizers must report nothing."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests.conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1801_09803_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")


def _tools():
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    llvm = "/opt/rocm/llvm/bin"
    clang, clangxx = os.path.join(llvm, "clang"), os.path.join(llvm, "clang++")
    if not all(os.path.exists(t) for t in (hipcc, clang, clangxx)):
        pytest.skip("ROCm compilers not found")
    return hipcc, clang, clangxx


def test_host_validation_under_asan_and_ubsan(tmp_path):
    from paper_1801_09803_amd.build import SOURCES
    hipcc, clang, clangxx = _tools()
    # sanitizers on the host pass only (each -fsanitize= right after -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I", INCLUDE]
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([hipcc] + flags + san + ["-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, (src, r.stdout[-2000:], r.stderr[-2000:])
        return obj

    jobs = max(1, min(len(srcs), len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libxsec_san.so")
    subprocess.run([clangxx, "-shared", "-fsanitize=address,undefined"] + objs +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", lib], check=True)
    drv = str(tmp_path / "validate_host")
    subprocess.run([clang, "-fsanitize=address,undefined", "-g", "-I", INCLUDE,
                    os.path.join(ROOT, "tests", "host", "validate_host.c"), lib,
                    f"-Wl,-rpath,{tmp_path}", "-lm", "-o", drv], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "OK: 0 failure(s)" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
