"""Build libxsec.so (the HIP/CDNA4 cross-section library) for gfx950, in-tree.

    python -m paper_1801_09803_amd.build        # or: python paper_1801_09803_amd/build.py

Every call compiles from source (no caching): each source file is compiled to an
object in parallel (objects under _build/ at the repository root), then the objects are
linked into the shared library next to this file, which the Python binding loads.
"""
import os
import shlex
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxsec.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build", "xsec")
ARCH = os.environ.get("XSEC_OFFLOAD_ARCH", "gfx950")

SOURCES = ["xs_api.cpp", "xs_quadrature.cpp", "xs_lineprep.hip", "xs_core.hip",
           "xs_forward_f32.hip", "xs_far.hip", "xs_forward_f64.hip", "xs_adjoint.hip", "xs_stream.hip", "xs_vv.hip", "xs_threshold.hip",
           "xs_states.hip", "xs_noalloc.hip", "xs_probe.hip"]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 (v_pk_*_f32) code generation disabled on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-variable", "-Wno-unused-function",
    "-I", os.path.join(os.path.dirname(HERE), "include"),
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _jobs():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 4
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [cc] + FLAGS + ["-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(shlex.quote(c) for c in cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return src, obj, r

    objs = []
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        for src, obj, r in ex.map(compile_one, [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]):
            out = "\n".join(ln for ln in r.stdout.splitlines()
                            if "packed-fp32-ops' is not a recognized feature" not in ln)
            if out.strip():
                print(out, flush=True)
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, f"hipcc {src}")
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(shlex.quote(c) for c in cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
