"""Build libxsec.so (the HIP/CDNA4 cross-section library) for gfx950, in-tree.

    python -m paper_1801_09803_amd.build        # or: python paper_1801_09803_amd/build.py

Every call compiles from source (no caching); the shared library lands next to
this file and is what the Python binding loads.
"""
import os
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxsec.so")
ARCH = os.environ.get("XSEC_OFFLOAD_ARCH", "gfx950")

SOURCES = ["xs_api.cpp", "xs_quadrature.cpp", "xs_lineprep.hip", "xs_core.hip",
           "xs_forward_f32.hip", "xs_forward_f64.hip", "xs_adjoint.hip", "xs_stream.hip", "xs_vv.hip", "xs_threshold.hip",
           "xs_states.hip"]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
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


def build(verbose: bool = True) -> str:
    srcs = []
    for s in SOURCES:
        p = os.path.join(CSRC, s)
        if s.endswith(".cpp"):
            srcs += ["-x", "hip", p]
        else:
            srcs += ["-x", "hip", p]
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(shlex.quote(c) for c in cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
