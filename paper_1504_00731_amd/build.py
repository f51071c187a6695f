"""Build the HIP libraries for gfx950 (in-tree, next to this file): libwenotheta.so, the
solver, and libwt_probe.so, elementwise probes of its device arithmetic for the tests."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libwenotheta.so")
SOURCES = ["wenotheta.hip", "batched.hip"]
PROBE_LIB = os.path.join(HERE, "libwt_probe.so")
PROBE_SOURCES = ["arith_probe.hip"]
ARCH = os.environ.get("WENOTHETA_ARCH", "gfx950")

# No floating-point contraction (the kernels reproduce a fixed sequence of
# IEEE operations); packed FP32 instructions disabled.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _build_one(out: str, sources: list, verbose: bool) -> str:
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH] + FLAGS + ["-I" + INCLUDE, "-I" + CSRC,
                                                         "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building " + os.path.basename(out))
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Builds both libraries; returns the solver library's path."""
    _build_one(PROBE_LIB, PROBE_SOURCES, verbose)
    return _build_one(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
