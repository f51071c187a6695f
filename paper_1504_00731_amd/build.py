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


def _run(cmd: list, verbose: bool, what: str):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True), what


def _wait(jobs):
    failed = []
    for proc, what in jobs:
        out, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(out)
            failed.append(what)
    if failed:
        raise RuntimeError("hipcc failed building " + ", ".join(failed))


def _build_one(out: str, sources: list, verbose: bool) -> str:
    """Each source compiled to an object in parallel, then linked."""
    tag = ".tmp%d" % os.getpid()
    objs = [os.path.join(HERE, os.path.splitext(s)[0] + tag + ".o") for s in sources]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs = [_run([hipcc(), "--offload-arch=" + ARCH] + compile_flags +
                 ["-I" + INCLUDE, "-I" + CSRC, "-c", "-o", o, os.path.join(CSRC, src)],
                 verbose, src) for src, o in zip(sources, objs)]
    try:
        _wait(jobs)
        tmp = out + tag
        _wait([_run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs,
                    verbose, os.path.basename(out))])
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


def build(verbose: bool = False) -> str:
    """Builds both libraries; returns the solver library's path."""
    _build_one(PROBE_LIB, PROBE_SOURCES, verbose)
    return _build_one(LIB, SOURCES, verbose)


def build_solver(verbose: bool = False) -> str:
    """Builds the solver library only."""
    return _build_one(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
