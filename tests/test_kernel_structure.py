"""CPU checks of the compiled device code's loop structure (gfx950 assembly of
the library's own sources, cross-compiled here).

Every loop that contains a workgroup barrier must take its back edge on a
wave-uniform (scalar) condition.  The persistent batched kernel once compiled
to a job loop whose latch let only thread 0 leave an inner loop to fetch the
next job while the other lanes went back to the fetch barrier: the block then
re-read a stale job index for ever.  These tests keep that shape out of every
kernel, and test the checker itself on small hand-written listings.
"""
import os
import re
import shutil
import subprocess

import pytest

from tests.isa_loops import divergent_barrier_loops, kernel_symbols

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_00731_amd", "csrc")
BUILD = os.path.join(ROOT, "tests", "_build")


def _hipcc():
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


def _device_asm(src):
    """gfx950 assembly of one library source, rebuilt when any source is newer."""
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc is not available")
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, os.path.basename(src) + ".s")
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(ROOT, "include", "wenotheta.h")]
    if not os.path.exists(out) or os.path.getmtime(out) < max(os.path.getmtime(d) for d in deps):
        # the same code-generation flags as the library build
        from paper_1504_00731_amd import build as B
        flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
        cmd = [hipcc, "--offload-arch=gfx950", *flags, "-I" + os.path.join(ROOT, "include"),
               "-I" + CSRC, "--cuda-device-only", "-S", "-o", out, os.path.join(CSRC, src)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


def _kernels(asm):
    """The functions of the listing (device data such as the fixed scratch array of the
    allocation-free entry point is an @object symbol and has no code)."""
    funcs = set(re.findall(r"^\s*\.type\s+(_Z\w+),@function", asm, re.M))
    return sorted(set(re.findall(r"^(_Z\w+):", asm, re.M)) & funcs)


@pytest.mark.parametrize("src", ["wenotheta.hip", "batched.hip"])
def test_barrier_loops_are_wave_uniform(src):
    asm = _device_asm(src)
    names = _kernels(asm)
    assert names
    bad = {k: divergent_barrier_loops(asm, k) for k in names}
    bad = {k: v for k, v in bad.items() if v}
    assert not bad, bad


def test_batched_job_fetch_is_in_the_job_loop():
    """After the queue atomic, the fetch barrier follows with no loop header in between,
    and the job index is read as a scalar (one value per wave)."""
    asm = _device_asm("batched.hip")
    syms1 = kernel_symbols(asm, "_ZN2wt14batched_kernel")
    syms2 = kernel_symbols(asm, "_ZN2wt16batched2d_kernel")
    assert len(syms1) == 6 and len(syms2) == 6         # 3 precisions x 2 tile variants each
    syms = syms1 + syms2
    lines = asm.split("\n")
    for s in syms:
        a = next(i for i, l in enumerate(lines) if l.startswith(s + ":"))
        e = next(i for i in range(a, len(lines)) if lines[i].startswith(".Lfunc_end"))
        body = lines[a:e]
        k = next(i for i, l in enumerate(body) if "global_atomic_add" in l)
        j = next(i for i in range(k, len(body)) if "s_barrier" in body[i])
        assert not any("Loop Header" in body[i] for i in range(k, j)), s
        after = [l.strip() for l in body[j:j + 12]]
        assert any(l.startswith("v_readfirstlane_b32") for l in after), s
        assert any(l.startswith("s_cbranch_scc") for l in after), s


# --- the checker on small listings ---------------------------------------------

_UNIFORM = """\
_Zuniform:
	s_mov_b32 s4, 0
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
	ds_write_b32 v0, v1
	s_waitcnt lgkmcnt(0)
	s_barrier
	s_add_i32 s4, s4, 1
	s_cmp_lt_i32 s4, s5
	s_cbranch_scc1 .LBB0_1
; %bb.2:
	s_endpgm
.Lfunc_end0:
"""

_DIVERGENT = """\
_Zdivergent:
	s_mov_b64 s[0:1], 0
	s_branch .LBB1_2
.LBB1_1:                                ;   in Loop: Header=BB1_2 Depth=1
	s_or_b64 s[0:1], vcc, s[0:1]
	s_andn2_b64 exec, exec, s[0:1]
	s_cbranch_execz .LBB1_3
.LBB1_2:                                ; =>This Inner Loop Header: Depth=1
	s_barrier
	v_cmp_eq_u32_e32 vcc, 0, v0
	s_branch .LBB1_1
.LBB1_3:
	s_endpgm
.Lfunc_end1:
"""

_DIVERGENT_NO_BARRIER = _DIVERGENT.replace("_Zdivergent", "_Zplain").replace("\ts_barrier\n", "")


def test_checker_accepts_scalar_latch():
    assert divergent_barrier_loops(_UNIFORM, "_Zuniform") == []


def test_checker_flags_exec_latch_around_barrier():
    bad = divergent_barrier_loops(_DIVERGENT, "_Zdivergent")
    assert len(bad) == 1 and bad[0].startswith("BB1_2")


def test_checker_ignores_exec_loops_without_barrier():
    # per-lane loops (e.g. over a thread's cells) may diverge freely
    assert divergent_barrier_loops(_DIVERGENT_NO_BARRIER, "_Zplain") == []
