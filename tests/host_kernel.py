"""Host build of the kernels' per-interface arithmetic (csrc/host_check.cpp),
for CPU-only checks of the device code's operation sequence against the oracle."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_00731_amd", "csrc")
LIB = os.path.join(ROOT, "tests", "_build", "libhostcheck.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".cpp"))]
        srcs.append(os.path.join(ROOT, "include", "wenotheta.h"))
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(map(os.path.getmtime, srcs)):
            os.makedirs(os.path.dirname(LIB), exist_ok=True)
            tmp = LIB + ".tmp%d" % os.getpid()
            subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                            "-Wno-unknown-pragmas", "-fPIC", "-shared",
                            "-I" + os.path.join(ROOT, "include"), "-o", tmp,
                            os.path.join(CSRC, "host_check.cpp")], check=True)
            os.replace(tmp, LIB)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.wth_weno.restype = ctypes.c_double
        L.wth_weno.argtypes = [dp, ctypes.c_double, ctypes.c_double]
        L.wth_weno_fast.restype = ctypes.c_double
        L.wth_weno_fast.argtypes = [dp, ctypes.c_double, ctypes.c_double]
        L.wth_rhs.restype = ctypes.c_int
        L.wth_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), dp,
                              ctypes.POINTER(ctypes.c_int), dp, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def weno(s, eps=1e-10, alpha_R=50.0) -> float:
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib().wth_weno(_dp(s), eps, alpha_R)


def weno_fast(s, eps=1e-10, alpha_R=50.0) -> float:
    """The fast FP64 reconstruction of the device headers (host rounding of its fused
    multiply-adds, which are correctly rounded on both)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib().wth_weno_fast(_dp(s), eps, alpha_R)


def rhs(P, u, alpha, f=None, prec=0):
    """L(u) with the device arithmetic in precision mode prec (0: plain FP64 order,
    1: FP32 reconstruction, 2: fast FP64; the host's own rounding of the fast forms);
    P is an oracle.Problem (grid description only), alpha the [ndim][m] Lax-Friedrichs
    speeds."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = (ctypes.c_int64 * 3)(*([int(v) for v in P.n] + [1] * (3 - len(P.n))))
    dx = (ctypes.c_double * 3)(*([float(v) for v in P.dx] + [1.0] * (3 - len(P.dx))))
    bc = (ctypes.c_int * 3)(*([int(v) for v in P.bc] + [0] * (3 - len(P.bc))))
    al = np.zeros((3, 5))
    a = np.asarray(alpha, dtype=np.float64).reshape(P.ndim, -1)
    al[:P.ndim, :a.shape[1]] = a
    if P.system != 2 and f is None:
        f = P.a * u if P.system == 0 else 0.5 * u * u
    f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    L = np.zeros_like(u)
    grav = np.ascontiguousarray(list(P.gravity) + [0.0] * (3 - len(P.gravity)), dtype=np.float64)
    bad = lib().wth_rhs(int(prec), P.system, P.ndim, n, dx, bc, _dp(al), P.gamma, P.eps, P.alpha_R,
                        _dp(u), _dp(f), _dp(L), _dp(grav))
    return L, bad


def div_finish(q, a, b) -> float:
    f = lib().wth_div_finish
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_double] * 3
    return f(q, a, b)


def sqrt_finish(s, x) -> float:
    f = lib().wth_sqrt_finish
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_double] * 2
    return f(s, x)


def div_by_recip(a, b, y) -> float:
    f = lib().wth_div_by_recip
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_double] * 3
    return f(a, b, y)


def div_by_recip_checked(a, b, y) -> float:
    f = lib().wth_div_by_recip_checked
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_double] * 3
    return f(a, b, y)


def recip_refine(b, y0) -> float:
    f = lib().wth_recip_refine
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_double] * 2
    return f(b, y0)


def map_index(i, n, bc) -> int:
    f = lib().wth_map_index
    f.restype = ctypes.c_int64
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    return f(i, n, bc)


def reflected(i, n, bc) -> bool:
    f = lib().wth_reflected
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    return bool(f(i, n, bc))


def pack_chunks(W, nl, qt, rmax):
    """(q0, nq) of the packed chunks of nl lines of W interfaces (batched 2D passes)."""
    L = lib()
    cap = nl * W + 1
    q0 = (ctypes.c_int32 * cap)()
    nq = (ctypes.c_int32 * cap)()
    f = L.wth_pack_chunks
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_int32)] * 2 + [ctypes.c_int]
    k = f(W, nl, qt, rmax, q0, nq, cap)
    assert k <= cap
    return [(q0[i], nq[i]) for i in range(k)]


def pack_rows(q0, nq, W) -> int:
    f = lib().wth_pack_rows
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] * 3
    return f(q0, nq, W)


def pack_base(q0, q, W) -> int:
    f = lib().wth_pack_base
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] * 3
    return f(q0, q, W)


def pack_point(q0, row, W):
    f = lib().wth_pack_point
    f.restype = None
    f.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_int)] * 2
    line, g = ctypes.c_int(), ctypes.c_int()
    f(q0, row, W, ctypes.byref(line), ctypes.byref(g))
    return line.value, g.value


def pack_limits():
    """(lanes per line, interface rows per chunk, staged rows per chunk) of the packed chunks."""
    lim = (ctypes.c_int * 3)()
    f = lib().wth_pack_limits
    f.restype = None
    f.argtypes = [ctypes.POINTER(ctypes.c_int)]
    f(lim)
    return lim[0], lim[1], lim[2]
