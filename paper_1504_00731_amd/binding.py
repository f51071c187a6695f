"""ctypes binding of libwenotheta.so (the C ABI of include/wenotheta.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Torch is used for device memory and streams.  The
library must have been built (``paper_1504_00731_amd.build``); without it,
every call raises ``LibraryMissing`` -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwenotheta.so")

WT_OK, WT_ERR_ARG, WT_ERR_UNSUPPORTED, WT_ERR_NONPHYSICAL = 0, 1, 2, 3
WT_ERR_NONFINITE, WT_ERR_DEVICE, WT_ERR_NOMEM, WT_ERR_SCRATCH = 4, 5, 6, 7
WT_LINEAR, WT_BURGERS, WT_EULER = 0, 1, 2
WT_PERIODIC, WT_TRANSMISSIVE, WT_REFLECTIVE, WT_SIDES = 0, 1, 2, 3
WT_SIDE_TRANSMISSIVE, WT_SIDE_REFLECTIVE, WT_SIDE_STATE = 1, 2, 3
WT_FP64, WT_FP32_RECON, WT_FP64_FAST = 0, 1, 2

EXPORTED = ("wenotheta_ctx_create", "wenotheta_ctx_destroy", "wenotheta_status_string",
            "wenotheta_rhs", "wenotheta_step", "wenotheta_solve", "wenotheta_sync",
            "wenotheta_profile", "wenotheta_profile_read", "wenotheta_solve_batched",
            "wenotheta_solve_batched_2d", "wenotheta_tune_batched", "wenotheta_tune_batched_2d",
            "wenotheta_set_batched_tiles", "wenotheta_tune", "wenotheta_set_tiles",
            "wenotheta_set_sides", "wenotheta_rhs_noalloc")
PROFILE_KINDS = ("sweep_x", "sweep_y", "sweep_z", "sweep_x_final", "sweep_y_final",
                 "sweep_z_final", "stage_2d")


class LibraryMissing(RuntimeError):
    pass


class WenoThetaError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib().wenotheta_status_string(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} (status {code})")
        self.code = code


class wt_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 3),
                ("reserved1", ctypes.c_int32)]


class wt_side(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32 * 2), ("state", (ctypes.c_double * 5) * 2),
                ("split0", ctypes.c_double), ("split_speed", ctypes.c_double)]


class wt_params(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("a", ctypes.c_double), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("eps", ctypes.c_double), ("alpha_R", ctypes.c_double),
                ("gravity", ctypes.c_double * 3)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built; run `python -m paper_1504_00731_amd.build` "
                "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        G, P = ctypes.POINTER(wt_grid), ctypes.POINTER(wt_params)
        dp = ctypes.POINTER(ctypes.c_double)
        L.wenotheta_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32]
        L.wenotheta_ctx_destroy.argtypes = [vp]
        L.wenotheta_status_string.argtypes = [ctypes.c_int32]
        L.wenotheta_status_string.restype = ctypes.c_char_p
        L.wenotheta_rhs.argtypes = [vp, G, P, vp, vp, dp, vp, vp]
        L.wenotheta_rhs_noalloc.argtypes = [G, P, vp, vp, dp, vp, vp, vp]
        L.wenotheta_step.argtypes = [vp, G, P, vp, ctypes.c_double, vp, vp]
        L.wenotheta_solve.argtypes = [vp, G, P, vp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int64), vp]
        L.wenotheta_sync.argtypes = [vp, vp]
        L.wenotheta_profile.argtypes = [vp, ctypes.c_int32]
        i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
        L.wenotheta_solve_batched.argtypes = [vp, ctypes.c_int64, i64p, i64p, dp, dp, i32p, P, vp,
                                              ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp]
        L.wenotheta_solve_batched_2d.argtypes = [vp, ctypes.c_int64, i64p, i64p, i64p, dp, dp, i32p,
                                                 P, vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp,
                                                 vp]
        L.wenotheta_tune_batched.argtypes = [vp, ctypes.c_int64, i64p, i64p, dp, dp, i32p, P, vp,
                                             ctypes.c_int64, ctypes.c_int64, i32p, vp]
        L.wenotheta_tune_batched_2d.argtypes = [vp, ctypes.c_int64, i64p, i64p, i64p, dp, dp, i32p,
                                                P, vp, ctypes.c_int64, ctypes.c_int64, i32p, vp]
        L.wenotheta_set_batched_tiles.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.wenotheta_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
        i32p3 = ctypes.POINTER(ctypes.c_int32)
        L.wenotheta_tune.argtypes = [vp, G, P, vp, i32p3, vp]
        L.wenotheta_set_tiles.argtypes = [vp, G, P, i32p3]
        L.wenotheta_set_sides.argtypes = [vp, ctypes.POINTER(wt_side), ctypes.c_double, vp]
        for name in EXPORTED:
            if name != "wenotheta_status_string":
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(code: int, what: str):
    if code != WT_OK:
        raise WenoThetaError(code, what)


@dataclass
class Grid:
    """Uniform grid: n points per dimension (x first), [lo, hi] per dimension, bc per dimension."""
    n: tuple
    lo: tuple
    hi: tuple
    bc: tuple

    @property
    def ndim(self) -> int:
        return len(self.n)

    def c_struct(self) -> wt_grid:
        g = wt_grid()
        g.ndim = self.ndim
        for k in range(3):
            inside = k < self.ndim
            g.n[k] = int(self.n[k]) if inside else 1
            g.lo[k] = float(self.lo[k]) if inside else 0.0
            g.hi[k] = float(self.hi[k]) if inside else 1.0
            g.bc[k] = int(self.bc[k]) if inside else 0
        return g


@dataclass
class Side:
    """One end of a WT_SIDES dimension (``wt_side``): rule kind[0] (WT_SIDE_TRANSMISSIVE,
    WT_SIDE_REFLECTIVE or WT_SIDE_STATE) on the grid lines whose coordinate along the
    next axis is below split0 + split_speed * t, kind[1] on the others; a WT_SIDE_STATE
    part puts state[part] (conserved, ndim + 2 entries) into the ghost points."""
    kind: tuple = (WT_SIDE_TRANSMISSIVE, WT_SIDE_TRANSMISSIVE)
    state: tuple = ((), ())
    split0: float = math.inf
    split_speed: float = 0.0


@dataclass
class Params:
    system: int = WT_EULER
    a: float = 1.0
    gamma: float = 1.4
    cfl: float = 0.5
    eps: float = 1e-10
    alpha_R: float = 50.0
    precision: int = WT_FP64
    gravity: tuple = (0.0, 0.0, 0.0)

    def c_struct(self) -> wt_params:
        p = wt_params()
        p.system, p.precision = int(self.system), int(self.precision)
        p.a, p.gamma, p.cfl = float(self.a), float(self.gamma), float(self.cfl)
        p.eps, p.alpha_R = float(self.eps), float(self.alpha_R)
        g = list(self.gravity) + [0.0] * (3 - len(self.gravity))
        for k in range(3):
            p.gravity[k] = float(g[k])
        return p


class Context:
    """Owns a wt_ctx (workspace on one device)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(_lib().wenotheta_ctx_create(ctypes.byref(h), int(device)), "wenotheta_ctx_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _lib().wenotheta_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, name, shape=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _dev_int_ptr(t, name, n, bits):
    import torch
    if t is None:
        return None
    want = torch.int32 if bits == 32 else torch.int64
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA (HIP) int{bits} tensor")
    if tuple(t.shape) != (n,):
        raise ValueError(f"{name} must have shape ({n},)")
    return ctypes.c_void_p(t.data_ptr())


def state_shape(grid: Grid, params: Params) -> tuple:
    m = grid.ndim + 2 if params.system == WT_EULER else 1
    return (m,) + tuple(reversed(tuple(int(v) for v in grid.n)))


# --- the C entry points, same names ------------------------------------------------

def wenotheta_rhs(ctx: Context, grid: Grid, params: Params, u, L_out, f=None, alpha_host=None,
                  stream=None):
    shp = state_shape(grid, params)
    al = None
    if alpha_host is not None:
        vals = [float(v) for v in alpha_host]
        al = (ctypes.c_double * len(vals))(*vals)
    _check(_lib().wenotheta_rhs(ctx.handle, ctypes.byref(grid.c_struct()),
                                ctypes.byref(params.c_struct()), _dev_ptr(u, "u", shp),
                                _dev_ptr(f, "f", shp), al, _dev_ptr(L_out, "L_out", shp),
                                _stream_ptr(stream)), "wenotheta_rhs")
    return L_out


def wenotheta_rhs_noalloc(grid: Grid, params: Params, u, L_out, f=None, alpha_host=None,
                          status=None, stream=None):
    """L(u) as wenotheta_rhs computes it, with no context and no allocation: the
    library's fixed per-GPU scratch buffer holds the intermediates (calls on one GPU
    must not overlap).  status: optional int32 device tensor of shape (1,) that
    receives the device-detected status."""
    shp = state_shape(grid, params)
    al = None
    if alpha_host is not None:
        vals = [float(v) for v in alpha_host]
        al = (ctypes.c_double * len(vals))(*vals)
    _check(_lib().wenotheta_rhs_noalloc(ctypes.byref(grid.c_struct()),
                                        ctypes.byref(params.c_struct()), _dev_ptr(u, "u", shp),
                                        _dev_ptr(f, "f", shp), al, _dev_ptr(L_out, "L_out", shp),
                                        _dev_int_ptr(status, "status", 1, 32),
                                        _stream_ptr(stream)), "wenotheta_rhs_noalloc")
    return L_out


def wenotheta_step(ctx: Context, grid: Grid, params: Params, u, dt=0.0, dt_used=None,
                   stream=None):
    shp = state_shape(grid, params)
    _check(_lib().wenotheta_step(ctx.handle, ctypes.byref(grid.c_struct()),
                                 ctypes.byref(params.c_struct()), _dev_ptr(u, "u", shp),
                                 float(dt), _dev_ptr(dt_used, "dt_used", (1,)),
                                 _stream_ptr(stream)), "wenotheta_step")
    return u


def wenotheta_solve(ctx: Context, grid: Grid, params: Params, u, t_end, t0=0.0, max_steps=-1,
                    stream=None):
    shp = state_shape(grid, params)
    t = ctypes.c_double(0.0)
    k = ctypes.c_int64(0)
    _check(_lib().wenotheta_solve(ctx.handle, ctypes.byref(grid.c_struct()),
                                  ctypes.byref(params.c_struct()), _dev_ptr(u, "u", shp),
                                  float(t0), float(t_end), int(max_steps), ctypes.byref(t),
                                  ctypes.byref(k), _stream_ptr(stream)), "wenotheta_solve")
    return t.value, k.value


TILE_SHAPES = ((8, 31), (16, 15), (4, 63), (32, 7))   # (TX, TN) of the y/z-sweep tile variants
X_TILE_SHAPES = ((1, 255), (8, 31), (15, 31))        # (rows, TN) of the x-sweep tile variants;
                                                      # 2: the fused 2D stage (31 x 15 tiles)


def wenotheta_tune(ctx: Context, grid: Grid, params: Params, u, stream=None) -> tuple:
    """Times the y/z-sweep tile shapes on u and keeps the fastest for this grid in the
    context; returns the chosen variant per direction.  Synchronises the stream."""
    out = (ctypes.c_int32 * 3)(0, 0, 0)
    _check(_lib().wenotheta_tune(ctx.handle, ctypes.byref(grid.c_struct()),
                                 ctypes.byref(params.c_struct()),
                                 _dev_ptr(u, "u", state_shape(grid, params)), out,
                                 _stream_ptr(stream)), "wenotheta_tune")
    return tuple(out[:grid.ndim])


def wenotheta_set_tiles(ctx: Context, grid: Grid, params: Params, tiles) -> None:
    """Sets the tile variant per direction (0..3) for this grid."""
    t = list(tiles) + [0] * (3 - len(tiles))
    arr = (ctypes.c_int32 * 3)(*[int(v) for v in t[:3]])
    _check(_lib().wenotheta_set_tiles(ctx.handle, ctypes.byref(grid.c_struct()),
                                      ctypes.byref(params.c_struct()), arr), "wenotheta_set_tiles")


def wenotheta_set_sides(ctx: Context, sides, t: float = 0.0, stream=None) -> None:
    """Sets the context's side table (6 Side entries [dim][lower, upper], or None to
    remove it) for grids with WT_SIDES dimensions, and the context's time t."""
    ptr = None
    if sides is not None:
        if len(sides) != 6:
            raise ValueError("sides: 6 entries [dim][lower, upper]")
        arr = (wt_side * 6)()
        for i, sd in enumerate(sides):
            for k in range(2):
                arr[i].kind[k] = int(sd.kind[k])
                for c, v in enumerate(sd.state[k]):
                    arr[i].state[k][c] = float(v)
            arr[i].split0 = float(sd.split0)
            arr[i].split_speed = float(sd.split_speed)
        ptr = ctypes.cast(arr, ctypes.POINTER(wt_side))
    _check(_lib().wenotheta_set_sides(ctx.handle, ptr, float(t), _stream_ptr(stream)),
           "wenotheta_set_sides")


def wenotheta_sync(ctx: Context, stream=None):
    _check(_lib().wenotheta_sync(ctx.handle, _stream_ptr(stream)), "wenotheta_sync")


def wenotheta_profile(ctx: Context, enable: bool):
    _check(_lib().wenotheta_profile(ctx.handle, 1 if enable else 0), "wenotheta_profile")


def wenotheta_profile_read(ctx: Context) -> dict:
    """{kind: (total_ms, launches)} since profiling was enabled."""
    nk = len(PROFILE_KINDS)
    ms = (ctypes.c_double * nk)()
    cnt = (ctypes.c_int64 * nk)()
    _check(_lib().wenotheta_profile_read(ctx.handle, ms, cnt, nk), "wenotheta_profile_read")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PROFILE_KINDS)}


def wenotheta_solve_batched(ctx: Context, params: Params, u, n, offset, lo, hi, bc, nsteps,
                            t_out=None, status_out=None, steps_out=None, stream=None):
    """Advance packed independent 1D Euler problems (u: [3, total] device tensor)."""
    import numpy as np
    n = np.ascontiguousarray(n, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    bc = np.ascontiguousarray(bc, dtype=np.int32)
    nprob = int(n.size)
    if not (offset.size == lo.size == hi.size == bc.size == nprob):
        raise ValueError("problem tables must have one entry per problem")
    if u.dim() != 2 or u.shape[0] != 3:
        raise ValueError("u must have shape (3, total)")
    total = int(u.shape[1])
    i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(_lib().wenotheta_solve_batched(
        ctx.handle, nprob, n.ctypes.data_as(i64p), offset.ctypes.data_as(i64p),
        lo.ctypes.data_as(dp), hi.ctypes.data_as(dp), bc.ctypes.data_as(i32p),
        ctypes.byref(params.c_struct()), _dev_ptr(u, "u"), total, int(nsteps),
        _dev_ptr(t_out, "t_out", (nprob,)), _dev_int_ptr(status_out, "status_out", nprob, 32),
        _dev_int_ptr(steps_out, "steps_out", nprob, 64), _stream_ptr(stream)),
        "wenotheta_solve_batched")
    return u


def wenotheta_solve_batched_2d(ctx: Context, params: Params, u, nx, ny, offset, lo, hi, bc, nsteps,
                               t_out=None, status_out=None, steps_out=None, stream=None):
    """Advance packed independent 2D Euler problems (u: [4, total] device tensor; problem b
    in columns offset[b] .. offset[b] + nx[b] ny[b] - 1, x fastest; lo, hi, bc: [nprob, 2])."""
    import numpy as np
    nx = np.ascontiguousarray(nx, dtype=np.int64)
    ny = np.ascontiguousarray(ny, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    bc = np.ascontiguousarray(bc, dtype=np.int32)
    nprob = int(nx.size)
    if not (ny.size == offset.size == nprob and lo.shape == hi.shape == bc.shape == (nprob, 2)):
        raise ValueError("problem tables must have one entry (two for lo, hi, bc) per problem")
    if u.dim() != 2 or u.shape[0] != 4:
        raise ValueError("u must have shape (4, total)")
    total = int(u.shape[1])
    i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(_lib().wenotheta_solve_batched_2d(
        ctx.handle, nprob, nx.ctypes.data_as(i64p), ny.ctypes.data_as(i64p),
        offset.ctypes.data_as(i64p), lo.ctypes.data_as(dp), hi.ctypes.data_as(dp),
        bc.ctypes.data_as(i32p), ctypes.byref(params.c_struct()), _dev_ptr(u, "u"), total,
        int(nsteps), _dev_ptr(t_out, "t_out", (nprob,)),
        _dev_int_ptr(status_out, "status_out", nprob, 32),
        _dev_int_ptr(steps_out, "steps_out", nprob, 64), _stream_ptr(stream)),
        "wenotheta_solve_batched_2d")
    return u


def _batch_tables_1d(n, offset, lo, hi, bc):
    import numpy as np
    t = (np.ascontiguousarray(n, dtype=np.int64), np.ascontiguousarray(offset, dtype=np.int64),
         np.ascontiguousarray(lo, dtype=np.float64), np.ascontiguousarray(hi, dtype=np.float64),
         np.ascontiguousarray(bc, dtype=np.int32))
    if not all(a.size == t[0].size for a in t):
        raise ValueError("problem tables must have one entry per problem")
    return t


def wenotheta_tune_batched(ctx: Context, params: Params, u, n, offset, lo, hi, bc, probe_steps=2,
                           stream=None) -> int:
    """Times the tile variants of the 1D batched kernel on a scratch copy of u and keeps
    the fastest in the context for batches of these sizes; returns it."""
    n, offset, lo, hi, bc = _batch_tables_1d(n, offset, lo, hi, bc)
    if u.dim() != 2 or u.shape[0] != 3:
        raise ValueError("u must have shape (3, total)")
    i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    v = ctypes.c_int32(-1)
    _check(_lib().wenotheta_tune_batched(
        ctx.handle, int(n.size), n.ctypes.data_as(i64p), offset.ctypes.data_as(i64p),
        lo.ctypes.data_as(dp), hi.ctypes.data_as(dp), bc.ctypes.data_as(i32p),
        ctypes.byref(params.c_struct()), _dev_ptr(u, "u"), int(u.shape[1]), int(probe_steps),
        ctypes.byref(v), _stream_ptr(stream)), "wenotheta_tune_batched")
    return v.value


def wenotheta_tune_batched_2d(ctx: Context, params: Params, u, nx, ny, offset, lo, hi, bc,
                              probe_steps=2, stream=None) -> int:
    """Times the tile variants of the 2D batched kernel on a scratch copy of u and keeps
    the fastest in the context for batches of these sizes; returns it."""
    import numpy as np
    nx = np.ascontiguousarray(nx, dtype=np.int64)
    ny = np.ascontiguousarray(ny, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    bc = np.ascontiguousarray(bc, dtype=np.int32)
    nprob = int(nx.size)
    if not (ny.size == offset.size == nprob and lo.shape == hi.shape == bc.shape == (nprob, 2)):
        raise ValueError("problem tables must have one entry (two for lo, hi, bc) per problem")
    if u.dim() != 2 or u.shape[0] != 4:
        raise ValueError("u must have shape (4, total)")
    i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    v = ctypes.c_int32(-1)
    _check(_lib().wenotheta_tune_batched_2d(
        ctx.handle, nprob, nx.ctypes.data_as(i64p), ny.ctypes.data_as(i64p),
        offset.ctypes.data_as(i64p), lo.ctypes.data_as(dp), hi.ctypes.data_as(dp),
        bc.ctypes.data_as(i32p), ctypes.byref(params.c_struct()), _dev_ptr(u, "u"),
        int(u.shape[1]), int(probe_steps), ctypes.byref(v), _stream_ptr(stream)),
        "wenotheta_tune_batched_2d")
    return v.value


def wenotheta_set_batched_tiles(ctx: Context, ndim: int, variant: int):
    """Forces the tile variant of every later batch of ndim (1 or 2) dimensions."""
    _check(_lib().wenotheta_set_batched_tiles(ctx.handle, int(ndim), int(variant)),
           "wenotheta_set_batched_tiles")


def loaded_library_path() -> str:
    _lib()
    return LIB_PATH


INF = math.inf
