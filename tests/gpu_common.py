"""Shared helpers of the GPU tests: run the library through its C ABI and the
oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W


def grid_params(case: W.Case, alpha_R=None, cfl=None):
    g = wt.Grid(n=case.n, lo=case.lo, hi=case.hi, bc=case.bc)
    p = wt.Params(system=case.system, a=case.a, gamma=case.gamma,
                  cfl=case.cfl if cfl is None else cfl,
                  alpha_R=case.alpha_R if alpha_R is None else alpha_R,
                  gravity=tuple(case.gravity))
    return g, p


def oracle_sides(sides):
    """The oracle's form of a workload's side table (None stays None)."""
    if sides is None:
        return None
    return tuple(oracle.Side(kind=s.kind, state=s.state, split0=s.split0,
                             split_speed=s.split_speed) for s in sides)


def oracle_problem(case: W.Case, alpha_R=None, cfl=None, t=0.0) -> oracle.Problem:
    return oracle.Problem(ndim=case.ndim, system=case.system, n=case.n, dx=case.dx, bc=case.bc,
                          a=case.a, gamma=case.gamma, cfl=case.cfl if cfl is None else cfl,
                          alpha_R=case.alpha_R if alpha_R is None else alpha_R,
                          gravity=tuple(case.gravity), lo=tuple(case.lo),
                          sides=oracle_sides(case.sides), t=t)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_rhs(ctx, case, u=None, f=None, alpha=None, alpha_R=None):
    import torch
    g, p = grid_params(case, alpha_R=alpha_R)
    ud = to_dev(case.u if u is None else u)
    L = torch.empty_like(ud)
    fd = None if f is None else to_dev(f)
    al = None if alpha is None else np.asarray(alpha, dtype=np.float64).ravel()
    wt.wenotheta_rhs(ctx, g, p, ud, L, f=fd, alpha_host=al)
    wt.wenotheta_sync(ctx)
    return L.cpu().numpy()


def gpu_steps(ctx, case, nsteps, dt=0.0, alpha_R=None):
    g, p = grid_params(case, alpha_R=alpha_R)
    ud = to_dev(case.u)
    for _ in range(nsteps):
        wt.wenotheta_step(ctx, g, p, ud, dt=dt)
    wt.wenotheta_sync(ctx)
    return ud.cpu().numpy()


def gpu_solve(ctx, case, t_end, t0=0.0, max_steps=-1, alpha_R=None):
    g, p = grid_params(case, alpha_R=alpha_R)
    ud = to_dev(case.u)
    t, k = wt.wenotheta_solve(ctx, g, p, ud, t_end, t0=t0, max_steps=max_steps)
    return ud.cpu().numpy(), t, k


def max_rel(a, b):
    """max |a - b| per component over max |b| per component (normwise, per component)."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float((np.abs(a - b).max(axis=1) / scale).max())


def assert_parity(gpu, ref, tol, what=""):
    """The tolerance bar of a floating-point result; also reports whether the two are
    bit-identical (the kernels reproduce the oracle's operation order)."""
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    assert np.all(np.isfinite(gpu)), what
    err = max_rel(gpu, ref)
    assert err <= tol, f"{what}: max-relative error {err:.3e} > {tol:.1e}"
    return err, bool(np.array_equal(gpu, ref))
