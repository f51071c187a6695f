"""Benchmark of the WENO-theta hot path on one MI355X.

A "step" is one full 3-stage TVD Runge-Kutta step (three RHS evaluations and
three stage updates, all directions) over the whole grid.  The default
workload is the 2D Euler one: 4096 x 4096 points, seeded four-quadrant Riemann
data, transmissive boundaries, CFL 0.5, 200 steps, FP64.

Prints ONE JSON line (rank 0):
  value  = grid points x timed steps / wall time of the timed region (inputs
           resident in HBM before the timed region starts), in cell-updates/s;
  roofline = the dominant kernel against the FP64 vector ALU peak (the path is
           ALU-bound), from HIP events recorded around every kernel launch of
           the timed region on the launch stream;
  hbm    = algorithmic state traffic per step against the HBM peak;
  cpu_baseline = the oracle (plain C, OpenMP over pencils) on the host cores,
           timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP64_VALU_OPS_PEAK = 256 * 64 * 2.4e9      # FP64 lane operations per second (FMA = 1 op)

WENO_OPS = 132          # FP64 operations of one WENO-theta reconstruction (9 divisions)


def euler_interface_ops(ndim: int) -> int:
    """Algorithmic FP64 operations of one characteristic-wise interface flux."""
    m, nt = ndim + 2, ndim - 1
    roe = 6 * ndim + 14                 # averages, q^2, c^2, sqrt, b1, b2, u/c, 1/c
    left = 13 + 5 * nt                  # non-trivial entries of L
    right = 5                           # u -+ c, u c, H -+ u c
    fluxes = 6 * (4 + nt)               # normal flux at the 6 stencil points
    proj = 6 * (6 * (2 * m - 1) + 4 * nt)   # q = L u, w = L f (sparse rows)
    split = 6 * m * 5                   # (w +- alpha q) / 2
    recon = 2 * m * WENO_OPS
    back = m + 12 + 8 * nt              # h+ + h-, F = R h
    return roe + left + right + fluxes + proj + split + recon + back


def euler_cell_ops(ndim: int, final: bool) -> int:
    """Per-cell operations of a sweep: primitives, flux difference, and for the
    final sweep of a stage the divergence sum, stage update and new speeds."""
    m = ndim + 2
    ops = (3 * ndim + 7) + 2 * m
    if final:
        ops += (m if ndim > 1 else 0) + 4 * m + (3 * ndim + 10) + 3 * ndim
    return ops


def sweep_ops(ndim: int, n: tuple, d: int, final: bool) -> float:
    cells = 1
    for k in range(ndim):
        cells *= n[k]
    interfaces = cells // n[d] * (n[d] + 1)
    return interfaces * euler_interface_ops(ndim) + cells * euler_cell_ops(ndim, final)


def build_case(workload: str, n: int | None):
    from paper_1504_00731_amd import workloads as W
    if workload == "euler2d":
        return W.euler2d_seeded(0, n or 4096), "2D Euler, seeded four-quadrant Riemann data"
    if workload == "euler1d":
        return W.euler1d_seeded(0, n or 65536), "1D Euler, seeded Riemann data with density wave"
    if workload == "euler3d":
        return W.euler3d_seeded(0, n or 512), "3D Euler, seeded vortex with density spheres"
    raise SystemExit(f"unknown workload {workload}")


def cpu_baseline(case, workload):
    """The oracle on the host: one full RK3 step of the workload (bounded sample)."""
    import oracle
    P = oracle.Problem(ndim=case.ndim, system=case.system, n=case.n, dx=case.dx, bc=case.bc,
                       gamma=case.gamma, cfl=case.cfl, alpha_R=case.alpha_R)
    oracle.lib()
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    cells = 1
    for v in case.n:
        cells *= v
    t0 = time.perf_counter()
    oracle.step(P, case.u)
    wall = time.perf_counter() - t0
    return {"value": cells / wall, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"1 RK3 step of the full {workload} grid {'x'.join(map(str, case.n))} "
                      f"({wall:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="euler2d", choices=["euler2d", "euler1d", "euler3d"])
    ap.add_argument("--n", type=int, default=None, help="points per dimension (default: full size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1504_00731_amd as wt

    case, desc = build_case(args.workload, args.n)
    cells = int(np.prod(case.n))
    print(f"[bench] workload {args.workload} {case.n} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    ctx = wt.Context(0)
    g = wt.Grid(n=case.n, lo=case.lo, hi=case.hi, bc=case.bc)
    p = wt.Params(system=case.system, gamma=case.gamma, cfl=case.cfl, alpha_R=case.alpha_R)
    u_init = torch.from_numpy(case.u).cuda()

    if args.warmup > 0:
        u = u_init.clone()
        wt.wenotheta_solve(ctx, g, p, u, float("inf"), max_steps=args.warmup)
        del u
    u = u_init.clone()
    torch.cuda.synchronize()
    wt.wenotheta_profile(ctx, True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    t_sim, k = wt.wenotheta_solve(ctx, g, p, u, float("inf"), max_steps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    prof = wt.wenotheta_profile_read(ctx)
    wt.wenotheta_profile(ctx, False)
    assert k == args.steps, (k, args.steps)
    assert bool(torch.isfinite(u).all()), "non-finite state after the timed steps"

    sec = ms / 1e3
    value = cells * args.steps / sec

    # dominant kernel: largest total time
    names = {"sweep_x": (0, False), "sweep_y": (1, False), "sweep_z": (2, False),
             "sweep_x_final": (0, True), "sweep_y_final": (1, True), "sweep_z_final": (2, True)}
    kind = max(prof, key=lambda kk: prof[kk][0])
    tot_ms, launches = prof[kind]
    d, final = names[kind]
    avg_s = tot_ms / launches / 1e3
    ops = sweep_ops(case.ndim, case.n, d, final)
    achieved = ops / avg_s
    bytes_per_step = 8 * (case.ndim + 2) * 8 * cells      # 8 state passes of m FP64 components

    line = {
        "metric": "cell-updates/s (RHS+RK3)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{desc}, {'x'.join(map(str, case.n))} points, "
                               f"{args.steps} RK3 steps, CFL {case.cfl}, FP64",
                   "grid": list(case.n), "steps": args.steps, "cfl": case.cfl,
                   "alpha_R": case.alpha_R, "precision": "fp64"},
        "roofline": {"bound": "alu", "kernel": kind, "achieved": achieved / 1e12,
                     "peak": FP64_VALU_OPS_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_OPS_PEAK, "traffic": None,
                     "avg_launch_ms": tot_ms / launches, "launches": launches,
                     "algorithmic_ops_per_launch": ops},
        "hbm": {"achieved": bytes_per_step * args.steps / sec / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": bytes_per_step * args.steps / sec / 1e9 / HBM_PEAK_GBS,
                "bytes_per_cell_update": bytes_per_step // cells},
        "kernel_ms": {kk: {"total": v[0], "launches": v[1]} for kk, v in prof.items() if v[1]},
        "wall_s": wall,
        "sim_time": t_sim,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(case, args.workload)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
