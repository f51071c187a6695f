"""Benchmark of the WENO-theta hot path on one MI355X.

A "step" is one full 3-stage TVD Runge-Kutta step (three RHS evaluations and
three stage updates, all directions) over the whole grid.  The default
workload is the 2D Euler one: 4096 x 4096 points, seeded four-quadrant Riemann
data, transmissive boundaries, CFL 0.5, 200 steps, in the fast FP64 mode
(fused multiply-adds, refined hardware reciprocals).  Beside it the same line
reports ("companions"): that workload in the plain FP64 order (bit-identical
to the oracle) and with FP32 weights, each with its difference to the plain
run; the batched workloads (4096 independent 1D Euler problems, N log-uniform
in [256, 16384], 500 steps; 4096 independent 2D problems, 32..96 points per
side, 100 steps), each solved as one captured graph in the form the batch
tuner picks, in plain FP64, fast FP64 and FP32 weights, with L1 (and for
FP32 Linf and conservation drift) against the plain FP64 result; the 1D Euler workload (65536 points to
t = 0.2) and the 3D one (512^3, 100 steps) in all three modes, each with its
own roofline entry and the oracle's CPU baseline.

Prints ONE JSON line (rank 0):
  value  = grid points x timed steps / wall time of the timed region (inputs
           resident in HBM before the timed region starts), in cell-updates/s;
  roofline = the dominant kernel against the FP64 vector ALU peak (the path is
           ALU-bound), from HIP events recorded around every kernel launch of
           the timed region on the launch stream;
  hbm    = algorithmic state traffic per step against the HBM peak;
  graph  = the same steps replayed from the solver's captured graph without the
           per-sweep events of the timed region (the production path; on short
           grids noticeably faster), checked to give the same state bit for bit;
  cpu_baseline = the oracle (plain C, OpenMP over pencils) on the host cores,
           timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_FLOPS_PEAK = 78.6e12           # FP64 vector FLOP/s (an FMA counts as 2 FLOPs)
# The same peak as an issue rate: 256 CUs x 64 FP64 lanes x 2.4 GHz = 39.3e12 lane
# instructions/s.  The method's formulas, evaluated as printed, have no fused
# multiply-adds, so every counted operation needs an instruction of its own: at most
# half the FLOP/s peak is reachable in that order of operations.
FP64_LANE_ISSUE_PEAK = 256 * 64 * 2.4e9

WENO_OPS = 132          # FP64 operations of one WENO-theta reconstruction (9 divisions)
W_EULER = 2             # wt_system of the Euler equations


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


# Scalar law (1D): the split f +- alpha u at the six stencil points (product, sum or
# difference, halving, per sign), both reconstructions and their sum; per cell the flux
# value, the difference quotient and, in the final sweep, the stage update and speed.
SCALAR_INTERFACE_OPS = 6 * 2 * 3 + 2 * WENO_OPS + 1


def scalar_cell_ops(final: bool) -> int:
    return 1 + 2 + (5 if final else 0)


def sweep_ops(ndim: int, n: tuple, d: int, final: bool, euler: bool = True) -> float:
    cells = 1
    for k in range(ndim):
        cells *= n[k]
    interfaces = cells // n[d] * (n[d] + 1)
    if not euler:
        return interfaces * SCALAR_INTERFACE_OPS + cells * scalar_cell_ops(final)
    return interfaces * euler_interface_ops(ndim) + cells * euler_cell_ops(ndim, final)


# Sources the grid sweep kernels are compiled from: the translation unit and the device
# headers (not the batched kernels, the arithmetic probes or the host-side context).
SWEEP_SOURCES = ("wenotheta.hip", "wt_bc.hpp", "wt_common.hpp", "wt_device.hpp", "wt_flux.hpp",
                 "wt_physics.hpp", "wt_round.hpp", "wt_weno.hpp")


def kernel_sources_hash() -> str:
    """SHA-256 over the sources of the grid sweep kernels, in name order."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1504_00731_amd", "csrc")
    for f in sorted(SWEEP_SOURCES):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, y_tile: str, precision: str = "fp64_fast"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary of the
    2D Euler 4096^2 sweeps in that precision mode, or None when there is none, the kernel
    sources have changed since the counters were taken, or the y sweep runs another tile
    shape."""
    path = os.path.join(ROOT, "profiles", f"traffic_euler2d_4096_{precision}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != kernel_sources_hash() or kernel + ".bytes" not in kv:
        return None
    if kernel.startswith("sweep_y") and kv.get("y_tile") != y_tile:
        return None
    return float(kv[kernel + ".bytes"])


def roofline_entry(kind, ops, tot_ms, launches, traffic=None, fp32_recon=False):
    """The dominant kernel against the published FP64 vector peak: algorithmic FLOPs per
    launch (every add, multiply, division and square root of the method's formulas
    counted as one FLOP) over the kernel's average launch duration from HIP events on
    its launch stream.  The same rate is also given against the lane issue rate."""
    avg_s = tot_ms / launches / 1e3
    achieved = ops / avg_s
    e = {"bound": "alu", "kernel": kind, "achieved": achieved / 1e12,
         "peak": FP64_VECTOR_FLOPS_PEAK / 1e12, "unit": "TFLOP/s",
         "frac": achieved / FP64_VECTOR_FLOPS_PEAK, "traffic": traffic,
         "avg_launch_ms": tot_ms / launches, "launches": launches,
         "algorithmic_flops_per_launch": ops,
         "frac_of_lane_issue_rate": achieved / FP64_LANE_ISSUE_PEAK,
         "lane_issue_rate_note": "39.3e12 FP64 lane instructions/s (256 CUs x 64 lanes x "
                                 "2.4 GHz): the reachable peak for formulas evaluated without "
                                 "fused multiply-adds, half the FLOP/s peak"}
    if fp32_recon:
        e["flops_counted_as"] = ("the FP64 formulas' operations, the reconstructions (run in "
                                 "FP32) counted alike; without packed FP32 instructions (left "
                                 "off in this build) FP32 issues at the FP64 lane rate, so the "
                                 "same peak applies")
    return e


def build_case(workload: str, n: int | None):
    from paper_1504_00731_amd import workloads as W
    if workload == "euler2d":
        # seed 0 draws a quadrant pressure of 0.034 that the unlimited scheme drives to a
        # non-physical state within 200 steps (the oracle fails alike); seed 1 is the
        # first seed whose data stays physical
        return W.euler2d_seeded(1, n or 4096), "2D Euler, seeded four-quadrant Riemann data (seed 1)"
    if workload == "euler1d":
        return W.euler1d_seeded(0, n or 65536), "1D Euler, seeded Riemann data with density wave"
    if workload == "euler3d":
        return W.euler3d_seeded(0, n or 512), "3D Euler, seeded vortex with density spheres"
    if workload == "scalar":
        return (W.scalar_modes(0, n or 200),
                "1D linear advection (a = 1), seeded three-mode periodic data, vertex grid")
    if workload == "double_mach":
        ny = n or 200
        return (W.double_mach(4 * ny, ny),
                "2D Euler, double Mach reflection of a Mach 10 shock (Sec. 4.3 TEST 9)")
    raise SystemExit(f"unknown workload {workload}")


def cpu_baseline(case, workload, sample_n=None):
    """The oracle on the host, timed on a bounded sample of the workload: whole RK3 steps
    of its full grid, or with sample_n, of the same workload generated at sample_n points
    per dimension (the oracle's per-cell work does not depend on the grid size)."""
    import oracle
    if sample_n is not None:
        case = build_case(workload, sample_n)[0]
    sides = None
    if case.sides is not None:
        sides = tuple(oracle.Side(kind=sd.kind, state=sd.state, split0=sd.split0,
                                  split_speed=sd.split_speed) for sd in case.sides)
    P = oracle.Problem(ndim=case.ndim, system=case.system, n=case.n, dx=case.dx, bc=case.bc,
                       gamma=case.gamma, cfl=case.cfl, alpha_R=case.alpha_R, lo=tuple(case.lo),
                       sides=sides)
    oracle.lib()
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    cells = 1
    for v in case.n:
        cells *= v
    # whole RK3 steps of the full grid from the initial state until about 10 s have
    # passed (at least one step), at most 400
    u = case.u
    k = 0
    t0 = time.perf_counter()
    while True:
        u, _ = oracle.step(P, u)
        k += 1
        wall = time.perf_counter() - t0
        if wall >= 10.0 or k >= 400:
            break
    grid = "x".join(map(str, case.n))
    what = (f"the full {workload} grid {grid}" if sample_n is None else
            f"the {workload} workload generated on a {grid} grid")
    return {"value": cells * k / wall, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} RK3 step{'s' if k > 1 else ''} of {what} ({wall:.2f} s)"}


def l1_rel(a, b):
    """Sum |a - b| / sum |b| per component (leading axis)."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return [float(x) for x in ((a - b).abs().sum(dim=1) / b.abs().sum(dim=1)).cpu()]


def differences(a, b):
    """Per component (leading axis) of a against the reference b: L1 and Linf of the
    difference relative to those of b, and the drift of the component's total (the
    conservation sum) relative to the L1 of b."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    d = a - b
    l1 = d.abs().sum(dim=1) / b.abs().sum(dim=1)
    linf = d.abs().amax(dim=1) / b.abs().amax(dim=1)
    drift = (a.sum(dim=1) - b.sum(dim=1)).abs() / b.abs().sum(dim=1)
    return {"l1_rel_vs_fp64": [float(x) for x in l1.cpu()],
            "linf_rel_vs_fp64": [float(x) for x in linf.cpu()],
            "conservation_drift_vs_fp64": [float(x) for x in drift.cpu()]}


def timed(stream, fn):
    """(milliseconds between HIP events recorded on `stream` around fn, fn's result)."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    r = fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), r


def run_grid(wt, ctx, case, precision, steps, warmup, profile, tile_choice=None, graph=True,
             t_end=None):
    """Times `steps` CFL steps (or, with t_end, the steps to that time) of the workload
    from its initial state; returns the timing, the kernel profile and the final state."""
    import torch
    t_stop = float("inf") if t_end is None else float(t_end)
    max_steps = -1 if t_end is not None else steps
    g = wt.Grid(n=case.n, lo=case.lo, hi=case.hi, bc=case.bc)
    p = wt.Params(system=case.system, gamma=case.gamma, cfl=case.cfl, alpha_R=case.alpha_R,
                  precision=precision)
    u_init = torch.from_numpy(case.u).cuda()
    if case.sides is not None:
        wt.wenotheta_set_sides(ctx, [wt.Side(kind=sd.kind, state=sd.state, split0=sd.split0,
                                             split_speed=sd.split_speed) for sd in case.sides], 0.0)
    if tile_choice is None:
        tiles = wt.wenotheta_tune(ctx, g, p, u_init)      # untimed set-up: tile shapes
    else:
        xv, yv = tile_choice
        tiles = tuple([xv] + [yv] * (case.ndim - 1))
        wt.wenotheta_set_tiles(ctx, g, p, tiles)
    if warmup > 0:
        # single CFL steps, queued like the timed ones (the solver's graph would also
        # run its no-op tail steps, which a kernel trace would count)
        u = u_init.clone()
        for _ in range(warmup):
            wt.wenotheta_step(ctx, g, p, u)
        wt.wenotheta_sync(ctx)
        del u
    u = u_init.clone()
    if profile:
        wt.wenotheta_profile(ctx, True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    ms, (t_sim, k) = timed(stream, lambda: wt.wenotheta_solve(ctx, g, p, u, t_stop,
                                                              max_steps=max_steps))
    wall = time.perf_counter() - t0
    prof = None
    if profile:
        prof = wt.wenotheta_profile_read(ctx)
        wt.wenotheta_profile(ctx, False)
    assert t_end is not None or k == steps, (k, steps)
    steps = k
    assert bool(torch.isfinite(u).all()), "non-finite state after the timed steps"
    # The profiled region queues the sweeps one by one with an event pair around each;
    # the solver itself replays them from a captured graph.  The same steps once more
    # that way (after one untimed solve that captures the graph), for the production
    # path's rate; the state must come out the same.
    ms_graph = None
    if profile and graph:
        ug = u_init.clone()            # the graph is captured for this state's address
        wt.wenotheta_solve(ctx, g, p, ug, float("inf"), max_steps=min(steps, 8))
        ug.copy_(u_init)
        ms_graph, (_, kg) = timed(stream, lambda: wt.wenotheta_solve(ctx, g, p, ug, t_stop,
                                                                   max_steps=max_steps))
        assert kg == steps and torch.equal(ug, u), "graph replay differs from the queued steps"
        del ug
    del u_init
    return {"ms": ms, "ms_graph": ms_graph, "wall": wall, "t_sim": t_sim, "u": u, "prof": prof,
            "steps": steps,
            "tiles": [list(wt.TILE_SHAPES[v]) if d > 0 else
                      (list(wt.X_TILE_SHAPES[v]) if case.system == wt.WT_EULER and case.ndim > 1
                       else [1, 255]) for d, v in enumerate(tiles)]}


PROFILE_NAMES = {"sweep_x": (0, False), "sweep_y": (1, False), "sweep_z": (2, False),
                 "sweep_x_final": (0, True), "sweep_y_final": (1, True),
                 "sweep_z_final": (2, True), "stage_2d": (None, True)}


def kernel_ops(case, kind, euler):
    """Algorithmic operations of one launch of a kernel kind: a sweep, or the fused 2D
    stage (both directions' interfaces, the x cell phase and the stage-finishing one)."""
    d, final = PROFILE_NAMES[kind]
    if d is None:
        return (sweep_ops(case.ndim, case.n, 0, False, euler) +
                sweep_ops(case.ndim, case.n, 1, True, euler))
    return sweep_ops(case.ndim, case.n, d, final, euler)
PRECISIONS = {"fp64_fast": 2, "fp64": 0, "fp32": 1}     # wt_precision values


def grid_block(wt, ctx, case, prec_name, steps, warmup, tile_choice=None, graph=True, t_end=None):
    """One timed run of a grid workload in one precision mode: cell-updates/s, the
    dominant kernel's roofline entry, the graph-replay rate, and the final state."""
    prec = PRECISIONS[prec_name]
    r = run_grid(wt, ctx, case, prec, steps, warmup, profile=True, tile_choice=tile_choice,
                 graph=graph, t_end=t_end)
    cells = int(np.prod(case.n))
    prof = r["prof"]
    kind = max(prof, key=lambda kk: prof[kk][0])
    euler = case.system == W_EULER
    ops = kernel_ops(case, kind, euler)
    out = {"value": cells * r["steps"] / (r["ms"] / 1e3), "unit": "cell-updates/s",
           "precision": prec_name, "steps": r["steps"], "ms_per_step": r["ms"] / r["steps"],
           "tiles_tx_tn": r["tiles"],
           "roofline": roofline_entry(kind, ops, prof[kind][0], prof[kind][1],
                                      fp32_recon=prec == 1),
           "kernel_ms": {kk: {"total": v[0], "launches": v[1]} for kk, v in prof.items() if v[1]}}
    if r["ms_graph"] is not None:
        out["graph"] = {"value": cells * r["steps"] / (r["ms_graph"] / 1e3),
                        "ms_per_step": r["ms_graph"] / r["steps"]}
    return out, r


def rel_diff(a, b):
    """Max-relative and L1-relative differences of a against b, per component."""
    m = b.shape[0]
    a2, b2 = a.reshape(m, -1), b.reshape(m, -1)
    d = (a2 - b2).abs()
    mx = b2.abs().amax(dim=1)
    scale = torch_max(mx, 1e-3 * mx.max())
    return {"max_rel": [float(x) for x in (d.amax(dim=1) / scale).cpu()],
            "l1_rel": [float(x) for x in (d.sum(dim=1) / b2.abs().sum(dim=1)).cpu()]}


def torch_max(a, floor):
    import torch
    return torch.maximum(a, torch.as_tensor(floor, dtype=a.dtype, device=a.device))


def perturbation_response(wt, ctx, case, steps, t_end, u_plain):
    """The conditioning of a run: the plain FP64 result's change when every initial value
    is moved by about one unit in the last place (relative 2^-52, seeded random signs),
    in the same measures as the differences of the fast and FP32 forms."""
    rng = np.random.default_rng(2)
    cp = dataclasses.replace(case, u=case.u * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0],
                                                                               size=case.u.shape)))
    r = run_grid(wt, ctx, cp, PRECISIONS["fp64"], steps, 0, profile=False, graph=False,
                 t_end=t_end, tile_choice=None)
    out = rel_diff(r["u"], u_plain)
    del r
    return out


def grid_companion(wt, ctx, case, desc, steps, warmup, t_end=None, graph=True):
    """The FP64 fast, FP64 plain and FP32-weight runs of one grid workload, with the
    differences of the fast and FP32 forms to the plain FP64 run (bit-identical to the
    oracle) and the oracle's CPU baseline."""
    out = {"workload": desc}
    res = {}
    for name in ("fp64_fast", "fp64", "fp32"):
        print(f"[bench] {desc}: {name}", file=sys.stderr, flush=True)
        e, r = grid_block(wt, ctx, case, name, steps, warmup, graph=graph, t_end=t_end)
        out[name] = e
        res[name] = r["u"]
        del r
    out["fp64_fast"]["vs_fp64"] = rel_diff(res["fp64_fast"], res["fp64"])
    out["fp32"].update(differences(res["fp32"], res["fp64"]))
    out["fp64_response_to_1ulp_input_perturbation"] = perturbation_response(
        wt, ctx, case, steps, t_end, res["fp64"])
    out["fp64_fast_over_fp64"] = out["fp64_fast"]["value"] / out["fp64"]["value"]
    out["fp32_over_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    del res
    return out


def run_batched(wt, ctx, B, precision, steps, warmup, tune=True):
    """A batched workload (1D: Batch, 2D: Batch2) through its persistent entry point;
    returns the timed launch's milliseconds, the final state and the per-problem status."""
    import torch
    u_init = torch.from_numpy(B.u).cuda()
    st = torch.empty(B.nprob, dtype=torch.int32, device="cuda")
    p = wt.Params(system=wt.WT_EULER, precision=precision, alpha_R=B.alpha_R, cfl=B.cfl)
    variant = None
    if tune:      # the batch tuner picks the kernel's tile variant before the timed launch
        if hasattr(B, "nx"):
            variant = wt.wenotheta_tune_batched_2d(ctx, p, u_init, B.nx, B.ny, B.offset, B.lo, B.hi,
                                                   B.bc, probe_steps=2)
        else:
            variant = wt.wenotheta_tune_batched(ctx, p, u_init, B.n, B.offset, B.lo, B.hi, B.bc,
                                                probe_steps=2)
    if hasattr(B, "nx"):
        def launch(u):
            wt.wenotheta_solve_batched_2d(ctx, p, u, B.nx, B.ny, B.offset, B.lo, B.hi, B.bc, steps,
                                          status_out=st)
    else:
        def launch(u):
            wt.wenotheta_solve_batched(ctx, p, u, B.n, B.offset, B.lo, B.hi, B.bc, steps,
                                       status_out=st)
    for _ in range(warmup):
        u = u_init.clone()
        launch(u)
        wt.wenotheta_sync(ctx)
    u = u_init.clone()
    stream = torch.cuda.current_stream()
    ms, _ = timed(stream, lambda: launch(u))
    wt.wenotheta_sync(ctx)
    return {"ms": ms, "u": u, "status": st.cpu().numpy(), "variant": variant}


def batched_companions(wt, ctx, steps):
    """Plain FP64, fast FP64 and FP32-weight runs of the batched workload.  L1 is taken over the
    problems that every run completes (the unlimited scheme drives about 2% of the
    seeded problems to a non-physical state; they are reported, not counted), over
    all of them and over the well-conditioned ones: a problem is ill-conditioned at
    FP32 scale when its FP64 result moves by more than 1e-4 (relative L1, 100x the
    FP32 target) under a 2^-24 perturbation of its initial data, about what rounding
    the data to FP32 does.  The same perturbation's effect on all problems is
    reported beside the FP32 difference."""
    from paper_1504_00731_amd import workloads as W
    B = W.batched_1d(seed=0, steps=steps)
    out = compare_batched(wt, ctx, B, B.n, steps)
    out["workload"] = (f"batched 1D Euler, {B.nprob} problems, N log-uniform in [256, 16384] "
                       f"({int(B.n.sum())} cells), seeded piecewise-constant states, transmissive, "
                       f"{steps} RK3 steps, CFL {B.cfl}")
    return out


def batched2d_companions(wt, ctx, steps):
    """The same comparison for the batched 2D workload (independent 2D Euler problems of
    uneven sizes in one persistent launch)."""
    from paper_1504_00731_amd import workloads as W
    B = W.batched_2d(seed=0, steps=steps)
    out = compare_batched(wt, ctx, B, B.nx * B.ny, steps)
    out["workload"] = (f"batched 2D Euler, {B.nprob} problems, nx and ny log-uniform in [32, 96] "
                       f"({int((B.nx * B.ny).sum())} cells), seeded four-quadrant Riemann data, "
                       f"transmissive, {steps} RK3 steps, CFL {B.cfl}")
    return out


def compare_batched(wt, ctx, B, cells_per_problem, steps):
    """Plain FP64, fast FP64 and FP32-weight runs of a batch, timed, and their differences
    to the plain FP64 run."""
    import numpy as np
    import torch
    from paper_1504_00731_amd import workloads as W
    cells = int(cells_per_problem.sum())
    m = B.u.shape[0]
    print(f"[bench] batched {B.nprob} problems ({m} components), {cells} cells, {steps} steps",
          file=sys.stderr, flush=True)
    r64 = run_batched(wt, ctx, B, wt.WT_FP64, steps, 1)
    rfast = run_batched(wt, ctx, B, wt.WT_FP64_FAST, steps, 1)
    r32 = run_batched(wt, ctx, B, wt.WT_FP32_RECON, steps, 1)
    # sensitivity of each problem at FP32 scale: the FP64 result's response to a 2^-24
    # perturbation of the initial data (untimed)
    rng = np.random.default_rng(1)
    Bp = dataclasses.replace(B, u=B.u * (1.0 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=B.u.shape)))
    rp = run_batched(wt, ctx, Bp, wt.WT_FP64, steps, 0, tune=False)
    ok = (r64["status"] == 0) & (r32["status"] == 0) & (rp["status"] == 0) & (rfast["status"] == 0)
    # problems are packed in order: per-problem sums as differences of a running sum at
    # the problems' ends (relative error ~1e-12 here, far below the figures reported).
    # The columns of problems that failed in any run (unspecified, possibly NaN or huge)
    # are zeroed first so that they cannot reach the sums of the others.
    sizes = np.asarray(cells_per_problem, dtype=np.int64)
    ends = torch.from_numpy(np.cumsum(sizes)).cuda()
    starts = ends - torch.from_numpy(sizes).cuda()
    keep = torch.from_numpy(np.repeat(ok, sizes)).cuda()

    def per_problem(x):            # [m, total] -> [nprob, m] sums per problem (0 if failed)
        x = torch.where(keep, x, torch.zeros((), dtype=x.dtype, device=x.device))
        cs = torch.cat([torch.zeros(m, 1, dtype=torch.float64, device="cuda"),
                        torch.cumsum(x, dim=1)], dim=1)
        return (cs[:, ends] - cs[:, starts]).t()

    den = per_problem(r64["u"].abs())
    dpert = per_problem((rp["u"] - r64["u"]).abs())
    resp = (dpert / den).max(dim=1).values.cpu().numpy()
    ill = ok & (resp > 1e-4)
    well = ok & ~ill
    d32 = per_problem((r32["u"] - r64["u"]).abs())
    s32 = per_problem(r32["u"] - r64["u"])
    okt, wellt = torch.from_numpy(ok).cuda(), torch.from_numpy(well).cuda()
    out = {}
    for name, r in (("fp64", r64), ("fp64_fast", rfast), ("fp32_recon", r32)):
        out[name] = {"value": cells * steps / (r["ms"] / 1e3), "unit": "cell-updates/s",
                     "ms": r["ms"], "failed_problems": int((r["status"] != 0).sum()),
                     "tile_variant": r["variant"]}
    dfast = per_problem((rfast["u"] - r64["u"]).abs())
    ff = out["fp64_fast"]
    ff["fp64_fast_over_fp64_same_workload"] = ff["value"] / out["fp64"]["value"]
    ff["l1_rel_vs_fp64_well_conditioned"] = [
        float(x) for x in (dfast[wellt].sum(0) / den[wellt].sum(0)).cpu()]
    ff["l1_rel_vs_fp64_all"] = [float(x) for x in (dfast[okt].sum(0) / den[okt].sum(0)).cpu()]
    f32 = out["fp32_recon"]
    f32["fp32_recon_over_fp64_same_workload"] = f32["value"] / out["fp64"]["value"]
    f32["l1_rel_vs_fp64_well_conditioned"] = [
        float(x) for x in (d32[wellt].sum(0) / den[wellt].sum(0)).cpu()]
    f32["l1_rel_vs_fp64_all"] = [float(x) for x in (d32[okt].sum(0) / den[okt].sum(0)).cpu()]
    f32["ill_conditioned_problems"] = int(ill.sum())
    f32["fp64_response_to_2^-24_input_perturbation_all"] = [
        float(x) for x in (dpert[okt].sum(0) / den[okt].sum(0)).cpu()]
    # per-problem maxima on the host (a segmented max over packed problems)
    first = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    dmax = np.maximum.reduceat((r32["u"] - r64["u"]).abs().cpu().numpy(), first, axis=1).T
    bmax = np.maximum.reduceat(r64["u"].abs().cpu().numpy(), first, axis=1).T
    f32["linf_rel_vs_fp64_all"] = [float(x) for x in dmax[ok].max(0) / bmax[ok].max(0)]
    f32["conservation_drift_vs_fp64"] = [
        float(x) for x in (s32[okt].sum(0).abs() / den[okt].sum(0)).cpu()]
    return out


def achievable_copy_bandwidth():
    """HBM bandwidth a plain device copy reaches (read + write bytes / time), the best of
    10 copies of 1 GiB: the achievable figure beside the published peak."""
    import torch
    n = 2 ** 30 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * 2 ** 30 / (best / 1e3) / 1e9


def copy_calibration(reps):
    """A plain device copy of a known size, for scaling the HBM traffic counters
    (FETCH_SIZE / WRITE_SIZE per dispatch) of the sweep kernels."""
    import torch
    nbytes = 512 * 2 ** 20
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="euler2d", choices=["euler2d", "euler1d", "euler3d", "double_mach", "scalar"])
    ap.add_argument("--precision", default="fp64_fast", choices=["fp64_fast", "fp64", "fp32"],
                    help="fp64_fast: FP64 with fused multiply-adds and fast reciprocals (within "
                         "1e-12 per RHS of the oracle); fp64: the plain operation order "
                         "(bit-identical to the oracle); fp32: FP32 nonlinear weights")
    ap.add_argument("--n", type=int, default=None,
                    help="points per dimension (double_mach: in y, 4n in x; default: full size)")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--batched2d-steps", type=int, default=100)
    ap.add_argument("--steps-3d", type=int, default=100)
    ap.add_argument("--tiles", default="auto", choices=["auto", "0", "1", "2", "3"],
                    help="y/z-sweep tile shape: tuned (auto) or forced variant")
    ap.add_argument("--x-tile", default="0", choices=["0", "1", "2"],
                    help="with a forced --tiles: the x variant (2: the fused 2D stage)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companions", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="of the companions, run only the two batched workloads (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="REPS",
                    help="only run a plain 512 MiB device copy REPS times (counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch

    import paper_1504_00731_amd as wt
    from paper_1504_00731_amd import workloads as W

    case, desc = build_case(args.workload, args.n)
    cells = int(np.prod(case.n))
    print(f"[bench] workload {args.workload} {case.n} {args.precision} steps={args.steps} "
          f"warmup={args.warmup}", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    ctx = wt.Context(0)
    tile_choice = None if args.tiles == "auto" else (int(args.x_tile), int(args.tiles))
    head, r = grid_block(wt, ctx, case, args.precision, args.steps, args.warmup,
                         tile_choice=tile_choice)
    u_head = r["u"]
    ms = r["ms"]
    sec = ms / 1e3
    value = head["value"]
    euler = case.system == W_EULER
    m = case.ndim + 2 if euler else 1
    bytes_per_step = 8 * m * 8 * cells                   # 8 state passes of m FP64 components
    kind = head["roofline"]["kernel"]
    step_traffic = None
    if args.workload == "euler2d" and case.n == (4096, 4096):
        y_tile = "x".join(map(str, r["tiles"][1]))
        head["roofline"]["traffic"] = measured_traffic(kind, y_tile, args.precision)
        tx = measured_traffic("sweep_x", y_tile, args.precision)
        ty = measured_traffic("sweep_y_final", y_tile, args.precision)
        if tx is not None and ty is not None:
            step_traffic = 3 * (tx + ty)                 # one x and one y sweep per stage

    line = {
        "metric": "cell-updates/s (RHS+RK3), FP64 plain vs FP32 batched; % of HBM peak",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{desc}, {'x'.join(map(str, case.n))} points, "
                               f"{args.steps} RK3 steps, CFL {case.cfl}, {args.precision}",
                   "grid": list(case.n), "steps": args.steps, "cfl": case.cfl,
                   "alpha_R": case.alpha_R, "precision": args.precision,
                   "tiles_tx_tn": r["tiles"]},
        "roofline": head["roofline"],
        "hbm": {"achieved": bytes_per_step * args.steps / sec / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": bytes_per_step * args.steps / sec / 1e9 / HBM_PEAK_GBS,
                "bytes_per_cell_update": bytes_per_step // cells,
                "measured_traffic_per_step": step_traffic,
                "measured_over_algorithmic": (None if step_traffic is None
                                              else step_traffic / bytes_per_step),
                "achievable_copy": achievable_copy_bandwidth()},
        "kernel_ms": head["kernel_ms"],
        "graph": dict(head.get("graph", {}), note="the same steps replayed from the solver's "
                      "captured graph without the per-sweep events of the timed region"),
        "wall_s": r["wall"],
        "sim_time": r["t_sim"],
    }
    del r
    if not args.no_companions and args.precision == "fp64_fast":
        comp = {}
        # the same workload in the plain FP64 order (bit-identical to the oracle) and with
        # FP32 weights; the headline's difference to the plain run
        for name in (() if args.batched_only else ("fp64", "fp32")):
            print(f"[bench] companion: same workload, {name}", file=sys.stderr, flush=True)
            e, rr = grid_block(wt, ctx, case, name, args.steps, args.warmup,
                               tile_choice=tile_choice)
            if name == "fp64":
                u_plain = rr["u"]
                e["note"] = "plain operation order, bit-identical to the oracle"
                line["vs_fp64_plain"] = rel_diff(u_head, u_plain)
                line["fp64_plain_response_to_1ulp_input_perturbation"] = perturbation_response(
                    wt, ctx, case, args.steps, None, u_plain)
                line["speedup_over_fp64_plain"] = value / e["value"]
            else:
                e.update(differences(rr["u"], u_plain))
                e["fp32_over_fp64_plain"] = e["value"] / comp["euler2d_fp64_plain"]["value"]
            comp[f"{args.workload}_{'fp64_plain' if name == 'fp64' else 'fp32_weights'}"] = e
            del rr
            if name == "fp32":
                del u_plain
        if args.workload == "euler2d":
            comp["batched"] = batched_companions(wt, ctx, args.batched_steps)
            comp["batched_2d"] = batched2d_companions(wt, ctx, args.batched2d_steps)
        if args.workload == "euler2d" and not args.batched_only:
            # the other grid workloads: 1D Euler to t = 0.2, 3D Euler 512^3
            c1 = W.euler1d_seeded(0, 65536)
            d1 = (f"1D Euler, seeded Riemann data with density wave, 65536 points, to t = "
                  f"{c1.t_end} (CFL {c1.cfl})")
            comp["euler1d"] = grid_companion(wt, ctx, c1, d1, None, args.warmup, t_end=c1.t_end)
            if not args.no_cpu_baseline:
                comp["euler1d"]["cpu_baseline"] = cpu_baseline(c1, "euler1d")
            del c1
            c3 = W.euler3d_seeded(0, 512)
            d3 = (f"3D Euler, seeded vortex with density spheres, 512^3 points, "
                  f"{args.steps_3d} RK3 steps (CFL {c3.cfl})")
            comp["euler3d"] = grid_companion(wt, ctx, c3, d3, args.steps_3d, args.warmup,
                                             graph=False)
            if not args.no_cpu_baseline:
                comp["euler3d"]["cpu_baseline"] = cpu_baseline(c3, "euler3d", sample_n=192)
            del c3
        line["companions"] = comp
    del u_head
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        big = cells > 64 * 2 ** 20           # one oracle step would take over a minute
        line["cpu_baseline"] = cpu_baseline(case, args.workload,
                                            sample_n=192 if big and case.ndim == 3 else None)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
