"""GPU tests of the batched persistent solve and of the FP32-reconstruction mode.

Batched FP64: every problem of a batch must equal, bit for bit, the oracle's
solve of that problem alone (and the library's single-problem solve).
FP32 reconstruction: L1 error relative to the FP64 result <= 1e-6 (the
precision target of the FP32 form), conservation sums in FP64.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import grid_params, oracle_problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _run_batched(ctx, B, steps, precision=wt.WT_FP64):
    """Returns (u, t, status, steps) per problem; failed problems are reported per problem."""
    import torch
    u = to_dev(B.u)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    st = torch.full((B.nprob,), -1, dtype=torch.int32, device="cuda")
    k = torch.full((B.nprob,), -1, dtype=torch.int64, device="cuda")
    p = wt.Params(system=wt.WT_EULER, precision=precision, alpha_R=B.alpha_R, cfl=B.cfl)
    wt.wenotheta_solve_batched(ctx, p, u, B.n, B.offset, B.lo, B.hi, B.bc, steps, t_out=t,
                               status_out=st, steps_out=k)
    wt.wenotheta_sync(ctx)
    return u.cpu().numpy(), t.cpu().numpy(), st.cpu().numpy(), k.cpu().numpy()


def _oracle_solve(B, b, steps):
    """(state, t) of the oracle's solve of problem b alone, or None if it fails."""
    P, u0 = _oracle_problem(B, b)
    try:
        ref, t_ref, _ = oracle.solve(P, u0, math.inf, max_steps=steps)
    except oracle.OracleError as e:
        assert e.code in (3, 4)
        return None
    return ref, t_ref


def _oracle_problem(B, b):
    o, k = int(B.offset[b]), int(B.n[b])
    P = oracle.Problem(ndim=1, system=oracle.EULER, n=(k,), dx=((B.hi[b] - B.lo[b]) / k,),
                       bc=(int(B.bc[b]),), gamma=B.gamma, cfl=B.cfl, alpha_R=B.alpha_R)
    return P, B.u[:, o:o + k]


def l1_rel(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


@pytest.mark.parametrize("seed,steps", [(3, 15), (5, 10)])
def test_batched_fp64_matches_oracle_per_problem(ctx, seed, steps):
    """Every problem equals the oracle's solve of it alone, bit for bit; a problem the
    unlimited scheme drives to a non-physical state (seed 5 has one) is reported as
    such, exactly where the oracle fails too, while the others continue."""
    B = W.batched_1d(seed=seed, nprob=40 if seed == 3 else 30, nmin=6 if seed == 3 else 50,
                     nmax=700 if seed == 3 else 900)
    got, t, st, k = _run_batched(ctx, B, steps)
    failed = 0
    for b in range(B.nprob):
        r = _oracle_solve(B, b, steps)
        o, n = int(B.offset[b]), int(B.n[b])
        if r is None:
            assert st[b] in (3, 4) and k[b] < steps, (b, st[b], k[b])
            failed += 1
            continue
        assert st[b] == 0 and k[b] == steps
        assert np.array_equal(got[:, o:o + n], r[0]), f"problem {b} (n={n})"
        assert t[b] == r[1]
    assert failed == (1 if seed == 5 else 0)


def test_batched_equals_single_problem_solves(ctx):
    B = W.batched_1d(seed=4, nprob=12, nmin=100, nmax=3000)
    got, t, st, _ = _run_batched(ctx, B, 25)
    for b in range(B.nprob):
        if st[b] != 0:
            continue
        o, k = int(B.offset[b]), int(B.n[b])
        case = W.Case("p", W.EULER, B.u[:, o:o + k].copy(), (B.lo[b],), (B.hi[b],), (int(B.bc[b]),))
        g, p = grid_params(case)
        ud = to_dev(case.u)
        tt, kk = wt.wenotheta_solve(ctx, g, p, ud, math.inf, max_steps=25)
        assert kk == 25 and tt == t[b]
        assert np.array_equal(ud.cpu().numpy(), got[:, o:o + k])


def test_batched_graph_replays(ctx):
    """The batch runs as a captured graph; replay it several times with eager work and
    synchronisations in between, each replay on a fresh copy of the same input."""
    import torch
    B = W.batched_1d(seed=3, nprob=30, nmin=50, nmax=900)
    ref, _, st, _ = _run_batched(ctx, B, 10)
    assert np.all(st == 0)
    u_init = to_dev(B.u)
    p = wt.Params(system=wt.WT_EULER, alpha_R=B.alpha_R, cfl=B.cfl)
    u = u_init.clone()
    for rep in range(4):
        u.copy_(u_init)                      # eager work between replays
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        wt.wenotheta_solve_batched(ctx, p, u, B.n, B.offset, B.lo, B.hi, B.bc, 10)
        wt.wenotheta_sync(ctx)
        assert np.array_equal(u.cpu().numpy(), ref), f"replay {rep}"
        del junk


def test_batched_argument_errors(ctx):
    B = W.batched_1d(seed=6, nprob=4, nmin=10, nmax=20)
    p = wt.Params(system=wt.WT_EULER)
    u = to_dev(B.u)
    bad_off = B.offset.copy()
    bad_off[1] = bad_off[0]                  # overlapping problems
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_solve_batched(ctx, p, u, B.n, bad_off, B.lo, B.hi, B.bc, 1)
    assert e.value.code == 1
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_solve_batched(ctx, wt.Params(system=wt.WT_LINEAR), u, B.n, B.offset, B.lo,
                                   B.hi, B.bc, 1)
    assert e.value.code == 2


@pytest.mark.parametrize("variant", [0, 2])
def test_batched_full_size_sampled(variant):
    """The batched workload at full size (4096 problems, N log-uniform in [256, 16384],
    500 steps), persistent (0) and flat (2) form: the 6 smallest problems against the
    oracle, bit for bit."""
    B = W.batched_1d(seed=0)
    with wt.Context(0) as ctx:
        wt.wenotheta_set_batched_tiles(ctx, 1, variant)
        got, t, st, k = _run_batched(ctx, B, 500)
    ok = st == 0
    assert ok.sum() >= 0.97 * B.nprob           # ~2% of the seeded problems fail (no limiter)
    assert np.all(k[ok] == 500) and np.all(k[~ok] < 500)
    checked = 0
    for b in np.argsort(B.n, kind="stable"):
        r = _oracle_solve(B, b, 500)
        if r is None:
            assert not ok[b]
            continue
        o, n = int(B.offset[b]), int(B.n[b])
        assert ok[b] and np.array_equal(got[:, o:o + n], r[0]), f"problem {b}"
        assert t[b] == r[1]
        checked += 1
        if checked == 6:
            break


# Sensitivity of each problem at FP32 scale: how far its FP64 result moves (relative
# L1, worst component) when its initial data are perturbed by 2^-24 relative, random
# sign per value -- about what rounding the data to FP32 does.  A problem that moves
# by more than ILL_CONDITIONED (100x the FP32 target) under that perturbation is
# ill-conditioned at FP32 scale: no FP32 form can be held to 1e-6 on it.
ILL_CONDITIONED = 1e-4


def _per_problem_l1(B, a, b):
    num = np.zeros((B.nprob, 3))
    den = np.zeros((B.nprob, 3))
    for p in range(B.nprob):
        o, n = int(B.offset[p]), int(B.n[p])
        num[p] = np.abs(a[:, o:o + n] - b[:, o:o + n]).sum(axis=1)
        den[p] = np.abs(b[:, o:o + n]).sum(axis=1)
    return num, den


def test_batched_fp32_l1_full_size(ctx):
    """FP32 reconstruction against the FP64 path (bit-identical to the oracle) on the
    full batched workload, 500 steps:
      - summed over the problems that are not ill-conditioned at FP32 scale, the L1
        relative difference is <= 1e-6 per component, and such problems are rare;
      - summed over all problems, the difference is no larger than the one a 2^-24
        perturbation of the initial data alone causes in the FP64 result."""
    B = W.batched_1d(seed=0)
    u64, _, st64, _ = _run_batched(ctx, B, 500)
    rng = np.random.default_rng(1)
    Bp = W.Batch(u=B.u * (1.0 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=B.u.shape)), n=B.n,
                 offset=B.offset, lo=B.lo, hi=B.hi, bc=B.bc)
    up, _, stp, _ = _run_batched(ctx, Bp, 500)
    u32, _, st32, _ = _run_batched(ctx, B, 500, precision=wt.WT_FP32_RECON)
    ok = (st64 == 0) & (stp == 0) & (st32 == 0)
    assert ok.sum() >= 0.97 * B.nprob
    # the FP32-weight form completes every problem the FP64 path completes
    assert not np.any((st32 != 0) & (st64 == 0)), np.flatnonzero((st32 != 0) & (st64 == 0))
    pn, pd = _per_problem_l1(B, up, u64)
    ill = ok & ((pn / pd).max(axis=1) > ILL_CONDITIONED)
    well = ok & ~ill
    n32, _ = _per_problem_l1(B, u32, u64)
    e_well = n32[well].sum(axis=0) / pd[well].sum(axis=0)
    e_all = n32[ok].sum(axis=0) / pd[ok].sum(axis=0)
    e_input = pn[ok].sum(axis=0) / pd[ok].sum(axis=0)
    print(f"FP32 vs FP64 L1: well-conditioned {e_well}, all {e_all}; FP64 under a 2^-24 "
          f"input perturbation {e_input}; ill-conditioned {int(ill.sum())} of {int(ok.sum())}")
    assert ill.sum() <= 0.01 * B.nprob, int(ill.sum())
    assert np.all(e_well <= 1e-6), e_well
    assert np.all(e_all <= e_input), (e_all, e_input)


def test_fp32_rhs_close_to_fp64(ctx):
    """FP32 reconstruction RHS against the oracle's FP64 RHS on smooth and discontinuous
    2D and 1D data: max error relative to max |L| per component well below 1e-4."""
    import torch
    for case in (W.euler2d_seeded(2, 96), W.euler2d_smooth_periodic(1, 64), W.euler1d_seeded(1, 4000),
                 W.sod(300)):
        ref = oracle.rhs(oracle_problem(case), case.u)
        g, p = grid_params(case)
        p.precision = wt.WT_FP32_RECON
        ud = to_dev(case.u)
        L = torch.empty_like(ud)
        wt.wenotheta_rhs(ctx, g, p, ud, L)
        wt.wenotheta_sync(ctx)
        got = L.cpu().numpy().reshape(ref.shape[0], -1)
        r = ref.reshape(ref.shape[0], -1)
        err = (np.abs(got - r).max(axis=1) / np.abs(r).max(axis=1)).max()
        assert err < 1e-4, (case.name, err)


def test_fp32_free_stream_exact(ctx):
    import torch
    u = W.conserved(np.full((40, 50), 0.9), [0.2, -0.4], 1.3)
    case = W.Case("c", W.EULER, u, (0.0, 0.0), (1.0, 1.0), (W.PERIODIC, W.PERIODIC))
    g, p = grid_params(case)
    p.precision = wt.WT_FP32_RECON
    ud = to_dev(u)
    L = torch.empty_like(ud)
    wt.wenotheta_rhs(ctx, g, p, ud, L)
    wt.wenotheta_sync(ctx)
    assert int(torch.count_nonzero(L)) == 0


def test_fp32_2d_workload_l1(ctx):
    """2D workload shape at 512^2, 40 steps: FP32 reconstruction vs the FP64 path
    (bit-identical to the oracle), L1 relative error per component <= 1e-6."""
    case = W.euler2d_seeded(0, 512)
    g, p = grid_params(case)
    u64 = to_dev(case.u)
    wt.wenotheta_solve(ctx, g, p, u64, math.inf, max_steps=40)
    p.precision = wt.WT_FP32_RECON
    u32 = to_dev(case.u)
    wt.wenotheta_solve(ctx, g, p, u32, math.inf, max_steps=40)
    a, b = u32.cpu().numpy(), u64.cpu().numpy()
    for c in range(4):
        assert l1_rel(a[c], b[c]) <= 1e-6, (c, l1_rel(a[c], b[c]))


def test_fp32_periodic_conservation(ctx):
    """Conservation sums stay FP64: periodic 2D data, 20 FP32-reconstruction steps,
    relative drift of every component's total <= 1e-13."""
    case = W.euler2d_smooth_periodic(5, 96)
    g, p = grid_params(case)
    p.precision = wt.WT_FP32_RECON
    ud = to_dev(case.u)
    wt.wenotheta_solve(ctx, g, p, ud, math.inf, max_steps=20)
    got = ud.cpu().numpy().reshape(4, -1)
    ref = case.u.reshape(4, -1)
    drift = np.abs(got.sum(axis=1) - ref.sum(axis=1)) / np.abs(ref).sum(axis=1)
    assert np.all(drift <= 1e-13), drift
