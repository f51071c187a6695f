"""GPU parity of the batched 2D solves (independent 2D Euler problems of uneven sizes in
one persistent launch) against the oracle solving each problem alone, bit for bit in
FP64: ragged tiles in both passes, every boundary condition per direction, problems
that go non-physical, the per-problem outputs, the grid path on the same problem, the
FP32 reconstruction, argument checks, and sampled problems of the full-size batch."""
import math

import numpy as np
import pytest

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _params(B, precision=wt.WT_FP64):
    return wt.Params(system=wt.WT_EULER, gamma=B.gamma, cfl=B.cfl, alpha_R=B.alpha_R,
                     precision=precision)


def _run(ctx, B, nsteps, precision=wt.WT_FP64):
    import torch
    u = to_dev(B.u)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    st = torch.full((B.nprob,), -1, dtype=torch.int32, device="cuda")
    ks = torch.full((B.nprob,), -1, dtype=torch.int64, device="cuda")
    wt.wenotheta_solve_batched_2d(ctx, _params(B, precision), u, B.nx, B.ny, B.offset, B.lo, B.hi,
                                  B.bc, nsteps, t_out=t, status_out=st, steps_out=ks)
    wt.wenotheta_sync(ctx)
    return u.cpu().numpy(), t.cpu().numpy(), st.cpu().numpy(), ks.cpu().numpy()


def _oracle_problem(B, b):
    nx, ny = int(B.nx[b]), int(B.ny[b])
    dx = ((B.hi[b, 0] - B.lo[b, 0]) / nx, (B.hi[b, 1] - B.lo[b, 1]) / ny)
    return oracle.Problem(ndim=2, system=oracle.EULER, n=(nx, ny), dx=dx,
                          bc=(int(B.bc[b, 0]), int(B.bc[b, 1])), gamma=B.gamma, cfl=B.cfl,
                          alpha_R=B.alpha_R)


def _check_against_oracle(B, got, t, st, ks, nsteps, problems):
    failed = 0
    for b in problems:
        o, n = int(B.offset[b]), int(B.nx[b] * B.ny[b])
        P = _oracle_problem(B, b)
        try:
            ref, t_ref, k_ref = oracle.solve(P, B.problem(b), math.inf, max_steps=nsteps)
        except oracle.OracleError:
            assert st[b] != 0, b
            assert 0 <= ks[b] < nsteps
            failed += 1
            continue
        assert st[b] == 0 and ks[b] == nsteps, b
        assert t[b] == t_ref, b
        assert np.array_equal(got[:, o:o + n].reshape(ref.shape), ref), b
    return failed


def _mixed_batch():
    """Uneven sizes (tiles of 4 x 63 and 8 x 31 cut ragged in both passes, several
    segments per line), every boundary condition in each direction."""
    B = W.batched_2d(seed=5, nprob=18, smin=8, smax=48, steps=10)
    sizes = [(130, 70), (6, 6), (64, 31), (63, 32), (7, 129), (33, 9)]
    rng = np.random.default_rng(2)
    parts, nx, ny = [], [], []
    for b in range(B.nprob):
        if b < len(sizes):
            x, y = sizes[b]
            S = [[rng.uniform(0.3, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                  rng.uniform(0.3, 1.5)] for _ in range(4)]
            parts.append(W.quadrants_2d(S, x, ny=y).u.reshape(4, -1))
        else:
            x, y = int(B.nx[b]), int(B.ny[b])
            parts.append(B.problem(b).reshape(4, -1))
        nx.append(x)
        ny.append(y)
    B.nx, B.ny = np.asarray(nx, dtype=np.int64), np.asarray(ny, dtype=np.int64)
    B.offset = np.concatenate([[0], np.cumsum(B.nx * B.ny)[:-1]]).astype(np.int64)
    B.u = np.ascontiguousarray(np.concatenate(parts, axis=1))
    kinds = (W.PERIODIC, W.TRANSMISSIVE, W.REFLECTIVE)
    B.bc = np.array([[kinds[b % 3], kinds[(b // 3) % 3]] for b in range(B.nprob)], dtype=np.int32)
    B.hi = np.ones((B.nprob, 2)) * np.array([1.0, 0.75])
    return B


def test_batched_2d_matches_the_oracle_per_problem(ctx):
    B = _mixed_batch()
    got, t, st, ks = _run(ctx, B, 10)
    failed = _check_against_oracle(B, got, t, st, ks, 10, range(B.nprob))
    assert failed < B.nprob // 2


def test_batched_2d_reports_non_physical_problems(ctx):
    """Seeded problems of the 2D workload's distribution, some of which leave the
    physical states within 60 steps: those are reported, the others are exact."""
    B = W.batched_2d(seed=3, nprob=40, smin=12, smax=40, steps=60)
    got, t, st, ks = _run(ctx, B, 60)
    failed = _check_against_oracle(B, got, t, st, ks, 60, range(B.nprob))
    assert failed == int((st != 0).sum())


def test_batched_2d_equals_the_grid_path(ctx):
    """A problem solved in a batch equals the same problem solved alone by
    wenotheta_solve on the GPU (both FP64, both the oracle's operation order)."""
    B = _mixed_batch()
    got, _, st, _ = _run(ctx, B, 10)
    for b in (0, 4):
        assert st[b] == 0
        nx, ny = int(B.nx[b]), int(B.ny[b])
        g = wt.Grid(n=(nx, ny), lo=tuple(B.lo[b]), hi=tuple(B.hi[b]), bc=tuple(int(k) for k in B.bc[b]))
        u = to_dev(B.problem(b))
        tt, k = wt.wenotheta_solve(ctx, g, _params(B), u, math.inf, max_steps=10)
        assert k == 10
        o = int(B.offset[b])
        assert np.array_equal(got[:, o:o + nx * ny], u.cpu().numpy().reshape(4, -1))


# A problem whose FP64 result moves by more than this (relative L1, worst component) when
# its initial data are perturbed by 2^-24 relative (about what rounding them to FP32
# does) is ill-conditioned at FP32 scale: no FP32 form can be held to 1e-6 on it.
ILL_CONDITIONED = 1e-4


def _per_problem_l1(B, a, b):
    num, den = np.zeros((B.nprob, 4)), np.zeros((B.nprob, 4))
    for p in range(B.nprob):
        o, n = int(B.offset[p]), int(B.nx[p] * B.ny[p])
        num[p] = np.abs(a[:, o:o + n] - b[:, o:o + n]).sum(axis=1)
        den[p] = np.abs(b[:, o:o + n]).sum(axis=1)
    return num, den


def test_batched_2d_fp32_reconstruction(ctx):
    """FP32 reconstruction against the FP64 batch (bit-identical to the oracle), 40 steps:
    over the problems that are not ill-conditioned at FP32 scale the relative L1
    difference is <= 1e-6 per component; over all problems it is no larger than what a
    2^-24 perturbation of the initial data alone does to the FP64 result; a problem of
    constant state is reproduced exactly."""
    B = W.batched_2d(seed=8, nprob=64, smin=16, smax=64, steps=40)
    B.u[:, B.offset[1]:B.offset[1] + B.nx[1] * B.ny[1]] = np.array([[1.0], [0.1], [-0.2], [2.5]])
    u64, _, s64, _ = _run(ctx, B, 40)
    u32, _, s32, _ = _run(ctx, B, 40, wt.WT_FP32_RECON)
    Bp = W.Batch2(u=B.u * (1.0 + 2.0 ** -24 * np.random.default_rng(1).choice([-1.0, 1.0], size=B.u.shape)),
                  nx=B.nx, ny=B.ny, offset=B.offset, lo=B.lo, hi=B.hi, bc=B.bc)
    up, _, sp, _ = _run(ctx, Bp, 40)
    ok = (s64 == 0) & (s32 == 0) & (sp == 0)
    assert ok.sum() >= B.nprob // 2
    pn, pd = _per_problem_l1(B, up, u64)
    well = ok & ((pn / pd).max(axis=1) <= ILL_CONDITIONED)
    n32, _ = _per_problem_l1(B, u32, u64)
    e_well = n32[well].sum(axis=0) / pd[well].sum(axis=0)
    e_all = n32[ok].sum(axis=0) / pd[ok].sum(axis=0)
    e_input = pn[ok].sum(axis=0) / pd[ok].sum(axis=0)
    print(f"FP32 vs FP64 L1: well-conditioned {e_well}, all {e_all}; FP64 under a 2^-24 "
          f"input perturbation {e_input}; well-conditioned {int(well.sum())} of {int(ok.sum())}")
    assert well.sum() >= 0.9 * ok.sum()
    assert np.all(e_well <= 1e-6), e_well
    assert np.all(e_all <= e_input), (e_all, e_input)
    o, n = int(B.offset[1]), int(B.nx[1] * B.ny[1])
    assert np.array_equal(u32[:, o:o + n], u64[:, o:o + n])


def test_batched_2d_fp32_full_size(ctx):
    """The benchmark's batched 2D workload (4096 problems, 32..96 points per side, 100
    steps) in FP32 weights against the FP64 batch (bit-identical to the oracle): the L1
    difference summed over every problem that both complete is <= 1e-6 per component,
    and the FP32 form completes every problem the FP64 path completes."""
    B = W.batched_2d(seed=0)
    u64, _, s64, _ = _run(ctx, B, 100)
    u32, _, s32, _ = _run(ctx, B, 100, wt.WT_FP32_RECON)
    assert not np.any((s32 != 0) & (s64 == 0)), np.flatnonzero((s32 != 0) & (s64 == 0))
    ok = (s64 == 0) & (s32 == 0)
    assert ok.sum() >= 0.97 * B.nprob
    n32, pd = _per_problem_l1(B, u32, u64)
    e_all = n32[ok].sum(axis=0) / pd[ok].sum(axis=0)
    print(f"batched 2D FP32 vs FP64 L1 over all {int(ok.sum())} completed problems: {e_all}")
    assert np.all(e_all <= 1e-6), e_all


@pytest.mark.parametrize("variant", [0, 2, 4])
def test_batched_2d_full_size_sampled(variant):
    """The benchmark batch (4096 problems, 32..96 points per side, 100 steps), in the
    persistent form (0), the flat form (2) and the flat form with packed chunks (4): the
    largest, the smallest and seeded other problems against the oracle."""
    B = W.batched_2d(seed=0)
    with wt.Context(0) as ctx:
        wt.wenotheta_set_batched_tiles(ctx, 2, variant)
        got, t, st, ks = _run(ctx, B, B.steps)
    cells = B.nx * B.ny
    pick = [int(np.argmax(cells)), int(np.argmin(cells))]
    pick += [int(b) for b in np.random.default_rng(1).choice(B.nprob, 6, replace=False)]
    _check_against_oracle(B, got, t, st, ks, B.steps, pick)
    assert (st == 0).mean() > 0.9


def test_batched_2d_arguments(ctx):
    import torch
    B = _mixed_batch()
    u = to_dev(B.u)
    p = _params(B)
    bad_offset = B.offset.copy()
    bad_offset[1] = bad_offset[0] + 5                    # overlaps problem 0
    small = B.nx.copy()
    small[2] = 5
    for args in ((B.nx, B.ny, bad_offset, B.bc), (small, B.ny, B.offset, B.bc),
                 (B.nx, B.ny, B.offset, np.full_like(B.bc, 7))):
        with pytest.raises(wt.WenoThetaError) as e:
            wt.wenotheta_solve_batched_2d(ctx, p, u, args[0], args[1], args[2], B.lo, B.hi, args[3], 1)
        assert e.value.code == 1
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_solve_batched_2d(ctx, wt.Params(system=wt.WT_EULER, gravity=(0.0, 1.0, 0.0)),
                                      u, B.nx, B.ny, B.offset, B.lo, B.hi, B.bc, 1)
    assert e.value.code == 2
    with pytest.raises(ValueError):
        wt.wenotheta_solve_batched_2d(ctx, p, torch.zeros((3, 10), dtype=torch.float64, device="cuda"),
                                      B.nx, B.ny, B.offset, B.lo, B.hi, B.bc, 1)
