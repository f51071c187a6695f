"""GPU tests of the batched kernels' tile variants and their tuners: both variants give
bit-identical results (1D and 2D, FP64 and FP32, ragged tiles, every boundary
condition), the tuners leave the state untouched and report no error for batches with
non-physical problems, and later solves of the same batch use the tuned variant."""
import math

import numpy as np
import pytest

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import to_dev
from tests.test_gpu_batched_2d import _mixed_batch

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _batch_1d():
    B = W.batched_1d(seed=11, nprob=30, nmin=6, nmax=700, steps=12)
    B.bc = np.array([(W.PERIODIC, W.TRANSMISSIVE, W.REFLECTIVE)[b % 3] for b in range(B.nprob)],
                    dtype=np.int32)
    return B


def _run_1d(ctx, B, steps, precision):
    import torch
    u = to_dev(B.u)
    st = torch.full((B.nprob,), -1, dtype=torch.int32, device="cuda")
    p = wt.Params(system=wt.WT_EULER, precision=precision, alpha_R=B.alpha_R, cfl=B.cfl)
    wt.wenotheta_solve_batched(ctx, p, u, B.n, B.offset, B.lo, B.hi, B.bc, steps, status_out=st)
    wt.wenotheta_sync(ctx)
    return u.cpu().numpy(), st.cpu().numpy()


def _run_2d(ctx, B, steps, precision):
    import torch
    u = to_dev(B.u)
    st = torch.full((B.nprob,), -1, dtype=torch.int32, device="cuda")
    p = wt.Params(system=wt.WT_EULER, precision=precision, alpha_R=B.alpha_R, cfl=B.cfl)
    wt.wenotheta_solve_batched_2d(ctx, p, u, B.nx, B.ny, B.offset, B.lo, B.hi, B.bc, steps,
                                  status_out=st)
    wt.wenotheta_sync(ctx)
    return u.cpu().numpy(), st.cpu().numpy()


def _equal_where_completed(B, a, b, status):
    """Bitwise equality of the problems that completed (status 0).  A problem that went
    non-physical keeps being advanced and its columns are unspecified: with NaN speeds
    the block maxima depend on the reduction order, which differs between variants."""
    cells = B.nx * B.ny if hasattr(B, "nx") else B.n
    ok = status == 0
    assert ok.sum() >= len(ok) // 2
    for p in np.nonzero(ok)[0]:
        o, n = int(B.offset[p]), int(cells[p])
        if not np.array_equal(a[:, o:o + n].view(np.int64), b[:, o:o + n].view(np.int64)):
            return False
    return True


@pytest.mark.parametrize("precision", [wt.WT_FP64, wt.WT_FP32_RECON])
def test_batch_variants_are_bit_identical(ctx, precision):
    """1D: the persistent kernel with either workgroup size and the flat form (one launch
    per stage over all problems' segments); 2D: the persistent kernel and the flat form,
    each with either x tile, and the flat form with packed chunks in both passes."""
    B1, B2 = _batch_1d(), _mixed_batch()
    res1, res2 = {}, {}
    for v in (0, 1, 2):
        wt.wenotheta_set_batched_tiles(ctx, 1, v)
        res1[v] = _run_1d(ctx, B1, 12, precision)
    for v in (0, 1, 2, 3, 4):
        wt.wenotheta_set_batched_tiles(ctx, 2, v)
        res2[v] = _run_2d(ctx, B2, 10, precision)
    for B, res in ((B1, res1), (B2, res2)):
        a, sa = res[0]
        for v in res:
            b, sb = res[v]
            assert np.array_equal(sa, sb), v
            assert _equal_where_completed(B, a, b, sa), v
    if precision == wt.WT_FP64:                 # the flat 1D form against the oracle
        got, st = res1[2]
        for b in range(B1.nprob):
            o, n = int(B1.offset[b]), int(B1.n[b])
            P = oracle.Problem(ndim=1, system=oracle.EULER, n=(n,), dx=((B1.hi[b] - B1.lo[b]) / n,),
                               bc=(int(B1.bc[b]),), cfl=B1.cfl, alpha_R=B1.alpha_R)
            try:
                ref, _, _ = oracle.solve(P, B1.u[:, o:o + n], math.inf, max_steps=12)
            except oracle.OracleError:
                assert st[b] != 0
                continue
            assert st[b] == 0 and np.array_equal(got[:, o:o + n], ref), b


def test_batch_tuners_leave_the_state_and_are_used(ctx):
    import torch
    B1 = _batch_1d()
    B2 = W.batched_2d(seed=3, nprob=40, smin=12, smax=40, steps=6)   # some go non-physical
    p = wt.Params(system=wt.WT_EULER, alpha_R=B1.alpha_R, cfl=B1.cfl)
    u1, u2 = to_dev(B1.u), to_dev(B2.u)
    v1 = wt.wenotheta_tune_batched(ctx, p, u1, B1.n, B1.offset, B1.lo, B1.hi, B1.bc, probe_steps=3)
    v2 = wt.wenotheta_tune_batched_2d(ctx, p, u2, B2.nx, B2.ny, B2.offset, B2.lo, B2.hi, B2.bc,
                                      probe_steps=3)
    wt.wenotheta_sync(ctx)                      # no error left in the context
    assert v1 in (0, 1, 2) and v2 in (0, 1, 2, 3, 4)
    assert np.array_equal(u1.cpu().numpy(), B1.u) and np.array_equal(u2.cpu().numpy(), B2.u)
    tuned = (_run_1d(ctx, B1, 12, wt.WT_FP64), _run_2d(ctx, B2, 60, wt.WT_FP64))
    with wt.Context(0) as other:                # default variants on a fresh context
        plain = (_run_1d(other, B1, 12, wt.WT_FP64), _run_2d(other, B2, 60, wt.WT_FP64))
    for k, B in enumerate((B1, B2)):
        assert np.array_equal(tuned[k][1], plain[k][1])
        assert _equal_where_completed(B, tuned[k][0], plain[k][0], tuned[k][1])
    assert (tuned[1][1] != 0).any()             # the 2D batch does have failing problems


def test_batch_tile_arguments(ctx):
    for ndim, v in ((0, 0), (3, 0), (1, 3), (2, -1), (2, 5)):
        with pytest.raises(wt.WenoThetaError) as e:
            wt.wenotheta_set_batched_tiles(ctx, ndim, v)
        assert e.value.code == 1
    B = _batch_1d()
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_tune_batched(ctx, wt.Params(system=wt.WT_EULER), to_dev(B.u), B.n, B.offset,
                                  B.lo, B.hi, B.bc, probe_steps=0)
    assert e.value.code == 1
