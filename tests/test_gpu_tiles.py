"""GPU tests of the sweep tile shapes (x: one row segment or 8 rows x 31 points; y/z:
four shapes) and their tuner: every shape computes the same fluxes with the same
operations, so RHS and steps are bit-identical across shapes (and to the oracle in
FP64), on grids whose sizes are not multiples of the tile widths or heights."""
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


def _cases():
    c2 = W.euler2d_seeded(2, 70)
    c2b = W.quadrants_2d(c2.extra["states"], 37, ny=45, name="q2d_37x45")
    c3 = W.euler3d_seeded(1, 22)
    return [c2, c2b, c3]


def _rhs(ctx, case, tiles, precision=wt.WT_FP64):
    import torch
    g, p = grid_params(case)
    p.precision = precision
    wt.wenotheta_set_tiles(ctx, g, p, tiles)
    u = to_dev(case.u)
    L = torch.empty_like(u)
    wt.wenotheta_rhs(ctx, g, p, u, L)
    wt.wenotheta_sync(ctx)
    return L.cpu().numpy()


def _steps(ctx, case, tiles, k, precision=wt.WT_FP64):
    g, p = grid_params(case)
    p.precision = precision
    wt.wenotheta_set_tiles(ctx, g, p, tiles)
    u = to_dev(case.u)
    wt.wenotheta_solve(ctx, g, p, u, math.inf, max_steps=k)
    return u.cpu().numpy()


@pytest.mark.parametrize("xv", range(2))
@pytest.mark.parametrize("v", range(4))
def test_every_tile_shape_matches_oracle_rhs(ctx, xv, v):
    for case in _cases():
        ref = oracle.rhs(oracle_problem(case), case.u)
        got = _rhs(ctx, case, [xv, v, v])
        assert np.array_equal(got, ref), (case.name, xv, v)


def test_tile_shapes_give_identical_steps(ctx):
    for case in _cases():
        for prec in (wt.WT_FP64, wt.WT_FP32_RECON):
            ref = _steps(ctx, case, [0, 0, 0], 3, prec)
            for tiles in ([0, 1, 2], [0, 2, 3], [0, 3, 1], [0, 1, 1], [1, 0, 0], [1, 2, 3]):
                assert np.array_equal(_steps(ctx, case, tiles, 3, prec), ref), (case.name, prec, tiles)


def test_tune_picks_a_shape_and_keeps_results(ctx):
    import torch
    case = W.euler2d_seeded(0, 256)
    g, p = grid_params(case)
    u = to_dev(case.u)
    choice = wt.wenotheta_tune(ctx, g, p, u)
    assert len(choice) == 2 and 0 <= choice[0] < 3 and 0 <= choice[1] < 4
    assert np.array_equal(u.cpu().numpy(), case.u)         # tuning only reads u
    L = torch.empty_like(u)
    wt.wenotheta_rhs(ctx, g, p, u, L)
    wt.wenotheta_sync(ctx)
    assert np.array_equal(L.cpu().numpy(), oracle.rhs(oracle_problem(case), case.u))


def test_set_tiles_rejects_bad_variants(ctx):
    case = W.euler2d_seeded(0, 16)
    g, p = grid_params(case)
    for bad in ([0, 4], [0, -1], [3, 0], [-1, 0]):
        with pytest.raises(wt.WenoThetaError) as e:
            wt.wenotheta_set_tiles(ctx, g, p, bad)
        assert e.value.code == 1
