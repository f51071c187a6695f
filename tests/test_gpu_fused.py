"""The fused 2D stage kernel (x tile variant 2: both directions of a stage in one launch
on 31 x 15 tiles with 3-point halos, the x divergence kept on chip) against the oracle
and the two-sweep path: it runs the sweeps' interface routine on the same values in the
same order, so RHS and steps are bit-identical to the oracle in FP64 (and to the sweeps'
to rounding in the fast FP64 and FP32-weight modes), on grids that are not multiples of
the tile, with every boundary condition, the gravity source, and through the solver's
captured graph."""
import math

import numpy as np
import pytest

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import grid_params, oracle_problem, to_dev

pytestmark = pytest.mark.gpu

FUSED = [2, 0]
SWEEPS = [0, 0]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _cases():
    c2 = W.euler2d_seeded(2, 70)
    rng = np.random.default_rng(4)
    q = [(rng.uniform(0.1, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.03, 1.5))
         for _ in range(4)]
    return [c2,
            W.quadrants_2d(c2.extra["states"], 37, ny=45, name="q2d_37x45"),
            W.quadrants_2d(q, 300, ny=262, name="q2d_300x262"),
            W.quadrants_2d(q, 10, ny=7, name="q2d_10x7"),          # smaller than one tile
            W.quadrants_2d(q, 31, ny=15, name="q2d_31x15"),        # exactly one tile
            W.quadrants_2d(q, 62, ny=31, name="q2d_62x31"),        # two tiles and a row
            W.euler2d_smooth_periodic(3, 64),
            W.rayleigh_taylor(40, 120),                             # walls in y, gravity
            W.implosion(48)]                                        # walls all round


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
    t, n = wt.wenotheta_solve(ctx, g, p, u, math.inf, max_steps=k)
    assert n == k
    return u.cpu().numpy()


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c.name}-{'x'.join(map(str, c.n))}")
def test_fused_rhs_equals_oracle(ctx, case):
    print(f"fused rhs {case.name} {case.n}", flush=True)
    assert np.array_equal(_rhs(ctx, case, FUSED), oracle.rhs(oracle_problem(case), case.u))


def _max_rel(a, b):
    m = b.shape[0]
    a, b = a.reshape(m, -1), b.reshape(m, -1)
    mx = np.abs(b).max(axis=1)
    return float((np.abs(a - b).max(axis=1) / np.maximum(mx, 1e-3 * mx.max())).max())


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c.name}-{'x'.join(map(str, c.n))}")
def test_fused_steps_equal_sweeps_and_oracle(ctx, case):
    """FP64: three steps bit for bit with the oracle.  The fast FP64 and FP32-weight modes
    contract multiply-adds where the compiler finds them, which need not be the same
    places in the fused kernel as in the sweeps: there the two agree to rounding."""
    print(f"fused steps {case.name} {case.n}", flush=True)
    P = oracle_problem(case)
    ref, _, _ = oracle.solve(P, case.u, math.inf, max_steps=3)
    assert np.array_equal(_steps(ctx, case, FUSED, 3), ref)
    for prec in (wt.WT_FP32_RECON, wt.WT_FP64_FAST):
        err = _max_rel(_steps(ctx, case, FUSED, 3, prec), _steps(ctx, case, SWEEPS, 3, prec))
        print(f"  precision {prec}: fused vs sweeps max-rel {err:.2e}", flush=True)
        assert err <= 1e-12, (prec, err)


@pytest.mark.parametrize("prec", [wt.WT_FP64, wt.WT_FP32_RECON, wt.WT_FP64_FAST])
def test_fused_keeps_the_symmetries_bitwise(ctx, prec):
    """Both directions of the fused stage run the sweeps' direction-agnostic routine: the
    TEST 8 quadrants (symmetric under x <-> y) stay exactly symmetric and the
    Rayleigh-Taylor flow exactly mirror-symmetric in x, in every precision mode."""
    c = W.test8_quadrants(96)
    rho, mx, my, E = _steps(ctx, c, FUSED, 20, prec)
    assert np.array_equal(rho, rho.T) and np.array_equal(E, E.T) and np.array_equal(mx, my.T)
    c = W.rayleigh_taylor(64, 192)
    u = _steps(ctx, c, FUSED, 20, prec)
    idx = (-np.arange(c.u.shape[2])) % c.u.shape[2]
    m = u[:, :, idx]
    assert np.array_equal(u[0], m[0]) and np.array_equal(u[2], m[2]) and np.array_equal(u[3], m[3])
    assert np.array_equal(u[1], -m[1])


def test_fused_through_the_graph_with_clipped_end(ctx):
    """20 steps replayed from the solver graph (8-step chunks, a tail of no-op steps) and a
    solve clipped to a final time equal the sweeps' bit for bit."""
    case = W.euler2d_seeded(1, 96)
    assert np.array_equal(_steps(ctx, case, FUSED, 20), _steps(ctx, case, SWEEPS, 20))
    g, p = grid_params(case)
    out = []
    for tiles in (FUSED, SWEEPS):
        wt.wenotheta_set_tiles(ctx, g, p, tiles)
        u = to_dev(case.u)
        t, n = wt.wenotheta_solve(ctx, g, p, u, 0.01)
        out.append((u.cpu().numpy(), t, n))
    assert out[0][1] == out[1][1] == 0.01 and out[0][2] == out[1][2]
    assert np.array_equal(out[0][0], out[1][0])


def test_fused_reports_nonphysical_state(ctx):
    import torch
    case = W.quadrants_2d([(1.0, 0.0, 0.0, 1.0)] * 4, 40)
    bad = case.u.copy()
    bad[1, 20, 20] = 0.5                         # kinetic energy 0.125 > E: p < 0 there
    bad[3, 20, 20] = 1e-6
    g, p = grid_params(case)
    wt.wenotheta_set_tiles(ctx, g, p, FUSED)
    u = to_dev(bad)
    L = torch.empty_like(u)
    wt.wenotheta_rhs(ctx, g, p, u, L)
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_sync(ctx)
    assert e.value.code == wt.binding.WT_ERR_NONPHYSICAL


def test_fused_only_for_2d_euler_without_sides(ctx):
    c3 = W.euler3d_seeded(1, 12)
    g, p = grid_params(c3)
    with pytest.raises(wt.WenoThetaError):
        wt.wenotheta_set_tiles(ctx, g, p, [2, 0, 0])
    dm = W.double_mach(48, 12)
    g, p = grid_params(dm)
    wt.wenotheta_set_sides(ctx, [wt.Side(kind=sd.kind, state=sd.state, split0=sd.split0,
                                         split_speed=sd.split_speed) for sd in dm.sides], 0.0)
    with pytest.raises(wt.WenoThetaError):
        wt.wenotheta_set_tiles(ctx, g, p, FUSED)
    wt.wenotheta_set_sides(ctx, None, 0.0)
