"""GPU parity of the sides (bc WT_SIDES: per end two parts, each a given state, a wall or
zero gradient, split at a point that may move; Sec. 4.3 TEST 9) with the oracle, bit for
bit in FP64: right-hand sides at several times, steps whose stages take the moving splits
at t, t + dt, t + dt/2, solves through the captured step graph, 1D/2D/3D, every tile shape
of the y sweep; and the double Mach reflection at the paper's grid and final time."""
import math

import numpy as np
import pytest

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import grid_params, oracle_problem, to_dev

pytestmark = pytest.mark.gpu

ST, RF, TR = W.STATE, W.REFLECTIVE, W.TRANSMISSIVE


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _wt_sides(sides):
    return [wt.Side(kind=s.kind, state=s.state, split0=s.split0, split_speed=s.split_speed)
            for s in sides]


def _random_case(seed, n, lo, hi):
    """Random physical interior; every kind of part on some side, moving splits."""
    rng = np.random.default_rng(seed)
    ndim = len(n)
    shape = tuple(reversed(n))
    rho = rng.uniform(0.5, 2.0, shape)
    vel = [rng.uniform(-1.0, 1.0, shape) for _ in range(ndim)]
    p = rng.uniform(0.5, 2.0, shape)
    u = W.conserved(rho, vel, p)
    pt = lambda: tuple(float(v) for v in W.conserved(rng.uniform(0.5, 2.0), [rng.uniform(-1, 1)
                                                     for _ in range(ndim)], rng.uniform(0.5, 2.0)))
    sides = []
    for d in range(3):
        a = (d + 1) % ndim
        mid = 0.5 * (lo[a] + hi[a])
        span = hi[a] - lo[a]
        sides.append(W.SideSpec((ST, RF), (pt(), ()), split0=mid - 0.2 * span, split_speed=0.5 * span))
        sides.append(W.SideSpec((TR, ST), ((), pt()), split0=mid + 0.1 * span,
                                split_speed=-0.3 * span))
    c = W.Case("random_sides", W.EULER, u, lo, hi, (W.SIDES,) * ndim, sides=tuple(sides))
    return c


def _gpu_rhs(ctx, c, t, precision=wt.WT_FP64):
    import torch
    g, p = grid_params(c)
    p.precision = precision
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), t)
    ud = to_dev(c.u)
    L = torch.empty_like(ud)
    wt.wenotheta_rhs(ctx, g, p, ud, L)
    wt.wenotheta_sync(ctx)
    return L.cpu().numpy()


@pytest.mark.parametrize("t", [0.0, 0.35, 0.9])
def test_rhs_2d_matches_oracle(ctx, t):
    """300 x 70: two x segments and three y segments, both ragged."""
    c = _random_case(1, (300, 70), (0.0, -1.0), (3.0, 0.4))
    got = _gpu_rhs(ctx, c, t)
    ref = oracle.rhs(oracle_problem(c, t=t), c.u)
    assert np.array_equal(got, ref)


def test_rhs_3d_and_1d_match_oracle(ctx):
    c3 = _random_case(2, (20, 18, 16), (0.0, 0.0, 0.0), (1.0, 0.9, 0.8))
    assert np.array_equal(_gpu_rhs(ctx, c3, 0.4), oracle.rhs(oracle_problem(c3, t=0.4), c3.u))
    c1 = _random_case(3, (300,), (-1.0,), (1.0,))
    assert np.array_equal(_gpu_rhs(ctx, c1, 0.2), oracle.rhs(oracle_problem(c1, t=0.2), c1.u))


def test_sides_with_gravity_match_oracle(ctx):
    """Sides and the gravity source together: a wall part on the bottom, a given state
    on the top and inflow on the left, with g along -y; RHS and two steps."""
    c = _random_case(12, (90, 70), (0.0, 0.0), (1.5, 1.0))
    c.gravity = (0.0, 0.7, 0.0)
    got = _gpu_rhs(ctx, c, 0.2)
    assert np.array_equal(got, oracle.rhs(oracle_problem(c, t=0.2), c.u))
    g, p = grid_params(c)
    ud = to_dev(c.u)
    P = oracle_problem(c, t=0.2)
    ref = c.u
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.2)
    for _ in range(2):
        wt.wenotheta_step(ctx, g, p, ud)
        ref, dt = oracle.step(P, ref)
        P.t = P.t + dt
    wt.wenotheta_sync(ctx)
    assert np.array_equal(ud.cpu().numpy(), ref)


def test_steps_match_oracle(ctx):
    """Three CFL steps from t = 0.01 of the double Mach problem at 240 x 60; the top split
    crosses grid lines within each step."""
    c = W.double_mach(240, 60)
    g, p = grid_params(c)
    t0 = 0.01
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), t0)
    ud = to_dev(c.u)
    P = oracle_problem(c, t=t0)
    ref = c.u
    for _ in range(3):
        wt.wenotheta_step(ctx, g, p, ud)
        ref, dt = oracle.step(P, ref)
        P.t = P.t + dt
    wt.wenotheta_sync(ctx)
    assert np.array_equal(ud.cpu().numpy(), ref)
    # the context's time advanced with the steps: a RHS now takes the splits at P.t
    import torch
    L = torch.empty_like(ud)
    wt.wenotheta_rhs(ctx, g, p, ud, L)
    wt.wenotheta_sync(ctx)
    assert np.array_equal(L.cpu().numpy(), oracle.rhs(P, ref))


def test_solve_matches_oracle_through_the_graph(ctx):
    c = W.double_mach(160, 40)
    g, p = grid_params(c)
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.0)
    ud = to_dev(c.u)
    t, k = wt.wenotheta_solve(ctx, g, p, ud, c.t_end, max_steps=30)
    ref, t_ref, k_ref = oracle.solve(oracle_problem(c), c.u, c.t_end, max_steps=30)
    assert (t, k) == (t_ref, k_ref) == (t, 30)
    assert np.array_equal(ud.cpu().numpy(), ref)


@pytest.mark.parametrize("n", [(6, 6), (6, 7), (9, 6)])
def test_smallest_grids(ctx, n):
    """Six points per line (the stencil's minimum): every tile reaches far past the
    ghost points; the given states, walls and zero-gradient parts still equal the
    oracle's."""
    c = _random_case(7 + n[0], n, (0.0, 0.0), (1.0, 1.0))
    for t in (0.0, 0.6):
        assert np.array_equal(_gpu_rhs(ctx, c, t), oracle.rhs(oracle_problem(c, t=t), c.u))
    c3 = _random_case(11, (6, 6, 6), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    assert np.array_equal(_gpu_rhs(ctx, c3, 0.3), oracle.rhs(oracle_problem(c3, t=0.3), c3.u))


def test_split_on_a_line_coordinate(ctx):
    """A split exactly at a grid line's coordinate puts that line in part 1 (part 0 is
    strictly below), on both paths; so does a moving split that reaches a line at the
    stage time."""
    c = _random_case(9, (40, 30), (0.0, 0.0), (1.0, 0.75))
    dx = c.dx[0]
    sides = list(c.sides)
    x17 = 0.0 + (17 + 0.5) * dx
    sides[2] = W.SideSpec((ST, RF), (sides[2].state[0], ()), split0=x17, split_speed=0.0)
    sides[3] = W.SideSpec((ST, TR), (sides[3].state[1], ()), split0=x17 - 0.5 * 2.0,
                          split_speed=2.0)          # at x17 when t = 0.5
    c.sides = tuple(sides)
    for t in (0.5, 0.25):
        assert np.array_equal(_gpu_rhs(ctx, c, t), oracle.rhs(oracle_problem(c, t=t), c.u))


def test_graph_follows_a_new_side_table(ctx):
    """The solver's captured graph holds the side table in its kernel arguments: after
    a solve, a new table (another split speed, a wall part turned into a given state)
    must be used by the next solve on the same grid, not the captured one."""
    c = W.double_mach(160, 40)
    g, p = grid_params(c)
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.0)
    ud = to_dev(c.u)
    wt.wenotheta_solve(ctx, g, p, ud, c.t_end, max_steps=16)
    sides = list(c.sides)
    sides[3] = W.SideSpec(sides[3].kind, sides[3].state, split0=sides[3].split0,
                          split_speed=0.5 * sides[3].split_speed)
    sides[2] = W.SideSpec((ST, ST), (sides[2].state[0], c.sides[3].state[1]),
                          split0=sides[2].split0)
    c.sides = tuple(sides)
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.0)
    ud = to_dev(c.u)
    t, k = wt.wenotheta_solve(ctx, g, p, ud, c.t_end, max_steps=16)
    ref, t_ref, k_ref = oracle.solve(oracle_problem(c), c.u, c.t_end, max_steps=16)
    assert (t, k) == (t_ref, k_ref)
    assert np.array_equal(ud.cpu().numpy(), ref)


@pytest.mark.parametrize("tiles", [(0, 0), (0, 1), (0, 2), (0, 3), (1, 0), (1, 2)])
def test_every_tile_shape(ctx, tiles):
    """2D: every y shape, and the 8-row x tile (each lane its own row, so its own side
    part along y); 3D with the 8-row x tile."""
    c = _random_case(4, (77, 50), (0.0, 0.0), (1.0, 0.7))
    g, p = grid_params(c)
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.3)
    wt.wenotheta_set_tiles(ctx, g, p, tiles)
    got = _gpu_rhs(ctx, c, 0.3)
    assert np.array_equal(got, oracle.rhs(oracle_problem(c, t=0.3), c.u))
    if tiles[0] == 1:
        c3 = _random_case(5, (20, 13, 11), (0.0, 0.0, 0.0), (1.0, 0.9, 0.8))
        g3, p3 = grid_params(c3)
        wt.wenotheta_set_sides(ctx, _wt_sides(c3.sides), 0.4)
        wt.wenotheta_set_tiles(ctx, g3, p3, (1, tiles[1], tiles[1]))
        assert np.array_equal(_gpu_rhs(ctx, c3, 0.4), oracle.rhs(oracle_problem(c3, t=0.4), c3.u))


def test_tuner_on_a_sides_grid(ctx):
    """The tuner leaves the state and the context's time as they were: a RHS after it
    takes the moving split at the time set before."""
    import torch
    c = W.double_mach(200, 50)
    g, p = grid_params(c)
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.05)
    ud = to_dev(c.u)
    tiles = wt.wenotheta_tune(ctx, g, p, ud)
    assert len(tiles) == 2
    assert np.array_equal(ud.cpu().numpy(), c.u)
    L = torch.empty_like(ud)
    wt.wenotheta_rhs(ctx, g, p, ud, L)
    wt.wenotheta_sync(ctx)
    assert np.array_equal(L.cpu().numpy(), oracle.rhs(oracle_problem(c, t=0.05), c.u))


@pytest.mark.parametrize("precision", [wt.WT_FP64, wt.WT_FP32_RECON])
def test_double_mach_at_the_paper_size_and_time(ctx, precision):
    """800 x 200 to t = 0.2: physical throughout; the FP64 run's first 20 steps equal
    the oracle's; along the top row the density falls from the post- to the pre-shock
    value where the exact shock line meets the top boundary."""
    c = W.double_mach(800, 200)
    g, p = grid_params(c)
    p.precision = precision
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.0)
    ud = to_dev(c.u)
    if precision == wt.WT_FP64:
        t, k = wt.wenotheta_solve(ctx, g, p, ud, c.t_end, max_steps=20)
        ref, t_ref, k_ref = oracle.solve(oracle_problem(c), c.u, c.t_end, max_steps=20)
        assert (t, k) == (t_ref, k_ref)
        assert np.array_equal(ud.cpu().numpy(), ref)
        ud = to_dev(c.u)
    t, k = wt.wenotheta_solve(ctx, g, p, ud, c.t_end)
    a = ud.cpu().numpy()
    assert t == c.t_end and k > 1000
    rho = a[0]
    assert np.isfinite(a).all() and rho.min() > 0.0
    assert 1.3 < rho.min() and rho.max() < 30.0
    top = c.sides[3]
    xs = top.split0 + top.split_speed * c.t_end
    x = W.grid_points(800, 0.0, 4.0, W.TRANSMISSIVE)
    row = rho[-1]
    cross = x[np.argmax(row < 0.5 * (8.0 + 1.4))]
    assert abs(cross - xs) < 2.0 * c.dx[0]
    assert np.all(np.abs(row[x > xs + 0.05] - 1.4) < 1e-3)


def test_side_arguments(ctx):
    import torch
    c = W.double_mach(40, 10)
    g, p = grid_params(c)
    ud = to_dev(c.u)
    L = torch.empty_like(ud)
    with pytest.raises(wt.WenoThetaError) as e:          # no side table yet
        wt.wenotheta_rhs(ctx, g, p, ud, L)
    assert e.value.code == 1
    bad = _wt_sides(c.sides)
    bad[1] = wt.Side(kind=(9, 1))
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_set_sides(ctx, bad, 0.0)
    assert e.value.code == 1
    bad[1] = wt.Side(split0=math.nan)
    with pytest.raises(wt.WenoThetaError):
        wt.wenotheta_set_sides(ctx, bad, 0.0)
    with pytest.raises(wt.WenoThetaError):
        wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), math.inf)
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.0)
    wt.wenotheta_rhs(ctx, g, p, ud, L)                  # now accepted
    wt.wenotheta_set_sides(ctx, None, 0.0)              # table removed
    with pytest.raises(wt.WenoThetaError):
        wt.wenotheta_rhs(ctx, g, p, ud, L)
    # scalar systems take no sides; batches take no WT_SIDES
    wt.wenotheta_set_sides(ctx, _wt_sides(c.sides), 0.0)
    gs = wt.Grid(n=(16,), lo=(0.0,), hi=(1.0,), bc=(wt.WT_SIDES,))
    us = to_dev(np.zeros((1, 16)))
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_rhs(ctx, gs, wt.Params(system=wt.WT_BURGERS), us, torch.empty_like(us))
    assert e.value.code == 2
    B = W.batched_1d(seed=1, nprob=3, nmin=8, nmax=20, steps=2)
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_solve_batched(ctx, wt.Params(), to_dev(B.u), B.n, B.offset, B.lo, B.hi,
                                   np.full(3, wt.WT_SIDES, dtype=np.int32), 2)
    assert e.value.code == 1
    wt.wenotheta_sync(ctx)
