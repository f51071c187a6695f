"""GPU parity of reflective walls and the gravity source (Sec. 4.2 TEST 5, Sec. 4.3
TESTs 6 and 7) against the oracle, bit for bit: RHS, steps and solves of the paper's
setups at reduced size, walls in each direction of 3D, the FP32 form's symmetry, and
batched problems with walls."""
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


def _rhs(ctx, case, precision=wt.WT_FP64):
    import torch
    g, p = grid_params(case)
    p.precision = precision
    u = to_dev(case.u)
    L = torch.empty_like(u)
    wt.wenotheta_rhs(ctx, g, p, u, L)
    wt.wenotheta_sync(ctx)
    return L.cpu().numpy()


def _steps(ctx, case, k, precision=wt.WT_FP64):
    g, p = grid_params(case)
    p.precision = precision
    u = to_dev(case.u)
    t, n = wt.wenotheta_solve(ctx, g, p, u, math.inf, max_steps=k)
    assert n == k
    return u.cpu().numpy()


def _oracle_steps(case, k):
    P = oracle_problem(case)
    u = case.u.copy()
    for _ in range(k):
        u, _ = oracle.step(P, u)
    return u


def _walls_3d():
    c = W.euler3d_seeded(4, 20, edge=2.0)
    c.bc = (W.REFLECTIVE, W.PERIODIC, W.REFLECTIVE)
    c.gravity = (0.0, 0.0, 0.2)
    return c


CASES = [lambda: W.blast_waves(300), lambda: W.rayleigh_taylor(40, 120), lambda: W.implosion(48),
         _walls_3d]


@pytest.mark.parametrize("make", CASES)
def test_rhs_matches_oracle(ctx, make):
    c = make()
    assert np.array_equal(_rhs(ctx, c), oracle.rhs(oracle_problem(c), c.u))


@pytest.mark.parametrize("make", CASES)
def test_steps_match_oracle(ctx, make):
    c = make()
    assert np.array_equal(_steps(ctx, c, 4), _oracle_steps(c, 4))


def test_rayleigh_taylor_symmetry_on_the_gpu(ctx):
    """x-mirror symmetry of the Rayleigh-Taylor flow in every precision mode.  The
    grid spacings are powers of two, so the grid points, and with them the initial data,
    are exactly mirror-symmetric (on a 48-wide grid x and -x differ in the last bit)."""
    c = W.rayleigh_taylor(64, 192)
    nx = c.u.shape[2]
    idx = (-np.arange(nx)) % nx
    for prec in (wt.WT_FP64, wt.WT_FP32_RECON, wt.WT_FP64_FAST):
        u = _steps(ctx, c, 30, prec)
        m = u[:, :, idx]
        assert np.array_equal(u[0], m[0]) and np.array_equal(u[2], m[2]) and np.array_equal(u[3], m[3])
        assert np.array_equal(u[1], -m[1])


def test_implosion_diagonal_symmetry_on_the_gpu(ctx):
    c = W.implosion(64)
    for prec in (wt.WT_FP64, wt.WT_FP32_RECON, wt.WT_FP64_FAST):
        u = _steps(ctx, c, 25, prec)
        assert np.array_equal(u[0], u[0].T) and np.array_equal(u[1], u[2].T)


def _mirror_double(u, axis, normal_comp):
    mir = np.flip(u, axis=axis).copy()
    mir[normal_comp] = -mir[normal_comp]
    return np.concatenate([mir, u], axis=axis)


def test_walls_are_the_mirrored_periodic_problem_on_the_gpu(ctx):
    """20 CFL steps of a 2D problem with walls all round equal, bit for bit, the same
    steps of the periodic problem on the doubled (mirrored) grid, both on the GPU: the
    walls' ghost points, the paired acoustic speeds and the time step agree with the
    mirror image everywhere (also with the y tiles reaching past the grid)."""
    c = W.euler2d_seeded(2, 72)
    ud = _mirror_double(_mirror_double(c.u, axis=1, normal_comp=2), axis=2, normal_comp=1)
    cw = W.Case("walls", W.EULER, c.u, (0.0, 0.0), (1.0, 1.0), (W.REFLECTIVE, W.REFLECTIVE))
    cd = W.Case("doubled", W.EULER, ud, (-1.0, -1.0), (1.0, 1.0), (W.PERIODIC, W.PERIODIC))
    for prec in (wt.WT_FP64, wt.WT_FP32_RECON):
        uw, udd = _steps(ctx, cw, 20, prec), _steps(ctx, cd, 20, prec)
        assert np.array_equal(uw, udd[:, 72:, 72:])


def test_implosion_at_the_paper_size_and_time(ctx):
    """TEST 7 as printed: 400 x 400, walls all round, alpha_R = 1, to t = 5 (about 17000
    CFL steps).  The density stays exactly symmetric about the diagonal (the paper's point
    for this test), and with walls all round mass and energy are conserved to rounding."""
    c = W.implosion(400)
    m0 = c.u.reshape(4, -1).sum(axis=1)
    for prec in (wt.WT_FP64, wt.WT_FP32_RECON):
        g, p = grid_params(c)
        p.precision = prec
        u = to_dev(c.u)
        t, k = wt.wenotheta_solve(ctx, g, p, u, c.t_end)
        a = u.cpu().numpy()
        assert t == c.t_end and k > 10000
        assert np.array_equal(a[0], a[0].T) and np.array_equal(a[1], a[2].T)
        m1 = a.reshape(4, -1).sum(axis=1)
        for comp in (0, 3):
            assert abs(m1[comp] - m0[comp]) <= 1e-11 * m0[comp], (prec, comp)


def test_rayleigh_taylor_at_the_paper_size_and_time(ctx):
    """TEST 6 as printed: 120 x 360, periodic in x, walls in y, gravity 0.1, to t = 9.5
    (about 17800 steps): mass is conserved to rounding, the heavy fluid has sunk (the
    centre of mass moved down) and the flow stayed physical."""
    c = W.rayleigh_taylor(120, 360)
    y = W.grid_points(360, -0.75, 0.75, W.REFLECTIVE)[:, None]
    g, p = grid_params(c)
    u = to_dev(c.u)
    t, k = wt.wenotheta_solve(ctx, g, p, u, c.t_end)
    a = u.cpu().numpy()
    assert t == c.t_end and k > 10000
    assert abs(a[0].sum() - c.u[0].sum()) <= 1e-11 * c.u[0].sum()
    assert (a[0] * y).sum() < (c.u[0] * y).sum() - 1e-3 * c.u[0].sum()
    assert a[0].min() > 0.5


def test_blast_waves_solve_until_the_collision(ctx):
    """TEST 5 at a reduced grid with the CFL step to t = 0.025, shortly before the two
    blast waves collide (about t = 0.027, where the scheme as read here turns the
    pressure between the shocks negative, in the oracle alike), against the oracle."""
    c = W.blast_waves(200)
    g, p = grid_params(c)
    u = to_dev(c.u)
    t, k = wt.wenotheta_solve(ctx, g, p, u, 0.025)
    ref, t_ref, k_ref = oracle.solve(oracle_problem(c), c.u, 0.025)
    assert (t, k) == (t_ref, k_ref) and t == 0.025
    assert np.array_equal(u.cpu().numpy(), ref)


def test_batched_problems_with_walls(ctx):
    import torch
    B = W.batched_1d(seed=7, nprob=24, nmin=40, nmax=600)
    B.bc[::2] = W.REFLECTIVE
    u = to_dev(B.u)
    st = torch.full((B.nprob,), -1, dtype=torch.int32, device="cuda")
    p = wt.Params(system=wt.WT_EULER, alpha_R=B.alpha_R, cfl=B.cfl)
    wt.wenotheta_solve_batched(ctx, p, u, B.n, B.offset, B.lo, B.hi, B.bc, 12, status_out=st)
    wt.wenotheta_sync(ctx)
    got, st = u.cpu().numpy(), st.cpu().numpy()
    for b in range(B.nprob):
        o, n = int(B.offset[b]), int(B.n[b])
        P = oracle.Problem(ndim=1, system=oracle.EULER, n=(n,), dx=((B.hi[b] - B.lo[b]) / n,),
                           bc=(int(B.bc[b]),), gamma=B.gamma, cfl=B.cfl, alpha_R=B.alpha_R)
        try:
            ref, _, _ = oracle.solve(P, B.u[:, o:o + n], math.inf, max_steps=12)
        except oracle.OracleError:
            assert st[b] != 0
            continue
        assert st[b] == 0 and np.array_equal(got[:, o:o + n], ref), b


def test_wall_and_gravity_arguments(ctx):
    import torch
    c = W.sod(64)
    g, p = grid_params(c)
    u = to_dev(c.u)
    L = torch.empty_like(u)
    for grav in ((0.0, 1.0, 0.0), (math.nan, 0.0, 0.0)):
        p.gravity = grav
        with pytest.raises(wt.WenoThetaError) as e:
            wt.wenotheta_rhs(ctx, g, p, u, L)
        assert e.value.code == 1
    s = W.scalar_modes(0, 64)
    gs, ps = grid_params(s)
    gs.bc = (wt.WT_REFLECTIVE,)
    us = to_dev(s.u)
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_rhs(ctx, gs, ps, us, torch.empty_like(us))
    assert e.value.code == 2
    B = W.batched_1d(seed=1, nprob=4, nmin=20, nmax=40)
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_solve_batched(ctx, wt.Params(system=wt.WT_EULER, gravity=(1.0, 0, 0)),
                                   to_dev(B.u), B.n, B.offset, B.lo, B.hi, B.bc, 1)
    assert e.value.code == 2
