"""GPU parity: the HIP library (through its C ABI) against the oracle on the same
seeded inputs.

Bar (floating point): per RHS evaluation max-relative error <= 1e-12, at final
time <= 1e-10, max-relative meaning max |gpu - oracle| / max |oracle| per
component.  The kernels evaluate every quantity with the oracle's sequence of
IEEE operations, so the results are expected to be bit-identical, and the tests
assert that as well: it is the evidence that no theta / restriction decision
flipped.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import (assert_parity, gpu_rhs, gpu_solve, gpu_steps, grid_params,
                              oracle_problem, to_dev)

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
FINAL_TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _check_rhs(ctx, case, alpha_R=None, f=None, alpha=None, what=""):
    P = oracle_problem(case, alpha_R=alpha_R)
    ref = oracle.rhs(P, case.u, f=f, alpha_=alpha)
    got = gpu_rhs(ctx, case, f=f, alpha=alpha, alpha_R=alpha_R)
    err, exact = assert_parity(got, ref, RHS_TOL, what or case.name)
    assert exact, f"{what or case.name}: within tolerance ({err:.2e}) but not bit-identical"


# ---------------------------------------------------------------------------
# Scalar
# ---------------------------------------------------------------------------

def _scalar_case(n, seed, system=W.LINEAR, rough=False, bc=W.PERIODIC, a=1.0):
    rng = np.random.default_rng(seed)
    if rough:
        u = rng.normal(size=n)
    else:
        u = W.scalar_modes(seed, n).u[0]
    c = W.Case("scalar", system, u[None].copy(), (-1.0,), (1.0,), (bc,), a=a)
    return c


@pytest.mark.parametrize("n", [6, 7, 200, 255, 256, 257, 1000])
@pytest.mark.parametrize("alpha_R", [50.0, 0.0, math.inf])
def test_rhs_linear(ctx, n, alpha_R):
    for rough in (False, True):
        _check_rhs(ctx, _scalar_case(n, n, rough=rough), alpha_R=alpha_R,
                   what=f"linear n={n} aR={alpha_R} rough={rough}")


@pytest.mark.parametrize("a", [-1.7, 0.0])
def test_rhs_linear_speed_and_transmissive(ctx, a):
    _check_rhs(ctx, _scalar_case(300, 3, rough=True, bc=W.TRANSMISSIVE, a=a), what=f"a={a}")


@pytest.mark.parametrize("n", [64, 511])
def test_rhs_burgers_and_caller_flux(ctx, n):
    c = _scalar_case(n, 11, system=W.BURGERS, rough=True)
    _check_rhs(ctx, c, what="burgers")
    P = oracle_problem(c)
    al, _ = oracle.alpha(P, c.u)
    f = 0.5 * c.u * c.u
    _check_rhs(ctx, c, f=f, alpha=al, what="burgers caller flux")
    # a flux the library does not know: f = u^3 / 3 with alpha = max u^2
    f3 = c.u ** 3 / 3.0
    _check_rhs(ctx, c, f=f3, alpha=[float((c.u ** 2).max())], what="cubic caller flux")


# ---------------------------------------------------------------------------
# Euler RHS
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [6, 255, 256, 511, 4096])
@pytest.mark.parametrize("seed", [0, 1])
def test_rhs_euler1d_seeded(ctx, n, seed):
    _check_rhs(ctx, W.euler1d_seeded(seed, n))


@pytest.mark.parametrize("make", [W.sod, W.lax, W.problem_123, W.shu_osher])
def test_rhs_euler1d_paper_problems(ctx, make):
    _check_rhs(ctx, make(300))
    _check_rhs(ctx, W.euler1d_smooth_periodic(4, 300), what="smooth periodic")


@pytest.mark.parametrize("shape", [(6, 6), (37, 64), (64, 37), (100, 100), (257, 33)])
def test_rhs_euler2d(ctx, shape):
    nx, ny = shape
    rng = np.random.default_rng(nx * 1000 + ny)
    states = [(rng.uniform(0.1, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1),
               rng.uniform(0.03, 1.5)) for _ in range(4)]
    c = W.quadrants_2d(states, nx, ny=ny, split=0.37)
    _check_rhs(ctx, c, what=f"quadrants {shape}")
    for aR in (0.0, math.inf):
        _check_rhs(ctx, c, alpha_R=aR, what=f"quadrants {shape} aR={aR}")
    s = W.euler2d_smooth_periodic(nx, 32)
    _check_rhs(ctx, s, what="smooth periodic 2D")


def _blocks_3d(shape, seed, bc):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    blk = (xx * 3 // nx) + 3 * (yy * 2 // ny) + 6 * (zz * 2 // nz)
    rho = rng.uniform(0.2, 2.0, 12)[blk]
    vel = [rng.uniform(-1, 1, 12)[blk] for _ in range(3)]
    p = rng.uniform(0.2, 2.0, 12)[blk]
    u = W.conserved(rho, vel, p)
    return W.Case("blocks3d", W.EULER, u, (0.0,) * 3, (1.0,) * 3, (bc,) * 3)


@pytest.mark.parametrize("shape", [(6, 6, 6), (20, 17, 9), (9, 33, 40)])
def test_rhs_euler3d(ctx, shape):
    _check_rhs(ctx, _blocks_3d(shape, sum(shape), W.TRANSMISSIVE), what=f"blocks {shape}")
    _check_rhs(ctx, _blocks_3d(shape, 7, W.PERIODIC), what=f"periodic blocks {shape}")


def test_rhs_euler3d_vortex(ctx):
    _check_rhs(ctx, W.euler3d_seeded(0, n=24), what="vortex 24^3")


# ---------------------------------------------------------------------------
# Steps and solves
# ---------------------------------------------------------------------------

def _check_steps(ctx, case, nsteps, dt=0.0):
    P = oracle_problem(case)
    ref = case.u
    for _ in range(nsteps):
        ref, _ = oracle.step(P, ref, dt)
    got = gpu_steps(ctx, case, nsteps, dt=dt)
    err, exact = assert_parity(got, ref, FINAL_TOL, f"{case.name} {nsteps} steps")
    assert exact, f"{case.name}: {err:.2e} but not bit-identical"


def test_steps_scalar(ctx):
    _check_steps(ctx, _scalar_case(200, 1), 25)
    _check_steps(ctx, _scalar_case(257, 2, system=W.BURGERS, rough=True), 10)
    _check_steps(ctx, _scalar_case(64, 3), 5, dt=(2 / 64) ** 2)


def test_steps_euler(ctx):
    _check_steps(ctx, W.euler1d_seeded(2, 777), 10)
    _check_steps(ctx, W.euler2d_seeded(3, 70), 4)
    _check_steps(ctx, _blocks_3d((14, 12, 10), 5, W.TRANSMISSIVE), 2)


def test_solve_scalar_workload(ctx):
    """The 1D scalar workload in full: N = 200, CFL 0.5, t_end = 2 (400 steps)."""
    c = W.scalar_modes(seed=0, n=200)
    P = oracle_problem(c)
    ref, t_ref, k_ref = oracle.solve(P, c.u, 2.0)
    got, t, k = gpu_solve(ctx, c, 2.0)
    assert (t, k) == (t_ref, k_ref) == (2.0, 400)
    err, exact = assert_parity(got, ref, FINAL_TOL, "scalar workload")
    assert exact


def test_solve_sod_paper_setup(ctx):
    """Sod's problem as in Sec. 4.2: N = 300, t = 1.7."""
    c = W.sod(300)
    P = oracle_problem(c)
    ref, t_ref, k_ref = oracle.solve(P, c.u, 1.7)
    got, t, k = gpu_solve(ctx, c, 1.7)
    assert t == t_ref == 1.7 and k == k_ref
    err, exact = assert_parity(got, ref, FINAL_TOL, "sod")
    assert exact


def test_solve_euler1d_seeded_reduced(ctx):
    c = W.euler1d_seeded(0, 2048)
    P = oracle_problem(c)
    ref, t_ref, k_ref = oracle.solve(P, c.u, 0.02)
    got, t, k = gpu_solve(ctx, c, 0.02)
    assert t == t_ref and k == k_ref
    err, exact = assert_parity(got, ref, FINAL_TOL, "euler1d seeded N=2048")
    assert exact


def test_solve_test8_reduced(ctx):
    c = W.test8_quadrants(48)
    P = oracle_problem(c)
    ref, t_ref, k_ref = oracle.solve(P, c.u, 0.05)
    got, t, k = gpu_solve(ctx, c, 0.05)
    assert t == t_ref and k == k_ref
    err, exact = assert_parity(got, ref, FINAL_TOL, "test8 48^2")
    assert exact
    assert np.array_equal(got[0], got[0].T) and np.array_equal(got[1], got[2].T)


def test_solve_max_steps_and_resume(ctx):
    c = W.lax(200)
    a, ta, ka = gpu_solve(ctx, c, 0.3)
    g, p = grid_params(c)
    ud = to_dev(c.u)
    t1, k1 = wt.wenotheta_solve(ctx, g, p, ud, 0.3, max_steps=5)
    assert k1 == 5 and t1 < 0.3
    t2, k2 = wt.wenotheta_solve(ctx, g, p, ud, 0.3, t0=t1)
    assert t2 == ta and k1 + k2 == ka
    assert np.array_equal(ud.cpu().numpy(), a)


# ---------------------------------------------------------------------------
# Full-size workloads (the configurations the benchmark times)
# ---------------------------------------------------------------------------

def test_full_size_euler1d_rhs_and_step(ctx):
    """1D Euler workload at full size, N = 65536: every output of one RHS and one step."""
    c = W.euler1d_seeded(0, 65536)
    _check_rhs(ctx, c, what="euler1d N=65536")
    _check_steps(ctx, c, 1)


def test_full_size_euler2d_rhs_sampled(ctx):
    """2D Euler workload at full size, 4096^2: RHS at sampled points (random, the
    quadrant boundaries, the domain edges and corners), each computed by the oracle."""
    n = 4096
    c = W.euler2d_seeded(0, n)
    got = gpu_rhs(ctx, c)
    rng = np.random.default_rng(0)
    pts = set(rng.integers(0, n * n, 1500).tolist())
    for j in (0, 1, 2, 3, n // 2 - 2, n // 2 - 1, n // 2, n // 2 + 1, n - 3, n - 2, n - 1):
        for i in rng.integers(0, n, 8).tolist() + [0, n - 1, n // 2 - 1, n // 2]:
            pts.add(j * n + i)
            pts.add(i * n + j)
    cells = np.array(sorted(pts), dtype=np.int64)
    P = oracle_problem(c)
    ref = oracle.rhs_points(P, c.u, cells)
    g = got.reshape(4, -1)[:, cells].T
    scale = np.abs(ref).max(axis=0)
    err = (np.abs(g - ref).max(axis=0) / scale).max()
    assert err <= RHS_TOL and np.array_equal(g, ref), err


def _full_size_step(ctx, c, precision):
    """One CFL step of a full-size workload in its tuned launch configuration, through
    the solver's captured step graph; returns the state and the step taken."""
    import torch
    g, p = grid_params(c)
    p.precision = precision
    ud = to_dev(c.u)
    wt.wenotheta_tune(ctx, g, p, ud)
    t, k = wt.wenotheta_solve(ctx, g, p, ud, math.inf, max_steps=1)
    assert k == 1
    got = ud.cpu().numpy()
    del ud
    torch.cuda.empty_cache()
    return got, t


def _check_fast_step(got, ref, what):
    """The fast FP64 mode after one step: within the final-time bar (1e-10 max-relative per
    component) and 1e-13 in L1, a component that vanishes in exact arithmetic (the
    z-momentum of a flow uniform in z) measured against 1e-3 of the largest; the cells over
    1e-12 (decisions flipped at near-ties) are counted."""
    m = ref.shape[0]
    a, b = got.reshape(m, -1), ref.reshape(m, -1)
    mx = np.abs(b).max(axis=1)
    rel = np.abs(a - b) / np.maximum(mx, 1e-3 * mx.max())[:, None]
    sb = np.abs(b).sum(axis=1)
    l1 = np.abs(a - b).sum(axis=1) / np.maximum(sb, 1e-3 * sb.max())
    print(f"{what} fast step: max-rel {rel.max():.2e}, L1 {l1.max():.2e}, "
          f"{int((rel > 1e-12).any(axis=0).sum())} cells over 1e-12", flush=True)
    assert rel.max() <= FINAL_TOL and l1.max() <= 1e-13


def test_full_size_euler2d_step_in_the_benchmark_configuration(ctx):
    """The benchmark's workload (seed 1, 4096^2) in its launch configuration (tuned tiles,
    the solver's captured step graph): one CFL step in FP64 equals the oracle's whole step,
    every output bit for bit; the fast FP64 mode (the benchmark's headline) is within the
    final-time bar of it."""
    c = W.euler2d_seeded(1, 4096)
    ref, dt = oracle.step(oracle_problem(c), c.u)
    got, t = _full_size_step(ctx, c, wt.WT_FP64)
    assert t == dt and np.array_equal(got, ref)
    got, _ = _full_size_step(ctx, c, wt.WT_FP64_FAST)
    _check_fast_step(got, ref, "euler2d 4096^2")


def test_full_size_euler3d_step_in_the_benchmark_configuration(ctx):
    """The 3D workload (seed 0, 512^3) in its launch configuration (tuned tiles, the step
    graph): one CFL step in FP64 equals the oracle's whole step (about half a minute on
    the host threads), all 671 M outputs bit for bit; the fast FP64 mode is within the
    final-time bar of it."""
    c = W.euler3d_seeded(0, 512)
    print("euler3d 512^3: oracle step ...", flush=True)
    ref, dt = oracle.step(oracle_problem(c), c.u)
    got, t = _full_size_step(ctx, c, wt.WT_FP64)
    assert t == dt and np.array_equal(got, ref)
    got, _ = _full_size_step(ctx, c, wt.WT_FP64_FAST)
    _check_fast_step(got, ref, "euler3d 512^3")


def test_full_size_euler3d_rhs_sampled(ctx):
    """3D Euler workload at full size, 512^3 (the launch configuration the benchmark
    times): RHS at sampled points -- random, on the sphere surfaces and through the
    vortex centre, on the periodic faces, edges and corners -- each computed by the
    oracle, bit for bit."""
    import torch
    n = 512
    c = W.euler3d_seeded(0, n)
    got = gpu_rhs(ctx, c)
    rng = np.random.default_rng(3)
    pts = set(rng.integers(0, n ** 3, 600).tolist())
    # steepest density gradients (sphere fronts) and the vortex centre line
    rho = c.u[0]
    gx = np.abs(np.roll(rho, -1, axis=2) - rho)
    steep = np.argpartition(gx.ravel(), -200)[-200:]
    pts.update(steep.tolist())
    xc, yc = c.extra["xc"], c.extra["yc"]
    ic, jc = int(xc * n), int(yc * n)
    for k in rng.integers(0, n, 20).tolist():
        pts.add((k * n + jc) * n + ic)
    for k in (0, n - 1):
        for j in (0, 1, n - 2, n - 1):
            for i in (0, 2, n - 3, n - 1):
                pts.add((k * n + j) * n + i)
    del gx
    cells = np.array(sorted(pts), dtype=np.int64)
    ref = oracle.rhs_points(oracle_problem(c), c.u, cells)
    g = got.reshape(5, -1)[:, cells].T
    assert np.array_equal(g, ref)
    torch.cuda.empty_cache()


def test_full_size_euler2d_symmetry_and_free_stream(ctx):
    """At 4096^2: diagonal-symmetric quadrant data stay exactly symmetric over two steps,
    and a constant state is preserved (to the ulp the printed stage form allows)."""
    import torch
    n = 4096
    c = W.euler2d_seeded(5, n, symmetric=True)
    g, p = grid_params(c)
    ud = to_dev(c.u)
    for _ in range(2):
        wt.wenotheta_step(ctx, g, p, ud)
    wt.wenotheta_sync(ctx)
    assert torch.equal(ud[0], ud[0].T) and torch.equal(ud[1], ud[2].T) and torch.equal(ud[3], ud[3].T)
    del ud
    const = W.conserved(np.full((n, n), 0.7), [0.3, -0.2], 1.1)
    u0 = to_dev(const)
    L = torch.empty_like(u0)
    wt.wenotheta_rhs(ctx, g, p, u0, L)
    wt.wenotheta_sync(ctx)
    assert int(torch.count_nonzero(L)) == 0


# ---------------------------------------------------------------------------
# Errors, determinism
# ---------------------------------------------------------------------------

def test_errors(ctx):
    import torch
    c = W.sod(64)
    g, p = grid_params(c)
    bad = c.u.copy()
    bad[0, 10] = -1.0
    ud = to_dev(bad)
    wt.wenotheta_step(ctx, g, p, ud)
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_sync(ctx)
    assert e.value.code == 3
    bad = c.u.copy()
    bad[2, 7] = np.nan
    ud = to_dev(bad)
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_solve(ctx, g, p, ud, 0.1)
    assert e.value.code == 4
    # the context recovers after the error was reported
    ud = to_dev(c.u)
    wt.wenotheta_step(ctx, g, p, ud)
    wt.wenotheta_sync(ctx)
    # argument errors are synchronous
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_step(ctx, wt.Grid(n=(5,), lo=(0.0,), hi=(1.0,), bc=(1,)), p,
                          to_dev(c.u[:, :5]))
    assert e.value.code == 1
    with pytest.raises(wt.WenoThetaError) as e:
        wt.wenotheta_rhs(ctx, g, wt.Params(system=wt.WT_EULER, gamma=1.0), ud, torch.empty_like(ud))
    assert e.value.code == 1


def test_deterministic(ctx):
    c = W.euler2d_seeded(9, 96)
    a = gpu_steps(ctx, c, 3)
    b = gpu_steps(ctx, c, 3)
    assert np.array_equal(a, b)
