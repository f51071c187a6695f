"""wenotheta_rhs_noalloc (the right-hand side for callers that cannot allocate)
against wenotheta_rhs, through the C ABI: the same seeded inputs must give the
same L(u) bit for bit, on two calls in a row with the second on a smaller grid
(the fixed scratch buffer keeps the first call's contents), in 1D, 2D and 3D,
and when the call is captured into a graph and replayed.  Argument checks that
need no GPU are in tests/test_abi.py."""
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


def _quadrants(n, ny=None, seed=0):
    rng = np.random.default_rng(seed)
    q = [(rng.uniform(0.1, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.03, 1.5))
         for _ in range(4)]
    return W.quadrants_2d(q, n, ny=ny)


def _cases():
    """(name, first case, second smaller case) per dimension."""
    big1 = W.euler1d_seeded(3, 4099)
    small1 = W.euler1d_seeded(4, 700)
    sc1 = W.scalar_modes(1, 1000)
    sc2 = W.scalar_modes(2, 200)
    q1 = _quadrants(300, ny=260, seed=1)
    q2 = _quadrants(70, ny=45, seed=2)
    v1 = W.euler3d_seeded(5, 40)
    v2 = W.euler3d_seeded(6, 18)
    return [("scalar", sc1, sc2), ("euler1d", big1, small1), ("euler2d", q1, q2),
            ("euler3d", v1, v2)]


def _rhs_ctx(ctx, case):
    import torch
    g, p = grid_params(case)
    ud = to_dev(case.u)
    L = torch.empty_like(ud)
    wt.wenotheta_rhs(ctx, g, p, ud, L)
    wt.wenotheta_sync(ctx)
    return L.cpu().numpy()


def _rhs_noalloc(case):
    import torch
    g, p = grid_params(case)
    ud = to_dev(case.u)
    L = torch.full_like(ud, float("nan"))
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    wt.wenotheta_rhs_noalloc(g, p, ud, L, status=st)
    torch.cuda.synchronize()
    return L.cpu().numpy(), int(st.item())


_CASES = _cases()


@pytest.mark.parametrize("name,first,second", _CASES, ids=[c[0] for c in _CASES])
def test_noalloc_equals_rhs_on_two_calls(ctx, name, first, second):
    print(f"noalloc {name}: shapes {first.u.shape} then {second.u.shape}", flush=True)
    for case in (first, second):
        ref = _rhs_ctx(ctx, case)
        got, status = _rhs_noalloc(case)
        assert status == wt.binding.WT_OK, status
        assert np.array_equal(got, ref), f"{name} {case.u.shape}: not bit-identical"
    # the second, smaller call also equals the oracle
    P = oracle_problem(second)
    assert np.array_equal(got, oracle.rhs(P, second.u)), f"{name}: differs from the oracle"


@pytest.mark.parametrize("precision", [wt.WT_FP64_FAST, wt.WT_FP32_RECON], ids=["fast", "fp32"])
def test_noalloc_equals_rhs_in_the_other_precision_modes(ctx, precision):
    """The fast FP64 and FP32-weight forms through the allocation-free entry point equal
    wenotheta_rhs in the same mode bit for bit, two calls in a row (2D, then 3D smaller)."""
    import torch
    for case in (_quadrants(300, ny=260, seed=1), W.euler3d_seeded(6, 18)):
        g, p = grid_params(case)
        p.precision = precision
        ud = to_dev(case.u)
        L1 = torch.empty_like(ud)
        wt.wenotheta_rhs(ctx, g, p, ud, L1)
        wt.wenotheta_sync(ctx)
        L2 = torch.full_like(ud, float("nan"))
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        wt.wenotheta_rhs_noalloc(g, p, ud, L2, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == wt.binding.WT_OK
        assert torch.equal(L1, L2), case.u.shape


def test_noalloc_caller_speeds_and_flux_values(ctx):
    """The scalar law with caller-evaluated flux values and speed (the paper's problem
    statement), as wenotheta_rhs takes them."""
    import torch
    case = W.scalar_modes(3, 257)
    g, p = grid_params(case)
    ud = to_dev(case.u)
    f = to_dev(0.5 * case.u * case.u)
    al = [float(np.abs(case.u).max())]
    p = wt.Params(system=wt.WT_BURGERS)
    L1 = torch.empty_like(ud)
    L2 = torch.empty_like(ud)
    wt.wenotheta_rhs(ctx, g, p, ud, L1, f=f, alpha_host=al)
    wt.wenotheta_sync(ctx)
    wt.wenotheta_rhs_noalloc(g, p, ud, L2, f=f, alpha_host=al)
    torch.cuda.synchronize()
    assert torch.equal(L1, L2)


def test_noalloc_reports_nonphysical_state():
    """A negative pressure is reported through status_dev (and the next call, on a
    physical state, clears it)."""
    import torch
    case = _quadrants(64, seed=3)
    bad = case.u.copy()
    bad[3, 10, 10] = 1e-6                        # tiny energy: p < 0 there
    g, p = grid_params(case)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    L = torch.empty_like(to_dev(bad))
    wt.wenotheta_rhs_noalloc(g, p, to_dev(bad), L, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == wt.binding.WT_ERR_NONPHYSICAL
    _, status = _rhs_noalloc(case)
    assert status == wt.binding.WT_OK


def test_noalloc_graph_replays(ctx):
    """Captured into a graph: every replay, with eager work and synchronisations in
    between, gives the eager result."""
    import torch
    case = _quadrants(96, ny=80, seed=4)
    ref = _rhs_ctx(ctx, case)
    g, p = grid_params(case)
    ud = to_dev(case.u)
    L = torch.zeros_like(ud)
    wt.wenotheta_rhs_noalloc(g, p, ud, L)        # first call outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        wt.wenotheta_rhs_noalloc(g, p, ud, L, stream=s)
    other = W.scalar_modes(5, 300)
    for k in range(3):
        L.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(L.cpu().numpy(), ref), f"replay {k}"
        _rhs_noalloc(other)                       # eager work on the same scratch
