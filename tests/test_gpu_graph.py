"""The solver replays its steps from a captured HIP graph (kGraphSteps = 8 steps per
graph); with the profiler on it queues the same kernels eagerly.  Replays with eager
work and synchronisations in between must give exactly the eager result, for step
counts that are and are not multiples of the graph's length, and for a time-limited
solve whose last step is clipped."""
import math

import numpy as np
import pytest

import paper_1504_00731_amd as wt
from paper_1504_00731_amd import workloads as W
from tests.gpu_common import grid_params, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wt.Context(0)
    yield c
    c.close()


def _eager(ctx, case, **kw):
    g, p = grid_params(case)
    u = to_dev(case.u)
    wt.wenotheta_profile(ctx, True)            # the profiler forces the eager path
    t, k = wt.wenotheta_solve(ctx, g, p, u, kw.get("t_end", math.inf), max_steps=kw.get("max_steps", -1))
    wt.wenotheta_profile(ctx, False)
    return u.cpu().numpy(), t, k


@pytest.mark.parametrize("case_fn,kw", [
    (lambda: W.sod(300), {"max_steps": 13}),
    (lambda: W.sod(300), {"max_steps": 16}),
    (lambda: W.sod(300), {"t_end": 0.4}),
    (lambda: W.euler2d_seeded(0, 64), {"max_steps": 11}),
    (lambda: W.euler3d_seeded(0, 16), {"max_steps": 9}),
])
def test_graph_replays_match_eager(ctx, case_fn, kw):
    import torch
    case = case_fn()
    ref, t_ref, k_ref = _eager(ctx, case, **kw)
    g, p = grid_params(case)
    u0 = to_dev(case.u)
    u = u0.clone()
    for rep in range(4):
        u.copy_(u0)                                     # same buffers: the graph is reused
        junk = torch.randn(4096, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        t, k = wt.wenotheta_solve(ctx, g, p, u, kw.get("t_end", math.inf),
                                  max_steps=kw.get("max_steps", -1))
        assert (t, k) == (t_ref, k_ref), rep
        assert np.array_equal(u.cpu().numpy(), ref), rep
        del junk


def test_graph_follows_new_buffers_and_parameters(ctx):
    """A different state buffer, CFL number or grid is captured anew."""
    case = W.sod(200)
    g, p = grid_params(case)
    ref, _, _ = _eager(ctx, case, max_steps=10)
    for _ in range(2):
        u = to_dev(case.u)                              # a new buffer each time
        wt.wenotheta_solve(ctx, g, p, u, math.inf, max_steps=10)
        assert np.array_equal(u.cpu().numpy(), ref)
    p2 = wt.Params(system=p.system, gamma=p.gamma, cfl=0.4, alpha_R=p.alpha_R)
    u = to_dev(case.u)
    wt.wenotheta_profile(ctx, True)
    wt.wenotheta_solve(ctx, g, p2, u, math.inf, max_steps=10)
    wt.wenotheta_profile(ctx, False)
    ref2 = u.cpu().numpy()
    u = to_dev(case.u)
    wt.wenotheta_solve(ctx, g, p2, u, math.inf, max_steps=10)
    assert np.array_equal(u.cpu().numpy(), ref2)
    assert not np.array_equal(ref, ref2)
