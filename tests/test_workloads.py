"""CPU checks that the seeded input generators follow their stated recipes: sizes and
layout of the packed batches, physical states, the quadrant structure, determinism."""
import numpy as np

from paper_1504_00731_amd import workloads as W


def _primitives(u):
    rho = u[0]
    vel = [u[1 + d] / rho for d in range(u.shape[0] - 2)]
    p = 0.4 * (u[-1] - 0.5 * rho * sum(v * v for v in vel))
    return rho, vel, p


def test_batched_1d_layout_and_ranges():
    B = W.batched_1d(seed=2, nprob=200)
    assert np.all((B.n >= 256) & (B.n <= 16384))
    assert B.offset[0] == 0 and np.array_equal(B.offset[1:], np.cumsum(B.n)[:-1])
    assert B.u.shape == (3, int(B.n.sum()))
    rho, (v,), p = _primitives(B.u)
    assert rho.min() >= 0.1 and rho.max() <= 4.0 and np.abs(v).max() <= 1.0 + 1e-12
    assert p.min() >= 0.1 - 1e-12 and p.max() <= 10.0 + 1e-12


def test_batched_2d_layout_ranges_and_quadrants():
    B = W.batched_2d(seed=4, nprob=120)
    assert np.all((B.nx >= 32) & (B.nx <= 96) & (B.ny >= 32) & (B.ny <= 96))
    assert len(set(zip(B.nx.tolist(), B.ny.tolist()))) > 100          # uneven sizes
    cells = B.nx * B.ny
    assert B.offset[0] == 0 and np.array_equal(B.offset[1:], np.cumsum(cells)[:-1])
    assert B.u.shape == (4, int(cells.sum()))
    assert B.lo.shape == B.hi.shape == B.bc.shape == (120, 2)
    for b in range(B.nprob):
        rho, (u, v), p = _primitives(B.problem(b))
        assert rho.min() >= 0.1 and rho.max() <= 1.5
        assert np.abs(u).max() <= 1.0 + 1e-12 and np.abs(v).max() <= 1.0 + 1e-12
        assert p.min() >= 0.03 - 1e-12 and p.max() <= 1.5 + 1e-12
        # four constant quadrants split at the middle of the cell-centred grid
        ny, nx = rho.shape
        for ys in (slice(0, ny // 2), slice(ny - ny // 2, ny)):
            for xs in (slice(0, nx // 2), slice(nx - nx // 2, nx)):
                q = B.problem(b)[:, ys, xs]
                assert np.all(q == q[:, :1, :1])


def test_generators_are_deterministic():
    a, b = W.batched_2d(seed=9, nprob=30), W.batched_2d(seed=9, nprob=30)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.nx, b.nx)
    c = W.batched_2d(seed=10, nprob=30)
    assert not np.array_equal(a.nx, c.nx)
    assert np.array_equal(W.euler2d_seeded(3, 64).u, W.euler2d_seeded(3, 64).u)
