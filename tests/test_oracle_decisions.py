"""Pins of the oracle's decision dump (theta and the restriction per reconstruction,
with margins in units of a rounding-error bound), used to account for legitimate
decision flips of evaluations with other rounding.

What fixes the expected values:
  * theta on smooth data: the Taylor expansions of tau_5 and tau_6 printed in
    Sec. 3.1 make tau_5 - tau_6 a positive-definite form at leading order, so
    theta = 0 everywhere, with a relative gap known in closed form;
  * the restriction on piecewise-constant data: R = max beta~ / (eps + min beta~)
    is 0 on a constant stencil and at least max beta~ / eps on a stencil with a
    jump (one of the four sub-stencils lies on one side of it, so min beta~ = 0);
  * the margins: a decision whose margin exceeds one unit is the decision of the
    exact (rational) evaluation of the same formulas on the same values, checked
    with Python fractions.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _plus_decisions(u, a=1.0, alpha_R=50.0):
    """Decisions of the + reconstructions of the scalar law f = a u on a periodic grid
    (a = 1: the + stencil values are the point values, the - ones are all zero)."""
    N = u.size
    P = oracle.linear_problem(N, a=a, alpha_R=alpha_R)
    dec, mar = oracle.decisions(P, u[None])
    return dec[0, 0, :, 0, :], mar[0, 0, :, 0, :]


@pytest.mark.parametrize("N,phase", [(160, 0.3), (320, 0.3), (320, 1.1), (640, 2.0)])
def test_theta_is_zero_on_smooth_data(N, phase):
    """Sec. 3.1's expansions about the interface x_{j+1/2}: with z = f3 / (f4 dx) there
    (f3, f4 the third and fourth derivatives), tau_5 - tau_6 = f4^2 dx^8 (z^2 + 1/12)
    + O(dx^9) and tau_5 = f4^2 dx^8 (z^2 + 13/12) + O(dx^9), a positive-definite gap:
    theta = 0 at every interface of smooth data, with the relative gap
    (tau_5 - tau_6) / tau_5 = (z^2 + 1/12) / (z^2 + 13/12), smallest (1/13) where f3
    vanishes."""
    x = -1.0 + np.arange(N) * (2.0 / N)
    u = np.sin(np.pi * x + phase)
    dec, mar = _plus_decisions(u)
    assert np.all(dec[:, 0] == 0)
    dx = 2.0 / N
    gaps, pred = [], []
    for i in range(-1, N):
        s = u[[(i - 2 + k) % N for k in range(6)]]
        d = oracle.weno_theta_diag(s, 1e-10, 50.0)
        gaps.append((d["tau5"] - d["tau6"]) / d["tau5"])
        xh = -1.0 + (i + 0.5) * dx
        f3 = -np.pi ** 3 * np.cos(np.pi * xh + phase)
        f4 = np.pi ** 4 * np.sin(np.pi * xh + phase)
        z2 = (f3 / (f4 * dx)) ** 2 if f4 != 0 else np.inf
        pred.append((z2 + 1 / 12) / (z2 + 13 / 12) if np.isfinite(z2) else 1.0)
    gaps, pred = np.array(gaps), np.array(pred)
    assert np.max(np.abs(gaps - pred)) < 20 * dx, np.max(np.abs(gaps - pred))
    # the interface nearest a zero of f3 has |z| <= 1/2: gap between 1/13 and 1/4
    assert 1 / 13 - 0.02 < gaps.min() < 0.25 + 0.02
    # the margins are far from a tie everywhere
    assert np.all(mar[:, 0] > 100)
    # the restriction holds everywhere on smooth data (all beta~_k ~ (f' dx)^2 alike,
    # and ~ f''^2 dx^4 alike where f' vanishes)
    assert np.all(dec[:, 1] == 1)
    # the - parts are zero stencils: a tie (theta = 1), restricted, no rounding can flip them
    P = oracle.linear_problem(N)
    d_all, m_all = oracle.decisions(P, u[None])
    assert np.all(d_all[0, 0, :, 0, 2] == 1) and np.all(d_all[0, 0, :, 0, 3] == 1)
    assert np.all(np.isinf(m_all[0, 0, :, 0, 2]))


def test_restriction_holds_exactly_on_constant_stencils():
    """Piecewise-constant data: restricted where the six points are equal, not where the
    stencil holds a jump (R >= max beta~ / eps there, far above alpha_R)."""
    rng = np.random.default_rng(7)
    N = 64
    levels = rng.choice([0.0, 1.0, 3.0, -2.5], size=6)
    u = np.repeat(levels, [7, 13, 9, 11, 10, 14])[:N]
    dec, _ = _plus_decisions(u)
    for i in range(-1, N):
        idx = [(i - 2 + k) % N for k in range(6)]
        const = np.all(u[idx] == u[idx[0]])
        assert dec[i + 1, 1] == (1 if const else 0), (i, u[idx])


def _exact(s, eps=1e-10):
    """tau_5, tau_6 and R of the stencil in exact rational arithmetic (Sec. 3.1)."""
    a, b, c, d, e, f = (Fraction(float(v)) for v in s)
    F = Fraction
    b0 = F(13, 12) * (a - 2 * b + c) ** 2 + (a - 3 * b + 2 * c) ** 2
    b1 = F(13, 12) * (b - 2 * c + d) ** 2 + (d - c) ** 2
    b2 = F(13, 12) * (c - 2 * d + e) ** 2 + (c - d) ** 2
    b3 = F(13, 48) * (3 * c - 7 * d + 5 * e - f) ** 2 + (2 * d - 3 * e + f) ** 2
    t5 = F(13, 12) * (a - 4 * b + 6 * c - 4 * d + e) ** 2 + (-b + 3 * c - 3 * d + e) ** 2
    t6 = F(13, 12) * (-a + 5 * b - 10 * c + 10 * d - 5 * e + f) ** 2 + \
        F(1, 4) * (a - 3 * b + 2 * c + 2 * d - 3 * e + f) ** 2
    R = max(b0, b1, b2, b3) / (Fraction(eps) + min(b0, b1, b2, b3))
    return t5, t6, R


def _near_tie_stencils(rng, n):
    """Stencils with tau_5 and tau_6 close: a smooth sample plus a multiple of a
    pattern, the multiple found by bisection on the sign of tau_6 - tau_5."""
    out = []
    pat = np.array([1.0, -5.0, 10.0, -10.0, 5.0, -1.0])
    while len(out) < n:
        base = np.sin(rng.uniform(0, 6) + np.arange(6) * rng.uniform(0.05, 0.6))
        def g(lam):
            d = oracle.weno_theta_diag(base + lam * pat, 1e-10, 50.0)
            return d["tau6"] - d["tau5"]
        lo, hi = 0.0, 1.0
        if g(lo) * g(hi) > 0:
            continue
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if g(lo) * g(mid) <= 0:
                hi = mid
            else:
                lo = mid
        out.append(base + lo * pat)
    return out


def test_margins_above_one_give_the_exact_decision():
    """A margin above one unit means the rounding of the oracle's own evaluation cannot
    have changed the decision: it equals the exact rational evaluation's.  Checked on
    random smooth and rough stencils and on stencils bisected to a theta tie (there the
    margins must be small, and only there may the decisions differ)."""
    rng = np.random.default_rng(11)
    stencils = [np.sin(rng.uniform(0, 6) + np.arange(6) * rng.uniform(0.001, 0.5))
                for _ in range(150)]
    stencils += [rng.normal(size=6) * 10.0 ** rng.integers(-6, 4) for _ in range(150)]
    ties = _near_tie_stencils(rng, 40)
    small = 0
    for k, s in enumerate(stencils + ties):
        u = np.roll(np.asarray(s, dtype=np.float64), 0)
        dec, mar = _plus_decisions(u)
        # interface i = 2 of the 6-point periodic grid: stencil points 0..5 in order
        th, rs, mth, mrs = dec[3, 0], dec[3, 1], mar[3, 0], mar[3, 1]
        t5, t6, R = _exact(s)
        if mth > 1.0:
            assert th == (0 if t6 < t5 else 1), (k, s, mth)
        if mrs > 1.0:
            assert rs == (1 if R <= 50 else 0), (k, s, mrs)
        if k >= len(stencils):
            small += mth < 1.0
    # the bisected ties sit within the rounding bound
    assert small >= 30, small


def test_decisions_cover_every_interface_of_each_direction():
    """Shape and consistency in 2D: per direction n + 1 interfaces per line, and the
    decisions of the x direction on data symmetric under x <-> y equal those of the y
    direction transposed (the two directions run one routine, Sec. 4.3 reading)."""
    from paper_1504_00731_amd import workloads as W
    case = W.euler2d_seeded(0, 24, symmetric=True)
    P = oracle.Problem(ndim=2, system=oracle.EULER, n=case.n, dx=case.dx, bc=case.bc)
    dx_, mx = oracle.decisions(P, case.u, direction=0)
    dy_, my = oracle.decisions(P, case.u, direction=1)
    assert dx_.shape == (1, 24, 25, 4, 4) and dy_.shape == (1, 25, 24, 4, 4)
    # transposing swaps the two directions; the shear field of each is its tangential
    assert np.array_equal(dx_[0], np.transpose(dy_[0], (1, 0, 2, 3)))
    assert np.array_equal(mx[0], np.transpose(my[0], (1, 0, 2, 3)))
    assert np.all(mx > 0)
