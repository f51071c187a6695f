"""CPU checks of the kernels' arithmetic, through a host build of the device
headers (no GPU): the finishing steps that make device division and square
root correctly rounded, and the per-interface flux / RHS operation sequence
against the oracle, bit for bit."""
import math

import numpy as np
import pytest

import oracle
from paper_1504_00731_amd import workloads as W
from tests import host_kernel as HK


def _neighbours(x):
    return [x, np.nextafter(x, np.inf), np.nextafter(x, -np.inf)]


def test_division_finish_recovers_the_nearest_quotient():
    """Given any faithful quotient (the nearest or either neighbour), the finishing
    step returns the IEEE quotient; includes the hard case met on the device."""
    rng = np.random.default_rng(0)
    cases = [(float.fromhex("0x1.6666666666663p-2"), float.fromhex("0x1.ffffffffffffbp-4"))]
    a = rng.normal(size=3000) * np.exp(rng.uniform(-40, 40, 3000))
    b = np.exp(rng.uniform(-40, 40, 3000))
    cases += list(zip(a.tolist(), b.tolist()))
    # divisors just below / above powers of two and numerators with long tails
    for k in range(1, 64):
        cases.append((0.35 * (1 - k * 2.0 ** -53), 0.125 * (1 - k * 2.0 ** -53)))
        cases.append((1.0 + k * 2.0 ** -52, 3.0 - k * 2.0 ** -51))
    for a_, b_ in cases:
        q = a_ / b_
        for qh in _neighbours(q):
            assert HK.div_finish(float(qh), a_, b_) == q, (a_, b_, qh, q)


def test_sqrt_finish_recovers_the_nearest_root():
    rng = np.random.default_rng(1)
    xs = np.exp(rng.uniform(-60, 60, 4000)).tolist()
    xs += [float(np.nextafter(4.0 ** k, 0)) for k in range(-5, 6)]
    xs += [float(np.nextafter(4.0 ** k, np.inf)) for k in range(-5, 6)]
    xs += [2.0, 0.125, 1.12, float.fromhex("0x1.ffffffffffffbp-4")]
    for x in xs:
        s = math.sqrt(x)
        for sh in _neighbours(s):
            assert HK.sqrt_finish(float(sh), x) == s, (x, sh, s)


def test_weno_operation_sequence_matches_oracle():
    rng = np.random.default_rng(2)
    for _ in range(3000):
        s = rng.normal(size=6) * rng.choice([1e-8, 1.0, 1e5])
        for aR in (50.0, 0.0, math.inf):
            assert HK.weno(s, 1e-10, aR) == oracle.weno_theta(s, 1e-10, aR)


def _compare(P, u):
    al, _ = oracle.alpha(P, u)
    ref = oracle.rhs(P, u)
    got, bad = HK.rhs(P, u, al)
    assert bad == 0
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [6, 37, 300])
def test_rhs_1d_matches_oracle(n):
    for seed in range(3):
        c = W.euler1d_seeded(seed, n)
        _compare(oracle.euler_problem(c.n, c.lo, c.hi), c.u)
    c = W.scalar_modes(0, n)
    P = oracle.linear_problem(n)
    al, _ = oracle.alpha(P, c.u)
    got, _ = HK.rhs(P, c.u, al)
    assert np.array_equal(got, oracle.rhs(P, c.u))


def test_rhs_2d_3d_match_oracle():
    c = W.euler2d_seeded(1, 40)
    _compare(oracle.euler_problem(c.n, c.lo, c.hi), c.u)
    c = W.euler2d_smooth_periodic(3, 24)
    _compare(oracle.euler_problem(c.n, c.lo, c.hi, bc=oracle.PERIODIC), c.u)
    c = W.euler3d_seeded(0, n=16)
    _compare(oracle.euler_problem(c.n, c.lo, c.hi, bc=oracle.PERIODIC), c.u)


def test_rhs_along_a_shock_tube_trajectory():
    """Sod's problem (Sec. 4.2), N = 300: every stage state of 40 oracle steps."""
    c = W.sod(300)
    P = oracle.euler_problem(c.n, c.lo, c.hi)
    u = c.u
    for _ in range(40):
        _compare(P, u)
        u, _ = oracle.step(P, u)


def test_restriction_threshold_band():
    """Stencils whose ratio R = max beta~ / (eps + min beta~) lies within a few ulps of
    alpha_R: the device's product pre-test must agree with the rounded quotient."""
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(60):
        base = rng.normal(size=6)
        direction = rng.normal(size=6)
        # find lam with R(lam) crossing alpha_R = 50 by bisection on the oracle's R
        R = lambda lam: oracle.weno_theta_diag(base + lam * direction, 1e-10, 50.0)["R"]
        lo, hi = 0.0, 1.0
        if (R(lo) - 50.0) * (R(hi) - 50.0) > 0:
            continue
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if (R(mid) - 50.0) * (R(lo) - 50.0) > 0:
                lo = mid
            else:
                hi = mid
        for lam in np.linspace(lo, hi, 5).tolist() + [np.nextafter(lo, -1), np.nextafter(hi, 2)]:
            s = base + lam * direction
            assert HK.weno(s, 1e-10, 50.0) == oracle.weno_theta(s, 1e-10, 50.0)
            checked += 1
    assert checked > 50


def test_markstein_quotients_on_hard_cases():
    """Quotients sharing a denominator use RN(1/b) and two FMA corrections; check them
    against IEEE division on numerators and denominators next to powers of two."""
    import math
    for ea in (-3, 0, 5):
        for eb in (-4, 3):
            for i in range(0, 120, 3):
                for j in range(1, 120, 5):
                    a = math.ldexp(1 + i * 2.0 ** -52, ea)
                    b = math.ldexp(1 - j * 2.0 ** -53, eb)
                    assert HK.div_by_recip(a, b, 1.0 / b) == a / b
    a_hard = float.fromhex("0x1.6666666666663p-2")
    b_hard = float.fromhex("0x1.ffffffffffffbp-4")
    assert HK.div_by_recip(a_hard, b_hard, 1.0 / b_hard) == a_hard / b_hard


def test_restricted_quotient_from_the_reciprocal_of_eps():
    """tau / eps in the restricted case is formed from RN(1/eps) with two FMA corrections
    where the first product is zero or normal and far from overflow, else by full division:
    equal to IEEE division for the paper's eps and others, over tau from 0 and subnormal to
    huge, including significands next to powers of two."""
    rng = np.random.default_rng(5)
    for eps in (1e-10, 1e-6, 1e-40, 3.0, float.fromhex("0x1.fffffffffffffp-34")):
        y = 1.0 / eps
        taus = [0.0, 5e-324, 1e-310, 2.0 ** -960, 1e-300, 1.0, 1e290, 1e300, 1.7e308]
        taus += [math.ldexp(1 + i * 2.0 ** -52, e) for i in range(0, 64) for e in (-40, -3, 0, 7, 60)]
        taus += [math.ldexp(1 - i * 2.0 ** -53, e) for i in range(1, 64) for e in (-20, 0, 30)]
        taus += list(np.exp(rng.uniform(-700, 700, 4000)))
        for tau in taus:
            got = HK.div_by_recip_checked(tau, eps, y)
            with np.errstate(over="ignore"):           # huge tau / small eps is inf on both
                want = tau / eps
            assert got == want or (math.isinf(got) and math.isinf(want)), (tau, eps, got, want)


def test_reciprocal_refinement_from_coarse_estimates():
    """The device reciprocal refines the hardware estimate with two Newton steps and the
    exact neighbour test: from any estimate within 2^-14 (relative) it must give RN(1/b).
    Estimates here are the nearest reciprocal perturbed by up to 2^-14, both ways, for b
    spread over [2^-1000, 2^1000] and b with all-ones or near-power-of-two significands."""
    rng = np.random.default_rng(6)
    bs = list(np.exp(rng.uniform(-690, 690, 3000)))
    bs += [math.ldexp(2 - k * 2.0 ** -52, e) for k in range(1, 40) for e in (-1000, -5, 0, 9, 999)]
    bs += [math.ldexp(1 + k * 2.0 ** -52, e) for k in range(0, 40) for e in (-3, 0, 11)]
    for b in bs:
        want = 1.0 / b
        for rel in (0.0, 2.0 ** -14, -(2.0 ** -14), 3e-6, -7e-9, 2.0 ** -40):
            assert HK.recip_refine(b, want * (1.0 + rel)) == want, (b, rel)


@pytest.mark.parametrize("make", [lambda: W.blast_waves(120), lambda: W.rayleigh_taylor(16, 48),
                                  lambda: W.implosion(24)])
def test_rhs_with_walls_and_gravity_matches_oracle(make):
    """Reflective walls and the gravity source through the kernels' arithmetic on the
    host: the RHS equals the oracle's bit for bit, also after the flow has moved."""
    from tests.gpu_common import oracle_problem
    c = make()
    P = oracle_problem(c)
    u = c.u
    for _ in range(2):
        al, _ = oracle.alpha(P, u)
        got, bad = HK.rhs(P, u, al)
        assert not bad
        assert np.array_equal(got, oracle.rhs(P, u, alpha_=al))
        u, _ = oracle.step(P, u)


def test_boundary_maps_stay_inside_the_line():
    """The kernels stage whole tiles (up to 261 points from 3 before the tile), which
    can reach far past the last ghost point of a short line: every boundary map must
    land inside the line for every such index, and on the ghost points -3..-1 and
    n..n+2 give the plain rule (wrap, nearest end point, mirror image with the flag).
    (A mirror 2n - 1 - i without the period 2n fell to -162 on a 48-point line.)"""
    for n in list(range(6, 40)) + [48, 100, 131, 255, 256, 300]:
        for bc in (0, 1, 2):
            for i in list(range(-300, -3)) + list(range(n + 3, n + 600, 7)):
                assert 0 <= HK.map_index(i, n, bc) < n, (n, bc, i)
            for i in list(range(-3, 0)) + list(range(n, n + 3)) + [0, 1, n - 1]:
                k = HK.map_index(i, n, bc)
                if bc == 0:
                    assert k == i % n
                elif bc == 1:
                    assert k == min(max(i, 0), n - 1)
                else:
                    want = -1 - i if i < 0 else (2 * n - 1 - i if i >= n else i)
                    assert k == want and HK.reflected(i, n, bc) == (i < 0 or i >= n)


@pytest.mark.parametrize("prec", [1, 2], ids=["fp32_recon", "fp64_fast"])
def test_fast_and_fp32_forms_close_to_oracle(prec):
    """The fast FP64 form (fused multiply-adds, fast reciprocals, linear weights taken
    exactly where the restriction holds) and the FP32-weight form, built for the host
    (its own rounding of those forms): L(u) within 1e-11 (fast FP64) or 1e-8 (weights
    from FP32: 1e-7 of the spread of the candidate fluxes where the restriction does not
    hold) of the oracle per component on 1D, 2D and 3D data with shocks (a component
    that vanishes in exact arithmetic is measured against 1e-3 of the largest), so the
    forms compute the same scheme."""
    tol = 1e-11 if prec == 2 else 1e-8
    cases = [(W.euler1d_seeded(1, 300), oracle.TRANSMISSIVE), (W.sod(200), oracle.TRANSMISSIVE),
             (W.euler2d_seeded(1, 40), oracle.TRANSMISSIVE),
             (W.euler2d_smooth_periodic(3, 24), oracle.PERIODIC),
             (W.euler3d_seeded(0, n=16), oracle.PERIODIC)]
    for c, bc in cases:
        P = oracle.euler_problem(c.n, c.lo, c.hi, bc=bc)
        al, _ = oracle.alpha(P, c.u)
        ref = oracle.rhs(P, c.u)
        got, bad = HK.rhs(P, c.u, al, prec=prec)
        assert bad == 0
        m = ref.shape[0]
        mx = np.abs(ref).reshape(m, -1).max(axis=1)
        scale = np.maximum(mx, 1e-3 * mx.max())
        err = (np.abs(got - ref).reshape(m, -1).max(axis=1) / scale).max()
        assert err <= tol, (c.name, err)
    # scalar law
    c = W.scalar_modes(0, 200)
    P = oracle.linear_problem(200)
    al, _ = oracle.alpha(P, c.u)
    got, _ = HK.rhs(P, c.u, al, prec=prec)
    ref = oracle.rhs(P, c.u)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_fast_restricted_reconstruction_is_the_linear_one():
    """Where the restriction holds, the weights are gamma^theta and the reconstruction is
    the linear one (Sec. 2): the 5th-order upwind form (theta = 1)
    (2 s0 - 13 s1 + 47 s2 + 27 s3 - 3 s4) / 60 or the 6th-order central form (theta = 0)
    (s0 - 8 s1 + 37 s2 + 37 s3 - 8 s4 + s5) / 60, here the gamma^theta-weighted sum of
    the four candidates in exact rational arithmetic.  The fast forms evaluate it from the
    indicators' second and fifth differences; on the side of the theta switch the oracle
    takes (decisions within 1e-9 of their threshold skipped), they must agree with the
    exact value to a few units of rounding of max|s_k|, and give constant stencils back
    exactly."""
    from fractions import Fraction as Fr
    cand = [[Fr(2, 6), Fr(-7, 6), Fr(11, 6), 0, 0, 0], [0, Fr(-1, 6), Fr(5, 6), Fr(2, 6), 0, 0],
            [0, 0, Fr(2, 6), Fr(5, 6), Fr(-1, 6), 0], [0, 0, 0, Fr(11, 6), Fr(-7, 6), Fr(2, 6)]]
    gamma = {0: [Fr(1, 20), Fr(9, 20), Fr(9, 20), Fr(1, 20)], 1: [Fr(2, 20), Fr(12, 20), Fr(6, 20), 0]}
    coef = {th: [sum(g[k] * cand[k][j] for k in range(4)) for j in range(6)] for th, g in gamma.items()}
    assert coef[1] == [Fr(2, 60), Fr(-13, 60), Fr(47, 60), Fr(27, 60), Fr(-3, 60), 0]
    assert coef[0] == [Fr(1, 60), Fr(-8, 60), Fr(37, 60), Fr(37, 60), Fr(-8, 60), Fr(1, 60)]
    rng = np.random.default_rng(31)
    x = np.arange(6) - 2.5
    seen = {0: 0, 1: 0}
    worst = 0.0
    for trial in range(3000):
        kind = trial % 3
        if kind == 0:       # smooth: polynomial plus a sine, of several scales and widths
            c = rng.normal(size=4) * 10.0 ** rng.uniform(-3, 3)
            h = math.exp(rng.uniform(-6, 0))
            s = c[0] + c[1] * h * x + c[2] * (h * x) ** 2 + c[3] * np.sin(h * x)
        elif kind == 1:     # near-constant
            s = rng.normal() * (1 + 1e-6 * rng.normal(size=6))
        else:               # constant
            s = np.full(6, rng.normal() * 10.0 ** rng.uniform(-5, 5))
        d = oracle.weno_theta_diag(s, 1e-10, 50.0)
        if not d["restricted"] or abs(d["R"] - 50.0) < 1e-9 * 50.0:
            continue
        if abs(d["tau5"] - d["tau6"]) <= 1e-9 * max(d["tau5"], d["tau6"]) and kind != 2:
            continue
        th = int(d["theta"])
        got = HK.weno_fast(s)
        if kind == 2:
            assert got == s[2], (s.tolist(), got)
        exact = sum(cj * Fr(float(v)) for cj, v in zip(coef[th], s))
        err = float(abs(Fr(got) - exact)) / (np.abs(s).max() * 2.0 ** -52)
        worst = max(worst, err)
        assert err <= 4.0, (th, s.tolist(), got, float(exact))
        seen[th] += 1
    print(f"restricted fast reconstructions: {seen}, worst {worst:.2f} x 2^-52 max|s|")
    assert seen[0] > 100 and seen[1] > 100, seen
