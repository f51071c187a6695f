"""GPU checks of the kernels' device arithmetic through libwt_probe.so, which
applies the sweep kernels' own division, reciprocal, square-root and WENO-theta
routines elementwise: every quotient, reciprocal and root must equal the IEEE
(correctly rounded) result computed on the host, and the FP64 WENO-theta must
equal the oracle's bit for bit, over millions of inputs including hard cases."""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
from paper_1504_00731_amd import build as B

pytestmark = pytest.mark.gpu

DIV, RECIP, DIV_BY_RECIP, SQRT, WENO, WENO_FP32, RCP_FAST, RCP_ESTIMATE, WENO_FAST, RSQ_FAST, SQRT_FAST = range(11)


@pytest.fixture(scope="module")
def probe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    if not os.path.exists(B.PROBE_LIB):
        raise RuntimeError(f"{B.PROBE_LIB} is missing: build the libraries first")
    L = ctypes.CDLL(B.PROBE_LIB)
    vp = ctypes.c_void_p
    L.wt_probe.argtypes = [ctypes.c_int, vp, vp, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, vp, ctypes.c_int64, vp]
    L.wt_probe.restype = ctypes.c_int

    def run(op, a=None, b=None, c=(0.0, 0.0, 0.0)):
        n = (len(a) // 6 if op in (WENO, WENO_FP32, WENO_FAST) else len(a)) if a is not None else len(b)
        da = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() if a is not None else None
        db = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).cuda() if b is not None else None
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        rc = L.wt_probe(op, da.data_ptr() if da is not None else None,
                        db.data_ptr() if db is not None else None, *c, out.data_ptr(), n,
                        torch.cuda.current_stream().cuda_stream)
        assert rc == 0, rc
        torch.cuda.synchronize()
        return out.cpu().numpy()
    return run


def _same(got, want):
    """Bitwise equality (NaNs compared by position)."""
    gb, wb = got.view(np.int64), want.view(np.int64)
    bad = np.nonzero(gb != wb)[0]
    return bad


def _hard_significands(rng, n):
    """Values whose significands sit next to powers of two or are all ones."""
    k = rng.integers(1, 1 << 20, n).astype(np.float64)
    e = rng.integers(-40, 40, n)
    up = np.ldexp(1.0 + k * 2.0 ** -52, e)
    down = np.ldexp(2.0 - k * 2.0 ** -52, e)
    return np.concatenate([up, down])


def test_division_is_correctly_rounded(probe):
    rng = np.random.default_rng(11)
    n = 2_000_000
    a = rng.normal(size=n) * np.exp(rng.uniform(-300, 300, n))
    b = np.exp(rng.uniform(-300, 300, n))
    a = np.concatenate([a, _hard_significands(rng, n // 4), [float.fromhex("0x1.6666666666663p-2")]])
    b = np.concatenate([b, _hard_significands(rng, n // 4)[::-1], [float.fromhex("0x1.ffffffffffffbp-4")]])
    bad = _same(probe(DIV, a, b), a / b)
    assert bad.size == 0, [(a[i].hex(), b[i].hex()) for i in bad[:5]]


def test_reciprocal_is_correctly_rounded(probe):
    rng = np.random.default_rng(12)
    b = np.concatenate([np.exp(rng.uniform(-690, 690, 3_000_000)), _hard_significands(rng, 500_000),
                        np.ldexp(np.ones(41), np.arange(-1000, 1001, 50))])
    bad = _same(probe(RECIP, b=b), 1.0 / b)
    assert bad.size == 0, [b[i].hex() for i in bad[:5]]


@pytest.mark.parametrize("eps", [1e-10, 1e-6, 1e-40])
def test_restricted_quotient_is_correctly_rounded(probe, eps):
    rng = np.random.default_rng(13)
    tau = np.concatenate([np.exp(rng.uniform(-700, 700, 1_000_000)), _hard_significands(rng, 200_000),
                          [0.0, 5e-324, 1e-310, 2.0 ** -900, 1e-300, 1e300, 1.7e308]])
    got = probe(DIV_BY_RECIP, tau, c=(eps, 1.0 / eps, 0.0))
    with np.errstate(over="ignore"):
        want = tau / eps
    bad = _same(got, want)
    assert bad.size == 0, [tau[i].hex() for i in bad[:5]]


def test_square_root_is_correctly_rounded(probe):
    rng = np.random.default_rng(14)
    x = np.concatenate([np.exp(rng.uniform(-700, 700, 2_000_000)), _hard_significands(rng, 500_000)])
    bad = _same(probe(SQRT, x), np.sqrt(x))
    assert bad.size == 0, [x[i].hex() for i in bad[:5]]


def _stencils(rng, n):
    """Six-point stencils of several kinds: smooth (polynomial + sine), with one jump,
    constant, near-constant, and random."""
    x = np.arange(6) - 2.5
    kinds = []
    m = n // 5
    c = rng.normal(size=(m, 4))
    h = np.exp(rng.uniform(-8, 0, (m, 1)))
    kinds.append(c[:, :1] + c[:, 1:2] * h * x + c[:, 2:3] * (h * x) ** 2 + c[:, 3:4] * np.sin(h * x))
    jump = rng.integers(1, 6, m)
    base = rng.normal(size=(m, 1)) + 0.01 * rng.normal(size=(m, 6))
    kinds.append(base + (np.arange(6)[None, :] >= jump[:, None]) * rng.normal(size=(m, 1)) * 3)
    kinds.append(np.repeat(rng.normal(size=(m, 1)), 6, axis=1))
    kinds.append(rng.normal(size=(m, 1)) * (1 + 1e-12 * rng.normal(size=(m, 6))))
    kinds.append(rng.normal(size=(n - 4 * m, 6)) * np.exp(rng.uniform(-5, 5, (n - 4 * m, 1))))
    return np.concatenate(kinds)


def test_weno_theta_matches_oracle(probe):
    """The device WENO-theta (restricted tau/eps from RN(1/eps), the shared reciprocal of
    sum alpha, the Markstein weights) equals the oracle's plain evaluation bit for bit."""
    rng = np.random.default_rng(15)
    S = _stencils(rng, 200_000)
    for eps, aR in ((1e-10, 50.0), (1e-10, 10.0), (1e-6, 0.0)):
        got = probe(WENO, S.ravel(), c=(eps, aR, 1.0 / eps))
        want = np.array([oracle.weno_theta(s, eps, aR) for s in S])
        bad = _same(got, want)
        assert bad.size == 0, (eps, aR, [S[i].tolist() for i in bad[:3]])


def test_weno_fp32_reconstruction_accuracy(probe):
    """FP32 weights against the oracle's FP64 value.  The FP32 rounding of the weights
    (about 2^-24 relative) moves the flux by that fraction of the spread of the candidate
    fluxes, which is of the order of the stencil's spread max|s_k - s_2|, while the FP64
    parts carry rounding of order 2^-50 of max|s_k|: the difference is measured against
    the sum of the two.  Constant stencils are restricted and reconstruct to s_2 exactly
    (the linear reconstruction is formed as (s_2 + s_3)/2 plus differences, all zero), so
    a constant region's flux differences vanish and constant states stay exact (checked by
    the solver tests).  A theta or
    restriction decision lying within rounding of its threshold (about 1 in 10^5 of these
    stencils) may differ more."""
    rng = np.random.default_rng(16)
    S = _stencils(rng, 100_000)
    got = probe(WENO_FP32, S.ravel(), c=(1e-10, 50.0, 0.0))
    want = np.array([oracle.weno_theta(s) for s in S])
    spread = np.abs(S - S[:, 2:3]).max(axis=1)
    const = spread == 0
    assert const.sum() > 1000 and np.array_equal(got[const], S[const, 2])
    scale = spread * 2.0 ** -24 + np.abs(S).max(axis=1) * 2.0 ** -50
    ratio = np.abs(got - want) / scale
    assert np.percentile(ratio, 99.9) <= 4.0, np.percentile(ratio, 99.9)
    assert (ratio > 16.0).mean() <= 1e-4, (ratio > 16.0).mean()


def _positive_normals(rng, n):
    """Positive normal values of exponents -500 .. 500 and hard significands."""
    e = rng.integers(-500, 500, n)
    return np.concatenate([np.ldexp(rng.uniform(1.0, 2.0, n), e), _hard_significands(rng, n // 4)])


def test_fast_reciprocal_within_one_ulp(probe):
    """The fast modes' reciprocal (hardware estimate refined by two Newton steps) against
    the IEEE reciprocal: within one unit in the last place.  The bare estimate's
    relative error is printed and bounded: it is what two Newton steps (error e -> e^2
    each) have to bring below 2^-53."""
    rng = np.random.default_rng(21)
    b = _positive_normals(rng, 400_000)
    want = 1.0 / b
    got = probe(RCP_FAST, b=b)
    ulps = np.abs(got - want) / np.spacing(want)
    est = probe(RCP_ESTIMATE, b=b)
    rel = float(np.max(np.abs(est - want) / want))
    print(f"rcp_fast: max {ulps.max():.2f} ulp, {(ulps > 0).mean():.2e} of the values not "
          f"correctly rounded; hardware estimate max relative error {rel:.3e} "
          f"(2^{math.log2(rel):.1f})", flush=True)
    assert ulps.max() <= 1.0, ulps.max()
    assert rel < 2.0 ** -13, rel


def test_fast_roots_within_two_ulps(probe):
    """The fast modes' reciprocal square root (hardware estimate refined by two Newton
    steps) against 1/sqrt(x) evaluated in extended precision, and their square root
    (x times it) against the IEEE square root: within two units in the last place over
    positive normal inputs of exponents -500 .. 500 and hard significands (the kernels
    take the roots of densities and squared sound speeds)."""
    rng = np.random.default_rng(23)
    b = _positive_normals(rng, 400_000)
    want = (1.0 / np.sqrt(b.astype(np.longdouble)))
    got = probe(RSQ_FAST, b=b)
    ulps = np.abs(got.astype(np.longdouble) - want) / np.spacing(want.astype(np.float64))
    sq = probe(SQRT_FAST, b=b)
    sq_ulps = np.abs(sq - np.sqrt(b)) / np.spacing(np.sqrt(b))
    print(f"rsq_fast: max {float(ulps.max()):.2f} ulp; sqrt_fast: max {sq_ulps.max():.2f} ulp, "
          f"{(sq_ulps > 0).mean():.2e} of the values not correctly rounded", flush=True)
    assert float(ulps.max()) <= 2.0, float(ulps.max())
    assert sq_ulps.max() <= 2.0, sq_ulps.max()


def test_weno_fast_matches_oracle_to_rounding(probe):
    """The fast FP64 reconstruction against the oracle over seeded stencils: the
    difference is rounding, of order 2^-52 of max|s_k|, except where a theta or
    restriction decision lies within rounding of its threshold (a legitimate flip,
    about 1 in 10^5 of these stencils).  Constant stencils reconstruct exactly (as in the
    FP32-weight form, which shares the restricted path)."""
    rng = np.random.default_rng(22)
    S = _stencils(rng, 100_000)
    got = probe(WENO_FAST, S.ravel(), c=(1e-10, 50.0, 0.0))
    want = np.array([oracle.weno_theta(s) for s in S])
    spread = np.abs(S - S[:, 2:3]).max(axis=1)
    const = spread == 0
    assert const.sum() > 1000 and np.array_equal(got[const], S[const, 2])
    ratio = np.abs(got - want) / (np.abs(S).max(axis=1) * 2.0 ** -52)
    print(f"weno_fast: 99.9th percentile {np.percentile(ratio, 99.9):.1f} x 2^-52 max|s|, "
          f"{(ratio > 1024).mean():.1e} over 1024", flush=True)
    assert np.percentile(ratio, 99.9) <= 64.0, np.percentile(ratio, 99.9)
    assert (ratio > 1024.0).mean() <= 1e-4, (ratio > 1024.0).mean()
