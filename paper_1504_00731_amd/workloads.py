"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle tests.

This module only builds initial states (point values on the grid) and grid
descriptions; it holds none of the scheme's arithmetic.  Every generator is
seeded (``numpy.random.default_rng(seed)``) and draws its numbers in the
order documented in its docstring, so the same seed gives the same input on
every machine.

Grids: a periodic grid of n points is the vertex grid x_j = lo + j dx,
j = 0..n-1, dx = (hi - lo)/n (the paper's grid of Sec. 2, with x_n identified
with x_0); a non-periodic grid is cell-centred, x_j = lo + (j + 1/2) dx, so a
jump at the middle of the domain lies on an interface.

States are returned as float64 arrays of conserved variables, component-major
with x fastest: (m, n) in 1D, (m, ny, nx) in 2D, (m, nz, ny, nx) in 3D, with
components (rho, rho u, [rho v, [rho w,]] E).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, TRANSMISSIVE, REFLECTIVE, SIDES = 0, 1, 2, 3
STATE = 3                 # side part holding a given state
LINEAR, BURGERS, EULER = 0, 1, 2


@dataclass
class SideSpec:
    """One end of a dimension whose boundary condition is SIDES: rule kind[0]
    (TRANSMISSIVE, REFLECTIVE or STATE) on the grid lines whose coordinate along the
    next axis ((d + 1) mod ndim) is below split0 + split_speed * t, kind[1] on the
    others; a STATE part puts the conserved state state[part] into the ghost points."""
    kind: tuple = (TRANSMISSIVE, TRANSMISSIVE)
    state: tuple = ((), ())
    split0: float = math.inf
    split_speed: float = 0.0


@dataclass
class Case:
    """An initial state with its grid and scheme parameters."""
    name: str
    system: int
    u: np.ndarray
    lo: tuple
    hi: tuple
    bc: tuple
    gamma: float = 1.4
    cfl: float = 0.5
    alpha_R: float = 50.0
    a: float = 1.0
    t_end: float | None = None
    steps: int | None = None
    extra: dict = field(default_factory=dict)
    gravity: tuple = (0.0, 0.0, 0.0)
    sides: tuple | None = None    # 6 SideSpec [dim][lower, upper] where bc is SIDES

    @property
    def ndim(self) -> int:
        return self.u.ndim - 1

    @property
    def n(self) -> tuple:
        """Points per dimension, x first."""
        return tuple(reversed(self.u.shape[1:]))

    @property
    def dx(self) -> tuple:
        return tuple((self.hi[k] - self.lo[k]) / self.n[k] for k in range(self.ndim))


def grid_points(n: int, lo: float, hi: float, bc: int) -> np.ndarray:
    dx = (hi - lo) / n
    j = np.arange(n, dtype=np.float64)
    return lo + j * dx if bc == PERIODIC else lo + (j + 0.5) * dx


def conserved(rho, vel, p, gamma=1.4) -> np.ndarray:
    """Conserved variables (rho, rho*v..., E) from density, velocity list and pressure,
    with E = p/(gamma-1) + rho |v|^2 / 2 (ideal gas)."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    ke = sum(v * v for v in vel)
    E = p / (gamma - 1.0) + 0.5 * rho * ke
    return np.stack([rho] + [rho * v for v in vel] + [E])


# --------------------------------------------------------------------------
# Scalar workloads
# --------------------------------------------------------------------------

def scalar_modes(seed: int = 0, n: int = 200) -> Case:
    """1D linear advection u_t + u_x = 0 on [-1, 1], periodic, n points,
    u0 = sum_{k=1..3} A_k sin(k pi x + phi_k).  Draws: A_1..A_3 ~ U(0,1), then
    phi_1..phi_3 ~ U(0, 2 pi).  CFL 0.5, t_end = 2 (one period)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.0, 1.0, 3)
    phi = rng.uniform(0.0, 2.0 * np.pi, 3)
    x = grid_points(n, -1.0, 1.0, PERIODIC)
    u = sum(A[k] * np.sin((k + 1) * np.pi * x + phi[k]) for k in range(3))
    return Case("scalar_modes", LINEAR, u[None, :].copy(), (-1.0,), (1.0,), (PERIODIC,),
                t_end=2.0, extra={"A": A, "phi": phi})


def scalar_exact_modes(case: Case, t: float) -> np.ndarray:
    """Exact solution u0(x - t) of scalar_modes (period 2)."""
    n = case.n[0]
    x = grid_points(n, -1.0, 1.0, PERIODIC)
    A, phi = case.extra["A"], case.extra["phi"]
    return sum(A[k] * np.sin((k + 1) * np.pi * (x - case.a * t) + phi[k]) for k in range(3))


# --------------------------------------------------------------------------
# 1D Euler workloads
# --------------------------------------------------------------------------

def riemann_1d(left, right, n: int, lo=-5.0, hi=5.0, x0=0.0, gamma=1.4, name="riemann",
               t_end=None, alpha_R=50.0) -> Case:
    """Piecewise-constant primitive states (rho, u, p) left/right of x0,
    cell-centred transmissive grid."""
    x = grid_points(n, lo, hi, TRANSMISSIVE)
    L = x < x0
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    return Case(name, EULER, conserved(rho, [u], p, gamma), (lo,), (hi,), (TRANSMISSIVE,),
                gamma=gamma, t_end=t_end, alpha_R=alpha_R,
                extra={"left": tuple(left), "right": tuple(right), "x0": x0})


def sod(n=300) -> Case:
    """Sod's problem as set up in Sec. 4.2 (TEST 3), t = 1.7."""
    return riemann_1d((0.125, 0.0, 0.1), (1.0, 0.0, 1.0), n, name="sod", t_end=1.7)


def lax(n=300) -> Case:
    """Lax's problem of Sec. 4.2 (TEST 3), t = 1.3, alpha_R = 10."""
    return riemann_1d((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), n, name="lax", t_end=1.3,
                      alpha_R=10.0)


def problem_123(n=300) -> Case:
    """The 123 problem of Sec. 4.2 (TEST 3), t = 1."""
    return riemann_1d((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), n, name="123", t_end=1.0)


def shu_osher(n=200) -> Case:
    """Shock / density-wave interaction of Sec. 4.2 (TEST 4), zero-gradient BC, t = 1.8."""
    x = grid_points(n, -5.0, 5.0, TRANSMISSIVE)
    L = x < -4.0
    rho = np.where(L, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(L, 2.629369, 0.0)
    p = np.where(L, 31.0 / 3.0, 1.0)
    return Case("shu_osher", EULER, conserved(rho, [u], p), (-5.0,), (5.0,), (TRANSMISSIVE,),
                t_end=1.8)


def euler1d_seeded(seed: int = 0, n: int = 65536) -> Case:
    """Seeded Riemann data with a density wave on [-5, 5], transmissive, CFL 0.5,
    t_end = 0.2.  Draws: rho_L, p_L, u_L, rho_R, p_R, u_R with rho ~ U(0.1, 4),
    p ~ U(0.1, 10), u ~ U(-1, 2); then k ~ U(3, 8).  The right state's density
    carries the perturbation rho_R (1 + 0.2 sin(k x)) (multiplicative, so the
    density stays positive for rho_R down to 0.1)."""
    rng = np.random.default_rng(seed)
    rl, pl, ul = rng.uniform(0.1, 4.0), rng.uniform(0.1, 10.0), rng.uniform(-1.0, 2.0)
    rr, pr, ur = rng.uniform(0.1, 4.0), rng.uniform(0.1, 10.0), rng.uniform(-1.0, 2.0)
    k = rng.uniform(3.0, 8.0)
    x = grid_points(n, -5.0, 5.0, TRANSMISSIVE)
    L = x < 0.0
    rho = np.where(L, rl, rr * (1.0 + 0.2 * np.sin(k * x)))
    u = np.where(L, ul, ur)
    p = np.where(L, pl, pr)
    return Case("euler1d_seeded", EULER, conserved(rho, [u], p), (-5.0,), (5.0,),
                (TRANSMISSIVE,), t_end=0.2,
                extra={"left": (rl, ul, pl), "right": (rr, ur, pr), "k": k})


def euler1d_smooth_periodic(seed: int = 0, n: int = 256) -> Case:
    """Smooth periodic 1D Euler data on [0, 1] (for conservation checks).
    Draws: a_rho, a_u, a_p ~ U(0, 0.3), then phases ~ U(0, 2 pi) (3)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 0.3, 3)
    ph = rng.uniform(0.0, 2 * np.pi, 3)
    x = grid_points(n, 0.0, 1.0, PERIODIC)
    rho = 1.0 + amp[0] * np.sin(2 * np.pi * x + ph[0])
    u = 0.5 + amp[1] * np.sin(2 * np.pi * x + ph[1])
    p = 1.0 + amp[2] * np.sin(4 * np.pi * x + ph[2])
    return Case("euler1d_smooth", EULER, conserved(rho, [u], p), (0.0,), (1.0,), (PERIODIC,))


# --------------------------------------------------------------------------
# 2D Euler workloads
# --------------------------------------------------------------------------

def quadrants_2d(states, n, lo=0.0, hi=1.0, split=0.5, bc=TRANSMISSIVE, name="quadrants",
                 gamma=1.4, ny=None) -> Case:
    """Four constant primitive states (rho, u, v, p) for quadrants 1..4 (x>s,y>s),
    (x<s,y>s), (x<s,y<s), (x>s,y<s) as numbered in Sec. 4.3 (TEST 8)."""
    nx = n
    ny = n if ny is None else ny
    x = grid_points(nx, lo, hi, bc)[None, :]
    y = grid_points(ny, lo, hi, bc)[:, None]
    right, top = x > split, y > split
    q = np.where(top, np.where(right, 0, 1), np.where(right, 3, 2))
    S = np.asarray(states, dtype=np.float64)
    rho, u, v, p = (S[q, k] for k in range(4))
    return Case(name, EULER, conserved(rho, [u, v], p, gamma), (lo, lo), (hi, hi), (bc, bc),
                gamma=gamma, extra={"states": S})


def test8_quadrants(n=1000) -> Case:
    """The 2D Riemann configuration of Sec. 4.3 (TEST 8), t = 0.25."""
    states = [(0.5313, 0.0, 0.0, 0.4), (1.0, 0.7276, 0.0, 1.0), (0.8, 0.0, 0.0, 1.0),
              (1.0, 0.0, 0.7276, 1.0)]
    c = quadrants_2d(states, n, name="test8")
    c.t_end = 0.25
    return c


def euler2d_seeded(seed: int = 0, n: int = 4096, symmetric: bool = False) -> Case:
    """Seeded four-quadrant Riemann data on (0,1)^2, split at 0.5, transmissive,
    CFL 0.5, 200 steps.  Draws per quadrant 1..4 in order: rho ~ U(0.1, 1.5),
    u ~ U(-1, 1), v ~ U(-1, 1), p ~ U(0.03, 1.5).  symmetric=True then makes the
    data symmetric about the diagonal x = y: quadrant 4 becomes quadrant 2 with u
    and v exchanged, and quadrants 1 and 3 get v = u."""
    rng = np.random.default_rng(seed)
    S = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        p = rng.uniform(0.03, 1.5)
        S.append([rho, u, v, p])
    if symmetric:
        S[0][2] = S[0][1]
        S[2][2] = S[2][1]
        S[3] = [S[1][0], S[1][2], S[1][1], S[1][3]]
    c = quadrants_2d(S, n, name="euler2d_seeded" + ("_sym" if symmetric else ""))
    c.steps = 200
    return c


def euler2d_smooth_periodic(seed: int = 0, n: int = 64) -> Case:
    """Smooth periodic 2D data on (0,1)^2 (conservation checks).  Draws: amplitudes
    a_rho, a_u, a_v, a_p ~ U(0, 0.2), then phases ~ U(0, 2 pi) (4)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 0.2, 4)
    ph = rng.uniform(0.0, 2 * np.pi, 4)
    x = grid_points(n, 0.0, 1.0, PERIODIC)[None, :]
    y = grid_points(n, 0.0, 1.0, PERIODIC)[:, None]
    rho = 1.0 + amp[0] * np.sin(2 * np.pi * (x + y) + ph[0])
    u = 0.3 + amp[1] * np.sin(2 * np.pi * x + ph[1])
    v = -0.2 + amp[2] * np.sin(2 * np.pi * y + ph[2])
    p = 1.0 + amp[3] * np.sin(2 * np.pi * (x - y) + ph[3])
    return Case("euler2d_smooth", EULER, conserved(rho, [u, v], p), (0.0, 0.0), (1.0, 1.0),
                (PERIODIC, PERIODIC))


# --------------------------------------------------------------------------
# 3D Euler workload
# --------------------------------------------------------------------------

def euler3d_seeded(seed: int = 0, n: int = 512, nspheres: int = 8, edge: float = 2.0) -> Case:
    """Isentropic-vortex background in x-y, uniform in z, with spherical density
    jumps, on the periodic unit cube; CFL 0.5, 100 steps.
    Draws: centre (x_c, y_c) ~ U(0.25, 0.75)^2, strength beta ~ U(1, 5); then per
    sphere: centre ~ U(0,1)^3, radius ~ U(0.02, 0.1), density ratio ~ U(2, 10).
    Background (r = periodic distance to the centre / 0.1):
      rho = [1 - (gamma-1) beta^2/(8 gamma pi^2) e^{1-r^2}]^{1/(gamma-1)}, p = rho^gamma,
      (u, v, w) = (1, 1, 0) + beta/(2 pi) e^{(1-r^2)/2} (-dy, dx, 0)/0.1.
    Inside a sphere (periodic minimum image) rho is multiplied by the ratio, by the
    largest ratio where spheres overlap (so every density jump stays within the
    drawn range); p and the velocity are unchanged.  The sphere surface is a
    front of width edge * dx (tanh profile, edge = 2 by default; 0 gives the sharp
    jump): a sharp surface cut by grid lines leaves one-cell chords (a single
    dense cell between light ones) that the unlimited scheme turns into negative
    densities within a few steps."""
    g = 1.4
    rng = np.random.default_rng(seed)
    xc, yc = rng.uniform(0.25, 0.75, 2)
    beta = rng.uniform(1.0, 5.0)
    spheres = [(rng.uniform(0.0, 1.0, 3), rng.uniform(0.02, 0.1), rng.uniform(2.0, 10.0))
               for _ in range(nspheres)]
    x1 = grid_points(n, 0.0, 1.0, PERIODIC)

    def wrap(d):
        return d - np.round(d)

    dx2 = wrap(x1[None, :] - xc)
    dy2 = wrap(x1[:, None] - yc)
    r2 = (dx2 * dx2 + dy2 * dy2) / 0.01
    rho2 = (1.0 - (g - 1.0) * beta * beta / (8.0 * g * np.pi ** 2) * np.exp(1.0 - r2)) ** (1.0 / (g - 1.0))
    p2 = rho2 ** g
    fac = beta / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2)) / 0.1
    u2 = 1.0 - fac * dy2
    v2 = 1.0 + fac * dx2
    U = np.empty((5, n, n, n))
    for kz in range(n):
        z = x1[kz]
        fac_rho = np.ones_like(rho2)
        for (c, rad, ratio) in spheres:
            dz = wrap(z - c[2])
            if abs(dz) > rad + 4.0 * edge / n:
                continue
            d2 = wrap(x1[None, :] - c[0]) ** 2 + wrap(x1[:, None] - c[1]) ** 2 + dz * dz
            if edge > 0.0:
                w = edge / n
                inside = 0.5 * (1.0 - np.tanh((np.sqrt(d2) - rad) / (0.5 * w)))
                fac_rho = np.maximum(fac_rho, 1.0 + (ratio - 1.0) * inside)
            else:
                fac_rho = np.where(d2 < rad * rad, np.maximum(fac_rho, ratio), fac_rho)
        rho = rho2 * fac_rho
        U[:, kz] = conserved(rho, [u2, v2, np.zeros_like(u2)], p2, g)
    c = Case("euler3d_seeded", EULER, U, (0.0,) * 3, (1.0,) * 3, (PERIODIC,) * 3, steps=100,
             extra={"xc": xc, "yc": yc, "beta": beta})
    return c


# --------------------------------------------------------------------------
# Batched 1D Euler workload
# --------------------------------------------------------------------------

@dataclass
class Batch:
    """Independent 1D Euler problems packed back to back: u has shape (3, sum n_b);
    problem b occupies columns offset[b] .. offset[b] + n[b] - 1 on [lo[b], hi[b]]."""
    u: np.ndarray
    n: np.ndarray
    offset: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    bc: np.ndarray
    gamma: float = 1.4
    cfl: float = 0.5
    alpha_R: float = 50.0
    steps: int = 500

    @property
    def nprob(self) -> int:
        return int(self.n.size)

    def problem(self, b: int) -> np.ndarray:
        o, k = int(self.offset[b]), int(self.n[b])
        return self.u[:, o:o + k]


def batched_1d(seed: int = 0, nprob: int = 4096, nmin: int = 256, nmax: int = 16384,
               steps: int = 500) -> Batch:
    """Batched independent 1D Euler problems on [0, 1], cell-centred, transmissive.
    Draws per problem, in problem order: N_b = round(exp(U(ln nmin, ln nmax)));
    K_b ~ U{2..5} segments; K_b - 1 breakpoints ~ U(0, 1) (sorted); then per segment
    rho ~ U(0.1, 4), p ~ U(0.1, 10), u ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    ns, parts = [], []
    for _ in range(nprob):
        nb = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        nb = max(nb, 6)
        K = int(rng.integers(2, 6))
        bp = np.sort(rng.uniform(0.0, 1.0, K - 1))
        seg = [(rng.uniform(0.1, 4.0), rng.uniform(0.1, 10.0), rng.uniform(-1.0, 1.0))
               for _ in range(K)]
        x = grid_points(nb, 0.0, 1.0, TRANSMISSIVE)
        idx = np.searchsorted(bp, x)
        S = np.asarray(seg)
        rho, p, u = S[idx, 0], S[idx, 1], S[idx, 2]
        ns.append(nb)
        parts.append(conserved(rho, [u], p))
    n = np.asarray(ns, dtype=np.int64)
    offset = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    return Batch(u=np.ascontiguousarray(np.concatenate(parts, axis=1)), n=n, offset=offset,
                 lo=np.zeros(nprob), hi=np.ones(nprob),
                 bc=np.full(nprob, TRANSMISSIVE, dtype=np.int32), steps=steps)


@dataclass
class Batch2:
    """Independent 2D Euler problems packed back to back: u has shape (4, sum nx_b ny_b);
    problem b occupies columns offset[b] .. offset[b] + nx[b] ny[b] - 1 (x fastest) on
    [lo[b, 0], hi[b, 0]] x [lo[b, 1], hi[b, 1]] with boundary conditions bc[b, 0..1]."""
    u: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    offset: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    bc: np.ndarray
    gamma: float = 1.4
    cfl: float = 0.5
    alpha_R: float = 50.0
    steps: int = 100

    @property
    def nprob(self) -> int:
        return int(self.nx.size)

    def problem(self, b: int) -> np.ndarray:
        """State of problem b as (4, ny, nx)."""
        o, nx, ny = int(self.offset[b]), int(self.nx[b]), int(self.ny[b])
        return self.u[:, o:o + nx * ny].reshape(4, ny, nx)


def batched_2d(seed: int = 0, nprob: int = 4096, smin: int = 32, smax: int = 96,
               steps: int = 100) -> Batch2:
    """Batched independent 2D Euler problems on (0,1)^2, cell-centred, transmissive, each
    with the four-quadrant Riemann data of the 2D workload at its own uneven grid size.
    Draws per problem, in problem order: nx, ny = round(exp(U(ln smin, ln smax))) (x
    first), then per quadrant 1..4 rho ~ U(0.1, 1.5), u ~ U(-1, 1), v ~ U(-1, 1),
    p ~ U(0.03, 1.5); split at 0.5."""
    rng = np.random.default_rng(seed)
    nxs, nys, parts = [], [], []
    for _ in range(nprob):
        nx = max(int(round(np.exp(rng.uniform(np.log(smin), np.log(smax))))), 6)
        ny = max(int(round(np.exp(rng.uniform(np.log(smin), np.log(smax))))), 6)
        S = [[rng.uniform(0.1, 1.5), rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0),
              rng.uniform(0.03, 1.5)] for _ in range(4)]
        c = quadrants_2d(S, nx, ny=ny)
        nxs.append(nx)
        nys.append(ny)
        parts.append(c.u.reshape(4, -1))
    nx = np.asarray(nxs, dtype=np.int64)
    ny = np.asarray(nys, dtype=np.int64)
    offset = np.concatenate([[0], np.cumsum(nx * ny)[:-1]]).astype(np.int64)
    return Batch2(u=np.ascontiguousarray(np.concatenate(parts, axis=1)), nx=nx, ny=ny,
                  offset=offset, lo=np.zeros((nprob, 2)), hi=np.ones((nprob, 2)),
                  bc=np.full((nprob, 2), TRANSMISSIVE, dtype=np.int32), steps=steps)


# ---------------------------------------------------------------------------
# Reflective walls and gravity (Sec. 4.2 TEST 5, Sec. 4.3 TESTs 6 and 7)
# ---------------------------------------------------------------------------

def blast_waves(n: int = 801) -> Case:
    """Two interacting blast waves (Sec. 4.2, TEST 5): (rho, u, p) = (1, 0, 1000) on
    (0, 0.1), (1, 0, 0.01) on (0.1, 0.9), (1, 0, 100) on (0.9, 1); reflective walls at
    both ends; alpha_R = 10 (Sec. 4.2 sets 10 for this problem and Lax's); t = 0.038."""
    x = grid_points(n, 0.0, 1.0, REFLECTIVE)
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    u = conserved(np.ones(n), [np.zeros(n)], p)
    return Case("blast_waves", EULER, u, (0.0,), (1.0,), (REFLECTIVE,), t_end=0.038, alpha_R=10.0)


def rayleigh_taylor(nx: int = 120, ny: int = 360, g: float = 0.1) -> Case:
    """Rayleigh-Taylor instability (Sec. 4.3, TEST 6) on (-0.25, 0.25) x (-0.75, 0.75):
    rho = 2 for y >= 0, 1 below; p = 2.5 - rho g y; u = 0,
    v = 0.01/4 (1 + cos 4 pi x)(1 + cos 4 pi y / 3); periodic in x, reflective in y;
    gravity g = 0.1 along -y (source -g rho, -g rho v); t = 9.5."""
    x = grid_points(nx, -0.25, 0.25, PERIODIC)[None, :]
    y = grid_points(ny, -0.75, 0.75, REFLECTIVE)[:, None]
    rho = np.where(y >= 0.0, 2.0, 1.0) * np.ones_like(x)
    p = 2.5 - rho * g * y
    v = 0.01 / 4.0 * (1.0 + np.cos(4.0 * np.pi * x)) * (1.0 + np.cos(4.0 * np.pi * y / 3.0))
    u = conserved(rho, [np.zeros_like(rho), v], p)
    return Case("rayleigh_taylor", EULER, u, (-0.25, -0.75), (0.25, 0.75), (PERIODIC, REFLECTIVE),
                t_end=9.5, gravity=(0.0, g, 0.0))


def implosion(n: int = 400) -> Case:
    """Implosion problem (Sec. 4.3, TEST 7) on (0, 1)^2: (rho, p) = (1, 1) for
    x + y > 1/2, (0.125, 0.14) otherwise, at rest; reflective walls all round;
    alpha_R = 1; t = 5."""
    x = grid_points(n, 0.0, 1.0, REFLECTIVE)[None, :]
    y = grid_points(n, 0.0, 1.0, REFLECTIVE)[:, None]
    outer = (x + y) > 0.5
    rho = np.where(outer, 1.0, 0.125)
    p = np.where(outer, 1.0, 0.14)
    z = np.zeros_like(rho)
    u = conserved(rho, [z, z], p)
    return Case("implosion", EULER, u, (0.0, 0.0), (1.0, 1.0), (REFLECTIVE, REFLECTIVE),
                t_end=5.0, alpha_R=1.0)


def double_mach(nx: int = 800, ny: int = 200) -> Case:
    """Double Mach reflection of a Mach 10 shock (Sec. 4.3, TEST 9) on (0, 4) x (0, 1),
    t = 0.2 (the paper's grid is 800 x 200).  The shock leaves the bottom at
    x0 = 1/6 at 60 degrees to the x axis; behind it (x < x0 + y / tan 60)
    (rho, u, v, p) = (8, 8.25 cos 30, -8.25 sin 30, 116.5), ahead (1.4, 0, 0, 1).
    Sides: inflow of the post-shock state on the left, zero gradient on the right; at
    the bottom the post-shock state for x < x0 and a wall beyond; at the top the
    post-shock state for x < x_s(t) and the pre-shock state beyond, with
    x_s(t) = x0 + 1 / tan 60 + M_s a_pre t / cos 30 (M_s = 10, a_pre the pre-shock
    sound speed).  alpha_R = 10: the paper gives none for this problem, asks for a
    small one where there are shocks and takes 10 for its strongest 1D shocks (Sec.
    4.2); at the default 50 the first step already leaves a non-physical state."""
    gamma = 1.4
    x0 = 1.0 / 6.0
    c30, s30, t60 = math.cos(math.pi / 6.0), math.sin(math.pi / 6.0), math.tan(math.pi / 3.0)
    post = (8.0, 8.25 * c30, -8.25 * s30, 116.5)
    pre = (1.4, 0.0, 0.0, 1.0)
    a_pre = math.sqrt(gamma * pre[3] / pre[0])
    cons = lambda w: tuple(float(v) for v in conserved(w[0], [w[1], w[2]], w[3], gamma))
    U_post, U_pre = cons(post), cons(pre)
    x = grid_points(nx, 0.0, 4.0, TRANSMISSIVE)[None, :]
    y = grid_points(ny, 0.0, 1.0, TRANSMISSIVE)[:, None]
    behind = x < x0 + y / t60
    u = np.stack([np.where(behind, a, b) for a, b in zip(U_post, U_pre)])
    sides = (SideSpec((STATE, STATE), (U_post, U_post)),              # x = 0: inflow
             SideSpec((TRANSMISSIVE, TRANSMISSIVE)),                  # x = 4
             SideSpec((STATE, REFLECTIVE), (U_post, ()), split0=x0),  # y = 0
             SideSpec((STATE, STATE), (U_post, U_pre), split0=x0 + 1.0 / t60,
                      split_speed=10.0 * a_pre / c30),                 # y = 1
             SideSpec(), SideSpec())
    return Case("double_mach", EULER, u, (0.0, 0.0), (4.0, 1.0), (SIDES, SIDES), gamma=gamma,
                t_end=0.2, sides=sides, alpha_R=10.0,
                extra={"x0": x0, "post": post, "pre": pre, "mach": 10.0, "a_pre": a_pre})
