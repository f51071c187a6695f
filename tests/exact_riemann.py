"""Exact solution of the Riemann problem of the 1D Euler equations (ideal gas).

An independent reference for the shock-tube tests of Sec. 4.2 (Sod, Lax and
123 problems), which the paper measures against "the exact solution".  The
method is the classical one: the star-region pressure p* is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot)
branch for p > p_K and the rarefaction (isentropic) branch otherwise; the
solution is then sampled along rays x/t.  Written here from the textbook
derivation; it shares nothing with the oracle or the GPU library.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, gamma):
    """Velocity jump across the wave connecting state K with pressure p, and its derivative."""
    c = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    r = (p / pk) ** e
    return 2.0 * c / (gamma - 1.0) * (r - 1.0), (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * c)


def star_state(left, right, gamma=1.4):
    """p*, u* of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    # bracket and bisect-safeguarded Newton on f(p) = f_L + f_R + du
    def f(p):
        a, da = _fk(p, rl, pl, gamma)
        b, db = _fk(p, rr, pr, gamma)
        return a + b + (ur - ul), da + db
    lo, hi = 1e-14, max(pl, pr)
    while f(hi)[0] < 0.0:
        hi *= 2.0
    p = 0.5 * (lo + hi)
    for _ in range(200):
        val, der = f(p)
        if val > 0.0:
            hi = p
        else:
            lo = p
        pn = p - val / der if der > 0 else 0.5 * (lo + hi)
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= 1e-15 * max(p, 1e-300):
            p = pn
            break
        p = pn
    u = 0.5 * (ul + ur) + 0.5 * (_fk(p, rr, pr, gamma)[0] - _fk(p, rl, pl, gamma)[0])
    return p, u


def sample(left, right, xi, gamma=1.4):
    """Primitive variables (rho, u, p) on rays xi = x / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    vel = np.empty_like(xi)
    pre = np.empty_like(xi)
    for k, s in enumerate(xi.ravel()):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    r, v, q = rl, ul, pl
                else:
                    r = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                    v, q = us, ps
            else:  # left rarefaction
                cs = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                head, tail = ul - cl, us - cs
                if s <= head:
                    r, v, q = rl, ul, pl
                elif s >= tail:
                    r, v, q = rl * (ps / pl) ** (1 / gamma), us, ps
                else:
                    v = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + s)
                    c = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (gamma - 1))
                    q = pl * (c / cl) ** (2 * gamma / (gamma - 1))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    r, v, q = rr, ur, pr
                else:
                    r = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                    v, q = us, ps
            else:  # right rarefaction
                cs = cr * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                head, tail = ur + cr, us + cs
                if s >= head:
                    r, v, q = rr, ur, pr
                elif s <= tail:
                    r, v, q = rr * (ps / pr) ** (1 / gamma), us, ps
                else:
                    v = 2 / (gamma + 1) * (-cr + (gamma - 1) / 2 * ur + s)
                    c = 2 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (gamma - 1))
                    q = pr * (c / cr) ** (2 * gamma / (gamma - 1))
        rho.ravel()[k], vel.ravel()[k], pre.ravel()[k] = r, v, q
    return rho, vel, pre
