"""Exact solution of the one-dimensional Riemann problem of the Euler
equations for an ideal gas (test infrastructure only).

The textbook construction (e.g. Toro, Riemann Solvers and Numerical Methods
for Fluid Dynamics, ch. 4): the star-region pressure p* is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the velocity jump across a
shock (p > p_K, Rankine-Hugoniot) or a rarefaction (p <= p_K, isentropic);
the solution is self-similar in x/t and is sampled wave by wave.  Written
from those definitions; it shares nothing with the solver or its oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma=1.4):
    """p*, u* of the Riemann problem between primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = lambda p: _f(p, rl, pl, gamma) + _f(p, rr, pr, gamma) + (ur - ul)
    hi = 10.0 * max(pl, pr)
    while g(hi) < 0:
        hi *= 10.0
    ps = brentq(g, 1e-14 * min(pl, pr), hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, gamma) - _f(ps, rl, pl, gamma))
    return ps, us


def sample(left, right, xi, gamma=1.4):
    """Primitive fields (rho, u, p) of the self-similar solution at x/t = xi
    (array), the discontinuity initially at x = 0."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    gm, gp = gamma - 1.0, gamma + 1.0
    xi = np.asarray(xi, dtype=np.float64)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    for n, s in enumerate(xi.ravel()):
        if s <= us:  # left of the contact
            if ps > pl:
                sl = ul - al * math.sqrt(gp / (2 * gamma) * ps / pl + gm / (2 * gamma))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    w = (rl * (ps / pl + gm / gp) / (gm / gp * ps / pl + 1.0), us, ps)
            else:
                a_star = al * (ps / pl) ** (gm / (2 * gamma))
                if s <= ul - al:
                    w = (rl, ul, pl)
                elif s >= us - a_star:
                    w = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    uf = 2.0 / gp * (al + gm / 2.0 * ul + s)
                    af = 2.0 / gp * (al + gm / 2.0 * (ul - s))
                    w = (rl * (af / al) ** (2.0 / gm), uf, pl * (af / al) ** (2.0 * gamma / gm))
        else:  # right of the contact
            if ps > pr:
                sr = ur + ar * math.sqrt(gp / (2 * gamma) * ps / pr + gm / (2 * gamma))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    w = (rr * (ps / pr + gm / gp) / (gm / gp * ps / pr + 1.0), us, ps)
            else:
                a_star = ar * (ps / pr) ** (gm / (2 * gamma))
                if s >= ur + ar:
                    w = (rr, ur, pr)
                elif s <= us + a_star:
                    w = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    uf = 2.0 / gp * (-ar + gm / 2.0 * ur + s)
                    af = 2.0 / gp * (ar - gm / 2.0 * (ur - s))
                    w = (rr * (af / ar) ** (2.0 / gm), uf, pr * (af / ar) ** (2.0 * gamma / gm))
        rho.flat[n], u.flat[n], p.flat[n] = w
    return rho, u, p


def shock_speed(left, right, gamma=1.4):
    """Speed of the right-running shock (requires p* > p_R)."""
    rr, ur, pr = right
    ps, _ = star_state(left, right, gamma)
    ar = math.sqrt(gamma * pr / rr)
    return ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
