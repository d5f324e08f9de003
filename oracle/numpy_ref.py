"""Second, independent implementation of the residual in NumPy (test only).

Whole-array form with periodic ``np.roll`` shifts instead of the C++
oracle's explicit index loops, used to cross-check those loops on tiny
blocks.  Same equations (Sec. 3 of the paper and the readings of the open
points), written again from them rather than from the C++ source.
"""
from __future__ import annotations

import numpy as np

_AXIS = {0: 2, 1: 1, 2: 0}   # direction xi/eta/zeta -> axis of a (nk, nj, ni) array


def _at(f, d, off):
    """f at node + off * e_d (periodic)."""
    return np.roll(f, -off, axis=_AXIS[d] + (f.ndim - 3))


def residual(dims, P, m, q) -> np.ndarray:
    ni, nj, nk = dims
    sh = (nk, nj, ni)
    Q = np.asarray(q, dtype=np.float64).reshape(5, *sh)
    M = np.asarray(m, dtype=np.float64).reshape(10, *sh)
    S = M[:9].reshape(3, 3, *sh)          # S[d, a]
    J = M[9]
    gam = P["gamma"]
    cp = 1.0 / (gam - 1.0)
    mu_inf = P["mach_j"] / P["re_d"] if np.isfinite(P["re_d"]) and P["re_d"] > 0 else 0.0

    rho = Q[0]
    vel = Q[1:4] / rho
    p = (gam - 1.0) * (Q[4] - 0.5 * rho * np.sum(vel * vel, axis=0))
    T = gam * p / rho
    a = np.sqrt(T)

    def grad(f):
        dd = np.stack([0.5 * (_at(f, d, 1) - _at(f, d, -1)) for d in range(3)])  # [d]
        return J * np.einsum("da...,d...->a...", S, dd)                          # [a]

    G = np.stack([grad(vel[0]), grad(vel[1]), grad(vel[2])])   # G[a, b] = du_a/dx_b
    gT = grad(T)
    mu = mu_inf * T ** 1.5 * (1.0 + P["sutherland_s"]) / (T + P["sutherland_s"])
    Sab = 0.5 * (G + np.swapaxes(G, 0, 1))
    smag = np.sqrt(2.0 * np.sum(Sab * Sab, axis=(0, 1)))
    delta = (1.0 / J) ** (1.0 / 3.0)
    mut = rho * (P["cs"] * delta) ** 2 * smag
    kap = cp * mu / P["prandtl"] + cp * mut / P["prandtl_t"]
    div = G[0, 0] + G[1, 1] + G[2, 2]
    eye = np.eye(3)[:, :, None, None, None]
    tau = (mu + mut) * (G + np.swapaxes(G, 0, 1) - 2.0 / 3.0 * eye * div)
    qh = -kap * gT

    # Cartesian flux columns E_c - V_c, c = x, y, z  -> EV[c, v]
    EV = np.empty((3, 5) + sh)
    for c in range(3):
        EV[c, 0] = rho * vel[c]
        for r in range(3):
            EV[c, 1 + r] = Q[1 + r] * vel[c] + (p if r == c else 0.0) - tau[r, c]
        EV[c, 4] = (Q[4] + p) * vel[c] - (np.sum(vel * tau[:, c], axis=0) - qh[c])
    F = np.einsum("dc...,cv...->dv...", S, EV)               # F[d, v]

    lam = np.stack([np.abs(J * np.einsum("a...,a...->...", S[d], vel))
                    + a * np.abs(J) * np.sqrt(np.sum(S[d] * S[d], axis=0)) for d in range(3)])
    sig = np.empty_like(lam)
    for d in range(3):
        phi = 1.0 + sum((lam[e] / lam[d]) ** P["tv_alpha"] for e in range(3) if e != d)
        sig[d] = phi * lam[d] / J

    C = np.zeros((5,) + sh)
    D = np.zeros((5,) + sh)
    for d in range(3):
        C += 0.5 * (_at(F[d], d, 1) - _at(F[d], d, -1))
        nu = np.abs(_at(p, d, 1) - 2 * p + _at(p, d, -1)) / (_at(p, d, 1) + 2 * p + _at(p, d, -1))
        # face flux at i+1/2 stored at node i
        eps2 = P["k2"] * np.maximum(nu, _at(nu, d, 1))
        eps4 = np.maximum(0.0, P["k4"] - eps2)
        sg = 0.5 * (sig[d] + _at(sig[d], d, 1))
        third = (_at(Q, d, 2) - _at(Q, d, -1)) - 3 * (_at(Q, d, 1) - Q)
        dface = sg * (eps2 * (_at(Q, d, 1) - Q) - eps4 * third)
        D += dface - _at(dface, d, -1)
    return (J * (C - D)).reshape(5, -1)
