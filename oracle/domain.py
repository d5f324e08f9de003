"""Domain decomposition of one periodic block, on the CPU (test
infrastructure only: it checks the splitting rule, not the kernels).

The paper partitions the mesh along the axial and azimuthal directions into
parts of balanced size (Sec. 4.1: the node count divided by the number of
parts, the remainder spread over the parts) and gives each part a fringe of
two ghost layers at both ends of each split direction, since the
dissipation stencil reaches two nodes to either side (Sec. 4.3); the ghosts
are refreshed between Runge-Kutta stages so that no stage reads outdated
neighbour data.  Here every part is a padded block whose residual comes
from the oracle itself: with two ghost layers, no stencil of a node of the
part reaches past its padding, so treating the padded block as periodic
changes nothing at the part's own nodes.  The stage update
Q(k) = Q(0) - alpha_k dt R(Q(k-1)) and the CFL rule are the oracle's
(Sec. 3, time integration); the exchange after each stage copies, along
xi, the two last own layers of each part into the low ghosts of its upper
neighbour and the two first into the high ghosts of its lower neighbour
(periodic between the first and last part) over every zeta layer, then the
same along zeta over the whole padded xi width, which carries the corner
ghosts.  The result must be bitwise that of the unsplit oracle.
"""
from __future__ import annotations

import numpy as np

from . import core


def part_sizes(n: int, parts: int) -> list:
    """Balanced part lengths along one direction: n // parts each, the first
    n % parts parts one node longer (Sec. 4.1, balancing)."""
    if parts < 1 or n < 2 * parts:
        raise ValueError("every part needs at least two nodes")
    base, rem = divmod(n, parts)
    return [base + (1 if a < rem else 0) for a in range(parts)]


class _Part:
    def __init__(self, lo_i, len_i, lo_k, len_k, gi, gk):
        self.lo = (lo_i, lo_k)
        self.len = (len_i, len_k)
        self.g = (gi, gk)   # ghost layers along xi and zeta (2 when split, else 0)


def _pad_index(lo, ln, g, n):
    return np.arange(lo - g, lo + ln + g) % n


def advance(dims, params: core.Params, m, q, nsteps: int, parts=(1, 1), corners: bool = True):
    """nsteps steps of the block split into parts[0] x parts[1] parts along
    xi and zeta.  Returns (q_new, t, rms[5], linf[5]) like core.advance.
    corners=False leaves the corner ghosts stale (the zeta exchange then
    covers only the own xi nodes) -- a deliberately wrong variant that the
    tests use to show the corners matter."""
    ni, nj, nk = dims
    P = params
    if any(P.bc[f] != core.BC_PERIODIC for f in range(6)):
        raise ValueError("the split mirror takes periodic blocks")
    pi, pk = parts
    si, sk = part_sizes(ni, pi), part_sizes(nk, pk)
    oi = np.concatenate([[0], np.cumsum(si)[:-1]])
    ok = np.concatenate([[0], np.cumsum(sk)[:-1]])
    gi, gk = (2 if pi > 1 else 0), (2 if pk > 1 else 0)
    Q = np.asarray(q, dtype=np.float64).reshape(5, nk, nj, ni)
    M = np.asarray(m, dtype=np.float64).reshape(10, nk, nj, ni)

    parts_list = {}
    for c in range(pk):
        for a in range(pi):
            pt = _Part(oi[a], si[a], ok[c], sk[c], gi, gk)
            ii = _pad_index(oi[a], si[a], gi, ni)
            kk = _pad_index(ok[c], sk[c], gk, nk)
            pt.m = np.ascontiguousarray(M[:, kk][:, :, :, ii])
            pt.q = np.ascontiguousarray(Q[:, kk][:, :, :, ii])
            pt.dims = (len(ii), nj, len(kk))
            parts_list[(a, c)] = pt

    def own(pt):
        return (slice(None), slice(pt.g[1], pt.g[1] + pt.len[1]), slice(None),
                slice(pt.g[0], pt.g[0] + pt.len[0]))

    def exchange(arrs):
        if pi > 1:
            for c in range(pk):
                for a in range(pi):
                    dst, lo, hi = arrs[(a, c)], arrs[((a - 1) % pi, c)], arrs[((a + 1) % pi, c)]
                    nlo = lo.shape[3]
                    dst[:, :, :, 0:2] = lo[:, :, :, nlo - 4:nlo - 2]
                    dst[:, :, :, dst.shape[3] - 2:] = hi[:, :, :, 2:4]
        if pk > 1:
            for c in range(pk):
                for a in range(pi):
                    dst, lo, hi = arrs[(a, c)], arrs[(a, (c - 1) % pk)], arrs[(a, (c + 1) % pk)]
                    xs = slice(None) if corners else slice(gi, gi + si[a])
                    nlo = lo.shape[1]
                    dst[:, 0:2, :, xs] = lo[:, nlo - 4:nlo - 2, :, xs]
                    dst[:, dst.shape[1] - 2:, :, xs] = hi[:, 2:4, :, xs]

    t = 0.0
    ntot = ni * nj * nk
    rms = np.zeros(5)
    linf = np.zeros(5)
    for _ in range(nsteps):
        # dt from the CFL rule over every part (a maximum: the same value as
        # over the unsplit block)
        if P.dt_fixed > 0.0:
            dt = P.dt_fixed
        else:
            lmax = max(core.cfl_dt(pt.dims, P, pt.m.reshape(10, -1), pt.q.reshape(5, -1))[1]
                       for pt in parts_list.values())
            dt = P.cfl / lmax
        q0 = {key: pt.q.copy() for key, pt in parts_list.items()}
        qk = {key: pt.q.copy() for key, pt in parts_list.items()}
        for s in range(P.n_stages):
            ad = P.rk_alpha[s] * dt
            new = {}
            ss = np.zeros(5)
            mx = np.zeros(5)
            for key, pt in parts_list.items():
                r = core.residual(pt.dims, P, pt.m.reshape(10, -1), qk[key].reshape(5, -1))
                r = r.reshape(qk[key].shape)
                out = qk[key].copy()
                o = own(pt)
                out[o] = q0[key][o] - ad * r[o]
                new[key] = out
                if s == 0:
                    ro = r[o].reshape(5, -1)
                    ss += (ro * ro).sum(axis=1)
                    mx = np.maximum(mx, np.abs(ro).max(axis=1))
            if s == 0:
                rms = np.sqrt(ss / ntot)
                linf = mx
            exchange(new)
            qk = new
        for key, pt in parts_list.items():
            pt.q = qk[key]
        t += dt

    out = np.empty_like(Q)
    for (a, c), pt in parts_list.items():
        o = own(pt)
        out[:, ok[c]:ok[c] + sk[c], :, oi[a]:oi[a] + si[a]] = pt.q[o]
    return out.reshape(5, -1), t, rms, linf
