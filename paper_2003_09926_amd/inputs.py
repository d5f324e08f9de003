"""Seeded synthetic inputs for the jet LES hot path.

Grids (coordinates, periodic shift vectors, analytic metrics of separable
maps), initial conserved states and workload mixes.  Both the HIP path and the
CPU oracle receive their inputs from here, so this module holds none of the
solver's own arithmetic: no fluxes, no dissipation, no time stepping, no
metric differencing.  Every random number is drawn from a counter-based
generator (splitmix64, Steele, Lea and Flood, OOPSLA 2014) keyed by the seed,
the node's global linear index and the component, so a subsampled grid gets
exactly the subsampled perturbation field.

Layout conventions shared with the C-ABI:
  node (i, j, k) of an ni x nj x nk block sits at linear index
  i + ni * (j + nj * k)  (i = xi, the streamwise index, fastest);
  the conserved state is 5 x N FP64 structure-of-arrays
  [rho, rho u, rho v, rho w, e];
  the metric set is 10 x N FP64: m[3 d + a] = (d/dx_a of xi_d) / J for
  d, a in {0, 1, 2} and m[9] = J = 1 / det d(x, y, z)/d(xi, eta, zeta).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GAMMA = 1.4

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


# ----------------------------------------------------------------------------
# counter-based random numbers
# ----------------------------------------------------------------------------
def splitmix64(x) -> np.ndarray:
    """splitmix64 finaliser applied elementwise to uint64 counters."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counter) -> np.ndarray:
    """Uniform [0, 1) doubles from (seed, counter): 53 high bits of
    splitmix64(splitmix64(seed) + counter)."""
    key = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        v = splitmix64(np.asarray(counter, dtype=np.uint64) + key)
    return (v >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------
@dataclass
class Grid:
    """One structured block.  ``period[d]`` is the coordinate shift picked up
    when index d wraps once in the positive direction."""
    ni: int
    nj: int
    nk: int
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    period: np.ndarray
    metrics: Optional[np.ndarray] = None   # 10 x N analytic metrics, or None
    name: str = ""
    # 1-D axis positions for separable grids (used by initial conditions)
    axes: Optional[tuple] = None
    # exact mapping derivatives d x_a / d xi_d (3 x 3 x N), when known
    jacobian: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return self.ni * self.nj * self.nk

    @property
    def dims(self) -> tuple:
        return (self.ni, self.nj, self.nk)


def _broadcast(xa: np.ndarray, ya: np.ndarray, za: np.ndarray):
    """1-D axis arrays -> flat coordinate arrays in i-fastest order."""
    ni, nj, nk = xa.size, ya.size, za.size
    X = np.broadcast_to(xa[None, None, :], (nk, nj, ni)).ravel().copy()
    Y = np.broadcast_to(ya[None, :, None], (nk, nj, ni)).ravel().copy()
    Z = np.broadcast_to(za[:, None, None], (nk, nj, ni)).ravel().copy()
    return X, Y, Z


def _separable_metrics(dx: np.ndarray, dy: np.ndarray, dz: np.ndarray) -> np.ndarray:
    """Analytic metric set of x = X(xi), y = Y(eta), z = Z(zeta): the mapping
    matrix is diag(X', Y', Z'), so S^xi = (Y'Z', 0, 0), S^eta = (0, X'Z', 0),
    S^zeta = (0, 0, X'Y') and J = 1 / (X'Y'Z')."""
    ni, nj, nk = dx.size, dy.size, dz.size
    n = ni * nj * nk
    DX, DY, DZ = _broadcast(dx, dy, dz)
    m = np.zeros((10, n), dtype=np.float64)
    m[0] = DY * DZ
    m[4] = DX * DZ
    m[8] = DX * DY
    m[9] = 1.0 / (DX * DY * DZ)
    return m


def uniform_box(ni: int, nj: int, nk: int, lo=(0.0, -1.5, -1.5),
                size=(4.0, 3.0, 3.0), name: str = "uniform") -> Grid:
    """Uniform Cartesian periodic box: node i at lo_x + i * size_x / ni etc."""
    h = [size[0] / ni, size[1] / nj, size[2] / nk]
    xa = lo[0] + np.arange(ni, dtype=np.float64) * h[0]
    ya = lo[1] + np.arange(nj, dtype=np.float64) * h[1]
    za = lo[2] + np.arange(nk, dtype=np.float64) * h[2]
    X, Y, Z = _broadcast(xa, ya, za)
    period = np.diag(np.asarray(size, dtype=np.float64))
    m = _separable_metrics(np.full(ni, h[0]), np.full(nj, h[1]), np.full(nk, h[2]))
    return Grid(ni, nj, nk, X, Y, Z, period, m, name, axes=(xa, ya, za))


# face boundary types, indexed xi-, xi+, eta-, eta+, zeta-, zeta+
BC_PERIODIC, BC_INFLOW, BC_FARFIELD, BC_AXIS = 0, 1, 2, 3
# the jet domain: jet exit (supersonic inflow) at xi-, far field elsewhere
JET_DOMAIN_BC = (BC_INFLOW, BC_FARFIELD, BC_FARFIELD, BC_FARFIELD, BC_FARFIELD, BC_FARFIELD)
# the cylindrical jet mesh: jet exit at xi-, far field at the outflow and the
# lateral surface, the centreline at eta = 0, periodic azimuth
JET_CYLINDER_BC = (BC_INFLOW, BC_FARFIELD, BC_AXIS, BC_FARFIELD, BC_PERIODIC, BC_PERIODIC)


def bounded_box(ni: int, nj: int, nk: int, lo=(0.0, -1.5, -1.5), size=(4.0, 3.0, 3.0),
                bounded=(True, True, True), name: str = "bounded") -> Grid:
    """Uniform Cartesian block whose bounded directions carry nodes on both
    end faces (spacing size / (n - 1)); periodic directions keep spacing
    size / n and their period."""
    n = (ni, nj, nk)
    h = [size[d] / (n[d] - 1) if bounded[d] else size[d] / n[d] for d in range(3)]
    ax = [lo[d] + np.arange(n[d], dtype=np.float64) * h[d] for d in range(3)]
    X, Y, Z = _broadcast(*ax)
    period = np.diag([0.0 if bounded[d] else size[d] for d in range(3)])
    m = _separable_metrics(np.full(ni, h[0]), np.full(nj, h[1]), np.full(nk, h[2]))
    return Grid(ni, nj, nk, X, Y, Z, period, m, name, axes=tuple(ax))


def bounded_wavy_grid(ni: int, nj: int, nk: int, lo=(0.0, -1.5, -1.5), size=(4.0, 3.0, 3.0),
                      amp=(0.1, 0.08, 0.06), bounded=(True, True, True), name: str = "bounded-wavy") -> Grid:
    """Curvilinear block like ``wavy_grid`` whose bounded directions span
    [lo, lo + size] with nodes on both ends (the wave phase 2 pi i / (n - 1)
    there).  Coordinates only; ``jacobian`` holds the exact d x_a / d xi_d."""
    n = (ni, nj, nk)
    den = [n[d] - 1 if bounded[d] else n[d] for d in range(3)]
    h = np.asarray(size, dtype=np.float64) / np.asarray(den, dtype=np.float64)
    ii = np.arange(ni, dtype=np.float64)[None, None, :]
    jj = np.arange(nj, dtype=np.float64)[None, :, None]
    kk = np.arange(nk, dtype=np.float64)[:, None, None]
    w = [2 * np.pi / den[d] for d in range(3)]
    ti, tj, tk = w[0] * ii, w[1] * jj, w[2] * kk
    ax, ay, az = amp
    shp = (nk, nj, ni)
    X = np.broadcast_to(lo[0] + h[0] * ii + ax * np.sin(tj) * np.sin(tk), shp).ravel().copy()
    Y = np.broadcast_to(lo[1] + h[1] * jj + ay * np.sin(tk) * np.sin(ti), shp).ravel().copy()
    Z = np.broadcast_to(lo[2] + h[2] * kk + az * np.sin(ti) * np.sin(tj), shp).ravel().copy()
    jac = np.zeros((3, 3, ni * nj * nk))
    bc = lambda a: np.broadcast_to(a, shp).ravel()
    jac[0, 0] = h[0]
    jac[0, 1] = bc(ax * w[1] * np.cos(tj) * np.sin(tk))
    jac[0, 2] = bc(ax * np.sin(tj) * w[2] * np.cos(tk))
    jac[1, 0] = bc(ay * np.sin(tk) * w[0] * np.cos(ti))
    jac[1, 1] = h[1]
    jac[1, 2] = bc(ay * w[2] * np.cos(tk) * np.sin(ti))
    jac[2, 0] = bc(az * w[0] * np.cos(ti) * np.sin(tj))
    jac[2, 1] = bc(az * np.sin(ti) * w[1] * np.cos(tj))
    jac[2, 2] = h[2]
    period = np.diag([0.0 if bounded[d] else size[d] for d in range(3)])
    return Grid(ni, nj, nk, X, Y, Z, period, None, name, jacobian=jac)


def cylindrical_grid(ni: int, nj: int, nk: int, length: float = 4.0, radius: float = 1.5,
                     name: str = "cylinder") -> Grid:
    """Cylindrical mesh around the jet axis: xi axial (x = i length/(ni-1)),
    eta radial (r = j radius/(nj-1), j = 0 on the centreline), zeta azimuthal
    (theta = 2 pi k / nk, periodic with nk distinct points; the coordinates
    repeat exactly, so the period shift is zero).  ``metrics`` holds the exact
    metric set of the mapping: with h = (hx, hr, htheta) and
    det = hx hr r htheta, S^xi = (hr r htheta, 0, 0),
    S^eta = hx r htheta (0, cos, sin), S^zeta = hx hr (0, -sin, cos),
    J = 1/det (infinite on the axis, where the cells have no volume)."""
    hx, hr, ht = length / (ni - 1), radius / (nj - 1), 2.0 * np.pi / nk
    x = np.arange(ni, dtype=np.float64) * hx
    r = np.arange(nj, dtype=np.float64) * hr
    th = np.arange(nk, dtype=np.float64) * ht
    shp = (nk, nj, ni)
    X = np.broadcast_to(x[None, None, :], shp).ravel().copy()
    Y = np.broadcast_to(r[None, :, None] * np.cos(th)[:, None, None], shp).ravel().copy()
    Z = np.broadcast_to(r[None, :, None] * np.sin(th)[:, None, None], shp).ravel().copy()
    R = np.broadcast_to(r[None, :, None], shp).ravel()
    C = np.broadcast_to(np.cos(th)[:, None, None], shp).ravel()
    S = np.broadcast_to(np.sin(th)[:, None, None], shp).ravel()
    m = np.zeros((10, ni * nj * nk))
    m[0] = hr * R * ht
    m[4] = hx * R * ht * C
    m[5] = hx * R * ht * S
    m[7] = -hx * hr * S
    m[8] = hx * hr * C
    with np.errstate(divide="ignore"):
        m[9] = 1.0 / (hx * hr * R * ht)
    return Grid(ni, nj, nk, X, Y, Z, np.zeros((3, 3)), m, name, axes=(x, r, th))


def _sech2_map(n: int, s0: float, s1: float, centres, amp: float, width: float):
    """Nodes of a periodic 1-D map whose point density is
    g(s) = 1 + amp * sum_c sech^2((s - c) / width) on [s0, s1).
    Returns (positions, d position / d index)."""
    centres = np.asarray(centres, dtype=np.float64)

    def G(s):
        return (s - s0) + amp * width * np.sum(
            np.tanh((s[:, None] - centres[None, :]) / width)
            - np.tanh((s0 - centres[None, :]) / width), axis=1)

    def g(s):
        c = np.cosh((s[:, None] - centres[None, :]) / width)
        return 1.0 + amp * np.sum(1.0 / (c * c), axis=1)

    gtot = float(G(np.array([s1]))[0])
    target = np.arange(n, dtype=np.float64) * (gtot / n)
    lo = np.full(n, float(s0))
    hi = np.full(n, float(s1))
    for _ in range(64):    # bisection on the monotone map G(s) = target
        mid = 0.5 * (lo + hi)
        below = G(mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    s = 0.5 * (lo + hi)
    for _ in range(3):     # Newton polish to full FP64 accuracy
        s = s - (G(s) - target) / g(s)
    s[0] = s0
    return s, gtot / (n * g(s))


def stretched_jet_grid(ni: int, nj: int, nk: int, stride: int = 1) -> Grid:
    """Separable tanh-stretched periodic jet grid on [0,16) x [-4,4)^2.

    Radial (y, z): density clustered at |s| = r0 = 0.5 (amp 4, width 0.25);
    axial (x): clustered near the inflow plane x = 0 (and its periodic image
    x = 16; amp 3, width 1).  Positions come from Newton inversion of the
    integrated tanh map in FP64; metrics are the analytic derivatives.
    ``stride`` > 1 returns every stride-th node of the ni x nj x nk grid.
    """
    xa, dxa = _sech2_map(ni, 0.0, 16.0, (0.0, 16.0), 3.0, 1.0)
    ya, dya = _sech2_map(nj, -4.0, 4.0, (-0.5, 0.5), 4.0, 0.25)
    za, dza = _sech2_map(nk, -4.0, 4.0, (-0.5, 0.5), 4.0, 0.25)
    if stride > 1:
        xa, ya, za = xa[::stride], ya[::stride], za[::stride]
        dxa, dya, dza = dxa[::stride] * stride, dya[::stride] * stride, dza[::stride] * stride
    X, Y, Z = _broadcast(xa, ya, za)
    period = np.diag([16.0, 8.0, 8.0])
    m = _separable_metrics(dxa, dya, dza)
    return Grid(xa.size, ya.size, za.size, X, Y, Z, period, m,
                f"stretched_jet_{ni}x{nj}x{nk}" + (f"_s{stride}" if stride > 1 else ""),
                axes=(xa, ya, za))


def wavy_grid(ni: int, nj: int, nk: int, lo=(0.0, -1.5, -1.5), size=(4.0, 3.0, 3.0),
              amp=(0.1, 0.08, 0.06), name: str = "wavy") -> Grid:
    """Non-separable periodic curvilinear grid:
    x = lo_x + h_x i + A_x sin(2 pi j / nj) sin(2 pi k / nk), cyclically for
    y and z.  ``amp`` holds the absolute amplitudes A, so refining the grid
    keeps the geometry fixed.  No analytic metric set is attached;
    ``jacobian`` holds the exact d x_a / d xi_d."""
    h = np.asarray(size, dtype=np.float64) / np.array([ni, nj, nk])
    ii = np.arange(ni, dtype=np.float64)[None, None, :]
    jj = np.arange(nj, dtype=np.float64)[None, :, None]
    kk = np.arange(nk, dtype=np.float64)[:, None, None]
    ti, tj, tk = 2 * np.pi * ii / ni, 2 * np.pi * jj / nj, 2 * np.pi * kk / nk
    ax, ay, az = amp
    shp = (nk, nj, ni)
    X = np.broadcast_to(lo[0] + h[0] * ii + ax * np.sin(tj) * np.sin(tk), shp).ravel().copy()
    Y = np.broadcast_to(lo[1] + h[1] * jj + ay * np.sin(tk) * np.sin(ti), shp).ravel().copy()
    Z = np.broadcast_to(lo[2] + h[2] * kk + az * np.sin(ti) * np.sin(tj), shp).ravel().copy()
    jac = np.zeros((3, 3, ni * nj * nk))
    bc = lambda a: np.broadcast_to(a, shp).ravel()
    jac[0, 0] = h[0]
    jac[0, 1] = bc(ax * (2 * np.pi / nj) * np.cos(tj) * np.sin(tk))
    jac[0, 2] = bc(ax * np.sin(tj) * (2 * np.pi / nk) * np.cos(tk))
    jac[1, 0] = bc(ay * np.sin(tk) * (2 * np.pi / ni) * np.cos(ti))
    jac[1, 1] = h[1]
    jac[1, 2] = bc(ay * (2 * np.pi / nk) * np.cos(tk) * np.sin(ti))
    jac[2, 0] = bc(az * (2 * np.pi / ni) * np.cos(ti) * np.sin(tj))
    jac[2, 1] = bc(az * np.sin(ti) * (2 * np.pi / nj) * np.cos(tj))
    jac[2, 2] = h[2]
    period = np.diag(np.asarray(size, dtype=np.float64))
    return Grid(ni, nj, nk, X, Y, Z, period, None, name, jacobian=jac)


# ----------------------------------------------------------------------------
# initial states (conserved variables from primitive fields)
# ----------------------------------------------------------------------------
def conserved(rho, u, v, w, p, gamma: float = GAMMA) -> np.ndarray:
    """Pack primitive fields into the 5 x N conserved array with
    e = p / (gamma - 1) + rho |u|^2 / 2 (ideal-gas total energy)."""
    n = np.broadcast(rho, u, v, w, p).shape[0]
    q = np.empty((5, n), dtype=np.float64)
    q[0] = rho
    q[1] = rho * u
    q[2] = rho * v
    q[3] = rho * w
    q[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return q


def jet_state(grid: Grid, mach: float, seed: int, noise: float = 0.01,
              r0: float = 0.5, theta: Optional[float] = None, gamma: float = GAMMA,
              centre=(0.0, 0.0), global_dims: Optional[tuple] = None,
              stride: int = 1) -> np.ndarray:
    """Round jet along x: U(r) = U_j/2 (1 - tanh((r - r0) / (2 theta))),
    r = distance from the axis (y, z) = centre, rho = 1, p = 1/gamma (so the
    ambient sound speed is 1 and U_j = mach), plus seeded white noise
    noise * U_j * (2 xi - 1) on all three velocity components.

    The noise of node (i, j, k) is keyed by its linear index in the grid of
    ``global_dims`` at (stride i, stride j, stride k), so a subsampled grid
    carries the subsample of the full grid's perturbation."""
    theta = r0 / 20.0 if theta is None else theta
    uj = float(mach)
    r = np.sqrt((grid.y - centre[0]) ** 2 + (grid.z - centre[1]) ** 2)
    U = 0.5 * uj * (1.0 - np.tanh((r - r0) / (2.0 * theta)))
    gi_n, gj_n, gk_n = global_dims if global_dims is not None else grid.dims
    i = np.arange(grid.ni, dtype=np.uint64) * np.uint64(stride)
    j = np.arange(grid.nj, dtype=np.uint64) * np.uint64(stride)
    k = np.arange(grid.nk, dtype=np.uint64) * np.uint64(stride)
    gidx = (i[None, None, :] + np.uint64(gi_n) * (j[None, :, None]
            + np.uint64(gj_n) * k[:, None, None])).ravel()
    ctr = gidx * np.uint64(3)
    du = noise * uj * (2.0 * uniform01(seed, ctr) - 1.0)
    dv = noise * uj * (2.0 * uniform01(seed, ctr + np.uint64(1)) - 1.0)
    dw = noise * uj * (2.0 * uniform01(seed, ctr + np.uint64(2)) - 1.0)
    one = np.ones(grid.n)
    return conserved(one, U + du, dv, dw, one / gamma, gamma)


def vortex_fields(x, y, t: float, beta: float = 5.0, u_inf: float = 0.5,
                  v_inf: float = 0.3, x0: float = 0.0, y0: float = 0.0,
                  period=(10.0, 10.0), gamma: float = GAMMA):
    """Isentropic vortex (Shu 1998; Yee, Sandham and Djomehri 1999) in units
    with rho_inf = 1, p_inf = 1/gamma (a_inf = 1), convected by (u_inf, v_inf)
    for time t on a doubly periodic [x0 - Lx/2, x0 + Lx/2) x ... domain.
    Returns primitive fields (rho, u, v, w, p).  Exact Euler solution."""
    Lx, Ly = period
    xc = x0 + u_inf * t
    yc = y0 + v_inf * t
    dx = np.mod(x - xc + 0.5 * Lx, Lx) - 0.5 * Lx
    dy = np.mod(y - yc + 0.5 * Ly, Ly) - 0.5 * Ly
    r2 = dx * dx + dy * dy
    f = beta / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    T = 1.0 - 0.5 * (gamma - 1.0) * (beta / (2.0 * np.pi)) ** 2 * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T / gamma
    return rho, u_inf - f * dy, v_inf + f * dx, np.zeros_like(rho), p


def vortex_state(grid: Grid, t: float = 0.0, gamma: float = GAMMA, **kw) -> np.ndarray:
    rho, u, v, w, p = vortex_fields(grid.x, grid.y, t, gamma=gamma, **kw)
    return conserved(rho, u, v, w, p, gamma)


def shear_wave_state(grid: Grid, amp: float, modes: int = 1, gamma: float = GAMMA) -> np.ndarray:
    """u = amp sin(2 pi modes (y - y_0) / L_y), v = w = 0, rho = 1, p = 1/gamma."""
    ly = grid.period[1, 1]
    y0 = grid.y.min()
    u = amp * np.sin(2 * np.pi * modes * (grid.y - y0) / ly)
    one = np.ones(grid.n)
    return conserved(one, u, 0 * one, 0 * one, one / gamma, gamma)


def entropy_wave_state(grid: Grid, amp: float, u0: float, modes: int = 1,
                       gamma: float = GAMMA) -> np.ndarray:
    """rho = 1 + amp sin(2 pi modes (x - x_0) / L_x), u = (u0, 0, 0), p = 1/gamma."""
    lx = grid.period[0, 0]
    x0 = grid.x.min()
    rho = 1.0 + amp * np.sin(2 * np.pi * modes * (grid.x - x0) / lx)
    one = np.ones(grid.n)
    return conserved(rho, u0 * one, 0 * one, 0 * one, one / gamma, gamma)


def uniform_state(grid: Grid, u=(0.7, -0.3, 0.2), rho: float = 1.3, p: float = 0.9,
                  gamma: float = GAMMA) -> np.ndarray:
    one = np.ones(grid.n)
    return conserved(rho * one, u[0] * one, u[1] * one, u[2] * one, p * one, gamma)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def jet_box_case(dims=(64, 48, 48), mach: float = 1.4, seed: int = 1):
    """Periodic jet box [0,4) x [-1.5,1.5)^2 with uniform spacing; the jet
    axis passes through the node row y = z = 0 when nj, nk are even."""
    g = uniform_box(*dims)
    return g, jet_state(g, mach, seed)


def shock_box_case(dims=(40, 24, 20), mach: float = 1.4, seed: int = 3, ratio: float = 4.0):
    """Periodic jet box [0,4) x [-1.5,1.5)^2 with a slab 1 <= x < 2 of
    `ratio` times the ambient pressure and twice its density (the jet and its
    noise unchanged): pressure jumps that start the second-difference branch
    of the artificial dissipation at once."""
    g = uniform_box(*dims)
    q = jet_state(g, mach, seed)
    rho0 = q[0]
    u, v, w = q[1] / rho0, q[2] / rho0, q[3] / rho0
    slab = (g.x >= 1.0) & (g.x < 2.0)
    rho = np.where(slab, 2.0, 1.0)
    p = np.where(slab, ratio, 1.0) / GAMMA
    return g, conserved(rho, u, v, w, p)


def stretched_jet_case(dims=(512, 256, 256), mach: float = 1.4, seed: int = 2, stride: int = 1):
    """Separable tanh-stretched jet grid with analytic metrics; ``stride``
    subsamples the grid and the perturbation field together."""
    g = stretched_jet_grid(*dims, stride=stride)
    q = jet_state(g, mach, seed, global_dims=dims, stride=stride)
    return g, q


def jet_domain_case(dims=(64, 48, 48), mach: float = 1.4, seed: int = 1, bc=JET_DOMAIN_BC,
                    size=(4.0, 3.0, 3.0), noise_radius: Optional[float] = None):
    """The jet in a bounded domain: x in [0, 4] from the jet exit, y, z in
    [-1.5, 1.5], nodes on every bounded face.  The jet profile with seeded
    noise fills the block (only within distance ``noise_radius`` of the axis
    when given; the ambient fluid outside is then exactly at rest); the two
    inflow layers at the jet exit (i = 0, 1) carry the clean profile.
    Returns (grid, state, bc)."""
    bounded = tuple(bc[2 * d] != BC_PERIODIC for d in range(3))
    g = bounded_box(*dims, size=size, bounded=bounded)
    q = jet_state(g, mach, seed)
    clean = jet_state(g, mach, seed, noise=0.0)
    if noise_radius is not None:
        far = np.sqrt(g.y ** 2 + g.z ** 2) >= noise_radius
        q[:, far] = clean[:, far]
    q = q.reshape(5, dims[2], dims[1], dims[0])
    clean = clean.reshape(5, dims[2], dims[1], dims[0])
    if bc[0] == BC_INFLOW:
        q[:, :, :, :2] = clean[:, :, :, :2]
    if bc[1] == BC_INFLOW:
        q[:, :, :, -2:] = clean[:, :, :, -2:]
    return g, q.reshape(5, -1).copy(), tuple(bc)


def jet_cylinder_case(dims=(40, 16, 24), mach: float = 1.4, seed: int = 1, noise_radius: Optional[float] = None,
                      noise: float = 0.01):
    """The jet on the cylindrical mesh (``cylindrical_grid``, jet axis on the
    centreline) with ``JET_CYLINDER_BC``: jet profile plus seeded noise (within
    ``noise_radius`` of the axis when given), the clean profile on the two
    inflow layers.  Returns (grid, state, bc)."""
    g = cylindrical_grid(*dims)
    q = jet_state(g, mach, seed, noise=noise)
    clean = jet_state(g, mach, seed, noise=0.0)
    if noise_radius is not None:
        far = np.sqrt(g.y ** 2 + g.z ** 2) >= noise_radius
        q[:, far] = clean[:, far]
    q = q.reshape(5, dims[2], dims[1], dims[0])
    q[:, :, :, :2] = clean.reshape(5, dims[2], dims[1], dims[0])[:, :, :, :2]
    return g, q.reshape(5, -1).copy(), JET_CYLINDER_BC


def batch_mix(seed: int = 4, nblocks: int = 64, lo: int = 32, hi: int = 160):
    """Uneven block mix: each of ni, nj, nk uniform in [lo, hi], Mach
    uniform in [1.2, 2.0], Re_D log-uniform in [1e5, 1e6] (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    dims = rng.integers(lo, hi + 1, size=(nblocks, 3))
    mach = rng.uniform(1.2, 2.0, size=nblocks)
    re = 10.0 ** rng.uniform(5.0, 6.0, size=nblocks)
    return [dict(dims=tuple(int(v) for v in dims[b]), mach=float(mach[b]),
                 re_d=float(re[b]), seed=seed * 1000 + b) for b in range(nblocks)]


def arrival_stream(seed: int = 5, nruns: int = 300, rate: float = 20.0,
                   lo: int = 48, hi: int = 192, steps: int = 200):
    """Poisson arrivals (exponential gaps of mean 1/rate seconds) of cubic
    jet runs n^3, n uniform in [lo, hi], Mach U[1.2, 2.0], Re_D log-uniform
    in [1e5, 1e6], each ``steps`` steps long."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nruns)
    t = np.cumsum(gaps) - gaps[0]
    n = rng.integers(lo, hi + 1, size=nruns)
    mach = rng.uniform(1.2, 2.0, size=nruns)
    re = 10.0 ** rng.uniform(5.0, 6.0, size=nruns)
    return [dict(arrival=float(t[r]), dims=(int(n[r]),) * 3, mach=float(mach[r]),
                 re_d=float(re[r]), steps=steps, seed=seed * 100000 + r) for r in range(nruns)]
