"""Helpers for the time-averaged statistics of Sec. 6 (host-side analysis of
what the library accumulates on the GPU): the radial bins of a cross-section
for the azimuthal average, and the length of the potential core."""
from __future__ import annotations

import numpy as np


def radial_bins(y: np.ndarray, z: np.ndarray, dims, i: int, nbins: int, rmax: float,
                centre=(0.0, 0.0)) -> np.ndarray:
    """Bin index (nj * nk ints, entry j + nj k) of every node of the
    cross-section xi = i by its distance r from the jet axis: bin
    floor(r / rmax * nbins), or -1 beyond rmax.  y, z: node coordinates
    (N each, node (i, j, k) at i + ni (j + nj k))."""
    ni, nj, nk = dims
    yy = np.asarray(y).reshape(nk, nj, ni)[:, :, i]
    zz = np.asarray(z).reshape(nk, nj, ni)[:, :, i]
    r = np.sqrt((yy - centre[0]) ** 2 + (zz - centre[1]) ** 2)       # (nk, nj)
    b = np.floor(r / rmax * nbins).astype(np.int64)
    b[r >= rmax] = -1
    return np.ascontiguousarray(b.reshape(-1), dtype=np.int32)    # index j + nj k


def potential_core_length(x: np.ndarray, mean_u_axis: np.ndarray, u_jet: float, frac: float = 0.95) -> float:
    """Length of the potential core (Sec. 6: the region where the time-averaged
    axial velocity is at least frac of the jet exit velocity) along the axis:
    the first position where <U> falls below frac * u_jet, linearly
    interpolated between nodes; the last x if it never does."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(mean_u_axis, dtype=np.float64)
    thr = frac * u_jet
    below = np.nonzero(u < thr)[0]
    if below.size == 0:
        return float(x[-1])
    k = int(below[0])
    if k == 0:
        return float(x[0])
    t = (u[k - 1] - thr) / (u[k - 1] - u[k])
    return float(x[k - 1] + t * (x[k] - x[k - 1]))
