"""Helpers shared by the GPU parity tests (comparison metrics, patches)."""
import numpy as np


def rel_l2(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def per_var_rel(a, b):
    return [rel_l2(a[v], b[v]) for v in range(a.shape[0])]


def patch(arr: np.ndarray, dims, centre, r: int) -> np.ndarray:
    """(c, N) field -> (c, (2r+1)^3) periodic patch around node ``centre``."""
    ni, nj, nk = dims
    c = arr.shape[0]
    a = arr.reshape(c, nk, nj, ni)
    i, j, k = centre
    ii = np.arange(i - r, i + r + 1) % ni
    jj = np.arange(j - r, j + r + 1) % nj
    kk = np.arange(k - r, k + r + 1) % nk
    return np.ascontiguousarray(a[:, kk][:, :, jj][:, :, :, ii].reshape(c, -1))


def flat(dims, i, j, k) -> int:
    ni, nj, _ = dims
    return i + ni * (j + nj * k)
