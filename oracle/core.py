"""ctypes wrapper of the FP64 C++ oracle (test infrastructure only).

Arrays are NumPy float64, C-contiguous, structure-of-arrays: a state is
5 x N, a metric set 10 x N, with node (i, j, k) at i + ni (j + nj k).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jetles_oracle.cpp")
_LIB = os.path.join(_HERE, "libjetles_oracle.so")
# JZO_LIB names another build of this same source (used to check, once, that
# each pin fails when a mistake is planted in a copy of the oracle)
_LOAD = os.environ.get("JZO_LIB", _LIB)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O3, OpenMP over outer loops; no other tuning)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("prandtl_t", ctypes.c_double), ("mach_j", ctypes.c_double),
                ("re_d", ctypes.c_double), ("sutherland_s", ctypes.c_double),
                ("cs", ctypes.c_double), ("k2", ctypes.c_double), ("k4", ctypes.c_double),
                ("tv_alpha", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double), ("rk_alpha", ctypes.c_double * 5),
                ("n_stages", ctypes.c_int), ("bc", ctypes.c_int * 6), ("mach_inf", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("rk_alpha", "bc")}
        d["rk_alpha"] = list(self.rk_alpha)
        d["bc"] = list(self.bc)
        return d


# boundary types of the faces (xi-, xi+, eta-, eta+, zeta-, zeta+)
BC_PERIODIC, BC_INFLOW, BC_FARFIELD, BC_AXIS = 0, 1, 2, 3


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _LOAD == _LIB and not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LOAD)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        i = ctypes.c_int
        lib.jzo_params_default.argtypes = [pp]
        lib.jzo_metrics_tl.argtypes = [i, i, i, dp, dp, dp, dp, dp]
        lib.jzo_metrics_tl_bc.argtypes = [i, i, i, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int), dp]
        lib.jzo_apply_bc.argtypes = [i, i, i, pp, dp, dp, dp]
        lib.jzo_residual.argtypes = [i, i, i, pp, dp, dp, dp]
        lib.jzo_fields.argtypes = [i, i, i, pp, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.jzo_cfl_dt.argtypes = [i, i, i, pp, dp, dp, dp, dp]
        lib.jzo_step.argtypes = [i, i, i, pp, dp, dp, ctypes.c_double, dp, dp, dp]
        lib.jzo_advance.argtypes = [i, i, i, pp, dp, dp, i, dp, dp, dp]
        lib.jzo_threads.argtypes = [i]
        for f in (lib.jzo_params_default, lib.jzo_metrics_tl, lib.jzo_metrics_tl_bc, lib.jzo_apply_bc,
                  lib.jzo_residual, lib.jzo_fields, lib.jzo_cfl_dt, lib.jzo_step, lib.jzo_advance,
                  lib.jzo_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_params(**kw) -> Params:
    p = Params()
    _load().jzo_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "rk_alpha":
            for s in range(5):
                p.rk_alpha[s] = v[s] if s < len(v) else 0.0
        elif k == "bc":
            for f in range(6):
                p.bc[f] = int(v[f])
        else:
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
    return p


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def metrics_tl(ni, nj, nk, x, y, z, period, bc=None) -> np.ndarray:
    """Thomas-Lombard metric set (10 x N) from node coordinates; bc (six face
    types) makes the directions with physical faces one-sided at their ends."""
    x, y, z = _c(x), _c(y), _c(z)
    per = _c(np.asarray(period, dtype=np.float64).reshape(9))
    m = np.empty((10, ni * nj * nk))
    if bc is None:
        rc = _load().jzo_metrics_tl(ni, nj, nk, _ptr(x), _ptr(y), _ptr(z), _ptr(per), _ptr(m))
    else:
        cb = (ctypes.c_int * 6)(*[int(t) for t in bc])
        rc = _load().jzo_metrics_tl_bc(ni, nj, nk, _ptr(x), _ptr(y), _ptr(z), _ptr(per), cb, _ptr(m))
    if rc:
        raise ValueError(f"jzo_metrics_tl failed ({rc})")
    return m


def residual(dims, params: Params, m, q) -> np.ndarray:
    ni, nj, nk = dims
    m, q = _c(m), _c(q)
    r = np.empty_like(q)
    rc = _load().jzo_residual(ni, nj, nk, ctypes.byref(params), _ptr(m), _ptr(q), _ptr(r))
    if rc:
        raise ValueError(f"jzo_residual failed ({rc})")
    return r


def fields(dims, params: Params, m, q) -> dict:
    ni, nj, nk = dims
    n = ni * nj * nk
    m, q = _c(m), _c(q)
    out = dict(mu=np.empty(n), mut=np.empty(n), lam=np.empty((3, n)), sig=np.empty((3, n)),
               nu=np.empty((3, n)), grad=np.empty((12, n)))
    rc = _load().jzo_fields(ni, nj, nk, ctypes.byref(params), _ptr(m), _ptr(q),
                            *[_ptr(out[k]) for k in ("mu", "mut", "lam", "sig", "nu", "grad")])
    if rc:
        raise ValueError(f"jzo_fields failed ({rc})")
    return out


def cfl_dt(dims, params: Params, m, q):
    ni, nj, nk = dims
    m, q = _c(m), _c(q)
    dt = ctypes.c_double()
    lm = ctypes.c_double()
    rc = _load().jzo_cfl_dt(ni, nj, nk, ctypes.byref(params), _ptr(m), _ptr(q),
                            ctypes.byref(dt), ctypes.byref(lm))
    if rc:
        raise ValueError(f"jzo_cfl_dt failed ({rc})")
    return dt.value, lm.value


def step(dims, params: Params, m, q, dt: float = 0.0):
    """One multistage step.  Returns (q_new, dt_used, rms[5], linf[5])."""
    ni, nj, nk = dims
    m = _c(m)
    qn = np.array(q, dtype=np.float64, order="C", copy=True)
    dtu = ctypes.c_double()
    rms = np.empty(5)
    linf = np.empty(5)
    rc = _load().jzo_step(ni, nj, nk, ctypes.byref(params), _ptr(m), _ptr(qn), float(dt),
                          ctypes.byref(dtu), _ptr(rms), _ptr(linf))
    if rc:
        raise ValueError(f"jzo_step failed ({rc})")
    return qn, dtu.value, rms, linf


def advance(dims, params: Params, m, q, nsteps: int):
    """nsteps steps.  Returns (q_new, t, rms[5], linf[5]) of the last step."""
    ni, nj, nk = dims
    m = _c(m)
    qn = np.array(q, dtype=np.float64, order="C", copy=True)
    t = ctypes.c_double(0.0)
    rms = np.empty(5)
    linf = np.empty(5)
    rc = _load().jzo_advance(ni, nj, nk, ctypes.byref(params), _ptr(m), _ptr(qn), int(nsteps),
                             ctypes.byref(t), _ptr(rms), _ptr(linf))
    if rc:
        raise ValueError(f"jzo_advance failed ({rc})")
    return qn, t.value, rms, linf


def threads(n: int = 0) -> int:
    """Worker threads of the oracle's loops: n > 0 sets them; returns the
    count in use."""
    return int(_load().jzo_threads(int(n)))


def apply_bc(dims, params: Params, m, q, q0) -> np.ndarray:
    """The boundary conditions alone: returns q with its boundary layers set
    (inflow layers from q0, far-field layers from q's first interior nodes)."""
    ni, nj, nk = dims
    m, q0 = _c(m), _c(q0)
    qn = np.array(q, dtype=np.float64, order="C", copy=True)
    rc = _load().jzo_apply_bc(ni, nj, nk, ctypes.byref(params), _ptr(m), _ptr(qn), _ptr(q0))
    if rc:
        raise ValueError(f"jzo_apply_bc failed ({rc})")
    return qn
