"""Thin ctypes binding of libjetles.so (see include/jetles.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch provides device memory (the solver workspace and device
state buffers) and the HIP stream.  There is no CPU fallback: importing the
binding on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libjetles.so")

JZ_OK, JZ_EINVAL, JZ_ENOMEM, JZ_EHIP, JZ_ENONFINITE, JZ_ESTATE = 0, -1, -2, -3, -4, -5
JZ_FP64, JZ_FP32_FLUX = 0, 1

_ERRNAMES = {JZ_EINVAL: "JZ_EINVAL", JZ_ENOMEM: "JZ_ENOMEM", JZ_EHIP: "JZ_EHIP",
             JZ_ENONFINITE: "JZ_ENONFINITE", JZ_ESTATE: "JZ_ESTATE"}


class JzError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("prandtl_t", ctypes.c_double), ("mach_j", ctypes.c_double),
                ("re_d", ctypes.c_double), ("sutherland_s", ctypes.c_double),
                ("cs", ctypes.c_double), ("k2", ctypes.c_double), ("k4", ctypes.c_double),
                ("tv_alpha", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double), ("rk_alpha", ctypes.c_double * 5),
                ("n_stages", ctypes.c_int), ("precision", ctypes.c_int),
                ("tile_i", ctypes.c_int), ("tile_j", ctypes.c_int), ("kchunk", ctypes.c_int),
                ("bc", ctypes.c_int * 6), ("mach_inf", ctypes.c_double), ("stats_interval", ctypes.c_int)]


# face boundary types (jz_bc), indexed xi-, xi+, eta-, eta+, zeta-, zeta+
JZ_BC_PERIODIC, JZ_BC_INFLOW, JZ_BC_FARFIELD, JZ_BC_AXIS = 0, 1, 2, 3


_lib = None


def library() -> ctypes.CDLL:
    """Load libjetles.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or python -m paper_2003_09926_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    S = ctypes.c_void_p
    dp = ctypes.c_void_p   # double* (host or device address)
    i, ll, d, sz = ctypes.c_int, ctypes.c_longlong, ctypes.c_double, ctypes.c_size_t
    sig = {
        "jz_params_default": ([P], i),
        "jz_workspace_bytes": ([i, i, i, P], sz),
        "jz_create": ([i, i, i, P, ctypes.c_void_p, sz, ctypes.c_void_p, ctypes.POINTER(S)], i),
        "jz_set_grid_coords": ([S, dp, dp, dp, dp], i),
        "jz_set_grid_metrics": ([S, dp, i], i),
        "jz_get_grid_metrics": ([S, dp, i], i),
        "jz_set_state": ([S, dp, i], i),
        "jz_advance": ([S, i], i),
        "jz_get_state": ([S, dp, i], i),
        "jz_get_residual_norms": ([S, dp, dp], i),
        "jz_get_clock": ([S, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(ll)], i),
        "jz_set_clock": ([S, d, ll], i),
        "jz_eval_residual": ([S, dp, i], i),
        "jz_eval_dt": ([S, ctypes.POINTER(d), ctypes.POINTER(d)], i),
        "jz_set_timing": ([S, i], i),
        "jz_get_occupancy": ([S, ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "jz_stats_reset": ([S], i),
        "jz_stats_sample": ([S], i),
        "jz_get_stats": ([S, dp, dp, dp, dp, ctypes.POINTER(ll), i], i),
        "jz_stats_profile": ([S, i, ctypes.c_void_p, i, dp, dp, dp, dp, ctypes.c_void_p], i),
        "jz_get_timing": ([S, ctypes.POINTER(d), ctypes.POINTER(ll), ctypes.POINTER(d)], i),
        "jz_destroy": ([S], i),
        "jz_set_tiling": ([S, i, i, i], i),
        "jz_get_tiling": ([S, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "jz_batch_create": ([ctypes.POINTER(S), i, ctypes.c_void_p, ctypes.POINTER(S)], i),
        "jz_batch_advance": ([S, i], i),
        "jz_batch_add": ([S, S], i),
        "jz_batch_remove": ([S, S], i),
        "jz_batch_members": ([S], i),
        "jz_batch_refresh": ([S], i),
        "jz_batch_set_graph": ([S, i], i),
        "jz_batch_autotune": ([S, i, ctypes.c_char_p, ctypes.POINTER(i), ctypes.POINTER(i),
                               ctypes.POINTER(i), ctypes.POINTER(d)], i),
        "jz_batch_set_timing": ([S, i], i),
        "jz_batch_get_timing": ([S, ctypes.POINTER(d), ctypes.POINTER(ll), ctypes.POINTER(ll)], i),
        "jz_batch_synchronize": ([S], i),
        "jz_batch_destroy": ([S], i),
        "jz_advance_static": ([i, i, i, P, dp, dp, dp, i, ctypes.c_void_p], i),
        "jz_domain_create": ([i, i, i, P, i, i, ctypes.c_void_p, ctypes.POINTER(S)], i),
        "jz_domain_set_grid_metrics": ([S, dp], i),
        "jz_domain_set_state": ([S, dp], i),
        "jz_domain_advance": ([S, i], i),
        "jz_domain_get_state": ([S, dp], i),
        "jz_domain_get_clock": ([S, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(ll)], i),
        "jz_domain_get_residual_norms": ([S, dp, dp], i),
        "jz_domain_destroy": ([S], i),
        "jz_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != JZ_OK:
        msg = library().jz_last_error().decode(errors="replace")
        raise JzError(rc, where, msg)


def params_default(**kw) -> Params:
    p = Params()
    _check(library().jz_params_default(ctypes.byref(p)), "jz_params_default")
    for k, v in kw.items():
        if k == "rk_alpha":
            for s in range(5):
                p.rk_alpha[s] = v[s] if s < len(v) else 0.0
        elif k == "bc":
            if len(v) != 6:
                raise ValueError("bc needs six face types")
            for f in range(6):
                p.bc[f] = int(v[f])
        elif hasattr(p, k):
            setattr(p, k, v)
        else:
            raise KeyError(k)
    return p


def advance_static(dims, params: Params, met, q, nsteps: int, info=None, stream=None):
    """jz_advance_static: nsteps steps of the state q (device tensor, 5 x N
    float64, advanced in place) on the metric set met (device tensor, 10 x N
    float64), with the library's static scratch and no device allocation.
    info: optional device tensor of 14 float64 (clock, norms, step count,
    flag).  stream: a torch.cuda.Stream (default: the current stream).  The
    call only queues work."""
    import torch
    ni, nj, nk = dims
    n = ni * nj * nk
    for name, a, rows in (("met", met, 10), ("q", q, 5)):
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
                and a.numel() == rows * n):
            raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of {rows} x {n} values")
    if info is not None and not (isinstance(info, torch.Tensor) and info.is_cuda and info.dtype == torch.float64
                                 and info.numel() >= 14):
        raise ValueError("info must be a CUDA float64 tensor of at least 14 values")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(library().jz_advance_static(ni, nj, nk, ctypes.byref(params), met.data_ptr(), q.data_ptr(),
                                       info.data_ptr() if info is not None else None, int(nsteps),
                                       ctypes.c_void_p(st.cuda_stream)), "jz_advance_static")


def workspace_bytes(dims, params: Optional[Params] = None) -> int:
    ni, nj, nk = dims
    p = params if params is not None else params_default()
    return int(library().jz_workspace_bytes(ni, nj, nk, ctypes.byref(p)))


def _host_ptr(a: np.ndarray) -> int:
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data


def _as_host(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _is_torch_cuda(a) -> bool:
    try:
        import torch
        return isinstance(a, torch.Tensor) and a.is_cuda
    except ImportError:   # pragma: no cover
        return False


class Solver:
    """One block resident in HBM.  Device memory: a torch uint8 tensor (the
    default) or a library allocation (workspace="library")."""

    def __init__(self, dims, params: Optional[Params] = None, workspace: str = "torch",
                 stream=None):
        import torch
        self.dims = tuple(int(x) for x in dims)
        self.n = self.dims[0] * self.dims[1] * self.dims[2]
        self.params = params if params is not None else params_default()
        lib = library()
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if workspace == "torch":
            ws_bytes = workspace_bytes(self.dims, self.params)
            if ws_bytes == 0:
                _check(JZ_EINVAL, "jz_workspace_bytes")
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
            ws_ptr = self._ws.data_ptr()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib.jz_create(*self.dims, ctypes.byref(self.params), ws_ptr, ws_bytes,
                             ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h)), "jz_create")
        self._h = h

    # -- geometry -----------------------------------------------------------
    def set_grid_coords(self, x, y, z, period):
        x, y, z = _as_host(x), _as_host(y), _as_host(z)
        per = _as_host(np.asarray(period).reshape(9))
        _check(library().jz_set_grid_coords(self._h, _host_ptr(x), _host_ptr(y), _host_ptr(z),
                                            _host_ptr(per)), "jz_set_grid_coords")

    def set_grid_metrics(self, m):
        if _is_torch_cuda(m):
            _check(library().jz_set_grid_metrics(self._h, m.contiguous().data_ptr(), 1), "jz_set_grid_metrics")
        else:
            m = _as_host(m)
            _check(library().jz_set_grid_metrics(self._h, _host_ptr(m), 0), "jz_set_grid_metrics")

    def get_grid_metrics(self) -> np.ndarray:
        out = np.empty((10, self.n))
        _check(library().jz_get_grid_metrics(self._h, _host_ptr(out), 0), "jz_get_grid_metrics")
        return out

    # -- state --------------------------------------------------------------
    def set_state(self, q):
        if _is_torch_cuda(q):
            _check(library().jz_set_state(self._h, q.contiguous().data_ptr(), 1), "jz_set_state")
        else:
            q = _as_host(q)
            _check(library().jz_set_state(self._h, _host_ptr(q), 0), "jz_set_state")

    def get_state(self, out=None):
        """Host copy (numpy) by default; pass a CUDA tensor of 5*N doubles for a device copy."""
        if out is not None and _is_torch_cuda(out):
            _check(library().jz_get_state(self._h, out.data_ptr(), 1), "jz_get_state")
            return out
        out = np.empty((5, self.n)) if out is None else out
        _check(library().jz_get_state(self._h, _host_ptr(out), 0), "jz_get_state")
        return out

    def advance(self, nsteps: int):
        _check(library().jz_advance(self._h, int(nsteps)), "jz_advance")

    def residual_norms(self):
        rms, linf = np.empty(5), np.empty(5)
        _check(library().jz_get_residual_norms(self._h, _host_ptr(rms), _host_ptr(linf)),
               "jz_get_residual_norms")
        return rms, linf

    def clock(self):
        t, dt, st = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        _check(library().jz_get_clock(self._h, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(st)),
               "jz_get_clock")
        return t.value, dt.value, st.value

    def set_clock(self, t: float, steps: int):
        _check(library().jz_set_clock(self._h, float(t), int(steps)), "jz_set_clock")

    def eval_residual(self) -> np.ndarray:
        out = np.empty((5, self.n))
        _check(library().jz_eval_residual(self._h, _host_ptr(out), 0), "jz_eval_residual")
        return out

    def eval_dt(self):
        dt, lm = ctypes.c_double(), ctypes.c_double()
        _check(library().jz_eval_dt(self._h, ctypes.byref(dt), ctypes.byref(lm)), "jz_eval_dt")
        return dt.value, lm.value

    def occupancy(self):
        """(stage workgroups per CU, CUs): their product is one round"""
        w, c = ctypes.c_int(), ctypes.c_int()
        _check(library().jz_get_occupancy(self._h, ctypes.byref(w), ctypes.byref(c)), "jz_get_occupancy")
        return w.value, c.value

    # -- statistics ---------------------------------------------------------
    def stats_reset(self):
        _check(library().jz_stats_reset(self._h), "jz_stats_reset")

    def stats_sample(self):
        _check(library().jz_stats_sample(self._h), "jz_stats_sample")

    def stats(self) -> dict:
        """per-node mean and RMS of the fluctuation of u and p, and the count"""
        out = {k: np.empty(self.n) for k in ("mean_u", "rms_u", "mean_p", "rms_p")}
        ns = ctypes.c_longlong()
        _check(library().jz_get_stats(self._h, *[_host_ptr(out[k]) for k in ("mean_u", "rms_u", "mean_p", "rms_p")],
                                      ctypes.byref(ns), 0), "jz_get_stats")
        out["samples"] = ns.value
        return out

    def stats_profile(self, i: int, bins, nbins: int) -> dict:
        """bin averages of the node statistics over the cross-section i"""
        b = np.ascontiguousarray(bins, dtype=np.int32)
        assert b.size == self.dims[1] * self.dims[2]
        out = {k: np.empty(nbins) for k in ("mean_u", "rms_u", "mean_p", "rms_p")}
        cnt = np.empty(nbins, dtype=np.int64)
        _check(library().jz_stats_profile(self._h, int(i), b.ctypes.data, int(nbins),
                                          *[_host_ptr(out[k]) for k in ("mean_u", "rms_u", "mean_p", "rms_p")],
                                          cnt.ctypes.data), "jz_stats_profile")
        out["count"] = cnt
        return out

    # -- timing -------------------------------------------------------------
    def set_timing(self, enable: bool):
        _check(library().jz_set_timing(self._h, 1 if enable else 0), "jz_set_timing")

    def timing(self):
        ms, n, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        _check(library().jz_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
               "jz_get_timing")
        return ms.value, n.value, b.value

    def set_tiling(self, tile_i: int, tile_j: int, kchunk: int = 0):
        _check(library().jz_set_tiling(self._h, tile_i, tile_j, kchunk), "jz_set_tiling")

    def tiling(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(library().jz_get_tiling(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "jz_get_tiling")
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            library().jz_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Advance several Solvers together (one persistent launch per stage,
    step replayed from a hipGraph).  The members stay owned by the caller."""

    def __init__(self, members, stream=None):
        import torch
        self.members = list(members)
        arr = (ctypes.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(library().jz_batch_create(arr, len(self.members), ctypes.c_void_p(self._stream.cuda_stream),
                                         ctypes.byref(h)), "jz_batch_create")
        self._h = h

    def advance(self, nsteps: int):
        _check(library().jz_batch_advance(self._h, int(nsteps)), "jz_batch_advance")

    def add(self, solver):
        """Join a member between steps (no new capture of the step)."""
        _check(library().jz_batch_add(self._h, solver._h), "jz_batch_add")
        self.members.append(solver)

    def remove(self, solver):
        """Take a member out between steps; the caller keeps it."""
        _check(library().jz_batch_remove(self._h, solver._h), "jz_batch_remove")
        self.members = [m for m in self.members if m is not solver]

    def __len__(self):
        n = library().jz_batch_members(self._h)
        if n < 0:
            _check(n, "jz_batch_members")
        return n

    def refresh(self):
        _check(library().jz_batch_refresh(self._h), "jz_batch_refresh")

    def set_graph(self, enable: bool):
        _check(library().jz_batch_set_graph(self._h, 1 if enable else 0), "jz_batch_set_graph")

    def autotune(self, trial_steps: int = 3, cache_path: Optional[str] = None):
        a, b, c, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(library().jz_batch_autotune(self._h, int(trial_steps),
                                           cache_path.encode() if cache_path else None,
                                           ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                           ctypes.byref(ms)), "jz_batch_autotune")
        return (a.value, b.value, c.value), ms.value

    def set_timing(self, enable: bool):
        _check(library().jz_batch_set_timing(self._h, 1 if enable else 0), "jz_batch_set_timing")

    def timing(self):
        ms, n, pts = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_longlong()
        _check(library().jz_batch_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pts)),
               "jz_batch_get_timing")
        return ms.value, n.value, pts.value

    def synchronize(self):
        _check(library().jz_batch_synchronize(self._h), "jz_batch_synchronize")

    def close(self):
        if getattr(self, "_h", None):
            library().jz_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Domain:
    """A periodic block split into parts_i x parts_k padded sub-blocks whose
    two-layer ghost fringes are refilled by halo copies after every stage;
    the whole-block arrays go in and come out in the Solver layouts (host)."""

    def __init__(self, dims, params: Optional[Params] = None, parts=(1, 1), stream=None):
        import torch
        self.dims = tuple(int(x) for x in dims)
        self.n = self.dims[0] * self.dims[1] * self.dims[2]
        self.params = params if params is not None else params_default()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(library().jz_domain_create(*self.dims, ctypes.byref(self.params), int(parts[0]), int(parts[1]),
                                          ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h)),
               "jz_domain_create")
        self._h = h

    def set_grid_metrics(self, m):
        m = _as_host(m)
        _check(library().jz_domain_set_grid_metrics(self._h, _host_ptr(m)), "jz_domain_set_grid_metrics")

    def set_state(self, q):
        q = _as_host(q)
        _check(library().jz_domain_set_state(self._h, _host_ptr(q)), "jz_domain_set_state")

    def advance(self, nsteps: int):
        _check(library().jz_domain_advance(self._h, int(nsteps)), "jz_domain_advance")

    def get_state(self) -> np.ndarray:
        out = np.empty((5, self.n))
        _check(library().jz_domain_get_state(self._h, _host_ptr(out)), "jz_domain_get_state")
        return out

    def clock(self):
        t, dt, st = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        _check(library().jz_domain_get_clock(self._h, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(st)),
               "jz_domain_get_clock")
        return t.value, dt.value, st.value

    def residual_norms(self):
        rms, linf = np.empty(5), np.empty(5)
        _check(library().jz_domain_get_residual_norms(self._h, _host_ptr(rms), _host_ptr(linf)),
               "jz_domain_get_residual_norms")
        return rms, linf

    def close(self):
        if getattr(self, "_h", None):
            library().jz_domain_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
