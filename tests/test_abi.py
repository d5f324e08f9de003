"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-only entry points behave (no GPU work is issued here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(jz_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return binding.library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_symbols()
    assert "jz_advance" in names and "jz_create" in names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_params_default_matches_oracle_defaults(lib):
    p = binding.params_default()
    o = oracle.default_params()
    for k in ("gamma", "prandtl", "prandtl_t", "mach_j", "re_d", "sutherland_s", "cs", "k2", "k4",
              "tv_alpha", "cfl", "dt_fixed", "n_stages"):
        assert getattr(p, k) == getattr(o, k), k
    assert list(p.rk_alpha) == list(o.rk_alpha)
    assert p.precision == binding.JZ_FP64
    assert list(p.bc) == list(o.bc) == [0] * 6 and p.mach_inf == o.mach_inf == 0.0


def test_params_struct_sizes_match_the_libraries(lib):
    """jz_params_default / jzo_params_default must write exactly the bytes of
    the ctypes mirrors: a guard pattern after the struct stays untouched."""
    for fill, size in ((lib.jz_params_default, ctypes.sizeof(binding.Params)),
                       (oracle.core._load().jzo_params_default, ctypes.sizeof(oracle.Params))):
        buf = (ctypes.c_ubyte * (size + 64))(*([0xAB] * (size + 64)))
        saved, fill.argtypes = fill.argtypes, None
        try:
            assert fill(ctypes.cast(buf, ctypes.c_void_p)) == 0
        finally:
            fill.argtypes = saved
        assert bytes(buf[size:]) == b"\xab" * 64


def test_workspace_bytes_covers_state_and_metrics(lib):
    p = binding.params_default()
    for dims in [(64, 48, 48), (512, 256, 256), (5, 5, 5), (37, 23, 19)]:
        n = dims[0] * dims[1] * dims[2]
        b = binding.workspace_bytes(dims, p)
        assert b >= n * 8 * (15 + 10)
        assert b < n * 8 * 26 + (1 << 22)
    assert binding.workspace_bytes((0, 4, 4), p) == 0


def test_invalid_sizes_and_params_rejected_on_host(lib):
    p = binding.params_default()
    h = ctypes.c_void_p()
    rc = lib.jz_create(0, 4, 4, ctypes.byref(p), None, 0, None, ctypes.byref(h))
    assert rc == binding.JZ_EINVAL and h.value is None
    assert b"sizes" in lib.jz_last_error()
    bad = binding.params_default(n_stages=7)
    assert lib.jz_create(8, 8, 8, ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == binding.JZ_EINVAL
    bad = binding.params_default(tile_i=13, tile_j=3)
    assert lib.jz_create(8, 8, 8, ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == binding.JZ_EINVAL
    bad = binding.params_default(gamma=1.0)
    assert binding.workspace_bytes((8, 8, 8), bad) == 0
    bad = binding.params_default(bc=[1, 0, 0, 0, 0, 0])           # periodic faces come in pairs
    assert binding.workspace_bytes((8, 8, 8), bad) == 0
    bad = binding.params_default(bc=[1, 2, 0, 0, 0, 0])           # bounded direction with 4 nodes
    assert binding.workspace_bytes((4, 8, 8), bad) == 0
    assert binding.workspace_bytes((5, 8, 8), bad) > 0
    bad = binding.params_default(bc=[3, 2, 0, 0, 0, 0])
    assert lib.jz_create(8, 8, 8, ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == binding.JZ_EINVAL
    assert lib.jz_advance(None, 1) == binding.JZ_EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        binding.library()
