"""CPU oracle of the jet-LES hot path -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product path (the HIP library and its
binding) never touches it, and it never touches the product path.

``oracle.core`` wraps the plain FP64 C++ oracle (``jetles_oracle.cpp``);
``oracle.numpy_ref`` is a second, independent NumPy implementation of the
same residual used only to cross-check the C++ loops on tiny blocks.
"""
from .core import (Params, default_params, metrics_tl, residual, fields, cfl_dt, step,  # noqa: F401
                   advance, apply_bc, build, lib_path, threads, BC_PERIODIC, BC_INFLOW, BC_FARFIELD)
from . import core  # noqa: F401
