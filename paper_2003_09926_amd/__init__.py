"""MI355X-native hot path of the supersonic-jet LES solver of arXiv:2003.09926.

* ``inputs``  -- seeded synthetic grids, states and workload mixes;
* ``binding`` -- ctypes binding of the HIP library ``_lib/libjetles.so``
  (C ABI in ``include/jetles.h``);
* ``build``   -- compiles the HIP sources for gfx950.

The binding is imported lazily so that the input generators can be used on a
machine without the built library.
"""
__all__ = ["inputs", "binding", "build"]
