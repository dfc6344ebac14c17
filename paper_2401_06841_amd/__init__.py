"""MI355X-native modal DG right-hand side and SSP-RK3 stage for 3D isothermal Euler.

The compute path is the HIP library ``libdg.so`` (built from ``csrc/``) behind the
C ABI declared in ``include/dg.h``; ``dg`` is its thin ctypes binding.
"""
