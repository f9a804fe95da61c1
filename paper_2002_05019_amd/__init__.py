"""MI355X-native direct domain-decomposition (D3M-style) FEM solver.

The solver lives in a C-ABI shared library (``libdd.so``, declared in
``include/dd.h``) built from the HIP/C++ sources in ``csrc/``; ``binding``
is a thin ctypes layer over it and ``problem`` builds seeded synthetic
curl-curl workloads.
"""
__all__ = ["problem", "binding"]
