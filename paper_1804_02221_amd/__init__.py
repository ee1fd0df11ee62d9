"""MI355X-native entropy-stable DGSEM for the 2D shallow water equations.

The solver is the HIP library ``libesdg.so`` behind the C ABI of
``include/esdg.h``; ``esdg`` is its ctypes binding and ``inputs`` builds the
seeded synthetic workloads.
"""
__all__ = ["esdg", "inputs", "build"]
