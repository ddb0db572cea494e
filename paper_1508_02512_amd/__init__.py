"""QMC integration of sector-decomposed Feynman integrals on AMD MI355X.

The integration runs in libqmc.so (hand-written HIP kernels for gfx950
behind the C ABI of include/qmc.h); ``qmc`` is its ctypes binding and
``frontend`` turns propagators into the sector list the library takes.
"""

__all__ = ["qmc", "frontend"]
