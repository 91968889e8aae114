"""MI355X (gfx950) matrix-free nonlinear-elasticity solvers: NK, iNK, L-BFGS.

The compute path is the HIP library libnlelast.so (C ABI in include/nlelast.h);
`nlelast` is its thin ctypes binding and `problems` assembles the synthetic
workloads (Cook's membrane) on top of it.
"""

from . import nlelast  # noqa: F401

__all__ = ["nlelast"]
