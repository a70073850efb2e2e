"""Block Krylov solves of the O(a)-improved Wilson-Dirac equation with many
right-hand sides on AMD Instinct MI355X (arXiv:0903.4936).

The work runs in libbkwd.so (hand-written HIP kernels for gfx950, C ABI in
include/bkwd.h); ``bkwd`` is its ctypes binding.  Importing this package does
not load the library; the first call does, and fails loudly if it is absent.
"""
from .bkwd import (  # noqa: F401
    BICGSTAB, BLOCK_BICGGR, BLOCK_BICGSTAB, COMPRESS12, FP32, FP64, MIXED, BkwdError, Lattice,
    NotConverged, SolveInfo, SolveOpts, lattice_bytes, lib,
)
from .autograd import block_solve  # noqa: F401,E402
