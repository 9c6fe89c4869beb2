"""MI355X (gfx950) library for the matrix-free SIPG Laplacian in the
Hermite-like basis (Kronbichler et al., Hermite-like basis for faster
matrix-free evaluation of interior penalty DG operators).

The compute path is the HIP library `libsipg.so` (C ABI in include/sipg.h);
this package is a thin ctypes binding over it.  Build the library with
`python -m paper_1907_08492_amd.build` (or `__graft_entry__.build()`).
"""
from .binding import (  # noqa: F401
    BASIS, BC_MODES, DTYPE, EXPORTED, GEOMETRY, LIB_PATH, SIPG_E_ARG, SIPG_E_BUDGET, SIPG_E_NOCONV, SIPG_OK,
    TORCH_ALLOCATOR, Batch, Multigrid, Operator, Server, SipgAllocator, SipgError, SipgSolveInfo, SolveInfo,
    host_block_order, host_fdm_tables, host_tables, launch_shape, lib, make_mesh,
)
