"""MI355X steady-state solver for Lindblad master equations.

Python binding of the C ABI in include/ss.h (argument marshalling only: every
step of the solve runs in the HIP library libss.so).  The library must have
been built (python paper_1504_06768_amd/build.py); importing this package
fails loudly otherwise.
"""
from .ss import (  # noqa: F401
    SS_OK, SS_E_INVALID_ARG, SS_E_NOT_CONVERGED, SS_E_BREAKDOWN,
    SS_FP64, SS_MIXED, SS_ILU0, SS_ILUT, SS_ORDER_RCM, SS_ORDER_NATURAL, SS_ORDER_COLOUR,
    SS_TRACE_BICGSTAB, SS_TRACE_GMRES, SS_INVPOW_BICGSTAB, SS_INVPOW_GMRES, SS_AUTO,
    SS_MAT_L, SS_MAT_A, SS_MAT_A_PERM, SS_MAT_LU, SS_MAT_SYM,
    SS_OP_SPMV_L, SS_OP_SPMV_APERM, SS_OP_PRECOND, SS_OP_LSOLVE, SS_OP_USOLVE, SS_OP_PRECOND_SYNCFREE,
    SS_OP_PRECOND_BLOCK, SS_OP_PRECOND_LEVELS, SS_OP_PRECOND_GROUPS, SS_OP_PRECOND_CLASSES, SS_OP_APPLY_L,
    SS_FLAG_MATRIX_FREE, SS_FLAG_TRSV_CLASSES,
    SolverError, Liouvillian, Server, apply, bandwidth_profile, build_liouvillian, build_liouvillian_batch,
    apply_noalloc, export_csr, export_perm, library_path, options, prepare, set_allocator, solve, solve_batch, time_operator,
    trim_cache, version,
)
