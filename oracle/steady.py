"""Dense fp64 steady state -- test infrastructure (oracle).

Paper, section "Direct factorization", eq. (linear): the unit-trace property
turns L vec(rho) = 0 into a non-singular linear system.  The oracle replaces
row 0 of L by the trace row t (ones at the diagonal positions of vec(rho)) and
solves A x = e_0 with LAPACK LU (partial pivoting).  Because t^T L = 0 (trace
preservation), row 0 of L is a linear combination of the other rows, so this
system has the same solution as the paper's L + w T form for any w != 0; the
paper-literal form is provided as well (steady_state_dense_weighted).
"""
from __future__ import annotations

import numpy as np

from .liouvillian import liouvillian_dense, trace_row, unvec


def steady_state_dense(H, c_ops) -> np.ndarray:
    """rho_ss (d x d, complex128) from the trace-replaced Liouvillian."""
    L = liouvillian_dense(H, c_ops)
    n = L.shape[0]
    d = int(round(np.sqrt(n)))
    A = L.copy()
    A[0, :] = trace_row(d)
    b = np.zeros(n, dtype=np.complex128)
    b[0] = 1.0
    x = np.linalg.solve(A, b)
    return unvec(x, d)


def steady_state_dense_weighted(H, c_ops, w: complex | None = None) -> np.ndarray:
    """Eq. (linear) as printed: (L + w T) x = w e_0, T = e_0 t^T.  Default w is
    the mean of the diagonal of L."""
    L = liouvillian_dense(H, c_ops)
    n = L.shape[0]
    d = int(round(np.sqrt(n)))
    if w is None:
        w = np.mean(np.diag(L))
    A = L.copy()
    A[0, :] += w * trace_row(d)
    b = np.zeros(n, dtype=np.complex128)
    b[0] = w
    return unvec(np.linalg.solve(A, b), d)
