"""Problem transforms of the Liouvillian -- test infrastructure (oracle).

modified  -- eq. (linear): L~ = L + w T, where T has ones in one row at the
             columns of the diagonal of rho (k (d + 1), k = 0..d-1) and w is a
             weight; right-hand side w e_row.  Default w = mean of the diagonal
             of L (the paper sets w to the average of the diagonal elements).
             The paper puts T in row 0 and notes the choice of row is
             arbitrary; any population row r = k (d + 1) works because the
             population rows of L sum to zero.  trace_population() is the rule
             the solver uses by default: the population row with the smallest
             |L_rr| (lowest k among ties), so a structurally zero diagonal
             (a ground state no channel leaves) receives the trace entry.
shifted   -- eq. (inverse): L - sigma I with sigma = 1e-15 (section "Eigenvalue
             Methods").
Entries that become exactly zero are dropped, as in the assembly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def mean_diagonal(L) -> complex:
    return complex(np.mean(sp.csr_matrix(L).diagonal()))


def trace_population(L) -> int:
    """k minimising |L[k (d + 1), k (d + 1)]| (lowest k among ties)."""
    L = sp.csr_matrix(L)
    d = int(round(np.sqrt(L.shape[0])))
    diag = np.abs(L.diagonal()[np.arange(d) * (d + 1)])
    return int(np.argmin(diag))


def modified(L, w: complex | None = None, pop: int = 0):
    """(L~, b, w) of eq. (linear) with T in row pop * (d + 1)."""
    L = sp.csr_matrix(L, dtype=np.complex128)
    n = L.shape[0]
    d = int(round(np.sqrt(n)))
    if w is None:
        w = mean_diagonal(L)
    row = pop * (d + 1)
    T = sp.csr_matrix((np.full(d, w, dtype=np.complex128),
                       (np.full(d, row, dtype=np.int64), np.arange(d) * (d + 1))), shape=(n, n))
    A = (L + T).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    b = np.zeros(n, dtype=np.complex128)
    b[row] = w
    return A, b, w


def shifted(L, sigma: float = 1e-15):
    """L - sigma I."""
    L = sp.csr_matrix(L, dtype=np.complex128)
    A = (L - sigma * sp.identity(L.shape[0], dtype=np.complex128, format="csr")).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A
