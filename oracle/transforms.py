"""Problem transforms of the Liouvillian -- test infrastructure (oracle).

modified  -- eq. (linear): L~ = L + w T, where T has ones in row 0 at the
             columns of the diagonal of rho (k (d + 1), k = 0..d-1) and w is a
             weight; right-hand side w e_0.  Default w = mean of the diagonal
             of L (the paper sets w to the average of the diagonal elements).
shifted   -- eq. (inverse): L - sigma I with sigma = 1e-15 (section "Eigenvalue
             Methods").
Entries that become exactly zero are dropped, as in the assembly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def mean_diagonal(L) -> complex:
    return complex(np.mean(sp.csr_matrix(L).diagonal()))


def modified(L, w: complex | None = None):
    """(L~, b, w) of eq. (linear)."""
    L = sp.csr_matrix(L, dtype=np.complex128)
    n = L.shape[0]
    d = int(round(np.sqrt(n)))
    if w is None:
        w = mean_diagonal(L)
    T = sp.csr_matrix((np.full(d, w, dtype=np.complex128),
                       (np.zeros(d, dtype=np.int64), np.arange(d) * (d + 1))), shape=(n, n))
    A = (L + T).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    b = np.zeros(n, dtype=np.complex128)
    b[0] = w
    return A, b, w


def shifted(L, sigma: float = 1e-15):
    """L - sigma I."""
    L = sp.csr_matrix(L, dtype=np.complex128)
    A = (L - sigma * sp.identity(L.shape[0], dtype=np.complex128, format="csr")).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A
