"""Liouvillian super-operator as a matrix -- test infrastructure (oracle).

Paper, section "Steady-state density matrix", eq. (lindblad) and the
dissipator D[C, rho] = (2 C rho C+ - rho C+C - C+C rho)/2, hbar = 1.  The
matrix form of eq. (eigval) uses column stacking: vec(rho)[i + d*j] = rho[i, j],
so that vec(A rho B) = (B^T kron A) vec(rho).  Hence

    L = -i (I kron H - H^T kron I)
        + sum_k [ conj(C_k) kron C_k - 1/2 I kron (C_k+ C_k) - 1/2 (C_k+ C_k)^T kron I ].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _dense(m) -> np.ndarray:
    return m.toarray().astype(np.complex128) if sp.issparse(m) else np.asarray(m, dtype=np.complex128)


def liouvillian_dense(H, c_ops) -> np.ndarray:
    """Dense n x n Liouvillian, n = d^2 (eq. lindblad, column stacking)."""
    H = _dense(H)
    d = H.shape[0]
    I = np.eye(d, dtype=np.complex128)
    L = -1j * (np.kron(I, H) - np.kron(H.T, I))
    for C in c_ops:
        C = _dense(C)
        CdC = C.conj().T @ C
        L = L + np.kron(C.conj(), C) - 0.5 * np.kron(I, CdC) - 0.5 * np.kron(CdC.T, I)
    return L


def liouvillian_sparse(H, c_ops) -> sp.csr_matrix:
    """The same matrix assembled with sparse Kronecker products (for sizes the
    dense form cannot hold).  Entries that sum to exactly zero are dropped."""
    H = sp.csr_matrix(H, dtype=np.complex128)
    d = H.shape[0]
    I = sp.identity(d, dtype=np.complex128, format="csr")
    L = -1j * (sp.kron(I, H, format="csr") - sp.kron(H.T, I, format="csr"))
    for C in c_ops:
        C = sp.csr_matrix(C, dtype=np.complex128)
        CdC = (C.conj().T @ C).tocsr()
        L = (L + sp.kron(C.conj(), C, format="csr") - 0.5 * sp.kron(I, CdC, format="csr")
             - 0.5 * sp.kron(CdC.T, I, format="csr"))
    L = sp.csr_matrix(L)
    L.sum_duplicates()
    L.eliminate_zeros()
    L.sort_indices()
    return L


def vec(rho: np.ndarray) -> np.ndarray:
    """Column stacking (eq. eigval)."""
    return np.asarray(rho).reshape(-1, order="F")


def unvec(x: np.ndarray, d: int) -> np.ndarray:
    return np.asarray(x).reshape(d, d, order="F")


def trace_row(d: int) -> np.ndarray:
    """Row vector t with ones at the positions of the diagonal of rho in
    vec(rho): t[k*(d+1)] = 1 (the non-zero row of the matrix T, eq. linear)."""
    t = np.zeros(d * d, dtype=np.complex128)
    t[np.arange(d) * (d + 1)] = 1.0
    return t
