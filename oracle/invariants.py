"""Density-matrix invariants and the residual certificate -- test
infrastructure (oracle).  A steady state must be Hermitian, positive
semidefinite, of unit trace, and annihilated by the Liouvillian (eq. ss)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .liouvillian import vec


def hermiticity_error(rho: np.ndarray) -> float:
    return float(np.max(np.abs(rho - rho.conj().T)))


def trace_error(rho: np.ndarray) -> float:
    return float(abs(np.trace(rho) - 1.0))


def min_eigenvalue(rho: np.ndarray) -> float:
    return float(np.min(np.linalg.eigvalsh(0.5 * (rho + rho.conj().T))))


def residual_l2(L, rho: np.ndarray) -> float:
    """||L vec(rho)||_2 for a dense or sparse Liouvillian matrix."""
    x = vec(rho)
    y = L @ x if sp.issparse(L) else np.asarray(L) @ x
    return float(np.linalg.norm(y))


def superop_action(H, c_ops, rho: np.ndarray) -> np.ndarray:
    """L[rho] evaluated with d x d matrix products, eq. (lindblad), without
    any vectorisation: -i[H, rho] + sum_k (C rho C+ - {C+C, rho}/2)."""
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H)
    out = -1j * (Hd @ rho - rho @ Hd)
    for C in c_ops:
        Cd = C.toarray() if sp.issparse(C) else np.asarray(C)
        CdC = Cd.conj().T @ Cd
        out = out + Cd @ rho @ Cd.conj().T - 0.5 * (rho @ CdC + CdC @ rho)
    return out
