"""Bandwidth, profile and (reverse) Cuthill-McKee ordering -- test
infrastructure (oracle).

Paper, section "Direct factorization":
  * upper/lower bandwidth ub = max_{a_ij != 0} (j - i), lb = max_{a_ij != 0} (i - j),
    total bandwidth B = ub + lb + 1;
  * upper profile up = sum over rows i of max_{a_ij != 0} (j - i), lower profile
    lp = sum over columns j of max_{a_ij != 0} (i - j), P = up + lp (each
    per-row / per-column maximum is taken as 0 when negative or absent);
  * RCM is computed on the structure of A + A^T and the same permutation is
    applied to rows and columns.

The Cuthill-McKee search itself is plain C (oracle/c/cm_order.c), compiled
with gcc on first use so large graphs stay fast.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import _clib


def build_c() -> str:
    """Compile the C part of the oracle (kept for the build step)."""
    return _clib.build_c()


def _load():
    return _clib.load()


def pattern(A) -> sp.csr_matrix:
    """Boolean structure of the non-zero entries of A (explicit zeros excluded)."""
    A = sp.csr_matrix(A)
    # copies of the index arrays: eliminate_zeros works in place, and A may
    # share its arrays with the caller's matrix
    P = sp.csr_matrix((A.data != 0, A.indices.copy(), A.indptr.copy()), shape=A.shape)
    P.eliminate_zeros()
    P = P.astype(np.int8)
    P.sort_indices()
    return P


def symmetrized_pattern(A) -> sp.csr_matrix:
    """Structure of A + A^T (the union of both patterns)."""
    P = pattern(A)
    S = ((P + P.T) != 0).astype(np.int8).tocsr()
    S.sort_indices()
    return S


def bandwidth(A) -> tuple[int, int, int]:
    """(ub, lb, B) of the non-zero structure."""
    C = pattern(A).tocoo()
    if C.nnz == 0:
        return 0, 0, 1
    diff = C.col.astype(np.int64) - C.row.astype(np.int64)
    ub = max(int(diff.max()), 0)
    lb = max(int((-diff).max()), 0)
    return ub, lb, ub + lb + 1


def profile(A) -> tuple[int, int, int]:
    """(up, lp, P) of the non-zero structure."""
    C = pattern(A).tocoo()
    n = A.shape[0]
    r = C.row.astype(np.int64)
    c = C.col.astype(np.int64)
    row_max = np.zeros(n, dtype=np.int64)
    np.maximum.at(row_max, r, c - r)
    col_max = np.zeros(A.shape[1], dtype=np.int64)
    np.maximum.at(col_max, c, r - c)
    up = int(row_max.sum())
    lp = int(col_max.sum())
    return up, lp, up + lp


def cuthill_mckee(S) -> np.ndarray:
    """Cuthill-McKee visit order of a symmetric pattern S (CSR)."""
    S = sp.csr_matrix(S)
    S.sort_indices()
    n = S.shape[0]
    indptr = np.ascontiguousarray(S.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(S.indices, dtype=np.int32)
    order = np.empty(n, dtype=np.int32)
    rc = _load().oracle_cuthill_mckee(n, indptr.ctypes.data, indices.ctypes.data, order.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle Cuthill-McKee: allocation failed")
    return order


def rcm(A) -> np.ndarray:
    """Reverse Cuthill-McKee permutation of A: perm[new] = old, computed on the
    structure of A + A^T."""
    return cuthill_mckee(symmetrized_pattern(A))[::-1].copy()


def permute(A, perm) -> sp.csr_matrix:
    """P A P^T with P the row permutation perm[new] = old."""
    A = sp.csr_matrix(A)
    B = A[perm, :][:, perm].tocsr()
    B.sort_indices()
    return B


def greedy_colouring(S, order) -> tuple[np.ndarray, int]:
    """(colour, number of colours) of the sequential greedy colouring of the
    symmetric pattern S visited in `order` (order[k] = vertex visited k-th):
    each vertex gets the smallest non-negative colour that none of its
    already visited neighbours carries; self-loops are not edges (plain C,
    oracle/c/colour.c).  Not a step of the paper: it serves the colour-class
    ordering below."""
    S = sp.csr_matrix(S)
    n = S.shape[0]
    order = np.ascontiguousarray(order, dtype=np.int32)
    if n == 0:
        return np.zeros(0, dtype=np.int32), 0
    if order.shape != (n,) or not np.array_equal(np.sort(order), np.arange(n)):
        raise ValueError("order must be a permutation of the vertices")
    indptr = np.ascontiguousarray(S.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(S.indices, dtype=np.int32)
    colour = np.empty(n, dtype=np.int32)
    used = _load().oracle_greedy_colour(n, indptr.ctypes.data, indices.ctypes.data, order.ctypes.data,
                                        colour.ctypes.data)
    if used < 0:
        raise MemoryError("oracle greedy colouring: allocation failed")
    return colour, int(used)


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(k) -> np.ndarray:
    """Outputs k = 0, 1, ... of SplitMix64 seeded with 0 (Steele, Lea and
    Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
    z = (k + 1) * 0x9E3779B97F4A7C15 mod 2^64, then z ^= z >> 30,
    z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB,
    z ^= z >> 31."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (k + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def random_visit(n: int) -> np.ndarray:
    """The vertices 0..n-1 in increasing (splitmix64(v), v) order: a seeded
    random visit order whose priorities each side can compute from the
    vertex index alone."""
    v = np.arange(n, dtype=np.int64)
    return np.lexsort((v, splitmix64(v))).astype(np.int32)


def colour_order(A, base=None) -> np.ndarray:
    """Colour-class ordering perm[new] = old: the greedy colouring of the
    structure of A + A^T visited in the random order random_visit(n),
    classes in increasing colour, each class in the base order (RCM of A by
    default).  Every off-diagonal entry of the reordered matrix then joins
    two different classes, so a zero-fill triangular factor has at most as
    many levels as there are colours."""
    if base is None:
        base = rcm(A)
    base = np.asarray(base, dtype=np.int32)
    colour, _ = greedy_colouring(symmetrized_pattern(A), random_visit(A.shape[0]))
    return base[np.argsort(colour[base], kind="stable")].astype(np.int32)
