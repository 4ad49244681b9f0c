"""Incomplete LU factorisations -- test infrastructure (oracle).

Paper, section "Iterative Solvers": the preconditioner M ~ L~ is an
incomplete LU factorisation of the (permuted) modified Liouvillian, and its
quality is judged by the condition estimate ||(LU)^{-1} e||_inf, e = (1,...,1).

ilu0  -- ILU with zero fill: L unit lower and U upper keep exactly the
         pattern of A, and (LU)_ij = a_ij on that pattern.  Computed in the
         row-wise (IKJ) elimination order, one row at a time.
ilu0_fixed_point -- the same zero-fill factors as the fixed point of their
         defining equations (LU)_ij = a_ij on the pattern, reached by
         synchronous sweeps (Chow and Patel, "Fine-grained parallel
         incomplete LU factorization", 2015; not in the paper, which builds
         its iLU by elimination): every entry is recomputed from the previous
         sweep's values, so a sweep has no order between entries.
ilut  -- dual-threshold ILU: during the elimination of row i, multipliers and
         fill entries smaller than drop_tol * ||a_i||_inf are dropped, and at
         most ceil(fill * nnz(a_i)) entries are kept in each of the strict lower
         and the strict upper part (largest magnitude first, ties to the lower
         column index); the diagonal is always kept.  No pivoting.
ilutp -- the same dual-threshold rules with column pivoting (the paper's
         "iLUT with dual-threshold and pivoting"): A Q = L U, where the
         column of largest magnitude among a row's kept upper entries becomes
         its pivot whenever permtol times its magnitude exceeds the diagonal
         candidate's (oracle/c/ilutp.c).  Factors in the permuted (position)
         numbering, with the permutation perm[position] = column.

Both return a single CSR matrix holding the strict lower part of L (the unit
diagonal is implicit) and U (diagonal included), with sorted column indices.
A pivot whose magnitude falls below guard * ||a_i||_inf is replaced by
boost * ||a_i||_inf times the pivot's phase (or by that value when it is
exactly zero) and counted; boost defaults to guard.  The solver uses
guard = 1e-8 and boost = 0.1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _guard(piv: complex, bound: float, value: float) -> tuple[complex, bool]:
    if abs(piv) >= bound:
        return piv, False
    if value <= 0:
        value = 1.0
    if piv == 0:
        return complex(value), True
    return piv / abs(piv) * value, True


def ilu0(A, guard: float = 0.0, boost: float | None = None):
    """ILU(0) of a square CSR matrix with a non-zero diagonal pattern.
    Returns (LU as csr_matrix, number of guarded pivots)."""
    boost = guard if boost is None else boost
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    n = A.shape[0]
    indptr, indices = A.indptr, A.indices
    vals = A.data.copy()
    # column -> position map per row, and the diagonal position
    pos = [dict(zip(indices[indptr[i]:indptr[i + 1]].tolist(),
                    range(indptr[i], indptr[i + 1]))) for i in range(n)]
    diag = np.array([pos[i].get(i, -1) for i in range(n)])
    if np.any(diag < 0):
        raise ValueError("ilu0: structurally zero diagonal")
    guarded = 0
    for i in range(n):
        rownorm = float(np.max(np.abs(A.data[indptr[i]:indptr[i + 1]]))) if indptr[i + 1] > indptr[i] else 0.0
        row_pos = pos[i]
        for e in range(indptr[i], diag[i]):          # k < i, ascending
            k = indices[e]
            vals[e] = vals[e] / vals[diag[k]]
            lik = vals[e]
            for f in range(diag[k] + 1, indptr[k + 1]):  # u_kj, j > k
                j = indices[f]
                p = row_pos.get(j)
                if p is not None:
                    vals[p] -= lik * vals[f]
        if guard > 0:
            v, g = _guard(complex(vals[diag[i]]), guard * rownorm, boost * rownorm)
            vals[diag[i]] = v
            guarded += int(g)
    return sp.csr_matrix((vals, indices.copy(), indptr.copy()), shape=A.shape), guarded


def ilu0_fixed_point(A, sweeps: int, guard: float = 0.0, boost: float | None = None):
    """ILU(0) factors after `sweeps` synchronous fixed-point sweeps.

    Unknowns: l_ij (j < i) and u_ij (j >= i) on the pattern of A, with
    l_ii = 1.  The equations (LU)_ij = a_ij give, for every pattern entry,
        u_ij = a_ij - sum_{k < i} l_ik u_kj                    (j >= i)
        l_ij = (a_ij - sum_{k < j} l_ik u_kj) / u_jj           (j < i)
    where the sums run over the k with (i, k) and (k, j) on the pattern.  A
    sweep evaluates every right-hand side with the previous sweep's values
    (the products subtracted from a_ij in increasing k, as the elimination
    does); the pivot guard of ilu0 is applied to each new u_ii.  Start:
    u_ii = a_ii through the same guard, l_ij = a_ij / u_jj, u_ij = a_ij
    (a structurally present zero or tiny a_jj, e.g. the shifted zero
    diagonal of inverse power, would otherwise put huge multipliers into the
    first sweeps).  After as many sweeps as the longest
    chain of dependencies between the unknowns, the values are those of
    ilu0 (up to rounding).  Returns (LU csr, pivots guarded in the last
    sweep)."""
    boost = guard if boost is None else boost
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    n = A.shape[0]
    indptr, indices, a = A.indptr, A.indices, A.data
    pos = [dict(zip(indices[indptr[i]:indptr[i + 1]].tolist(),
                    range(indptr[i], indptr[i + 1]))) for i in range(n)]
    diag = np.array([pos[i].get(i, -1) for i in range(n)])
    if np.any(diag < 0):
        raise ValueError("ilu0_fixed_point: structurally zero diagonal")
    rownorm = [float(np.max(np.abs(a[indptr[i]:indptr[i + 1]]))) for i in range(n)]
    x = a.copy()
    if guard > 0:
        for i in range(n):
            x[diag[i]] = _guard(complex(a[diag[i]]), guard * rownorm[i], boost * rownorm[i])[0]
    for i in range(n):
        for e in range(indptr[i], diag[i]):
            x[e] = a[e] / x[diag[indices[e]]]
    guarded = 0
    for _ in range(sweeps):
        new = np.empty_like(x)
        guarded = 0
        for i in range(n):
            for e in range(indptr[i], indptr[i + 1]):
                j = int(indices[e])
                v = complex(a[e])
                for e2 in range(indptr[i], diag[i]):      # k < i, ascending
                    k = int(indices[e2])
                    if k >= j:
                        break
                    f = pos[k].get(j)                      # u_kj, j > k
                    if f is not None:
                        v -= x[e2] * x[f]
                if j < i:
                    v = v / x[diag[j]]
                elif j == i and guard > 0:
                    v, g = _guard(v, guard * rownorm[i], boost * rownorm[i])
                    guarded += int(g)
                new[e] = v
        x = new
    return sp.csr_matrix((x, indices.copy(), indptr.copy()), shape=A.shape), guarded


def ilut(A, drop_tol: float = 1e-4, fill: float = 10.0, guard: float = 0.0, boost: float | None = None):
    """Dual-threshold ILUT without pivoting.  Returns (LU csr, guarded pivots)."""
    boost = guard if boost is None else boost
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    n = A.shape[0]
    U_rows: list[dict] = [None] * n   # j -> u_ij for j >= i
    out_rows = []
    guarded = 0
    for i in range(n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        nz = len(cols)
        rownorm = float(np.max(np.abs(vals))) if nz else 0.0
        tau = drop_tol * rownorm
        keep = int(math.ceil(fill * nz))
        w = dict(zip(cols.tolist(), vals.tolist()))
        L_part = {}
        while True:
            lower = [c for c in w if c < i and c not in L_part]
            if not lower:
                break
            k = min(lower)
            wk = w[k] / U_rows[k][k]
            if abs(wk) < tau:
                del w[k]
                continue
            L_part[k] = wk
            w[k] = wk
            for j, ukj in U_rows[k].items():
                if j > k:
                    w[j] = w.get(j, 0.0) - wk * ukj
        # second dropping rule on the remaining entries
        lo = [(c, v) for c, v in w.items() if c < i and abs(v) >= tau]
        up = [(c, v) for c, v in w.items() if c > i and abs(v) >= tau]
        lo.sort(key=lambda cv: (-abs(cv[1]), cv[0]))
        up.sort(key=lambda cv: (-abs(cv[1]), cv[0]))
        lo = lo[:keep]
        up = up[:keep]
        piv = w.get(i, 0.0)
        if guard > 0:
            piv, g = _guard(complex(piv), guard * rownorm, boost * rownorm)
            guarded += int(g)
        elif piv == 0:
            raise ZeroDivisionError(f"ilut: zero pivot in row {i}")
        U_rows[i] = dict(up)
        U_rows[i][i] = piv
        row = sorted(lo + up + [(i, piv)])
        out_rows.append(row)
    indptr = np.zeros(n + 1, dtype=np.int64)
    for i, row in enumerate(out_rows):
        indptr[i + 1] = indptr[i] + len(row)
    indices = np.array([c for row in out_rows for c, _ in row], dtype=np.int32)
    data = np.array([v for row in out_rows for _, v in row], dtype=np.complex128)
    return sp.csr_matrix((data, indices, indptr), shape=A.shape), guarded


def ilut_c(A, drop_tol: float = 1e-4, fill: float = 10.0, guard: float = 0.0, boost: float | None = None):
    """The same ILUT as ilut(), computed by the oracle's C routine
    (oracle/c/ilut.c) with identical arithmetic, for full-size systems.
    Returns (LU csr, guarded pivots)."""
    from . import _clib
    boost = guard if boost is None else boost
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    n = A.shape[0]
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.complex128)
    nz = np.diff(indptr).astype(np.float64)
    cap = int(n + 2 * np.sum(np.ceil(fill * nz)))
    lp = np.zeros(n + 1, dtype=np.int64)
    li = np.zeros(max(cap, 1), dtype=np.int32)
    lv = np.zeros(max(cap, 1), dtype=np.complex128)
    rc = _clib.load().oracle_ilut(n, indptr.ctypes.data, indices.ctypes.data, data.ctypes.data, float(drop_tol),
                                  float(fill), float(guard), float(boost), cap, lp.ctypes.data, li.ctypes.data,
                                  lv.ctypes.data)
    if rc == -3:
        raise ZeroDivisionError("ilut: zero pivot")
    if rc < 0:
        raise MemoryError(f"oracle_ilut failed ({rc})")
    m = int(lp[n])
    return sp.csr_matrix((lv[:m].copy(), li[:m].copy(), lp), shape=A.shape), rc


def ilutp_c(A, drop_tol: float = 1e-4, fill: float = 10.0, permtol: float = 0.5, guard: float = 0.0,
            boost: float | None = None):
    """ILUTP (oracle/c/ilutp.c): A[:, perm] ~ L U.  Returns (LU csr in the
    position numbering, perm, guarded pivots); permtol = 0 is ilut_c."""
    from . import _clib
    boost = guard if boost is None else boost
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sort_indices()
    n = A.shape[0]
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.complex128)
    nz = np.diff(indptr).astype(np.float64)
    cap = int(n + 2 * np.sum(np.ceil(fill * nz)))
    perm = np.zeros(max(n, 1), dtype=np.int32)
    lp = np.zeros(n + 1, dtype=np.int64)
    li = np.zeros(max(cap, 1), dtype=np.int32)
    lv = np.zeros(max(cap, 1), dtype=np.complex128)
    rc = _clib.load().oracle_ilutp(n, indptr.ctypes.data, indices.ctypes.data, data.ctypes.data, float(drop_tol),
                                   float(fill), float(permtol), float(guard), float(boost), cap, perm.ctypes.data,
                                   lp.ctypes.data, li.ctypes.data, lv.ctypes.data)
    if rc == -3:
        raise ZeroDivisionError("ilutp: zero pivot")
    if rc < 0:
        raise MemoryError(f"oracle_ilutp failed ({rc})")
    m = int(lp[n])
    return sp.csr_matrix((lv[:m].copy(), li[:m].copy(), lp), shape=A.shape), perm[:n].copy(), rc


def apply_inverse_perm(LU, perm, b):
    """M^{-1} b for A Q ~ L U: z = (L U)^{-1} b, then x = Q z (x[perm] = z)."""
    z = apply_inverse(LU, b)
    x = np.empty_like(z)
    x[perm] = z
    return x


def split(LU):
    """(unit lower L, upper U) as separate CSR matrices."""
    LU = sp.csr_matrix(LU)
    n = LU.shape[0]
    L = sp.tril(LU, k=-1, format="csr") + sp.identity(n, dtype=LU.dtype, format="csr")
    U = sp.triu(LU, k=0, format="csr")
    return L.tocsr(), U.tocsr()


def apply_inverse(LU, b):
    """(LU)^{-1} b by forward then backward substitution."""
    from scipy.sparse.linalg import spsolve_triangular
    L, U = split(LU)
    y = spsolve_triangular(L, b, lower=True, unit_diagonal=True)
    return spsolve_triangular(U, y, lower=False)


def condition_estimate(LU) -> float:
    """||(LU)^{-1} e||_inf with e the all-ones vector."""
    n = LU.shape[0]
    return float(np.max(np.abs(apply_inverse(LU, np.ones(n, dtype=np.complex128)))))
