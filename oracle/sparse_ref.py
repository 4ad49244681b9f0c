"""CPU fp64 sparse reference solve -- test infrastructure (oracle).

For systems too large for the dense LU of oracle.steady (n = d^2 beyond ~10^4:
the Kerr chain with n = 10^6, optomechanics with n = 3.6 * 10^5) the steady
state is computed the way the paper computes it with an iterative solver:

  * eq. (linear): L~ = L + w T with T in a population row (the row with the
    smallest |L_rr|, or row 0 as the paper prints it), b = w e_row;
  * section "Direct factorization": reverse Cuthill-McKee ordering of L~ on
    the pattern of L~ + L~^T, P L~ P^T;
  * section "Iterative Solvers", eq. (modified): an incomplete LU
    preconditioner (zero fill, oracle/c/sparse_ref.c, or the oracle's ILUT)
    and BiCGSTAB (van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992) 631),
    here preconditioned on the right so that its residual is the residual of
    L~ x = b, or scipy's restarted GMRES;
  * the solve is restarted from its own true residual until
    ||L vec(rho)||_2 <= tol with rho = unvec(x) / Tr, the certificate of
    eq. (ss).

Everything runs in complex128 on one CPU thread (plain C loops for the
factorisation and the triangular solves, scipy's CSR product, numpy vector
operations with BLAS limited to one thread by the caller where it matters).
It is written independently of the GPU solver and shares no code with it.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import scipy.sparse as sp

from . import _clib
from .liouvillian import liouvillian_sparse, unvec
from .ordering import permute, rcm
from .transforms import modified, trace_population


def _lib():
    lib = _clib.load()
    if not getattr(lib, "_sparse_ref_ready", False):
        lib.oracle_ilu0.restype = ctypes.c_int
        lib.oracle_ilu0.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_double]
        lib.oracle_lu_solve.restype = None
        lib.oracle_lu_solve.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib._sparse_ref_ready = True
    return lib


def with_diagonal(A) -> sp.csr_matrix:
    """A with an explicit (zero) entry at every structurally missing diagonal
    position, so that zero-fill ILU has a pivot position in every row."""
    A = sp.csr_matrix(A, dtype=np.complex128)
    n = A.shape[0]
    C = A.tocoo()
    have = np.zeros(n, dtype=bool)
    have[C.row[C.row == C.col]] = True
    miss = np.flatnonzero(~have)
    if miss.size == 0:
        A.sort_indices()
        return A
    rows = np.concatenate([C.row, miss])
    cols = np.concatenate([C.col, miss])
    vals = np.concatenate([C.data, np.zeros(miss.size, dtype=np.complex128)])
    B = sp.csr_matrix((vals, (rows, cols)), shape=A.shape)
    B.sum_duplicates()
    B.sort_indices()
    return B


class Ilu0:
    """Zero-fill ILU of a CSR matrix (C routine) and the application of its
    inverse by forward and backward substitution."""

    def __init__(self, A, guard: float = 0.0, boost: float | None = None):
        boost = guard if boost is None else boost
        A = with_diagonal(A)
        self.n = A.shape[0]
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.vals = np.ascontiguousarray(A.data, dtype=np.complex128).copy()
        rc = _lib().oracle_ilu0(self.n, self.indptr.ctypes.data, self.indices.ctypes.data, self.vals.ctypes.data,
                                float(guard), float(boost))
        if rc == -3:
            raise ZeroDivisionError("ilu0: zero pivot")
        if rc < 0:
            raise MemoryError(f"oracle_ilu0 failed ({rc})")
        self.guarded = rc
        self._diagonal()

    def _diagonal(self):
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.indptr))
        self.diag = np.ascontiguousarray(np.flatnonzero(self.indices == rows).astype(np.int64))


    def matrix(self) -> sp.csr_matrix:
        """The factors in one CSR: strict lower part of L, then U."""
        return sp.csr_matrix((self.vals.copy(), self.indices.copy(), self.indptr.copy()), shape=(self.n, self.n))

    def solve(self, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.complex128)
        x = np.empty_like(b)
        _lib().oracle_lu_solve(self.n, self.indptr.ctypes.data, self.indices.ctypes.data, self.vals.ctypes.data,
                               self.diag.ctypes.data, b.ctypes.data, x.ctypes.data)
        return x


class Ilut(Ilu0):
    """The dual-threshold ILUT of oracle.ilu (C routine), applied like Ilu0."""

    def __init__(self, A, drop_tol: float = 1e-4, fill: float = 10.0, guard: float = 0.0,
                 boost: float | None = None):
        from .ilu import ilut_c
        LU, self.guarded = ilut_c(with_diagonal(A), drop_tol, fill, guard=guard, boost=boost)
        LU.sort_indices()
        self.n = LU.shape[0]
        self.indptr = np.ascontiguousarray(LU.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(LU.indices, dtype=np.int32)
        self.vals = np.ascontiguousarray(LU.data, dtype=np.complex128).copy()
        self._diagonal()


def bicgstab(A, b: np.ndarray, M, x0: np.ndarray, rtol: float, maxiter: int):
    """Right-preconditioned BiCGSTAB for A x = b (M.solve applies M^-1).
    Stops at ||b - A x||_2 <= rtol ||b||_2 (recurrence residual, checked
    against the true residual on exit).  Returns (x, iterations, breakdown)."""
    x = x0.copy()
    r = b - A @ x
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, False
    rhat = r.copy()
    rho_prev = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for it in range(1, maxiter + 1):
        rho = np.vdot(rhat, r)
        if abs(rho) <= 1e-300:
            return x, it - 1, True
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = M.solve(p)
        v = A @ ph
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        if np.linalg.norm(s) <= rtol * bn:
            x = x + alpha * ph
            return x, it, False
        sh = M.solve(s)
        t = A @ sh
        tt = np.vdot(t, t)
        if tt == 0:
            return x + alpha * ph, it, True
        omega = np.vdot(t, s) / tt
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_prev = rho
        if np.linalg.norm(r) <= rtol * bn:
            return x, it, False
        if omega == 0:
            return x, it, True
    return x, maxiter, False


def gmres(A, b: np.ndarray, M, x0: np.ndarray, rtol: float, maxiter: int, restart: int = 50):
    """Restarted GMRES (scipy's) preconditioned with M.solve; returns
    (x, iterations, False) like bicgstab()."""
    import scipy.sparse.linalg as spla
    count = [0]
    Mop = spla.LinearOperator(A.shape, matvec=M.solve, dtype=np.complex128)
    x, _ = spla.gmres(A, b, x0=x0, M=Mop, rtol=rtol, restart=restart, maxiter=max(1, maxiter // restart),
                      callback=lambda _r: count.__setitem__(0, count[0] + 1), callback_type="pr_norm")
    return x, count[0], False


def steady_state_iterative(H, c_ops, tol: float = 1e-12, rtol_in: float = 1e-10, maxiter: int = 2000,
                           max_restarts: int = 10, pop: int | None = None, L=None, ilu: str = "ilu0",
                           krylov: str = "bicgstab", drop_tol: float = 1e-4, fill: float = 10.0):
    """rho_ss by RCM-ordered ILU-preconditioned BiCGSTAB (or GMRES) on the
    trace-row system, in fp64; ilu = "ilu0" or "ilut" (drop_tol, fill).
    Returns (rho, info) with the iteration counts, the certificate
    ||L vec rho||_2 and the times of the set-up and the solve."""
    t0 = time.perf_counter()
    if L is None:
        L = liouvillian_sparse(H, c_ops)
    if pop is None:
        pop = trace_population(L)
    A, b, w = modified(L, pop=pop)
    n = A.shape[0]
    d = int(round(np.sqrt(n)))
    perm = rcm(A)
    Ap = with_diagonal(permute(A, perm))
    bp = b[perm]
    M = Ilu0(Ap, guard=1e-8, boost=0.1) if ilu == "ilu0" else Ilut(Ap, drop_tol, fill, guard=1e-8, boost=0.1)
    krylov_solve = bicgstab if krylov == "bicgstab" else gmres
    t1 = time.perf_counter()
    x = np.zeros(n, dtype=np.complex128)
    its, outer, res, breakdowns = 0, 0, np.inf, 0
    rho = None
    for outer in range(1, max_restarts + 1):
        # refinement: the correction solves A delta = b - A x to rtol_in
        # relative to the current residual
        delta, k, bd = krylov_solve(Ap, bp - Ap @ x, M, np.zeros_like(x), rtol_in, maxiter)
        x = x + delta
        its += k
        breakdowns += int(bd)
        xn = np.empty_like(x)
        xn[perm] = x
        tr = np.trace(unvec(xn, d))
        rho = unvec(xn, d) / tr
        res = float(np.linalg.norm(L @ xn) / abs(tr))
        if res <= tol:
            break
    t2 = time.perf_counter()
    info = {"iterations": its, "restarts": outer, "resid_l2": res, "breakdowns": breakdowns,
            "guarded": M.guarded, "pop": pop, "weight": w, "t_setup_s": t1 - t0, "t_solve_s": t2 - t1,
            "nnz": int(Ap.nnz)}
    return rho, info
