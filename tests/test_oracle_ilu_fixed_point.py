"""Pins of the oracle's fixed-point ILU(0) (Chow and Patel's synchronous
sweeps over the equations (LU)_ij = a_ij on the pattern): the starting
guess, finite termination on a dependency chain, the complete LU of a dense
matrix (scipy's LU without row exchanges), and the elimination-order ILU(0)
of sparse matrices and of a transformed Liouvillian, with and without the
pivot guard."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import qsystems as qs
from oracle.ilu import ilu0, ilu0_fixed_point
from oracle.liouvillian import liouvillian_sparse
from oracle.ordering import permute, rcm
from oracle.transforms import modified, trace_population


def _rel(a, b):
    a, b = sp.csr_matrix(a), sp.csr_matrix(b)
    return abs(a - b).max() / abs(b).max()


def _sparse_dd(n, density, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=seed, format="csr")
    M.data = rng.normal(size=M.nnz) + 1j * rng.normal(size=M.nnz)
    M = M + sp.diags(np.abs(M).sum(axis=1).A1 + np.abs(M).sum(axis=0).A1 + 1.0)
    return sp.csr_matrix(M)


def test_zero_sweeps_is_the_starting_guess():
    A = _sparse_dd(30, 0.15, 1)
    A.sort_indices()
    LU, _ = ilu0_fixed_point(A, 0)
    for i in range(30):
        for e in range(A.indptr[i], A.indptr[i + 1]):
            j = A.indices[e]
            want = A.data[e] / A[j, j] if j < i else A.data[e]
            assert LU.data[e] == want


def test_starting_guess_takes_the_guarded_pivots():
    # a_11 = 1e-20 is below 1e-8 * ||a_1||_inf = 2e-8: u_11 starts at 0.1 * 2,
    # and l_21 = a_21 / u_11
    A = sp.csr_matrix(np.array([[3.0, 1.0, 0.0], [1.0, 1e-20, 2.0], [0.0, 5.0, 7.0]], dtype=np.complex128))
    LU, _ = ilu0_fixed_point(A, 0, guard=1e-8, boost=0.1)
    assert LU[1, 1] == 0.2
    assert LU[2, 1] == 5.0 / 0.2
    assert LU[1, 0] == 1.0 / 3.0 and LU[0, 0] == 3.0 and LU[2, 2] == 7.0


def test_tridiagonal_chain_terminates():
    # u_ii depends on u_{i-1,i-1}: the last pivot needs about n sweeps
    n = 8
    rng = np.random.default_rng(3)
    A = sp.diags([rng.normal(size=n - 1), 4.0 + rng.normal(size=n), rng.normal(size=n - 1)], [-1, 0, 1], format="csr")
    A = sp.csr_matrix(A, dtype=np.complex128)
    ref, _ = ilu0(A)
    assert _rel(ilu0_fixed_point(A, 2)[0], ref) > 1e-6
    assert _rel(ilu0_fixed_point(A, 2 * n)[0], ref) <= 1e-15


def test_dense_matrix_gives_the_complete_lu():
    n = 6
    rng = np.random.default_rng(5)
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    # column diagonal dominance: partial pivoting exchanges no rows
    M += np.diag(np.abs(M).sum(axis=0) + 1.0)
    P, Lr, Ur = sla.lu(M)
    assert np.array_equal(P, np.eye(n))
    LU, _ = ilu0_fixed_point(sp.csr_matrix(M), 2 * n)
    D = LU.toarray()
    assert np.max(np.abs(np.tril(D, -1) - np.tril(Lr, -1))) <= 1e-13 * np.max(np.abs(Lr))
    assert np.max(np.abs(np.triu(D) - Ur)) <= 1e-13 * np.max(np.abs(Ur))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sparse_matrices_reach_the_elimination_ilu0(seed):
    A = _sparse_dd(60, 0.06, seed)
    ref, _ = ilu0(A)
    assert _rel(ilu0_fixed_point(A, 60)[0], ref) <= 1e-14
    # a few sweeps already give a close approximation on diagonally dominant matrices
    assert _rel(ilu0_fixed_point(A, 3)[0], ref) < _rel(ilu0_fixed_point(A, 1)[0], ref)


def test_liouvillian_with_the_pivot_guard():
    s = qs.kerr(6)
    L = liouvillian_sparse(s.H, s.c_ops)
    A, _, _ = modified(L, pop=trace_population(L))
    A = permute(A, rcm(A))
    ref, gref = ilu0(A, guard=1e-8, boost=0.1)
    LU, g = ilu0_fixed_point(A, A.shape[0], guard=1e-8, boost=0.1)
    assert g == gref
    assert _rel(LU, ref) <= 1e-12


def test_guard_fires_at_the_fixed_point():
    # second pivot a_11 - a_10 a_01 / a_00 = 1 - 1 = 0: boosted to 0.1 * ||a_1||_inf
    A = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 3.0]], dtype=np.complex128))
    ref, gref = ilu0(A, guard=1e-8, boost=0.1)
    LU, g = ilu0_fixed_point(A, 6, guard=1e-8, boost=0.1)
    assert gref == 1 and g == 1
    assert abs(LU[1, 1] - 0.1) <= 1e-15
    assert _rel(LU, ref) <= 1e-15
