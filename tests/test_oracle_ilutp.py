"""Pins of the oracle's ILUTP (dual-threshold incomplete LU with column
pivoting, section "Iterative Solvers"): hand-worked factorisations, the
limit without pivoting (the oracle's ILUT, bit for bit) and the complete-LU
limit (Gaussian elimination with partial pivoting by columns, whose pivot
order LAPACK gives for the transpose)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import qsystems as qs
from oracle import ilu as oilu
from oracle.liouvillian import liouvillian_sparse
from oracle.ordering import permute, rcm
from oracle.transforms import modified, trace_population


def _dense(LU):
    L, U = oilu.split(LU)
    return L.toarray(), U.toarray()


def test_hand_worked_zero_diagonal_is_pivoted_away():
    # row 0 has no diagonal: column 1 becomes its pivot (perm = [1, 0, 2]);
    # row 1 then eliminates position 0 with l = 1/2 and keeps w = 1 as pivot
    A = sp.csr_matrix(np.array([[0, 2, 0], [1, 1, 0], [0, 0, 3]], dtype=complex))
    LU, perm, g = oilu.ilutp_c(A, drop_tol=0.0, fill=10.0, permtol=0.5)
    L, U = _dense(LU)
    assert perm.tolist() == [1, 0, 2] and g == 0
    assert np.array_equal(L, np.array([[1, 0, 0], [0.5, 1, 0], [0, 0, 1]], dtype=complex))
    assert np.array_equal(U, np.diag([2, 1, 3]).astype(complex))


@pytest.mark.parametrize("permtol,swap", [(0.5, True), (0.3, False)])
def test_hand_worked_threshold(permtol, swap):
    # row 0 = (1, 3): swapped when permtol * 3 > 1
    A = sp.csr_matrix(np.array([[1, 3], [2, 1]], dtype=complex))
    LU, perm, _ = oilu.ilutp_c(A, drop_tol=0.0, fill=10.0, permtol=permtol)
    L, U = _dense(LU)
    if swap:
        # A[:, [1, 0]] = [[3, 1], [1, 2]] = [[1, 0], [1/3, 1]] [[3, 1], [0, 5/3]]
        assert perm.tolist() == [1, 0]
        assert np.allclose(L, [[1, 0], [1 / 3, 1]], rtol=0, atol=1e-16)
        assert np.allclose(U, [[3, 1], [0, 5 / 3]], rtol=0, atol=1e-15)
    else:
        # no pivoting: [[1, 3], [2, 1]] = [[1, 0], [2, 1]] [[1, 3], [0, -5]]
        assert perm.tolist() == [0, 1]
        assert np.array_equal(L, np.array([[1, 0], [2, 1]], dtype=complex))
        assert np.array_equal(U, np.array([[1, 3], [0, -5]], dtype=complex))


def test_without_pivoting_it_is_the_oracle_ilut_bit_for_bit():
    mats = []
    for seed in range(4):
        A = (sp.random(60, 60, density=0.15, random_state=seed) + 1j * sp.random(60, 60, density=0.1,
             random_state=seed + 9) + 0.3 * sp.identity(60))
        mats.append(sp.csr_matrix(A))
    s = qs.jaynes_cummings(6, seed=2)
    Lq = liouvillian_sparse(s.H, s.c_ops)
    At, _, _ = modified(Lq, pop=trace_population(Lq))
    mats.append(permute(At, rcm(At)))
    for A in mats:
        A = sp.csr_matrix(A, dtype=complex)
        A.sort_indices()
        LU1, g1 = oilu.ilut_c(A, 1e-3, 3.0, guard=1e-8, boost=0.1)
        LU2, perm, g2 = oilu.ilutp_c(A, 1e-3, 3.0, permtol=0.0, guard=1e-8, boost=0.1)
        assert (perm == np.arange(A.shape[0])).all() and g1 == g2
        assert np.array_equal(LU1.indptr, LU2.indptr) and np.array_equal(LU1.indices, LU2.indices)
        assert np.array_equal(LU1.data, LU2.data)


@pytest.mark.parametrize("seed", range(4))
def test_complete_lu_is_partial_pivoting_by_columns(seed):
    """drop 0, no fill limit, permtol 1: A[:, perm] = L U exactly (up to
    rounding), with the column order LAPACK's row pivoting gives for A^T
    (real matrices, where LAPACK's |re| + |im| pivot measure is the modulus)."""
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(40, 40))
    M[np.abs(M) < 0.8] = 0.0
    np.fill_diagonal(M, 0.0)
    M += np.diag(rng.normal(size=40) * 0.01)
    LU, perm, g = oilu.ilutp_c(sp.csr_matrix(M.astype(complex)), 0.0, 1000.0, permtol=1.0)
    L, U = _dense(LU)
    assert g == 0
    assert np.max(np.abs(L @ U - M[:, perm])) <= 1e-13 * np.abs(M).max()
    P, _, _ = sla.lu(M.T)  # M^T = P L' U': row k of P^T M^T is row order[k] of M^T
    order = np.argmax(P, axis=0)
    assert np.array_equal(order, perm)


def test_apply_inverse_perm_solves_the_complete_factorisation():
    rng = np.random.default_rng(5)
    M = rng.normal(size=(30, 30)) + 1j * rng.normal(size=(30, 30))
    M[np.abs(M) < 1.0] = 0.0
    M += np.eye(30) * 0.05
    LU, perm, _ = oilu.ilutp_c(sp.csr_matrix(M), 0.0, 1000.0, permtol=1.0)
    b = rng.normal(size=30) + 0j
    x = oilu.apply_inverse_perm(LU, perm, b)
    assert np.max(np.abs(M @ x - b)) <= 1e-10 * np.abs(b).max() * np.linalg.cond(M)
