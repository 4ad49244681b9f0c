"""Pins of two oracle parts the dense-LU pins do not reach (no GPU):

* the pivot guard of the incomplete factorisations (a pivot below
  guard * ||a_i||_inf becomes boost * ||a_i||_inf times its phase), on a
  hand-worked 3 x 3 case whose values are written out below, through every
  oracle factorisation (Python ILU(0), Python ILUT, C ILUT, C ILU(0));
* the CPU fp64 sparse reference solve (oracle/sparse_ref.py): its ILU(0)
  against the Python one, its triangular solves against a dense solve, its
  BiCGSTAB against LAPACK, and its steady states against closed forms, the
  dense oracle and an exact product form at n = 15625.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import qsystems as qs
from oracle import ilu as oilu
from oracle import sparse_ref as sref
from oracle.steady import steady_state_dense

# ------------------------------------------------------------- pivot guard
# Row 1 eliminates with row 0: l_10 = 4 / 2 = 2 and
#   u_11 = a_11 - l_10 u_01 = (2 + (3 + 4i) 2^-30) - 2 = (3 + 4i) 2^-30,
# exactly (every operand is a short binary fraction).  |u_11| = 5 * 2^-30
# (4.7e-9) is below guard * ||a_1||_inf = 1e-8 * 4, so u_11 becomes
# boost * ||a_1||_inf * u_11 / |u_11| = 0.1 * 4 * (0.6 + 0.8i) = 0.24 + 0.32i.
# Row 2: l_21 = 1 / (0.24 + 0.32i) = 1.5 - 2i and
#   u_22 = 3 - (1.5 - 2i) * 1 = 1.5 + 2i, |u_22| = 2.5 above 1e-8 * 3.
EPS = 2.0 ** -30
A_GUARD = np.array([[2, 1, 0],
                    [4, 2 + (3 + 4j) * EPS, 1],
                    [0, 1, 3]], dtype=np.complex128)
LU_GUARD = np.array([[2, 1, 0],
                     [2, 0.24 + 0.32j, 1],
                     [0, 1.5 - 2j, 1.5 + 2j]], dtype=np.complex128)
# the same row with an exactly zero pivot: it becomes the real value 0.4,
# and row 2 follows with l_21 = 1 / 0.4 = 2.5, u_22 = 3 - 2.5 = 0.5
A_ZERO = A_GUARD.copy()
A_ZERO[1, 1] = 2
LU_ZERO = np.array([[2, 1, 0], [2, 0.4, 1], [0, 2.5, 0.5]], dtype=np.complex128)


def _factorisations():
    return {
        "ilu0": lambda A: oilu.ilu0(A, guard=1e-8, boost=0.1),
        "ilut": lambda A: oilu.ilut(A, drop_tol=0.0, fill=10.0, guard=1e-8, boost=0.1),
        "ilut_c": lambda A: oilu.ilut_c(A, drop_tol=0.0, fill=10.0, guard=1e-8, boost=0.1),
        "ilu0_c": lambda A: (lambda M: (M.matrix(), M.guarded))(sref.Ilu0(A, guard=1e-8, boost=0.1)),
    }


@pytest.mark.parametrize("name", ["ilu0", "ilut", "ilut_c", "ilu0_c"])
@pytest.mark.parametrize("A,LU", [(A_GUARD, LU_GUARD), (A_ZERO, LU_ZERO)], ids=["tiny", "zero"])
def test_pivot_guard_hand_example(name, A, LU):
    F, guarded = _factorisations()[name](sp.csr_matrix(A))
    assert guarded == 1
    assert np.max(np.abs(F.toarray() - LU)) <= 1e-15


@pytest.mark.parametrize("name", ["ilu0", "ilut", "ilut_c", "ilu0_c"])
def test_pivot_guard_uses_guard_for_the_test_and_boost_for_the_value(name):
    """A pivot between boost-scaled and guard-scaled bounds is left alone;
    with guard = 0 nothing is replaced and a zero pivot is an error."""
    A = A_GUARD.copy()
    A[1, 1] = 2 + 0.05  # u_11 = 0.05: above 1e-8 * 4, below 0.1 * 4
    F, guarded = _factorisations()[name](sp.csr_matrix(A))
    assert guarded == 0
    assert abs(F.toarray()[1, 1] - 0.05) <= 1e-15


# ------------------------------------------------------------ sparse ref
@pytest.mark.parametrize("sysf", [lambda: qs.kerr(8), lambda: qs.jaynes_cummings(4, seed=2),
                                  lambda: qs.random_lindblad(6, 2, seed=4)])
def test_sparse_ref_ilu0_equals_python_ilu0(sysf):
    from oracle.liouvillian import liouvillian_sparse
    from oracle.transforms import modified, trace_population
    from oracle.ordering import permute, rcm
    s = sysf()
    L = liouvillian_sparse(s.H, s.c_ops)
    A = modified(L, pop=trace_population(L))[0]
    Ap = sref.with_diagonal(permute(A, rcm(A)))
    LUp, gp = oilu.ilu0(Ap, guard=1e-8, boost=0.1)
    M = sref.Ilu0(Ap, guard=1e-8, boost=0.1)
    assert M.guarded == gp
    assert np.array_equal(M.matrix().indices, LUp.indices)
    assert np.max(np.abs(M.matrix().data - LUp.data)) <= 1e-13 * np.abs(LUp.data).max()


def test_sparse_ref_lu_solve_equals_dense_triangular_solves():
    rng = np.random.default_rng(3)
    n = 40
    D = sp.random(n, n, density=0.15, random_state=5, dtype=np.float64) + 4 * sp.identity(n)
    A = sp.csr_matrix(D.astype(np.complex128) * (1 + 0.5j))
    M = sref.Ilu0(A)
    F = M.matrix().toarray()
    Lf = np.tril(F, -1) + np.eye(n)
    Uf = np.triu(F)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x = M.solve(b)
    ref = sla.solve_triangular(Uf, sla.solve_triangular(Lf, b, lower=True, unit_diagonal=True))
    assert np.max(np.abs(x - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_sparse_ref_ilu0_is_exact_lu_without_fill():
    """A tridiagonal matrix has no fill: ILU(0) is its LU, one solve is exact."""
    n = 50
    rng = np.random.default_rng(1)
    A = sp.diags([rng.normal(size=n - 1) + 1j, 4 + rng.normal(size=n), rng.normal(size=n - 1) - 1j],
                 [-1, 0, 1], format="csr", dtype=np.complex128)
    b = rng.normal(size=n) + 0j
    x = sref.Ilu0(A).solve(b)
    assert np.max(np.abs(x - np.linalg.solve(A.toarray(), b))) <= 1e-13


def test_sparse_ref_bicgstab_solves_a_nonsymmetric_system():
    rng = np.random.default_rng(7)
    n = 300
    A = sp.csr_matrix(sp.random(n, n, density=0.02, random_state=2) * (1 + 1j) + 3 * sp.identity(n))
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    M = sref.Ilu0(A)
    x, its, bd = sref.bicgstab(A, b, M, np.zeros(n, complex), 1e-12, 500)
    assert not bd and its < 500
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)
    assert np.max(np.abs(x - np.linalg.solve(A.toarray(), b))) <= 1e-10


def test_sparse_ref_coherent_state_closed_form():
    """Driven damped cavity: rho = |alpha><alpha|, alpha = -iE/(kappa/2 + i Delta)."""
    N, delta, E, kappa = 40, 0.5, 1.0, 1.0
    s = qs.coherent_drive(N, delta, E, kappa)
    alpha = -1j * E / (kappa / 2 + 1j * delta)
    c = np.empty(N, dtype=np.complex128)
    c[0] = np.exp(-abs(alpha) ** 2 / 2)
    for k in range(1, N):
        c[k] = c[k - 1] * alpha / np.sqrt(k)
    rho, info = sref.steady_state_iterative(s.H, s.c_ops, tol=1e-13)
    assert info["resid_l2"] <= 1e-13
    assert np.max(np.abs(rho - np.outer(c, c.conj()))) <= 1e-10


@pytest.mark.parametrize("sysf", [lambda: qs.config(1), lambda: qs.jaynes_cummings(10, seed=1),
                                  lambda: qs.random_lindblad(8, 2, seed=9), lambda: qs.two_level_atom()])
def test_sparse_ref_matches_dense_oracle(sysf):
    s = sysf()
    rho, info = sref.steady_state_iterative(s.H, s.c_ops, tol=1e-12)
    assert info["resid_l2"] <= 1e-12
    assert np.max(np.abs(rho - steady_state_dense(s.H, s.c_ops))) <= 1e-10


def test_sparse_ref_kerr_chain_product_form():
    """Uncoupled chain (J = 0) of three 7-state Kerr cavities (d = 343,
    n = 117649): rho = rho_1 (x) rho_2 (x) rho_3, each factor from the dense
    oracle of one cavity."""
    s = qs.kerr_chain(3, 7, J=0.0)
    k = qs.kerr(7)
    r1 = steady_state_dense(k.H, k.c_ops)
    rho, info = sref.steady_state_iterative(s.H, s.c_ops, tol=1e-12)
    assert info["resid_l2"] <= 1e-12
    assert np.max(np.abs(rho - np.kron(np.kron(r1, r1), r1))) <= 1e-10
