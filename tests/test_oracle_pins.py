"""Pins of the CPU oracle against closed forms, invariants and the paper's
printed values (no GPU).  Each test fixes a part of the oracle with something
other than the oracle itself."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import qsystems as qs
from oracle import ilu as oilu
from oracle import invariants as inv
from oracle import ordering as oord
from oracle import transforms as otr
from oracle.liouvillian import liouvillian_dense, liouvillian_sparse, trace_row, unvec, vec
from oracle.steady import steady_state_dense, steady_state_dense_weighted

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _coherent(alpha, N):
    """Fock amplitudes exp(-|a|^2/2) a^n / sqrt(n!), built by the recursion
    c_n = c_{n-1} a / sqrt(n)."""
    c = np.empty(N, dtype=np.complex128)
    c[0] = np.exp(-abs(alpha) ** 2 / 2)
    for k in range(1, N):
        c[k] = c[k - 1] * alpha / np.sqrt(k)
    return c


def _rand_rho(d, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    return X


# ---------------------------------------------------------------- assembly
@pytest.mark.parametrize("sysf", [lambda: qs.random_lindblad(5, 2, seed=3),
                                  lambda: qs.kerr(6), lambda: qs.jaynes_cummings(3, seed=1),
                                  lambda: qs.two_level_atom()])
def test_liouvillian_matches_superoperator_action(sysf):
    """L vec(X) = vec(L[X]) with L[X] from d x d matrix products (eq. lindblad):
    pins the Kronecker formula and the column-stacking convention (eq. eigval)."""
    s = sysf()
    L = liouvillian_dense(s.H, s.c_ops)
    for seed in range(3):
        X = _rand_rho(s.dim, seed)
        lhs = L @ vec(X)
        rhs = vec(inv.superop_action(s.H, s.c_ops, X))
        assert np.max(np.abs(lhs - rhs)) <= 1e-12 * max(1.0, np.max(np.abs(rhs)))


def test_liouvillian_sparse_equals_dense():
    s = qs.jaynes_cummings(4, seed=2)
    Ld = liouvillian_dense(s.H, s.c_ops)
    Ls = liouvillian_sparse(s.H, s.c_ops).toarray()
    assert np.max(np.abs(Ld - Ls)) <= 1e-13


def test_trace_preservation_and_hermiticity_preservation():
    """t^T L = 0 (trace preserved), and L[X+] = L[X]+ (Hermiticity preserved)."""
    s = qs.random_lindblad(6, 3, seed=5)
    L = liouvillian_dense(s.H, s.c_ops)
    d = s.dim
    assert np.max(np.abs(trace_row(d) @ L)) <= 1e-12
    X = _rand_rho(d, 9)
    a = unvec(L @ vec(X.conj().T), d)
    b = unvec(L @ vec(X), d).conj().T
    assert np.max(np.abs(a - b)) <= 1e-12


# ---------------------------------------------------------------- closed forms
def test_coherent_state_closed_form():
    """Linear driven damped cavity: rho = |alpha><alpha|, alpha = -iE/(kappa/2 + i Delta).
    Needs a cutoff (N = 40) where |alpha|^2 = 2 is far from the truncation."""
    delta, E, kappa, N = 0.5, 1.0, 1.0, 40
    s = qs.coherent_drive(N, delta, E, kappa)
    rho = steady_state_dense(s.H, s.c_ops)
    alpha = -1j * E / (kappa / 2 + 1j * delta)
    c = _coherent(alpha, N)
    assert np.max(np.abs(rho - np.outer(c, c.conj()))) <= 1e-12


@pytest.mark.parametrize("N,nbar", [(20, 2.0), (8, 0.5), (30, 1.0)])
def test_thermal_oscillator_truncated_bose_einstein(N, nbar):
    """Thermal bath: diagonal rho with p_k = (1 - r) r^k / (1 - r^N), r = n/(1 + n),
    exact in the truncated space (detailed balance of the rate equations)."""
    s = qs.thermal_oscillator(N, nbar, kappa=0.7, omega=1.3)
    rho = steady_state_dense(s.H, s.c_ops)
    r = nbar / (1 + nbar)
    p = (1 - r) * r ** np.arange(N) / (1 - r ** N)
    assert np.max(np.abs(rho - np.diag(p))) <= 1e-12


@pytest.mark.parametrize("delta,omega_r,gamma", [(0.3, 0.7, 0.5), (0.0, 2.0, 1.0), (1.5, 0.2, 0.05)])
def test_two_level_atom_excited_population(delta, omega_r, gamma):
    """rho_ee = (Omega^2/4) / (Delta^2 + gamma^2/4 + Omega^2/2); index 0 is the
    excited state in the z basis used here."""
    s = qs.two_level_atom(delta, omega_r, gamma)
    rho = steady_state_dense(s.H, s.c_ops)
    ree = (omega_r ** 2 / 4) / (delta ** 2 + gamma ** 2 / 4 + omega_r ** 2 / 2)
    assert abs(rho[0, 0] - ree) <= 1e-13
    assert abs(np.trace(rho) - 1) <= 1e-13


def test_kerr_cutoff_convergence_and_linear_limit():
    """Kerr oscillator of the first workload: the N = 20 steady state agrees with
    the N = 40 one on the common block (cutoff converged), and chi -> 0 gives the
    coherent state."""
    r20 = steady_state_dense(qs.kerr(20).H, qs.kerr(20).c_ops)
    r40 = steady_state_dense(qs.kerr(40).H, qs.kerr(40).c_ops)
    assert np.max(np.abs(r20 - r40[:20, :20])) <= 1e-9
    s = qs.kerr(40, chi=1e-9)
    rho = steady_state_dense(s.H, s.c_ops)
    alpha = -1j * 1.0 / (0.5 + 0.5j)
    c = _coherent(alpha, 40)
    assert np.max(np.abs(rho - np.outer(c, c.conj()))) <= 1e-7


def test_product_form_special_cases():
    """Uncoupled subsystems have a product steady state (pins the composite
    operator order and the assembly): optomechanics with g0 = 0, Kerr chain with
    J = 0."""
    s = qs.optomechanics(3, 5, g0=0.0, E=0.3, gamma=0.2, nth=0.7)
    rho = steady_state_dense(s.H, s.c_ops)
    cav = qs.kerr(3, delta=0.0, chi=0.0, E=0.3, kappa=0.3)
    rc = steady_state_dense(cav.H, cav.c_ops)
    mech = qs.thermal_oscillator(5, 0.7, kappa=0.2, omega=1.0)
    rm = steady_state_dense(mech.H, mech.c_ops)
    assert np.max(np.abs(rho - np.kron(rc, rm))) <= 1e-12
    ch = qs.kerr_chain(2, 4, J=0.0)
    rho = steady_state_dense(ch.H, ch.c_ops)
    k = qs.kerr(4)
    r1 = steady_state_dense(k.H, k.c_ops)
    assert np.max(np.abs(rho - np.kron(r1, r1))) <= 1e-12


def test_weighted_trace_row_equals_trace_replacement():
    """Eq. (linear) as printed (L + w T, rhs w e_0) gives the same rho as row
    replacement, for the paper's w (mean diagonal) and an arbitrary w."""
    s = qs.jaynes_cummings(5, seed=3)
    r0 = steady_state_dense(s.H, s.c_ops)
    r1 = steady_state_dense_weighted(s.H, s.c_ops)
    r2 = steady_state_dense_weighted(s.H, s.c_ops, w=3.7 - 1.1j)
    assert np.max(np.abs(r0 - r1)) <= 1e-12
    assert np.max(np.abs(r0 - r2)) <= 1e-12


def test_trace_row_in_any_population_row():
    """The population rows of L sum to zero, so T may sit in any of them: the
    solution of L~ x = w e_row is the steady state for every choice, and the
    default choice for the Jaynes-Cummings workload is its ground state, whose
    diagonal entry in L is exactly zero."""
    s = qs.jaynes_cummings(6, seed=0)
    L = liouvillian_sparse(s.H, s.c_ops)
    ref = steady_state_dense(s.H, s.c_ops)
    d = s.dim
    for pop in (0, 1, 5, d - 1):
        A, b, _ = otr.modified(L, pop=pop)
        x = np.linalg.solve(A.toarray(), b)
        assert np.max(np.abs(unvec(x, d) - ref)) <= 1e-11
    k = otr.trace_population(L)
    assert k == 1 and L[k * (d + 1), k * (d + 1)] == 0  # |0, g> in cavity x qubit order
    assert otr.trace_population(liouvillian_sparse(qs.kerr(5).H, qs.kerr(5).c_ops)) == 0


@pytest.mark.parametrize("sysf", [lambda: qs.config(1), lambda: qs.jaynes_cummings(10, seed=0),
                                  lambda: qs.random_lindblad(8, 3, seed=11),
                                  lambda: qs.spin_chain(3)])
def test_invariants(sysf):
    s = sysf()
    rho = steady_state_dense(s.H, s.c_ops)
    L = liouvillian_sparse(s.H, s.c_ops)
    assert inv.hermiticity_error(rho) <= 1e-10
    assert inv.trace_error(rho) <= 1e-12
    assert inv.min_eigenvalue(rho) >= -1e-10
    assert inv.residual_l2(L, rho) <= 1e-10


# ---------------------------------------------------------------- transforms
def test_modified_and_shifted_definitions():
    s = qs.kerr(5)
    L = liouvillian_sparse(s.H, s.c_ops)
    A, b, w = otr.modified(L)
    d = 5
    Ad = L.toarray()
    Ad[0, np.arange(d) * (d + 1)] += w
    assert np.allclose(A.toarray(), Ad, atol=0, rtol=0)
    assert abs(w - np.mean(np.diag(L.toarray()))) < 1e-15
    assert w.real < 0  # a damped system has a negative mean diagonal
    S = otr.shifted(L, 1e-15)
    assert np.array_equal(S.toarray(), L.toarray() - 1e-15 * np.eye(25))


# ---------------------------------------------------------------- ordering
def test_bandwidth_profile_hand_examples():
    A = sp.csr_matrix(np.array([[1, 0, 2, 0],
                                [0, 1, 0, 0],
                                [0, 3, 1, 0],
                                [4, 0, 0, 1]]))
    # ub = 2 (0,2); lb = 3 (3,0); rows: max(j-i) = 2,0,0,0 -> up = 2;
    # columns: max(i-j) = 3 (col 0), 1 (col 1), 0, 0 -> lp = 4
    assert oord.bandwidth(A) == (2, 3, 6)
    assert oord.profile(A) == (2, 4, 6)
    T = sp.diags([np.ones(4), np.ones(5), np.ones(4)], [-1, 0, 1]).tocsr()
    assert oord.bandwidth(T)[2] == 3
    assert oord.profile(T) == (4, 4, 8)


def test_bandwidth_profile_skip_explicit_zeros_and_leave_the_input_alone():
    """Bandwidth and profile count non-zero entries only (an explicit zero,
    e.g. an added zero diagonal, is structure without value), and computing
    them does not change the matrix passed in."""
    indptr = np.array([0, 2, 3, 5])
    indices = np.array([0, 2, 1, 0, 2])
    data = np.array([1.0, 0.0, 1.0, 5.0, 1.0])  # (0, 2) stored as 0
    A = sp.csr_matrix((data, indices, indptr), shape=(3, 3))
    before = (A.indptr.copy(), A.indices.copy(), A.data.copy())
    # non-zeros: (0,0), (1,1), (2,0), (2,2): ub = 0, lb = 2; up = 0; lp = 2
    assert oord.bandwidth(A) == (0, 2, 3)
    assert oord.profile(A) == (0, 2, 2)
    assert oord.profile(A) == (0, 2, 2)  # a second call sees the same matrix
    assert all(np.array_equal(x, y) for x, y in zip(before, (A.indptr, A.indices, A.data)))


def test_cuthill_mckee_on_a_path_and_tie_free_graphs():
    """On a path graph RCM walks the path from one end (B = 3).  On graphs with
    a unique lowest-degree node and distinct neighbour degrees no tie-break is
    involved, so the order must equal scipy's reverse_cuthill_mckee."""
    n = 9
    rng = np.random.default_rng(0)
    p = rng.permutation(n)
    rows = np.r_[p[:-1], p[1:]]
    cols = np.r_[p[1:], p[:-1]]
    P = sp.csr_matrix((np.ones(2 * n - 2), (rows, cols)), shape=(n, n))
    perm = oord.rcm(P)
    assert sorted(perm.tolist()) == list(range(n))
    assert oord.bandwidth(oord.permute(P, perm))[2] == 3
    # a 5 x 6 grid with one pendant node: the lowest-degree node is unique, and
    # both implementations queue equal-degree neighbours in increasing index
    R, C = 5, 6
    edges = []
    for i in range(R):
        for j in range(C):
            u = i * C + j
            if j + 1 < C:
                edges.append((u, u + 1))
            if i + 1 < R:
                edges.append((u, u + C))
    m = R * C + 1
    edges.append((7, m - 1))
    r = [a for a, b in edges] + [b for a, b in edges]
    c = [b for a, b in edges] + [a for a, b in edges]
    G = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(m, m))
    ours = oord.rcm(G)
    ref = reverse_cuthill_mckee(G.tocsr(), symmetric_mode=True)
    assert np.array_equal(ours, ref)


def _paper_system(name):
    if name == "jc":
        return qs.jaynes_cummings_paper(16)
    if name == "spin":
        return qs.spin_chain(5)
    return qs.optomechanics(4, 8, nth=1.0)


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "rcm_paper_captions.json")))["cases"],
                         ids=lambda c: f"{c['system']}-{c['matrix']}")
def test_rcm_reproduces_paper_captions(case):
    s = _paper_system(case["system"])
    L = liouvillian_sparse(s.H, s.c_ops)
    A = otr.shifted(L) if case["matrix"] == "shifted" else otr.modified(L)[0]
    assert A.shape == (1024, 1024)
    perm = oord.rcm(A)
    Ap = oord.permute(A, perm)
    B = oord.bandwidth(Ap)[2]
    P = oord.profile(Ap)[2]
    assert B == case["B"]
    if case["exact"]:
        assert P == case["P"]
    else:
        assert abs(P - case["P"]) / case["P"] < 2e-3
    # RCM reduces both bandwidth and profile for these systems (Fig. 1 text)
    assert B < oord.bandwidth(A)[2] and P < oord.profile(A)[2]


def test_cm_order_is_a_breadth_first_level_order():
    """Every node after the start has an earlier-visited neighbour whose BFS level
    is one lower, and levels never decrease along the CM order (one component)."""
    s = qs.kerr(8)
    A = otr.modified(liouvillian_sparse(s.H, s.c_ops))[0]
    S = oord.symmetrized_pattern(A)
    order = oord.cuthill_mckee(S)
    n = S.shape[0]
    assert sorted(order.tolist()) == list(range(n))
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    level = np.zeros(n, dtype=np.int64)
    for k, u in enumerate(order[1:], start=1):
        nb = S.indices[S.indptr[u]:S.indptr[u + 1]]
        earlier = [v for v in nb if pos[v] < k]
        assert earlier, "node without an earlier neighbour in a connected graph"
        level[u] = min(level[v] for v in earlier) + 1
    assert np.all(np.diff(level[order]) >= 0)


# ---------------------------------------------------------------- ILU
def test_ilu0_is_exact_lu_without_fill():
    """A tridiagonal matrix has no fill, so ILU(0) = LU."""
    rng = np.random.default_rng(1)
    n = 30
    T = sp.diags([rng.normal(size=n - 1) + 1j * rng.normal(size=n - 1), 4 + rng.normal(size=n),
                  rng.normal(size=n - 1)], [-1, 0, 1]).tocsr()
    LU, g = oilu.ilu0(T)
    L, U = oilu.split(LU)
    assert g == 0
    assert np.max(np.abs((L @ U - T).toarray())) <= 1e-13


def test_ilu0_dense_equals_unpivoted_lu():
    """On a full pattern ILU(0) is Gaussian elimination; for a column-diagonally
    dominant matrix partial pivoting makes no swaps, so LAPACK's factors are the
    same."""
    rng = np.random.default_rng(2)
    n = 12
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    M += np.diag(3 * n * np.ones(n))
    Pm, Lr, Ur = sla.lu(M)
    assert np.allclose(Pm, np.eye(n))
    LU, _ = oilu.ilu0(sp.csr_matrix(M))
    L, U = oilu.split(LU)
    assert np.max(np.abs(L.toarray() - Lr)) <= 1e-13
    assert np.max(np.abs(U.toarray() - Ur)) <= 1e-12


def test_ilu0_reproduces_a_on_its_pattern():
    """Defining property of ILU(0): (LU)_ij = a_ij on the pattern of A."""
    s = qs.kerr(10)
    A = otr.modified(liouvillian_sparse(s.H, s.c_ops))[0]
    LU, _ = oilu.ilu0(A)
    L, U = oilu.split(LU)
    P = (L @ U).tocsr()
    Acoo = A.tocoo()
    prod = np.asarray(P[Acoo.row, Acoo.col]).ravel()
    assert np.max(np.abs(prod - Acoo.data)) <= 1e-12 * np.max(np.abs(A.data))
    # and L, U stay inside the pattern of A
    assert set(zip(*LU.nonzero())) <= set(zip(Acoo.row, Acoo.col))


def test_ilut_limits():
    """drop_tol = 0 with unlimited fill is the complete LU; with a large drop
    tolerance only the diagonal of U survives beyond the original pattern."""
    rng = np.random.default_rng(3)
    n = 10
    M = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.4) + 1j * rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.4)
    M += np.diag(2 * n * np.ones(n))
    LU, _ = oilu.ilut(sp.csr_matrix(M), drop_tol=0.0, fill=100.0)
    L, U = oilu.split(LU)
    assert np.max(np.abs((L @ U).toarray() - M)) <= 1e-12
    LU2, _ = oilu.ilut(sp.csr_matrix(M), drop_tol=10.0, fill=100.0)
    assert LU2.nnz == n  # everything off-diagonal dropped


def test_ilut_fill_cap():
    rng = np.random.default_rng(4)
    n = 16
    M = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.3)
    M = M + np.diag(n * np.ones(n))
    A = sp.csr_matrix(M.astype(np.complex128))
    LU, _ = oilu.ilut(A, drop_tol=0.0, fill=0.5)
    for i in range(n):
        nz = A.indptr[i + 1] - A.indptr[i]
        cols = LU.indices[LU.indptr[i]:LU.indptr[i + 1]]
        assert np.sum(cols < i) <= math.ceil(0.5 * nz)
        assert np.sum(cols > i) <= math.ceil(0.5 * nz)
        assert i in cols


def test_condition_estimate_of_exact_factors():
    """With complete factors, (LU)^{-1} e = A^{-1} e."""
    rng = np.random.default_rng(5)
    n = 8
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + np.diag(5 * np.ones(n))
    LU, _ = oilu.ilut(sp.csr_matrix(M), drop_tol=0.0, fill=100.0)
    ref = np.max(np.abs(np.linalg.solve(M, np.ones(n))))
    assert abs(oilu.condition_estimate(LU) - ref) <= 1e-12 * ref


def test_ilut_hand_example():
    """A 3 x 3 case worked by hand: A = [[4,0,1],[1,4,0],[0,1,4]].
    drop 0.1 (tau = 0.4): l_10 = l_21 = 1/4 are dropped, so L is empty and
    U = triu(A); drop 0.01 (tau = 0.04): l_10 = 1/4 is kept, fill u_12 = -1/4, then
    l_21 = 1/4 and u_22 = 4 + 1/16."""
    A = sp.csr_matrix(np.array([[4, 0, 1], [1, 4, 0], [0, 1, 4]], dtype=np.complex128))
    want_coarse = np.array([[4, 0, 1], [0, 4, 0], [0, 0, 4]])
    want_fine = np.array([[4, 0, 1], [0.25, 4, -0.25], [0, 0.25, 4.0625]])
    for f in (oilu.ilut, oilu.ilut_c):
        LU, _ = f(A, drop_tol=0.1, fill=10.0)
        assert np.array_equal(LU.toarray(), want_coarse)
        LU, _ = f(A, drop_tol=0.01, fill=10.0)
        assert np.array_equal(LU.toarray(), want_fine)


def _ilut_cases():
    rng = np.random.default_rng(11)
    n = 40
    M = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * (rng.random((n, n)) < 0.12)
    M += np.diag(rng.normal(size=n) + 3j)
    yield "random40", sp.csr_matrix(M)
    s = qs.kerr(10)
    A = otr.modified(liouvillian_sparse(s.H, s.c_ops))[0]
    yield "kerr10_rcm", oord.permute(A, oord.rcm(A))
    s = qs.jaynes_cummings(N=6)
    L = liouvillian_sparse(s.H, s.c_ops)
    A = otr.modified(L, pop=otr.trace_population(L))[0]
    yield "jc6_rcm", oord.permute(A, oord.rcm(A))


@pytest.mark.parametrize("drop,fill,guard", [(1e-4, 10.0, 1e-8), (1e-2, 2.0, 1e-8), (0.0, 100.0, 0.0),
                                             (1e-3, 1.0, 1e-8)])
def test_ilut_c_equals_python_ilut(drop, fill, guard):
    """The C ILUT and the Python ILUT are written independently from the same
    steps with the same complex arithmetic: they must agree bit for bit."""
    for name, A in _ilut_cases():
        LUp, gp = oilu.ilut(A, drop_tol=drop, fill=fill, guard=guard, boost=0.1 if guard else None)
        LUc, gc = oilu.ilut_c(A, drop_tol=drop, fill=fill, guard=guard, boost=0.1 if guard else None)
        assert gp == gc, name
        assert np.array_equal(LUp.indptr, LUc.indptr), name
        assert np.array_equal(LUp.indices, LUc.indices), name
        assert np.array_equal(LUp.data, LUc.data), name


def test_ilut_c_limits():
    """Complete LU at drop 0 / unlimited fill; ILU(0) where the exact LU has
    no fill (a tridiagonal matrix)."""
    rng = np.random.default_rng(12)
    n = 30
    M = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.3) + np.diag(4 * n * np.ones(n))
    LU, _ = oilu.ilut_c(sp.csr_matrix(M.astype(np.complex128)), drop_tol=0.0, fill=1000.0)
    L, U = oilu.split(LU)
    assert np.max(np.abs((L @ U).toarray() - M)) <= 1e-12 * np.max(np.abs(M))
    T = sp.diags([rng.normal(size=n - 1), 4 + rng.normal(size=n), rng.normal(size=n - 1)], [-1, 0, 1],
                 format="csr").astype(np.complex128)
    LUt, _ = oilu.ilut_c(T, drop_tol=0.0, fill=1.0)
    LU0, _ = oilu.ilu0(T)
    assert np.max(np.abs((LUt - LU0).toarray())) <= 1e-14
