"""Parity of every stage of the HIP path with the CPU oracle (GPU required).

Stages are exported through the C ABI (ss_export_csr / ss_export_perm /
ss_apply) and compared element by element with the oracle on the same seeded
inputs; the end-to-end solves are compared with the dense fp64 oracle.
Tolerances: integer and index results exact; assembled values to 1e-14
relative (sums of at most a few fp64 products in a different order); ILU
factors to 1e-11 relative; steady states to 1e-8 max-abs in fp64 mode and
1e-6 in mixed mode, with ||L rho||_2 <= 1e-10.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

import qsystems as qs
from oracle import ilu as oilu
from oracle import ordering as oord
from oracle import transforms as otr
from oracle.liouvillian import liouvillian_sparse
from oracle.steady import steady_state_dense

pytestmark = pytest.mark.gpu

from conftest import load_product

ssl = load_product()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


SMALL = {
    "kerr20": lambda: qs.config(1),
    "jc8": lambda: qs.jaynes_cummings(8, seed=0),
    "random7": lambda: qs.random_lindblad(7, 3, seed=4),
    "spin3": lambda: qs.spin_chain(3),
    "opto3x5": lambda: qs.optomechanics(3, 5, nth=1.0),
    "two_level": lambda: qs.two_level_atom(),
}


def _max_rel(a, b):
    a = sp.csr_matrix(a)
    b = sp.csr_matrix(b)
    scale = max(abs(b).max(), 1e-300)
    return abs(a - b).max() / scale


# ------------------------------------------------------------ assembly
@pytest.mark.parametrize("name", list(SMALL))
def test_assembly_matches_oracle(name):
    s = SMALL[name]()
    _say("assembly", name, s.dim)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    Lg = ssl.export_csr(L, ssl.SS_MAT_L)
    Lo = liouvillian_sparse(s.H, s.c_ops)
    assert Lg.shape == Lo.shape
    assert _max_rel(Lg, Lo) <= 1e-14
    # the structure equals the oracle's non-zero structure
    big = abs(Lo) > 1e-12 * abs(Lo).max()
    assert ((abs(Lg) > 0) != (abs(Lo) > 0)).multiply(big).nnz == 0
    # rows sorted, unique columns
    for i in range(Lg.shape[0]):
        c = Lg.indices[Lg.indptr[i]:Lg.indptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_assembly_full_size_sampled_rows():
    """Optomechanics 10 x 60 (n = 360000): sampled rows of L against the
    oracle's sparse Kronecker assembly."""
    s = qs.config(3)
    _say("assembly optomech 10x60")
    L = ssl.build_liouvillian(s.H, s.c_ops)
    Lg = ssl.export_csr(L, ssl.SS_MAT_L)
    Lo = liouvillian_sparse(s.H, s.c_ops)
    assert Lg.nnz == Lo.nnz
    rows = np.random.default_rng(0).choice(Lg.shape[0], 2000, replace=False)
    assert _max_rel(Lg[rows], Lo[rows]) <= 1e-14


# ------------------------------------------------------------ transforms
@pytest.mark.parametrize("name", ["kerr20", "jc8", "spin3"])
def test_transforms_match_oracle(name):
    s = SMALL[name]()
    Lo = liouvillian_sparse(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab")
    A = ssl.export_csr(L, ssl.SS_MAT_A)
    Ao, _, w = otr.modified(Lo, pop=otr.trace_population(Lo))
    assert _max_rel(A, Ao) <= 1e-14
    assert A.nnz == Ao.nnz
    ssl.prepare(L, "trace_bicgstab", trace_row=0)
    A0 = ssl.export_csr(L, ssl.SS_MAT_A)
    assert _max_rel(A0, otr.modified(Lo, pop=0)[0]) <= 1e-14
    ssl.prepare(L, "invpow_bicgstab")
    S = ssl.export_csr(L, ssl.SS_MAT_A)
    So = otr.shifted(Lo, 1e-15)
    assert _max_rel(S, So) <= 1e-14
    assert S.nnz == So.nnz


# ------------------------------------------------------------ ordering
def _paper(name):
    return {"jc": lambda: qs.jaynes_cummings_paper(16), "spin": lambda: qs.spin_chain(5),
            "opto": lambda: qs.optomechanics(4, 8, nth=1.0)}[name]()


@pytest.mark.parametrize("system", ["jc", "spin", "opto"])
@pytest.mark.parametrize("method", ["trace_bicgstab", "invpow_bicgstab"])
def test_rcm_permutation_bit_exact(system, method):
    """GPU RCM = oracle RCM exactly, on the paper's Fig. 1/3 systems."""
    s = _paper(system)
    _say("rcm", system, method)
    Lo = liouvillian_sparse(s.H, s.c_ops)
    # T in row 0, as in the paper's Fig. 3
    Ao = otr.modified(Lo, pop=0)[0] if method.startswith("trace") else otr.shifted(Lo)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, method, trace_row=0)
    perm = ssl.export_perm(L)
    assert np.array_equal(perm, oord.rcm(Ao))
    Sg = ssl.export_csr(L, ssl.SS_MAT_SYM)
    So = oord.symmetrized_pattern(Ao)
    assert (Sg != 0).astype(np.int8).nnz == So.nnz
    assert ((Sg != 0).astype(np.int8) - So).nnz == 0
    # the permutation moves values exactly
    Ag = ssl.export_csr(L, ssl.SS_MAT_A)
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    assert _max_rel(Ap, oord.permute(Ag, perm)) == 0.0
    B, P = ssl.bandwidth_profile(L, ssl.SS_MAT_A_PERM)
    stored = sp.csr_matrix((np.ones(Ap.nnz), Ap.indices, Ap.indptr), shape=Ap.shape)
    assert (B, P) == (oord.bandwidth(stored)[2], oord.profile(stored)[2])


@pytest.mark.parametrize("k,method", [(1, "trace_bicgstab"), (2, "trace_bicgstab"), (3, "trace_bicgstab"),
                                      (4, "trace_bicgstab"), (4, "invpow_bicgstab")])
def test_rcm_on_workloads(k, method):
    """Bit-exact RCM on the workloads: C1 and C2 take the one-workgroup
    search, C3 (n = 360000) and C4 (n = 10^6) the multi-kernel level search."""
    s = qs.config(k)
    _say("rcm workload", k, method)
    Lo = liouvillian_sparse(s.H, s.c_ops)
    Ao = otr.modified(Lo, pop=otr.trace_population(Lo))[0] if method.startswith("trace") else otr.shifted(Lo)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, method)
    assert np.array_equal(ssl.export_perm(L), oord.rcm(Ao))


# ------------------------------------------------------------ ILU(0)
@pytest.mark.parametrize("name", ["kerr20", "jc8", "random7", "opto3x5"])
def test_ilu0_matches_oracle(name):
    s = SMALL[name]()
    _say("ilu0", name)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab")
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    LUg = ssl.export_csr(L, ssl.SS_MAT_LU)
    LUo, g = oilu.ilu0(Ap, guard=1e-8, boost=0.1)
    assert np.array_equal(LUg.indptr, LUo.indptr) and np.array_equal(LUg.indices, LUo.indices)
    rel = np.abs(LUg.data - LUo.data) / np.maximum(np.abs(LUo.data), 1e-300)
    big = np.abs(LUo.data) > 1e-10 * np.abs(LUo.data).max()
    assert np.max(rel[big]) <= 1e-11
    # every entry, small ones included, to an absolute bound scaled to the factors
    assert np.max(np.abs(LUg.data - LUo.data)) <= 1e-12 * np.abs(LUo.data).max()


@pytest.mark.parametrize("method,ordering", [("invpow_bicgstab", "rcm"), ("trace_bicgstab", "natural"),
                                             ("invpow_bicgstab", "natural")])
def test_ilu0_pivot_guard_on_the_spin_chain(method, ordering):
    """Dephasing leaves structurally zero diagonals in L (7 of 64 for three
    spins).  In the shifted matrix L - sigma I they become -1e-15, and with
    the natural order the trace-row matrix meets them too before elimination
    has filled them: zero-fill ILU must guard those pivots.  The GPU guards
    as many as the oracle (1, 2 and 3 here), its factors equal the oracle's
    guarded ILU(0) (guard 1e-8, boost 0.1) entry by entry, and the solve
    reports the count and still reaches the steady state."""
    s = qs.spin_chain(3)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, method, ordering=ordering)
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    LUg = ssl.export_csr(L, ssl.SS_MAT_LU)
    LUo, g = oilu.ilu0(Ap, guard=1e-8, boost=0.1)
    _say("spin3 guarded pivots", method, ordering, g)
    assert g > 0
    assert np.array_equal(LUg.indptr, LUo.indptr) and np.array_equal(LUg.indices, LUo.indices)
    assert np.max(np.abs(LUg.data - LUo.data)) <= 1e-12 * np.abs(LUo.data).max()
    rho, info = ssl.solve(L, method, tol=1e-10, raise_on_error=False, path="device", ordering=ordering)
    assert info["pivots_guarded"] == g
    if info["status"] == 0:
        ref = steady_state_dense(s.H, s.c_ops)
        assert np.max(np.abs(rho - ref)) <= 1e-8


def test_ilu0_property_on_jc40():
    """(LU)_ij = a_ij on the pattern of A, on the Jaynes-Cummings workload."""
    s = qs.config(2)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab")
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    Lf, Uf = oilu.split(ssl.export_csr(L, ssl.SS_MAT_LU))
    P = (Lf @ Uf).tocsr()
    C = Ap.tocoo()
    prod = np.asarray(P[C.row, C.col]).ravel()
    assert np.max(np.abs(prod - C.data)) <= 1e-11 * np.abs(C.data).max()


# ------------------------------------------------------------ SpMV / trsv
PRECOND_OPS = (ssl.SS_OP_PRECOND, ssl.SS_OP_PRECOND_SYNCFREE, ssl.SS_OP_PRECOND_BLOCK, ssl.SS_OP_PRECOND_LEVELS,
               ssl.SS_OP_PRECOND_GROUPS, ssl.SS_OP_PRECOND_CLASSES)

@pytest.mark.parametrize("name", ["kerr20", "jc8", "spin3"])
def test_spmv_and_triangular_solves(name):
    s = SMALL[name]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab")
    Lo = liouvillian_sparse(s.H, s.c_ops)
    rng = np.random.default_rng(1)
    x = rng.normal(size=Lo.shape[0]) + 1j * rng.normal(size=Lo.shape[0])
    y = ssl.apply(L, ssl.SS_OP_SPMV_L, x)
    ref = Lo @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    y = ssl.apply(L, ssl.SS_OP_SPMV_APERM, x)
    assert np.max(np.abs(y - Ap @ x)) <= 1e-13 * np.max(np.abs(Ap @ x))
    Lf, Uf = oilu.split(ssl.export_csr(L, ssl.SS_MAT_LU))
    yl = ssl.apply(L, ssl.SS_OP_LSOLVE, x)
    refl = spsolve_triangular(Lf, x, lower=True, unit_diagonal=True)
    assert np.max(np.abs(yl - refl)) <= 1e-11 * np.max(np.abs(refl))
    yu = ssl.apply(L, ssl.SS_OP_USOLVE, x)
    refu = spsolve_triangular(Uf, x, lower=False)
    assert np.max(np.abs(yu - refu)) <= 1e-11 * np.max(np.abs(refu))
    refp = spsolve_triangular(Uf, refl, lower=False)
    for op in PRECOND_OPS:
        yp = ssl.apply(L, op, x)
        assert np.max(np.abs(yp - refp)) <= 1e-11 * np.max(np.abs(refp))


def test_mixed_precision_operators():
    s = SMALL["kerr20"]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab", prec="mixed")
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    x = np.random.default_rng(2).normal(size=Ap.shape[0]).astype(np.complex128)
    y = ssl.apply(L, ssl.SS_OP_SPMV_APERM, x, prec="mixed")
    ref = Ap @ x
    assert np.max(np.abs(y - ref)) <= 1e-5 * np.max(np.abs(ref))
    Lf, Uf = oilu.split(ssl.export_csr(L, ssl.SS_MAT_LU))
    refp = spsolve_triangular(Uf, spsolve_triangular(Lf, x, lower=True, unit_diagonal=True), lower=False)
    for op in PRECOND_OPS:
        yp = ssl.apply(L, op, x, prec="mixed")
        assert np.max(np.abs(yp - refp)) <= 1e-4 * np.max(np.abs(refp))


@pytest.mark.parametrize("k,prec,tol", [(2, "fp64", 1e-11), (2, "mixed", 1e-4), (4, "fp64", 1e-11),
                                        (4, "mixed", 1e-4)])
def test_level_scheduled_precond_on_workloads(k, prec, tol):
    """The single-workgroup level-scheduled (LU)^-1 on the workload matrices:
    factor rows longer than the packed width, levels wider than the
    workgroup (Kerr chain, n = 10^6)."""
    s = qs.config(k)
    _say("precond", k, prec)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "invpow_bicgstab" if k == 4 else "trace_bicgstab", prec=prec)
    Lf, Uf = oilu.split(ssl.export_csr(L, ssl.SS_MAT_LU))
    x = np.random.default_rng(3).normal(size=Lf.shape[0]) + 0j
    refp = spsolve_triangular(Uf, spsolve_triangular(Lf, x, lower=True, unit_diagonal=True), lower=False)
    outs = {}
    for op in PRECOND_OPS:
        _say("   op", op)
        yp = ssl.apply(L, op, x, prec=prec)
        assert np.max(np.abs(yp - refp)) <= tol * np.max(np.abs(refp))
        outs[op] = yp
    # the sync-free variants consume a row's entries in the factor's order
    # with the same arithmetic (no contraction): the same bits
    for op in (ssl.SS_OP_PRECOND_LEVELS, ssl.SS_OP_PRECOND_GROUPS):
        assert np.array_equal(outs[op], outs[ssl.SS_OP_PRECOND_SYNCFREE]), op


# ------------------------------------------------------------ end to end
METHODS = ["trace_bicgstab", "trace_gmres", "invpow_bicgstab", "invpow_gmres"]


CASES = [(name, m) for name in ["kerr20", "jc8", "random7", "opto3x5"] for m in METHODS]
# Pure dephasing leaves d - 1 population rows of L~ with a structurally zero
# diagonal, which zero-fill ILU without pivoting cannot precondition; as the
# paper recommends for its spin chain, the inverse-power method is used there.
CASES += [("spin3", "invpow_bicgstab"), ("spin3", "invpow_gmres")]


DEVICE_PATHS = ["device", "device_syncfree", "device_levels", "device_groups", "device_classes"]
CASES = [(n, m, p) for (n, m) in CASES for p in DEVICE_PATHS + (["workgroup"] if "bicgstab" in m else [])]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("name,method,path", CASES)
def test_steady_state_matches_dense_oracle(name, method, path, prec, tol):
    """Both execution paths: device-wide kernels, and the whole solve inside
    one workgroup (level-scheduled triangular solves in LDS)."""
    s = SMALL[name]()
    _say("solve", name, method, path, prec)
    ref = steady_state_dense(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    trsv = path.split("_")[1] if "_" in path else "auto"
    rho, info = ssl.solve(L, method, tol=1e-10, prec=prec, raise_on_error=False, path=path.split("_")[0],
                          trsv=trsv)
    _say("   info", info)
    assert info["status"] == 0
    err = np.max(np.abs(rho - ref))
    _say("   err", err, "resid", info["resid_l2"], "its", info["outer_its"], info["inner_its"])
    assert err <= tol
    assert info["resid_l2"] <= 1e-10
    assert abs(np.trace(rho) - 1) <= 1e-12


@pytest.mark.parametrize("path", ["device", "workgroup"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_jaynes_cummings_workload(prec, tol, path):
    """Driven Jaynes-Cummings, cavity 40 x qubit (n = 6400)."""
    s = qs.config(2)
    _say("solve jc40", prec, path)
    ref = steady_state_dense(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, info = ssl.solve(L, "trace_bicgstab", tol=1e-10, prec=prec, path=path)
    _say("   err", np.max(np.abs(rho - ref)), info)
    assert np.max(np.abs(rho - ref)) <= tol
    assert info["resid_l2"] <= 1e-10


def test_closed_forms_on_gpu():
    s = qs.coherent_drive(40, 0.5, 1.0, 1.0)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, _ = ssl.solve(L, "trace_bicgstab", tol=1e-10)
    alpha = -1j / (0.5 + 0.5j)
    c = np.empty(40, dtype=complex)
    c[0] = np.exp(-abs(alpha) ** 2 / 2)
    for k in range(1, 40):
        c[k] = c[k - 1] * alpha / np.sqrt(k)
    assert np.max(np.abs(rho - np.outer(c, c.conj()))) <= 1e-8
    s = qs.thermal_oscillator(20, 2.0, 0.7, 1.3)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, _ = ssl.solve(L, "invpow_bicgstab", tol=1e-10)
    r = 2.0 / 3.0
    p = (1 - r) * r ** np.arange(20) / (1 - r ** 20)
    assert np.max(np.abs(rho - np.diag(p))) <= 1e-8


# ------------------------------------------------------------ error paths
def test_invalid_inputs_are_rejected():
    s = SMALL["kerr20"]()
    H = s.H.toarray()
    H[0, 0] = np.nan
    with pytest.raises(ssl.SolverError) as e:
        ssl.build_liouvillian(H, s.c_ops)
    assert e.value.code == -1
    with pytest.raises(ssl.SolverError) as e:
        ssl.build_liouvillian(s.H, [sp.identity(3, dtype=complex, format="csr")])
    assert e.value.code == -1


def test_iteration_limit_reports_not_converged():
    s = qs.config(2)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    with pytest.raises(ssl.SolverError) as e:
        ssl.solve(L, "trace_bicgstab", tol=1e-12, maxiter=1, max_outer=1)
    assert e.value.code == -3
    assert e.value.info["inner_its"] >= 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("path", ["workgroup", "device"])
def test_repeated_solves_are_bitwise_identical(prec, path):
    """Every reduction and sweep runs in a fixed order, so repeating a solve
    gives the same bits (this caught a complex128 select that the compiler
    lowered through private memory inside the prefetching sweep)."""
    s = qs.jaynes_cummings(30, seed=0)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    runs = [ssl.solve(L, "trace_bicgstab", tol=1e-10, prec=prec, path=path) for _ in range(3)]
    for rho, info in runs[1:]:
        assert info["inner_its"] == runs[0][1]["inner_its"]
        assert np.array_equal(rho, runs[0][0])


# ------------------------------------------------------------ degenerate cases
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("path", ["auto", "device"])
def test_one_state_system(method, path):
    """N = 1: L = 0 and the only density matrix is [[1]]."""
    H = sp.csr_matrix(np.array([[0.3]], dtype=np.complex128))
    L = ssl.build_liouvillian(H, [])
    rho, info = ssl.solve(L, method, tol=1e-10, path=path)
    assert info["status"] == 0
    assert rho.shape == (1, 1) and rho[0, 0] == 1.0


def test_pure_decay_gives_the_ground_state():
    """H = 0 with one lowering operator: rho = |0><0| exactly."""
    a = qs.destroy(6)
    L = ssl.build_liouvillian(sp.csr_matrix((6, 6), dtype=np.complex128), [a])
    for method in METHODS:
        rho, info = ssl.solve(L, method, tol=1e-12)
        ref = np.zeros((6, 6))
        ref[0, 0] = 1.0
        assert np.max(np.abs(rho - ref)) <= 1e-10, method


def test_no_dissipation_returns_a_valid_steady_state():
    """Without collapse operators every state diagonal in the energy basis is
    stationary (no unique steady state); the solver returns one of them:
    unit trace, Hermitian, ||L rho|| within the tolerance."""
    s = qs.kerr(5)
    L = ssl.build_liouvillian(s.H, [])
    rho, info = ssl.solve(L, "invpow_gmres", tol=1e-10, raise_on_error=False)
    if info["status"] == 0:
        assert abs(np.trace(rho) - 1) <= 1e-12
        Lo = liouvillian_sparse(s.H, [])
        assert np.linalg.norm(Lo @ rho.reshape(-1, order="F")) <= 1e-8


def test_batches_with_degenerate_members():
    Ls = [ssl.build_liouvillian(sp.csr_matrix(np.array([[0.0]], dtype=np.complex128)), []),
          ssl.build_liouvillian(qs.kerr(6).H, qs.kerr(6).c_ops)]
    rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", 1e-10)
    assert [i["status"] for i in infos] == [0, 0]
    assert rhos[0][0, 0] == 1.0
    assert ssl.solve_batch([], "trace_bicgstab", 1e-10) == ([], [])


# ------------------------------------------------------------ method selection
def test_auto_method_follows_the_bandwidth_rule():
    """SS_AUTO: the spin chain's trace row inflates the RCM bandwidth
    (the paper's Fig. 1 vs Fig. 3 captions: 167 -> 405 for five spins), so
    inverse power is chosen; for the Jaynes-Cummings system the two
    bandwidths are alike and the trace-row driver is chosen, with BiCGSTAB
    in the workgroup-resident launch (n <= 4096) and GMRES, the paper's first
    choice, on the device-wide path (cavity 33: n = 4356).  Results match
    the dense oracle either way."""
    for s, want in ((qs.spin_chain(4), ssl.SS_INVPOW_BICGSTAB), (qs.jaynes_cummings(8, seed=0), ssl.SS_TRACE_BICGSTAB),
                    (qs.jaynes_cummings(33, seed=0), ssl.SS_TRACE_GMRES)):
        L = ssl.build_liouvillian(s.H, s.c_ops)
        rho, info = ssl.solve(L, "auto", tol=1e-10)
        _say("auto", s.name, info["method"], info["bandwidth"])
        assert info["method"] == want
        assert np.max(np.abs(rho - steady_state_dense(s.H, s.c_ops))) <= 1e-8


def test_info_reports_bandwidth_profile_and_condition_estimate():
    s = SMALL["kerr20"]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, info = ssl.solve(L, "trace_bicgstab", tol=1e-10, cond_est=True)
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    assert info["bandwidth"] == oord.bandwidth(Ap)[2]
    assert info["profile"] == oord.profile(Ap)[2]
    ref = oilu.condition_estimate(ssl.export_csr(L, ssl.SS_MAT_LU))
    assert abs(info["cond_est"] - ref) <= 1e-9 * ref


# ------------------------------------------------------------ breakdown
@pytest.mark.parametrize("path", ["workgroup", "device"])
def test_forced_breakdown_falls_back_to_gmres(path):
    """SS_FLAG_FORCE_BREAKDOWN makes every BiCGSTAB breakdown test fire: the
    solve restarts, gives up on BiCGSTAB and finishes with GMRES (or reports
    SS_E_BREAKDOWN when no fallback is allowed)."""
    s = qs.config(1)
    ref = steady_state_dense(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, info = ssl.solve(L, "trace_bicgstab", tol=1e-10, path=path, force_breakdown=True)
    _say("forced breakdown", path, info["breakdowns"], info["fell_back"], info["inner_its"])
    assert info["status"] == 0 and info["fell_back"] == 1 and info["breakdowns"] >= 1
    assert np.max(np.abs(rho - ref)) <= 1e-8
    with pytest.raises(ssl.SolverError) as e:
        ssl.solve(L, "trace_bicgstab", tol=1e-10, path=path, force_breakdown=True, no_fallback=True)
    assert e.value.code == ssl.SS_E_BREAKDOWN
    # without the flag the same solve needs no fallback
    _, info = ssl.solve(L, "trace_bicgstab", tol=1e-10, path=path)
    assert info["fell_back"] == 0 and info["breakdowns"] == 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_forced_breakdown_in_a_batch_and_in_the_server(prec, tol):
    systems = [qs.kerr(N, delta=0.2 * k, E=0.5 + 0.1 * k) for k, N in enumerate((8, 12, 16))]
    refs = [steady_state_dense(s.H, s.c_ops) for s in systems]
    Ls = [ssl.build_liouvillian(s.H, s.c_ops) for s in systems]
    rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", tol=1e-10, prec=prec, force_breakdown=True)
    for rho, info, ref in zip(rhos, infos, refs):
        assert info["status"] == 0 and info["fell_back"] == 1
        assert np.max(np.abs(rho - ref)) <= tol
    for L in Ls:
        L.free()
    S = ssl.Server(hbm_budget_bytes=1 << 30, max_slots=16)
    tk = [S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec=prec, force_breakdown=True) for s in systems]
    S.drain()
    for t, ref in zip(tk, refs):
        rho, info = S.poll(t)
        assert info["status"] == 0 and info["fell_back"] == 1
        assert np.max(np.abs(rho - ref)) <= tol
    S.close()
