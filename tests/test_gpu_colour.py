"""The colour-class ordering (SS_ORDER_COLOUR) through the C ABI against the
oracle: the permutation bit for bit (greedy colouring of the structure of
A + A^T visited in the seeded random order of SplitMix64 priorities, classes
in increasing colour, each in RCM order), the depth of the factors bounded by
the colour count, and steady
states against the dense oracle and, on the Kerr chain (n = 10^6), against
the oracle's CPU sparse reference.  Tolerances as everywhere: 1e-8 max-abs
in fp64 mode, 1e-6 in mixed mode, ||L rho||_2 <= 1e-10."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

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
}


def _transformed(s, method):
    Lo = liouvillian_sparse(s.H, s.c_ops)
    return otr.modified(Lo, pop=otr.trace_population(Lo))[0] if method.startswith("trace") else otr.shifted(Lo)


def _depths(LU):
    """Levels of the strictly lower and strictly upper parts (CPU loops)."""
    LU = sp.csr_matrix(LU)
    n = LU.shape[0]
    lo = np.zeros(n, dtype=np.int64)
    up = np.zeros(n, dtype=np.int64)
    for i in range(n):
        c = LU.indices[LU.indptr[i]:LU.indptr[i + 1]]
        c = c[c < i]
        lo[i] = lo[c].max() + 1 if c.size else 0
    for i in range(n - 1, -1, -1):
        c = LU.indices[LU.indptr[i]:LU.indptr[i + 1]]
        c = c[c > i]
        up[i] = up[c].max() + 1 if c.size else 0
    return int(lo.max()) + 1, int(up.max()) + 1


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("method", ["trace_bicgstab", "invpow_bicgstab"])
def test_colour_permutation_bit_exact(name, method):
    s = SMALL[name]()
    _say("colour perm", name, method)
    Ao = _transformed(s, method)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, method, ordering="colour")
    perm = ssl.export_perm(L)
    want = oord.colour_order(Ao)
    assert np.array_equal(perm, want)
    _, k = oord.greedy_colouring(oord.symmetrized_pattern(Ao), oord.random_visit(Ao.shape[0]))
    # zero fill keeps the pattern, so each substitution has at most k levels
    lo, up = _depths(ssl.export_csr(L, ssl.SS_MAT_LU))
    _say("   colours", k, "levels", lo, up)
    assert lo <= k and up <= k


@pytest.mark.parametrize("k,method", [(2, "trace_bicgstab"), (3, "trace_gmres"), (4, "invpow_gmres"),
                                      (4, "trace_gmres")])
def test_colour_permutation_on_workloads(k, method):
    """Bit-exact at the workloads' sizes (n = 6400, 360000 and 10^6)."""
    s = qs.config(k)
    _say("colour perm workload", k, method)
    Ao = _transformed(s, method)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, method, ordering="colour")
    assert np.array_equal(ssl.export_perm(L), oord.colour_order(Ao))


def test_colour_permutation_beyond_one_counter_window():
    """A dense Liouvillian (d = 36, n = 1296): its structure is a complete
    graph, so the greedy colouring takes n colours (one per round) -- more
    than one window of the class counters, and colours past 64 for every late
    vertex."""
    s = qs.random_lindblad(36, 2, density=1.0, seed=0)
    Ao = _transformed(s, "trace_bicgstab")
    _, k = oord.greedy_colouring(oord.symmetrized_pattern(Ao), oord.random_visit(Ao.shape[0]))
    assert k > 1024
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab", ordering="colour")
    assert np.array_equal(ssl.export_perm(L), oord.colour_order(Ao))


CASES = [(name, m) for name in ["kerr20", "jc8", "random7", "opto3x5"]
         for m in ["trace_bicgstab", "trace_gmres", "invpow_bicgstab", "invpow_gmres"]]
CASES += [("spin3", "invpow_gmres")]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("name,method", CASES)
@pytest.mark.parametrize("path", ["device", "device_classes", "device_groups", "workgroup"])
def test_colour_steady_state_matches_dense_oracle(name, method, path, prec, tol):
    if path == "workgroup" and "gmres" in method:
        pytest.skip("the workgroup-resident solver runs BiCGSTAB only")
    s = SMALL[name]()
    _say("colour solve", name, method, path, prec)
    ref = steady_state_dense(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    trsv = path.split("_")[1] if "_" in path else "auto"
    rho, info = ssl.solve(L, method, tol=1e-10, prec=prec, raise_on_error=False, path=path.split("_")[0],
                          trsv=trsv, ordering="colour")
    _say("   its", info["outer_its"], info["inner_its"], "colours", info["colours"], "resid", info["resid_l2"])
    assert info["status"] == 0
    At = _transformed(s, method)
    _, k = oord.greedy_colouring(oord.symmetrized_pattern(At), oord.random_visit(At.shape[0]))
    assert info["colours"] == k
    assert np.max(np.abs(rho - ref)) <= tol
    assert info["resid_l2"] <= 1e-10


def test_colour_info_is_zero_for_other_orderings():
    s = SMALL["kerr20"]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    _, info = ssl.solve(L, "trace_bicgstab", tol=1e-10)
    assert info["colours"] == 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_colour_in_a_batch(prec, tol):
    """ss_solve_batch with the colour order: every member's permutation is
    the oracle's and its steady state the dense oracle's."""
    systems = [qs.jaynes_cummings(10, seed=k) for k in range(4)]
    Ls = [ssl.build_liouvillian(s.H, s.c_ops) for s in systems]
    rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", tol=1e-10, prec=prec, ordering="colour")
    for s, L, rho, info in zip(systems, Ls, rhos, infos):
        assert info["status"] == 0
        assert np.array_equal(ssl.export_perm(L), oord.colour_order(_transformed(s, "trace_bicgstab")))
        assert np.max(np.abs(rho - steady_state_dense(s.H, s.c_ops))) <= tol


def _factor_positions(Ao):
    """cp[q]: the RCM position of row q of the colour-class factors."""
    base = oord.rcm(Ao)
    pos = np.empty(Ao.shape[0], dtype=np.int64)
    pos[base] = np.arange(Ao.shape[0])
    return pos[oord.colour_order(Ao)]


def test_colour_precond_matches_triangular_solves():
    """On the device-wide path the Krylov iteration stays in RCM order and
    the factors take the colour-class order: (LU)^-1 through the
    permutation, by every device-wide triangular solve, on the
    Jaynes-Cummings workload, against scipy's triangular solves of the
    exported factors; the sync-free variants agree bit for bit."""
    from scipy.sparse.linalg import spsolve_triangular
    s = qs.config(2)
    Ao = _transformed(s, "trace_gmres")
    cp = _factor_positions(Ao)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_gmres", ordering="colour")
    # the Krylov matrix is P A P^T in RCM order, the factors' order is the colour order
    assert _max_rel(ssl.export_csr(L, ssl.SS_MAT_A_PERM), oord.permute(Ao, oord.rcm(Ao))) <= 1e-14
    assert np.array_equal(ssl.export_perm(L), oord.colour_order(Ao))
    Lf, Uf = oilu.split(ssl.export_csr(L, ssl.SS_MAT_LU))
    x = np.random.default_rng(7).normal(size=Lf.shape[0]) + 0j
    ref = np.empty_like(x)
    ref[cp] = spsolve_triangular(Uf, spsolve_triangular(Lf, x[cp], lower=True, unit_diagonal=True), lower=False)
    outs = {}
    for op in (ssl.SS_OP_PRECOND_SYNCFREE, ssl.SS_OP_PRECOND_LEVELS, ssl.SS_OP_PRECOND_GROUPS,
               ssl.SS_OP_PRECOND_BLOCK, ssl.SS_OP_PRECOND_CLASSES, ssl.SS_OP_PRECOND):
        outs[op] = ssl.apply(L, op, x)
        assert np.max(np.abs(outs[op] - ref)) <= 1e-11 * np.max(np.abs(ref)), op
    for op in (ssl.SS_OP_PRECOND_LEVELS, ssl.SS_OP_PRECOND_GROUPS):
        assert np.array_equal(outs[op], outs[ssl.SS_OP_PRECOND_SYNCFREE]), op
    # the unit-lower and the upper solve alone, through the permutation
    yl = ssl.apply(L, ssl.SS_OP_LSOLVE, x)
    want = np.empty_like(x)
    want[cp] = spsolve_triangular(Lf, x[cp], lower=True, unit_diagonal=True)
    assert np.max(np.abs(yl - want)) <= 1e-11 * np.max(np.abs(want))


def _max_rel(a, b):
    a, b = sp.csr_matrix(a), sp.csr_matrix(b)
    return abs(a - b).max() / max(abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", ["jc8", "kerr20", "opto3x5", "kerr40"])
def test_level_ilu0_equals_sync_free_ilu0(name):
    """The ILU(0) run one launch per level (device-wide path, shallow
    schedule, factors of the colour-class reordering of the RCM-ordered
    matrix) gives the same factors, bit for bit, as the sync-free
    factorisation of the colour-ordered matrix (the workgroup path's
    set-up), and both match the oracle's ILU(0)."""
    # kerr40: the trace row (40 entries) is factored by one workgroup in LDS
    s = SMALL[name]() if name in SMALL else qs.kerr(40)
    La = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(La, "trace_gmres", ordering="colour", path="device")
    Lb = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(Lb, "trace_bicgstab", ordering="colour", path="workgroup")
    assert np.array_equal(ssl.export_perm(La), ssl.export_perm(Lb))
    Ab = ssl.export_csr(Lb, ssl.SS_MAT_A_PERM)
    LUa, LUb = ssl.export_csr(La, ssl.SS_MAT_LU), ssl.export_csr(Lb, ssl.SS_MAT_LU)
    assert np.array_equal(LUa.indptr, LUb.indptr) and np.array_equal(LUa.indices, LUb.indices)
    assert np.array_equal(LUa.data, LUb.data)
    LUo, _ = oilu.ilu0(Ab, guard=1e-8, boost=0.1)
    rel = np.abs(LUa.data - LUo.data) / np.maximum(np.abs(LUo.data), 1e-300)
    big = np.abs(LUo.data) > 1e-10 * np.abs(LUo.data).max()
    assert np.max(rel[big]) <= 1e-11
