"""Matrix-free application of L and the matrix-free fp64 residual (GPU
required).

SS_OP_APPLY_L evaluates vec(Gpre X + X Gpost^T + sum_k C_k X C_k^+) from the
d x d operators.  It is compared element by element with the oracle's
superoperator action L[X] (eq. lindblad written with d x d matrix products,
no vectorisation) and with the assembled SpMV (SS_OP_SPMV_L): both sums of
the same fp64 products in another order, so the bound is 1e-12 of
max_r sum_c |L_rc| max|x| (a few hundred terms at most, each rounded once).
Solves with SS_FLAG_MATRIX_FREE must meet the same bars as the assembled
residual (1e-8 fp64 / 1e-6 mixed against the dense oracle, ||L rho|| <= tol).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import qsystems as qs
from conftest import load_product
from oracle import invariants as inv
from oracle.liouvillian import liouvillian_sparse, vec
from oracle.steady import steady_state_dense

pytestmark = pytest.mark.gpu
ssl = load_product()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _zero_h(d):
    return sp.csr_matrix((d, d), dtype=np.complex128)


SYSTEMS = {
    "kerr20": lambda: qs.config(1),
    "jc8": lambda: qs.jaynes_cummings(8, seed=0),
    "random7": lambda: qs.random_lindblad(7, 3, seed=4),
    "spin4": lambda: qs.spin_chain(4),
    "opto3x5": lambda: qs.optomechanics(3, 5, nth=1.0),
    "two_level": lambda: qs.two_level_atom(),
    "jc40": lambda: qs.config(2),
    "kerr_chain2x4": lambda: qs.kerr_chain(2, 4, J=0.3),
    "no_dissipation": lambda: qs.System("kerr5_closed", qs.kerr(5).H, []),
    "pure_decay": lambda: qs.System("decay6", _zero_h(6), [qs.destroy(6)]),
    "one_state": lambda: qs.System("one", sp.csr_matrix(np.array([[0.3]], dtype=np.complex128)), []),
}


def _rand(d, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))


def _bound(Lo, x):
    return 1e-12 * max(float(abs(Lo).sum(axis=1).max()), 1.0) * max(float(np.abs(x).max()), 1e-300)


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_apply_l_matches_oracle_and_assembled_spmv(name):
    s = SYSTEMS[name]()
    _say("apply_l", name, s.dim)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    Lo = liouvillian_sparse(s.H, s.c_ops)
    for seed in range(2):
        X = _rand(s.dim, seed)
        x = vec(X)
        y = ssl.apply(L, ssl.SS_OP_APPLY_L, x)
        ref = vec(inv.superop_action(s.H, s.c_ops, X))
        tol = _bound(Lo, x)
        assert np.max(np.abs(y - ref)) <= tol
        assert np.max(np.abs(y - ssl.apply(L, ssl.SS_OP_SPMV_L, x))) <= tol


def test_apply_l_is_deterministic_and_needs_no_prepare():
    s = SYSTEMS["jc40"]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    x = vec(_rand(s.dim, 7))
    y0 = ssl.apply(L, ssl.SS_OP_APPLY_L, x)
    for _ in range(3):
        assert np.array_equal(ssl.apply(L, ssl.SS_OP_APPLY_L, x), y0)
    ssl.prepare(L, "trace_bicgstab")
    assert np.array_equal(ssl.apply(L, ssl.SS_OP_APPLY_L, x), y0)


@pytest.mark.parametrize("k", [3, 4])
def test_apply_l_full_size(k):
    """The two large workloads (optomechanics 10 x 60, n = 360 000; Kerr chain
    3 x 10, n = 10^6) against the oracle's d x d products, every element."""
    s = qs.config(k)
    _say("apply_l full size", s.name, s.dim)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    X = _rand(s.dim, 11)
    x = vec(X)
    y = ssl.apply(L, ssl.SS_OP_APPLY_L, x)
    ref = vec(inv.superop_action(s.H, s.c_ops, X))
    Lo = liouvillian_sparse(s.H, s.c_ops)
    err = np.max(np.abs(y - ref))
    _say("   err", err, "bound", _bound(Lo, x))
    assert err <= _bound(Lo, x)


SOLVES = [("kerr20", "trace_bicgstab"), ("kerr20", "invpow_bicgstab"), ("jc8", "trace_gmres"),
          ("opto3x5", "invpow_gmres"), ("random7", "trace_bicgstab"), ("spin4", "invpow_bicgstab"),
          ("jc40", "trace_bicgstab"), ("jc40", "invpow_bicgstab"), ("two_level", "trace_bicgstab")]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("name,method", SOLVES)
def test_matrix_free_solve_matches_oracle(name, method, prec, tol):
    s = SYSTEMS[name]()
    _say("matrix-free solve", name, method, prec)
    ref = steady_state_dense(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, info = ssl.solve(L, method, tol=1e-10, prec=prec, matrix_free=True, raise_on_error=False)
    rho_a, info_a = ssl.solve(L, method, tol=1e-10, prec=prec, path="device", raise_on_error=False)
    _say("   err", np.max(np.abs(rho - ref)), "resid", info["resid_l2"], info_a["resid_l2"], "outer",
         info["outer_its"], info_a["outer_its"], "inner", info["inner_its"], info_a["inner_its"])
    assert info["status"] == 0
    assert info["path"] == info_a["path"]
    assert np.max(np.abs(rho - ref)) <= tol
    assert info["resid_l2"] <= 1e-10
    # the certificate agrees with the oracle's ||L rho||
    Lo = liouvillian_sparse(s.H, s.c_ops)
    assert abs(info["resid_l2"] - inv.residual_l2(Lo, rho)) <= 1e-13 * max(1.0, float(abs(Lo).max()))


def test_matrix_free_degenerate_systems():
    for name in ("one_state", "pure_decay"):
        s = SYSTEMS[name]()
        L = ssl.build_liouvillian(s.H, s.c_ops)
        for method in ("trace_bicgstab", "invpow_gmres"):
            rho, info = ssl.solve(L, method, tol=1e-12, matrix_free=True)
            ref = np.zeros((s.dim, s.dim))
            ref[0, 0] = 1.0
            assert info["status"] == 0
            assert np.max(np.abs(rho - ref)) <= 1e-10, (name, method)


def test_matrix_free_takes_the_device_wide_path():
    """The flag implies the device-wide path (the workgroup-resident solver
    keeps its fp64 residual inside the kernel), so batched solves, which run
    only that solver, reject it."""
    s = SYSTEMS["kerr20"]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, info = ssl.solve(L, "trace_bicgstab", tol=1e-10, matrix_free=True, path="workgroup")
    assert info["path"] == 0
    with pytest.raises(ssl.SolverError):
        ssl.solve_batch([L], "trace_bicgstab", 1e-10, matrix_free=True)
