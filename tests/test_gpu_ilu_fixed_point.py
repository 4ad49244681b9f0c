"""Fixed-point ILU(0) (ss_options.ilu_sweeps, Chow and Patel's synchronous
sweeps) through the C ABI against the oracle: the factors after s sweeps
element by element, the elimination-order factors once the sweeps cover the
dependency chains, steady states with the approximate factors against the
dense oracle (1e-8 max-abs fp64, 1e-6 mixed, ||L rho||_2 <= 1e-10), and the
paths that refuse it."""
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


def _rel(a, b):
    a, b = sp.csr_matrix(a), sp.csr_matrix(b)
    return abs(a - b).max() / abs(b).max()


def _factored(L, s, method, ordering):
    """The matrix the device-wide set-up factorises: P A P^T in RCM order, or
    its colour-class reordering (the factors' order on that path)."""
    Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
    if ordering in ("rcm", "natural"):
        return Ap
    Lo = liouvillian_sparse(s.H, s.c_ops)
    Ao = otr.modified(Lo, pop=otr.trace_population(Lo))[0] if method.startswith("trace") else otr.shifted(Lo)
    base = oord.rcm(Ao)
    pos = np.empty(Ao.shape[0], dtype=np.int64)
    pos[base] = np.arange(Ao.shape[0])
    cp = pos[oord.colour_order(Ao)]
    return oord.permute(Ap, cp)


@pytest.mark.parametrize("sweeps", [1, 3])
@pytest.mark.parametrize("name,method,ordering", [("kerr20", "trace_gmres", "rcm"),
                                                  ("jc8", "invpow_gmres", "colour"),
                                                  ("opto3x5", "trace_gmres", "rcm"),
                                                  ("kerr40", "trace_gmres", "natural")])
def test_factors_after_s_sweeps_match_the_oracle(name, method, ordering, sweeps):
    # kerr40: the trace row has 40 entries, more than a lane group holds
    s = {"kerr20": lambda: qs.config(1), "jc8": lambda: qs.jaynes_cummings(8, seed=0),
         "opto3x5": lambda: qs.optomechanics(3, 5, nth=1.0), "kerr40": lambda: qs.kerr(40)}[name]()
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, method, ordering=ordering, path="device", ilu_sweeps=sweeps)
    F = _factored(L, s, method, ordering)
    LU = ssl.export_csr(L, ssl.SS_MAT_LU)
    ref, _ = oilu.ilu0_fixed_point(F, sweeps, guard=1e-8, boost=0.1)
    assert np.array_equal(LU.indptr, ref.indptr) and np.array_equal(LU.indices, ref.indices)
    r = _rel(LU, ref)
    _say(name, ordering, "sweeps", sweeps, "rel", r)
    assert r <= 1e-12
    L.free()


@pytest.mark.parametrize("ordering", ["rcm", "colour"])
def test_enough_sweeps_give_the_elimination_factors(ordering):
    s = qs.jaynes_cummings(8, seed=0)
    La = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(La, "trace_gmres", ordering=ordering, path="device", ilu_sweeps=300)
    Lb = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(Lb, "trace_gmres", ordering=ordering, path="device")
    r = _rel(ssl.export_csr(La, ssl.SS_MAT_LU), ssl.export_csr(Lb, ssl.SS_MAT_LU))
    _say("jc8", ordering, "300 sweeps vs elimination", r)
    assert r <= 1e-12
    La.free()
    Lb.free()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("ordering", ["rcm", "colour"])
def test_steady_state_with_approximate_factors(prec, tol, ordering):
    s = qs.config(2)
    ref = steady_state_dense(s.H, s.c_ops)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    rho, info = ssl.solve(L, "invpow_gmres", 1e-10, prec=prec, ordering=ordering, path="device", ilu_sweeps=3)
    err = float(np.max(np.abs(rho - ref)))
    _say("jc40", prec, ordering, "3 sweeps: inner its", info["inner_its"], "err", err)
    assert info["status"] == 0 and info["resid_l2"] <= 1e-10
    assert err <= tol
    L.free()


def test_refused_where_not_built():
    s = qs.config(1)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    with pytest.raises(ssl.SolverError):
        ssl.prepare(L, "trace_bicgstab", path="workgroup", ilu_sweeps=2)
    with pytest.raises(ssl.SolverError):
        ssl.prepare(L, "trace_bicgstab", path="device", ilu="ilut", ilu_sweeps=2)
    with pytest.raises(ssl.SolverError):
        ssl.solve_batch([L], "trace_bicgstab", 1e-10, ilu_sweeps=2)
    L.free()
