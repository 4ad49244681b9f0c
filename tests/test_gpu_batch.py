"""Batched solves (ss_solve_batch): one workgroup per system, results equal
to the dense oracle and bit-identical to a batch of one (GPU required)."""
import sys

import numpy as np
import pytest

import qsystems as qs
from conftest import load_product
from oracle.steady import steady_state_dense

pytestmark = pytest.mark.gpu
ssl = load_product()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _systems():
    return ([qs.jaynes_cummings(N, seed=k) for k, N in enumerate((6, 9, 12, 15))] +
            [qs.kerr(N, delta=dl, E=E) for N, dl, E in ((10, -0.5, 1.0), (17, 0.3, 0.5), (25, 1.0, 2.0))] +
            [qs.optomechanics(3, 5, nth=1.0), qs.random_lindblad(7, 3, seed=4)])


@pytest.mark.parametrize("method", ["trace_bicgstab", "invpow_bicgstab"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_batch_matches_oracle_and_batch_of_one(prec, tol, method):
    systems = _systems()
    Ls = [ssl.build_liouvillian(s.H, s.c_ops) for s in systems]
    rhos, infos = ssl.solve_batch(Ls, method, 1e-10, prec=prec)
    for s, L, rho, info in zip(systems, Ls, rhos, infos):
        _say(s.name, prec, method, "status", info["status"], "its", info["outer_its"], info["inner_its"],
             "resid", info["resid_l2"])
        assert info["status"] == 0
        assert info["resid_l2"] <= 1e-10
        ref = steady_state_dense(s.H, s.c_ops)
        assert np.max(np.abs(rho - ref)) <= tol
    for k in (0, 5):
        (alone,), _ = ssl.solve_batch([Ls[k]], method, 1e-10, prec=prec)
        assert np.array_equal(alone, rhos[k])


def test_batch_of_workload_systems():
    """Four seeded parameter draws of the Jaynes-Cummings workload (n = 6400)."""
    systems = [qs.jaynes_cummings(40, seed=k) for k in range(4)]
    Ls = [ssl.build_liouvillian(s.H, s.c_ops) for s in systems]
    for prec, tol in (("mixed", 1e-6), ("fp64", 1e-8)):
        rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", 1e-10, prec=prec)
        for s, rho, info in zip(systems[:2], rhos, infos):
            assert info["status"] == 0 and info["resid_l2"] <= 1e-10
            assert np.max(np.abs(rho - steady_state_dense(s.H, s.c_ops))) <= tol
        assert all(i["status"] == 0 and i["resid_l2"] <= 1e-10 for i in infos)


def test_batch_rejects_gmres_and_repeated_handles():
    s = qs.kerr(10)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    with pytest.raises(ssl.SolverError):
        ssl.solve_batch([L], "trace_gmres", 1e-10)
    with pytest.raises(ssl.SolverError):
        ssl.solve_batch([L, L], "trace_bicgstab", 1e-10)


def test_caller_allocator_is_used_and_gives_the_same_result():
    """ss_set_allocator with callbacks that call hipMalloc / hipFree of the
    HIP runtime the library uses: every device block of a solve goes
    through them, all are returned, and the result is bit-identical."""
    import ctypes
    # hipMalloc / hipFree looked up through libss.so's own dependencies: the
    # HIP runtime the library uses, whatever other copy (torch's) is loaded
    hip = ctypes.CDLL(ssl.library_path())
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    s = qs.jaynes_cummings(8, seed=0)
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ref, _ = ssl.solve(L, "trace_bicgstab", 1e-10, prec="mixed")
    L.free()
    ssl.trim_cache()
    live = set()
    calls = {"alloc": 0, "free": 0}

    def alloc(n):
        p = ctypes.c_void_p()
        if hip.hipMalloc(ctypes.byref(p), n) != 0:
            return 0
        calls["alloc"] += 1
        live.add(p.value)
        return p.value

    def free(p):
        calls["free"] += 1
        live.discard(p)
        hip.hipFree(ctypes.c_void_p(p))

    ssl.set_allocator(alloc, free)
    try:
        L = ssl.build_liouvillian(s.H, s.c_ops)
        rho, info = ssl.solve(L, "trace_bicgstab", 1e-10, prec="mixed")
        (rb,), _ = ssl.solve_batch([L], "trace_bicgstab", 1e-10, prec="mixed")
        L.free()
        ssl.trim_cache()
    finally:
        ssl.set_allocator(None, None)
    assert calls["alloc"] > 0 and calls["free"] == calls["alloc"] and not live
    assert np.array_equal(rho, ref)
    assert np.array_equal(rb, ref)
