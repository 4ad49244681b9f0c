"""Batched assembly (ss_build_liouvillian_batch) against assembly one system
at a time and against the oracle (GPU required).

Both assemblies add every entry's terms in the same order, so the batched L
must equal the single-system L bit for bit (row pointers, columns and
values), and the d x d operators kept for the matrix-free product must give
the same L x.  Against the oracle's Kronecker assembly the bar is the
assembly parity bar, 1e-14 relative.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import qsystems as qs
from conftest import load_product
from oracle.liouvillian import liouvillian_sparse

pytestmark = pytest.mark.gpu
ssl = load_product()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(m):
    A = sp.csr_matrix(m, dtype=np.complex128)
    A.sum_duplicates()
    A.sort_indices()
    return (torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.data)).cuda(), A.shape[0])


def _systems():
    k5 = qs.kerr(5)
    return [qs.config(1), qs.jaynes_cummings(8, seed=0), qs.random_lindblad(7, 3, seed=4), qs.spin_chain(3),
            qs.optomechanics(3, 5, nth=1.0), qs.two_level_atom(),
            qs.System("one", sp.csr_matrix(np.array([[0.3]], dtype=np.complex128)), []),
            qs.System("closed", k5.H, []),
            qs.System("decay", sp.csr_matrix((6, 6), dtype=np.complex128), [qs.destroy(6)]),
            qs.config(2)]


def _same(La, Lb):
    A = ssl.export_csr(La, ssl.SS_MAT_L)
    B = ssl.export_csr(Lb, ssl.SS_MAT_L)
    return (np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
            and np.array_equal(A.data, B.data))


def _check_batch(systems, Ls):
    for s, L in zip(systems, Ls):
        ref = ssl.build_liouvillian(s.H, s.c_ops)
        assert L.N == s.dim
        assert _same(L, ref), s.name
        Lo = liouvillian_sparse(s.H, s.c_ops)
        Lg = ssl.export_csr(L, ssl.SS_MAT_L)
        scale = max(abs(Lo).max(), 1e-300)
        assert abs(Lg - Lo).max() <= 1e-14 * scale, s.name
        x = np.random.default_rng(3).standard_normal(s.dim ** 2) * (1 + 0.5j)
        assert np.array_equal(ssl.apply(L, ssl.SS_OP_APPLY_L, x), ssl.apply(ref, ssl.SS_OP_APPLY_L, x)), s.name


def test_batch_build_equals_single_builds_device_inputs():
    systems = _systems()
    _say("batch build", [s.dim for s in systems])
    Ls = ssl.build_liouvillian_batch([(_dev(s.H), [_dev(c) for c in s.c_ops]) for s in systems])
    _check_batch(systems, Ls)


def test_batch_build_host_inputs_and_mixed_batches():
    """Host arrays take the one-system path; a batch may mix both kinds."""
    systems = _systems()[:6]
    items = [((s.H, s.c_ops) if k % 2 else (_dev(s.H), [_dev(c) for c in s.c_ops])) for k, s in enumerate(systems)]
    _check_batch(systems, ssl.build_liouvillian_batch(items))
    assert ssl.build_liouvillian_batch([]) == []


def test_batch_build_in_chunks(monkeypatch):
    """A staging cap of 1 MB splits 40 systems into several chunks."""
    monkeypatch.setenv("SS_ASM_STAGE_MB", "1")
    rng = np.random.default_rng(0)
    systems = [qs.kerr(int(n), delta=float(dl)) for n, dl in zip(rng.integers(10, 61, 40), rng.uniform(-1, 1, 40))]
    Ls = ssl.build_liouvillian_batch([(_dev(s.H), [_dev(c) for c in s.c_ops]) for s in systems])
    _check_batch(systems[:6], Ls[:6])
    for s, L in zip(systems, Ls):
        assert _same(L, ssl.build_liouvillian(s.H, s.c_ops))


def test_batch_build_then_batch_solve():
    from oracle.steady import steady_state_dense
    systems = [qs.kerr(int(n)) for n in (8, 12, 20, 31)] + [qs.jaynes_cummings(6, seed=1)]
    Ls = ssl.build_liouvillian_batch([(_dev(s.H), [_dev(c) for c in s.c_ops]) for s in systems])
    rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", 1e-10)
    for s, rho, info in zip(systems, rhos, infos):
        assert info["status"] == 0
        assert np.max(np.abs(rho - steady_state_dense(s.H, s.c_ops))) <= 1e-8


def _bad_cols(d, cols):
    ip = torch.tensor([0] + [len(cols)] * d, dtype=torch.int64).cuda()
    ix = torch.tensor(cols, dtype=torch.int32).cuda()
    dv = torch.ones(len(cols), dtype=torch.complex128).cuda()
    return (ip, ix, dv, d)


@pytest.mark.parametrize("cols,msg", [([2, 1], "strictly increasing"), ([0, 5], "in range")])
def test_batch_build_rejects_invalid_input(cols, msg):
    """An invalid system fails the whole batch and is named in the error;
    the valid systems of the batch are unaffected afterwards."""
    good = qs.kerr(5)
    items = [(_dev(good.H), [_dev(c) for c in good.c_ops]), (_bad_cols(5, cols), [])]
    with pytest.raises(ssl.SolverError) as e:
        ssl.build_liouvillian_batch(items)
    assert "system 1" in str(e.value) and msg in str(e.value)
    L = ssl.build_liouvillian_batch(items[:1])[0]
    assert _same(L, ssl.build_liouvillian(good.H, good.c_ops))


def _mats(L):
    return [ssl.export_csr(L, w) for w in (ssl.SS_MAT_A, ssl.SS_MAT_SYM, ssl.SS_MAT_A_PERM, ssl.SS_MAT_LU)]


@pytest.mark.parametrize("method,opts", [("trace_bicgstab", {}), ("invpow_bicgstab", {}),
                                         ("trace_bicgstab", {"weight": 0.7, "trace_row": 2}),
                                         ("trace_bicgstab", {"prec": "mixed"})])
def test_batched_setup_equals_prepare(method, opts):
    """The batch's set-up stages (transform, pattern, ordering, ILU(0)) give
    every handle the matrices ss_prepare gives it on its own, bit for bit.
    A system that ILU(0) cannot precondition (the three-spin chain's trace
    row) is solved again with iLUT and GMRES, which re-prepares its handle:
    it is checked for its result instead."""
    systems = _systems()[:6] + [qs.kerr(int(n)) for n in (9, 17, 33)]
    Ls = ssl.build_liouvillian_batch([(_dev(s.H), [_dev(c) for c in s.c_ops]) for s in systems])
    _, infos = ssl.solve_batch(Ls, method, 1e-10, raise_on_error=False, **opts)
    for s, L, info in zip(systems, Ls, infos):
        if opts.get("trace_row", -1) >= s.dim:
            assert info["status"] == ssl.SS_E_INVALID_ARG
            continue
        if info["fell_back"]:
            assert info["status"] == 0 and info["resid_l2"] <= 1e-10, s.name
            continue
        ref = ssl.build_liouvillian(s.H, s.c_ops)
        ssl.prepare(ref, method, **opts)
        for a, b in zip(_mats(L), _mats(ref)):
            assert np.array_equal(a.indptr, b.indptr) and np.array_equal(a.indices, b.indices), s.name
            assert np.array_equal(a.data, b.data), s.name
        assert np.array_equal(ssl.export_perm(L), ssl.export_perm(ref)), s.name


def test_batched_setup_rejects_a_bad_trace_row_for_that_system_only():
    systems = [qs.kerr(3), qs.kerr(8)]
    Ls = ssl.build_liouvillian_batch([(_dev(s.H), [_dev(c) for c in s.c_ops]) for s in systems])
    _, infos = ssl.solve_batch(Ls, "trace_bicgstab", 1e-10, raise_on_error=False, trace_row=5)
    assert infos[0]["status"] == ssl.SS_E_INVALID_ARG
    assert infos[1]["status"] == 0


def test_batched_finish_reports_what_the_one_system_finish_reports():
    """bandwidth and profile of P A P^T, trace and Hermiticity errors, and the
    certificate from the batched finish against the oracle's definitions."""
    from oracle import ordering as oord
    from oracle import invariants as oinv
    systems = _systems()[:6]
    Ls = ssl.build_liouvillian_batch([(_dev(s.H), [_dev(c) for c in s.c_ops]) for s in systems])
    rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", 1e-10, hermitize=True)
    for s, L, rho, info in zip(systems, Ls, rhos, infos):
        Ap = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
        assert info["bandwidth"] == oord.bandwidth(Ap)[2], s.name
        assert info["profile"] == oord.profile(Ap)[2], s.name
        assert info["herm_err"] == oinv.hermiticity_error(rho) == 0.0
        # trace_err: |Tr x - 1| of the solution before normalisation (the
        # trace row holds it to the tolerance); the returned rho has unit trace
        assert info["trace_err"] <= 1e-9
        assert abs(np.trace(rho) - 1.0) <= 1e-13
        Lo = liouvillian_sparse(s.H, s.c_ops)
        assert abs(info["resid_l2"] - oinv.residual_l2(Lo, rho)) <= 1e-13 * max(1.0, float(abs(Lo).max()))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_setup_and_solve_equal_one_system_on_the_workload(prec):
    """Driven Jaynes-Cummings, cavity 40 x qubit (n = 6400, several
    1024-row chunks in every batched set-up kernel): the batch's matrices,
    ordering and ILU(0) factors equal ss_prepare's bit for bit, and its solve
    takes the same iterations to the same bits as the one-system workgroup
    solve (the same kernel on the same factors)."""
    s = qs.config(2)
    Ls = ssl.build_liouvillian_batch([(s.H, s.c_ops)] * 3)
    rhos, infos = ssl.solve_batch(Ls, "trace_bicgstab", 1e-10, prec=prec)
    ref = ssl.build_liouvillian(s.H, s.c_ops)
    rho1, info1 = ssl.solve(ref, "trace_bicgstab", tol=1e-10, prec=prec, path="workgroup")
    print("batched", [(i["outer_its"], i["inner_its"]) for i in infos], "one system",
          (info1["outer_its"], info1["inner_its"]), file=sys.stderr, flush=True)
    for L, rho, info in zip(Ls, rhos, infos):
        for a, b in zip(_mats(L), _mats(ref)):
            assert np.array_equal(a.indptr, b.indptr) and np.array_equal(a.indices, b.indices)
            assert np.array_equal(a.data, b.data)
        assert np.array_equal(ssl.export_perm(L), ssl.export_perm(ref))
        assert (info["outer_its"], info["inner_its"]) == (info1["outer_its"], info1["inner_its"])
        assert np.array_equal(rho, rho1)
