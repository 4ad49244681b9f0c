"""ss_apply_noalloc against ss_apply through the C ABI: the same operators
with the scratch in the library's static device array instead of allocated
buffers.  Two calls in a row, the second on a smaller system, in both
precisions; the preconditioner runs the row-group triangular solves in both
entry points, so the results are the same bits.  Sizes beyond the scratch
array are refused."""
import ctypes
import sys

import numpy as np
import pytest

import qsystems as qs

pytestmark = pytest.mark.gpu

from conftest import load_product

ssl = load_product()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _prepared(system, prec, ordering="rcm"):
    L = ssl.build_liouvillian(system.H, system.c_ops)
    # the device-wide path, so that ss_prepare builds the triangular-solve
    # schedules the no-alloc preconditioner needs (in the colour-class order
    # the factors' permutation is applied around them)
    ssl.prepare(L, "trace_bicgstab", prec=prec, path="device", ordering=ordering)
    return L


def _both(L, op, prec, x):
    import torch
    xd = torch.from_numpy(x).cuda()
    yd = torch.full_like(xd, complex(np.nan, np.nan))
    ssl.apply_noalloc(L, op, xd, yd, prec=prec)
    torch.cuda.synchronize()
    y_noalloc = yd.cpu().numpy()
    ref_op = ssl.SS_OP_PRECOND_GROUPS if op == ssl.SS_OP_PRECOND else op
    y_ref = ssl.apply(L, ref_op, x, prec=prec)
    return y_noalloc, y_ref


@pytest.mark.parametrize("ordering", ["rcm", "colour"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_apply_on_two_calls_second_smaller(prec, ordering):
    big = qs.config(2)                       # Jaynes-Cummings 40 x qubit, n = 6400
    small = qs.jaynes_cummings(24, seed=3)   # n = 2304
    rng = np.random.default_rng(11)
    ops = [ssl.SS_OP_PRECOND, ssl.SS_OP_SPMV_APERM] + ([ssl.SS_OP_SPMV_L, ssl.SS_OP_APPLY_L] if prec == "fp64" else [])
    handles = [_prepared(big, prec, ordering), _prepared(small, prec, ordering)]
    try:
        for op in ops:
            for L in handles:   # the second call has the smaller input
                n = L.n
                x = rng.normal(size=n) + 1j * rng.normal(size=n)
                y0, y1 = _both(L, op, prec, x)
                _say("noalloc", prec, ordering, "op", op, "n", n, "max |diff|", float(np.max(np.abs(y0 - y1))))
                assert np.all(np.isfinite(y0))
                assert np.array_equal(y0, y1)
    finally:
        for L in handles:
            L.free()


def test_noalloc_refuses_what_it_cannot_do():
    import torch
    s = qs.jaynes_cummings(8, seed=0)   # n = 256: the workgroup path, no device-wide schedules
    L = ssl.build_liouvillian(s.H, s.c_ops)
    ssl.prepare(L, "trace_bicgstab")
    xd = torch.zeros(L.n, dtype=torch.complex128, device="cuda")
    yd = torch.zeros_like(xd)
    with pytest.raises(ssl.SolverError) as e:
        ssl.apply_noalloc(L, ssl.SS_OP_PRECOND, xd, yd)
    assert e.value.code == -7 and "schedules" in str(e.value)  # SS_E_STATE
    # host pointers are refused
    x = np.zeros(L.n, dtype=np.complex128)
    rc = ssl.ss._lib.ss_apply_noalloc(L.handle, ssl.SS_OP_SPMV_APERM, 0, x.ctypes.data, x.ctypes.data)
    assert rc == ssl.SS_E_INVALID_ARG
    L.free()


def test_noalloc_refuses_sizes_beyond_the_scratch():
    """Kerr chain 3 x 11 (n = 1 771 561) against the 64 MiB array: in the
    colour-class order the preconditioner needs 48 n B (fp64) or 40 n B
    (mixed), neither fits; in RCM order 16 n B and 24 n B both fit."""
    import torch
    ch = qs.kerr_chain(3, 11)
    L = ssl.build_liouvillian(ch.H, ch.c_ops)
    n = L.n
    assert 24 * n + 256 <= 64 << 20 < 40 * n + 256
    xd = torch.zeros(n, dtype=torch.complex128, device="cuda")
    xd[0] = 1.0
    yd = torch.zeros_like(xd)
    ssl.prepare(L, "invpow_bicgstab", prec="mixed", ordering="colour", path="device")
    for prec in ("fp64", "mixed"):
        with pytest.raises(ssl.SolverError) as e:
            ssl.apply_noalloc(L, ssl.SS_OP_PRECOND, xd, yd, prec=prec)
        assert e.value.code == ssl.SS_E_INVALID_ARG and "scratch" in str(e.value)
    ssl.prepare(L, "invpow_bicgstab", prec="mixed")
    for prec in ("fp64", "mixed"):
        ssl.apply_noalloc(L, ssl.SS_OP_PRECOND, xd, yd, prec=prec)
        torch.cuda.synchronize()
        y_ref = ssl.apply(L, ssl.SS_OP_PRECOND_GROUPS, xd.cpu().numpy(), prec=prec)
        assert np.array_equal(yd.cpu().numpy(), y_ref), prec
    L.free()
