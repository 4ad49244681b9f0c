"""Request server (continuous batching) on the GPU: results match the dense
oracle, are identical alone and in a mixed batch, and requests arriving
while a batch runs are admitted and finished."""
import sys
import time

import numpy as np
import pytest

import qsystems as qs
from oracle.steady import steady_state_dense

pytestmark = pytest.mark.gpu
from conftest import load_product

ssl = load_product()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _wait(server, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = server.poll(t)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.001)
    return out


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-6), ("fp64", 1e-8)])
def test_server_matches_oracle_and_is_batch_independent(prec, tol):
    stream = qs.serving_stream(12, rate=0.0, seed=3)
    systems = [qs.kerr(N, delta=dl, E=E) for (_, N, dl, E) in stream]
    S = ssl.Server(hbm_budget_bytes=4 << 30, max_slots=64)
    tickets = [S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec=prec) for s in systems]
    res = _wait(S, tickets)
    for t, s in zip(tickets, systems):
        rho, info = res[t]
        assert info["status"] == 0 and info["resid_l2"] <= 1e-10
        if s.dim <= 40:
            ref = steady_state_dense(s.H, s.c_ops)
            assert np.max(np.abs(rho - ref)) <= tol
    # the same request alone gives the same bits
    for k in (0, 5):
        t = S.submit(systems[k].H, systems[k].c_ops, "trace_bicgstab", 1e-10, prec=prec)
        rho_alone, _ = _wait(S, [t])[t]
        assert np.array_equal(rho_alone, res[tickets[k]][0])
    S.close()


def test_server_admits_late_arrivals_and_respects_the_budget():
    stream = qs.serving_stream(40, rate=2000.0, seed=5, n_min=10, n_max=30)
    S = ssl.Server(hbm_budget_bytes=64 << 20, max_slots=8)  # small budget forces queueing
    t0 = time.time()
    tickets = []
    for (arr, N, dl, E) in stream:
        while time.time() - t0 < arr:
            time.sleep(0.0002)
        s = qs.kerr(N, delta=dl, E=E)
        tickets.append(S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec="mixed"))
    res = _wait(S, tickets)
    ok = [res[t][1]["status"] == 0 and res[t][1]["resid_l2"] <= 1e-10 for t in tickets]
    _say("served", len(ok), "requests in", time.time() - t0, "s")
    assert all(ok)
    S.close()


def test_server_rejects_bad_requests():
    S = ssl.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    s = qs.kerr(10)
    with pytest.raises(ssl.SolverError):
        S.submit(s.H, s.c_ops, "trace_gmres", 1e-10)
    S.close()


def test_server_refuses_malformed_inputs_at_submission():
    """Inputs are checked on the host copy when submitted, so a malformed
    request never joins a group (the other requests are unaffected)."""
    import numpy as np
    import scipy.sparse as sp
    S = ssl.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    good = qs.kerr(6)
    A = sp.csr_matrix(good.H)
    A.sort_indices()
    ip = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(A.indices, dtype=np.int32).copy()
    dv = np.ascontiguousarray(A.data, dtype=np.complex128)
    r = next(i for i in range(6) if ip[i + 1] - ip[i] >= 2)
    seg = slice(ip[r], ip[r + 1])
    ix[seg] = ix[seg][::-1].copy()  # one row out of order
    t_ok = S.submit(good.H, good.c_ops, "trace_bicgstab", 1e-10)
    with pytest.raises(ssl.SolverError):
        S.submit((ip, ix, dv, 6), good.c_ops, "trace_bicgstab", 1e-10)
    bad_col = np.ascontiguousarray(A.indices, dtype=np.int32).copy()
    bad_col[0] = 6  # out of range
    with pytest.raises(ssl.SolverError):
        S.submit((ip, bad_col, dv, 6), good.c_ops, "trace_bicgstab", 1e-10)
    S.drain()
    rho, info = S.poll(t_ok)
    assert info["status"] == 0
    S.close()
