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
    budget = 64 << 20
    S = ssl.Server(hbm_budget_bytes=budget, max_slots=8)  # small budget forces queueing
    t0 = time.time()
    tickets, systems = [], []
    for (arr, N, dl, E) in stream:
        while time.time() - t0 < arr:
            time.sleep(0.0002)
        s = qs.kerr(N, delta=dl, E=E)
        systems.append(s)
        tickets.append(S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec="mixed"))
    res = _wait(S, tickets)
    st = S.stats()
    _say("served", len(tickets), "requests in", time.time() - t0, "s;", st)
    for t, s in zip(tickets, systems):
        rho, info = res[t]
        assert info["status"] == 0 and info["resid_l2"] <= 1e-10
        if s.dim <= 20:
            assert np.max(np.abs(rho - steady_state_dense(s.H, s.c_ops))) <= 1e-6
    # every request fits the budget alone, so the admitted footprint never exceeded it
    assert 0 < st["peak_resident_bytes"] <= budget
    assert st["resident_bytes"] == 0 and st["resident"] == 0 and st["queued"] == 0
    assert st["largest_group"] <= 8
    S.close()


def test_late_request_overtakes_a_running_group(monkeypatch):
    """Continuous batching: a request submitted while a long group is on the
    device starts on another worker and finishes first; its result is the
    same bits as when it runs alone."""
    big = [qs.jaynes_cummings(32, seed=k) for k in range(48)]  # n = 4096 each, fp64
    small = qs.kerr(10, delta=0.3, E=0.8)
    # a 5 ms batching window keeps the burst in one group
    monkeypatch.setenv("SS_SERVER_WINDOW_US", "5000")
    monkeypatch.setenv("SS_SERVER_WORKERS", "4")
    S = ssl.Server(hbm_budget_bytes=16 << 30, max_slots=1024)
    tb = [S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec="fp64") for s in big]
    # let the burst form its group and reach the device
    t_wait = time.time()
    while S.stats()["resident"] < len(big) and time.time() - t_wait < 10:
        time.sleep(0.001)
    time.sleep(0.005)
    ts = S.submit(small.H, small.c_ops, "trace_bicgstab", 1e-10, prec="fp64")
    done_small, big_pending_then = None, None
    res = {}
    t0 = time.time()
    while len(res) < len(tb) + 1:
        for t in tb + [ts]:
            if t in res:
                continue
            r = S.poll(t)
            if r is not None:
                res[t] = r
                if t == ts:
                    done_small = time.time() - t0
                    big_pending_then = sum(1 for b in tb if b not in res)
        assert time.time() - t0 < 120
        time.sleep(0.0005)
    st = S.stats()
    _say(f"late request done after {done_small * 1e3:.1f} ms with {big_pending_then} of {len(tb)} earlier requests "
         f"still running; {st}")
    assert st["largest_group"] == len(tb) and st["groups"] == 2
    assert big_pending_then == len(tb), "the late request waited for the running group"
    for t, s in zip(tb, big):
        assert res[t][1]["status"] == 0 and res[t][1]["resid_l2"] <= 1e-10
    rho_mix, info = res[ts]
    assert info["status"] == 0
    assert np.max(np.abs(rho_mix - steady_state_dense(small.H, small.c_ops))) <= 1e-8
    t1 = S.submit(small.H, small.c_ops, "trace_bicgstab", 1e-10, prec="fp64")
    rho_alone, _ = _wait(S, [t1])[t1]
    assert np.array_equal(rho_alone, rho_mix)
    S.close()


def test_fp64_burst_after_a_closed_mixed_server():
    """A server's device blocks outlive it in the library's cache; a later
    server must reuse them cleanly (no HIP error inherited from the first)."""
    stream = qs.serving_stream(300, rate=0.0, seed=7)
    systems = [qs.kerr(N, delta=dl, E=E) for (_, N, dl, E) in stream]
    S = ssl.Server(hbm_budget_bytes=8 << 30, max_slots=1024)
    t = [S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec="mixed") for s in systems[:100]]
    for tk, r in _wait(S, t).items():
        assert r[1]["status"] == 0
    S.close()
    S = ssl.Server(hbm_budget_bytes=8 << 30, max_slots=1024)
    t = [S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec="fp64") for s in systems]
    res = _wait(S, t)
    bad = [(i, res[tk][1]["status"]) for i, tk in enumerate(t) if res[tk][1]["status"] != 0]
    assert not bad, bad
    assert all(res[tk][1]["resid_l2"] <= 1e-10 for tk in t)
    S.close()


def test_server_solves_gmres_and_auto_requests():
    """Requests the batched path does not take are solved on their own."""
    S = ssl.Server(hbm_budget_bytes=1 << 30, max_slots=16)
    s = qs.kerr(12, delta=0.2, E=0.7)
    ref = steady_state_dense(s.H, s.c_ops)
    tk = {m: S.submit(s.H, s.c_ops, m, 1e-10) for m in ("trace_gmres", "invpow_gmres", "auto")}
    res = _wait(S, list(tk.values()))
    for m, t in tk.items():
        rho, info = res[t]
        assert info["status"] == 0, m
        assert np.max(np.abs(rho - ref)) <= 1e-8, m
    S.close()


def test_server_rejects_bad_requests():
    S = ssl.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    s = qs.kerr(10)
    with pytest.raises(ssl.SolverError):
        S.submit(s.H, s.c_ops, 7, 1e-10)       # unknown method
    with pytest.raises(ssl.SolverError):
        S.submit(s.H, s.c_ops, "trace_bicgstab", -1.0)  # bad tolerance
    with pytest.raises(ssl.SolverError):
        S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec=5)  # unknown precision
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
