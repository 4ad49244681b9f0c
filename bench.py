#!/usr/bin/env python3
"""Steady-state solver benchmark on one MI355X.

Headline workload: the chain of three coupled driven Kerr cavities, N = 10
each (Hilbert dimension 1000, Liouvillian 10^6 x 10^6 with 20.7 M non-zeros),
hopping J = 0.3; synthetic, no data files.  One step = one full solve through
the C ABI: Liouvillian assembly from H and the collapse operators already
resident in HBM, shift transform, RCM and the colour-class order over it,
ILU(0), the doubly-iterative inverse-power method (fp64 outer steps,
preconditioned inner Krylov solves), finish (unpermute, normalise,
certificate ||L rho||_2 <= 1e-10), rho left in HBM.

`value` is fp64 solves/s (complex128 throughout, BiCGSTAB inner solves); the
mixed path (complex64 inner solves and factors, fp64 outer steps, GMRES(40)
inner solves) is timed beside it on the same GPU, and so is the same solve
in plain RCM order.  Every result is checked against the oracle: for this size the CPU fp64
sparse reference (RCM-ordered ILU(0)-BiCGSTAB on the trace-row system, one
CPU thread), which is also the timed CPU baseline.

Secondary measurements, each recorded inside the one JSON line (a failure
is recorded there too, and makes the exit status non-zero):
  * the SpMV of the same matrix in complex128 and complex64 (GB/s) and the
    matrix-free L x;
  * a batched step of 256 seeded Jaynes-Cummings systems (cavity 40 x qubit,
    n = 6400, each with its own parameter draw), mixed and fp64;
  * the driven spin chain (8 spins) with the automatic method choice;
  * the serving stream (2000 Kerr requests): burst capacity in both
    precisions and Poisson arrivals at 0.5, 1 and 2 times that capacity,
    with p50/p99 submit-to-result latency.
"""
import argparse
import json
import os
import sys
import time
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _device_csr(m, torch):
    import scipy.sparse as sp
    A = sp.csr_matrix(m, dtype=np.complex128)
    A.sort_indices()
    ip = torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int64)).cuda()
    ix = torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).cuda()
    dv = torch.from_numpy(np.ascontiguousarray(A.data)).cuda()
    return (ip, ix, dv, A.shape[0])


def spmv_bytes(n, nnz, s):
    """Algorithmic bytes of one CSR SpMV: values + column indices, row
    pointers, x read once, y written once (s = bytes per complex value)."""
    return nnz * (s + 4) + 4 * (n + 1) + 2 * n * s


def trsv_pair_bytes(n, nnz_lu, s):
    """Algorithmic bytes of one L-solve + U-solve pair: factor values and
    indices once, row pointers and diagonal positions for both sweeps, and
    right-hand side, intermediate and result vectors."""
    return nnz_lu * (s + 4) + 8 * (n + 1) + 8 * n + 4 * n * s


def apply_l_bytes(n):
    """Algorithmic bytes of one matrix-free application of L: rho read once
    and the result written once (complex128); the d x d operators are a few
    kB and stay in the caches."""
    return 32 * n


# ------------------------------------------------------------------ traffic
# HBM bytes of the dominant kernel from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE), each scaled by what the same counter reads for a plain
# copy of COPY_BYTES bytes.  The dominant kernel is the complex128
# preconditioner application, two launches (lower and upper row-group
# triangular solve); the record holds the mean of each launch's dispatches
# and their sum per application.  It names the kernel and the SHA-256 of its
# sources and is used only while both still match.
KERNEL_SOURCE = "paper_1504_06768_amd/csrc/trsv_classes.hip"
KERNEL_MATCH = "k_trsv_level<HIP_vector_type<double"
COPY_BYTES = 256 << 20


def source_digest(rel, root=None):
    """SHA-256 over a kernel source and every local header it includes
    (transitively): the counters stay valid only while none of them changes."""
    import hashlib
    import re
    root = root or ROOT
    h, seen, todo = hashlib.sha256(), [], [os.path.normpath(os.path.join(root, rel))]
    while todo:
        f = todo.pop(0)
        if f in seen or not os.path.exists(f):
            continue
        seen.append(f)
        with open(f, "rb") as fh:
            data = fh.read()
        h.update(os.path.relpath(f, root).encode() + b"\0" + data)
        for inc in re.findall(rb'#include "([^"]+)"', data):
            todo.append(os.path.normpath(os.path.join(os.path.dirname(f), inc.decode())))
    return h.hexdigest()


def write_traffic(fetch_db, write_db, apps, out_path=None, root=None, match=KERNEL_MATCH, source=KERNEL_SOURCE,
                  workload="kerr_chain_3x10 (n = 1e6), colour-class order: complex128 preconditioner "
                           "application, one launch per level of the lower and the upper factor"):
    """profiles/traffic.json from two rocprofv3 --pmc runs of
    `bench.py --counter-apps apps`: FETCH_SIZE and WRITE_SIZE (KiB, summed
    over the counter's instances) of every dispatch whose kernel name
    contains `match`, summed and divided by the number of applications, each
    scaled by what the same counter reads for the calibration copy of
    COPY_BYTES."""
    import sqlite3

    def read(db, counter):
        con = sqlite3.connect(db)
        rows = list(con.execute(
            "select kernel_name, grid_size, sum(value) from counters_collection where counter_name = ? "
            "group by dispatch_id order by dispatch_id", (counter,)))
        con.close()
        per = [v for (k, g, v) in rows if match in k]
        # the calibration copy is bench.py's first device-to-device copy with
        # that grid (later copies of other sizes can share the grid)
        copy = [v for (k, g, v) in rows if "copyBuffer" in k and g == COPY_BYTES // 2048]
        if not per or not copy:
            raise SystemExit(f"{db}: no dispatch of {match} or no calibration copy of {COPY_BYTES} bytes")
        return float(sum(per)) / apps, copy[0], len(per), apps

    fetch, cf, nf, kf = read(fetch_db, "FETCH_SIZE")
    write, cw, nw, kw = read(write_db, "WRITE_SIZE")
    ff, fw = (COPY_BYTES / 1024) / cf, (COPY_BYTES / 1024) / cw
    fb, wb = fetch * 1024 * ff, write * 1024 * fw
    rec = {"kernel_match": match, "workload": workload, "source": source,
           "sources_sha256": source_digest(source, root), "dispatches": {"fetch": nf, "write": nw},
           "applications": apps,
           "fetch_size_kib": fetch, "write_size_kib": write,
           "calibration": {"copy_bytes": COPY_BYTES, "copy_fetch_size_kib": cf, "copy_write_size_kib": cw,
                           "fetch_factor": ff, "write_factor": fw},
           "hbm_bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb}
    with open(out_path or os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))
    return rec


def _traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    record, or None when it is missing, names another kernel, or its sources
    have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_match") != KERNEL_MATCH or rec.get("source") != KERNEL_SOURCE:
        return None
    if source_digest(rec["source"]) != rec.get("sources_sha256"):
        return None
    return rec["hbm_bytes_per_launch"]


# ---------------------------------------------------------------- headline
# Inverse power on the colour-class order (greedy colouring visited in a
# seeded random order, classes in RCM order): every ILU(0) substitution has
# about 14 levels instead of ~2200 in RCM order.  Measured per solve on this
# workload: fp64 131 ms with BiCGSTAB inner solves against 159 ms with
# GMRES(40); mixed 134 ms with GMRES(40) against 193 ms with BiCGSTAB (in
# complex64, BiCGSTAB needs 175 iterations for the three outer steps against
# 78 for one fp64 step).  In RCM order the same solve took 443 ms (fp64,
# GMRES(40)): bound by the ~2200 dependent levels of each preconditioner
# application.
HEADLINE_ORDERING = "colour"
HEADLINE = {"fp64": ("invpow_bicgstab", 20), "mixed": ("invpow_gmres", 40)}
RCM_COMPARE = ("invpow_gmres", 40)


def headline(ssl, qs, torch, args):
    """Full C4 solves, fp64 and mixed: per-step times, iteration counts,
    residuals; rho of the last step of each precision (host copy).  Then one
    solve per precision in plain RCM order, for comparison."""
    ch = qs.config(4)
    N = ch.dim
    Hd = _device_csr(ch.H, torch)
    Cd = [_device_csr(c, torch) for c in ch.c_ops]
    out = torch.empty(N * N, dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()

    def step(prec, method, m, ordering):
        L = ssl.build_liouvillian(Hd, Cd)
        _, info = ssl.solve(L, method, tol=1e-10, out=out, prec=prec, gmres_m=m, ordering=ordering)
        L.free()
        return info

    res = {}
    for prec in ("fp64", "mixed"):
        method, m = HEADLINE[prec]
        for _ in range(args.warmup):
            step(prec, method, m, HEADLINE_ORDERING)
        torch.cuda.synchronize()
        times, infos = [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            infos.append(step(prec, method, m, HEADLINE_ORDERING))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rho = out.cpu().numpy().reshape(N, N, order="F")
        last = infos[-1]
        res[prec] = {"method": method, "gmres_m": m if "gmres" in method else None, "ordering": HEADLINE_ORDERING,
                     "solves_per_s": args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
                     "median_ms": 1e3 * float(np.median(times)), "min_ms": 1e3 * float(np.min(times)),
                     "worst_resid_l2": max(i["resid_l2"] for i in infos), "outer_its": last["outer_its"],
                     "inner_its": last["inner_its"], "t_setup_ms": last["t_setup_ms"],
                     "t_solve_ms": last["t_solve_ms"], "colours": last["colours"], "bandwidth": last["bandwidth"],
                     "nnz_matrix": last["nnz_matrix"], "nnz_factors": last["nnz_factors"], "rho": rho}
        _log(f"kerr_chain_3x10 {prec} ({method}, colour order): {1e3 * dt / args.steps:.1f} ms per solve "
             f"(median {res[prec]['median_ms']:.1f}), set-up {last['t_setup_ms']:.1f} ms, "
             f"its {last['outer_its']}/{last['inner_its']}, resid {last['resid_l2']:.2e}")
    rcm = {"method": RCM_COMPARE[0], "gmres_m": RCM_COMPARE[1], "ordering": "rcm"}
    for prec in ("fp64", "mixed"):
        ts = time.perf_counter()
        info = step(prec, RCM_COMPARE[0], RCM_COMPARE[1], "rcm")
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - ts)
        rcm[prec] = {"ms": ms, "solves_per_s": 1e3 / ms, "inner_its": info["inner_its"],
                     "t_setup_ms": info["t_setup_ms"], "resid_l2": info["resid_l2"], "status": info["status"]}
        _log(f"kerr_chain_3x10 {prec} in RCM order ({RCM_COMPARE[0]}): {ms:.1f} ms, its {info['inner_its']}")
    res["rcm_order"] = rcm
    return ch, Hd, Cd, res


def _prepared_chain(ssl, Hd, Cd):
    L = ssl.build_liouvillian(Hd, Cd)
    ssl.prepare(L, HEADLINE["fp64"][0], prec="mixed", ordering=HEADLINE_ORDERING)
    return L


def dominant_kernel(ssl, ch, Hd, Cd, res):
    """The headline step's dominant kernels, timed live with HIP events on
    the handle's stream (ss_time_operator): the preconditioner application
    (lower then upper triangular solve, one launch per level) and the SpMV,
    both complex128; algorithmic bytes from the factor and matrix sizes."""
    L = _prepared_chain(ssl, Hd, Cd)
    try:
        _, n, nnzL = L.shape()
        A = ssl.export_csr(L, ssl.SS_MAT_A_PERM)
        LU = ssl.export_csr(L, ssl.SS_MAT_LU)
        t_pre = ssl.time_operator(L, ssl.SS_OP_PRECOND, "fp64", 20)
        t_pre32 = ssl.time_operator(L, ssl.SS_OP_PRECOND, "mixed", 20)
        t128 = ssl.time_operator(L, ssl.SS_OP_SPMV_APERM, "fp64", 50)
        t64 = ssl.time_operator(L, ssl.SS_OP_SPMV_APERM, "mixed", 50)
        tl = ssl.time_operator(L, ssl.SS_OP_SPMV_L, "fp64", 50)
        tm = ssl.time_operator(L, ssl.SS_OP_APPLY_L, "fp64", 50)
    finally:
        L.free()
    bp, bp32 = trsv_pair_bytes(n, LU.nnz, 16), trsv_pair_bytes(n, LU.nnz, 8)
    b128, b64 = spmv_bytes(n, A.nnz, 16), spmv_bytes(n, A.nnz, 8)
    bl, bm = spmv_bytes(n, nnzL, 16), apply_l_bytes(n)
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9
    kern = {
        "precond_c128": {"ms": t_pre, "bytes": bp, "GB/s": gbs(bp, t_pre), "frac": gbs(bp, t_pre) / PEAK_HBM_GBS},
        "precond_c64": {"ms": t_pre32, "bytes": bp32, "GB/s": gbs(bp32, t_pre32),
                        "frac": gbs(bp32, t_pre32) / PEAK_HBM_GBS},
        "spmv_c128": {"ms": t128, "bytes": b128, "GB/s": gbs(b128, t128), "frac": gbs(b128, t128) / PEAK_HBM_GBS},
        "spmv_c64": {"ms": t64, "bytes": b64, "GB/s": gbs(b64, t64), "frac": gbs(b64, t64) / PEAK_HBM_GBS,
                     "note": "268 MB working set: partly served by the 256 MB Infinity Cache"},
        "spmv_L_c128": {"ms": tl, "bytes": bl, "GB/s": gbs(bl, tl)},
        "apply_L_matrix_free": {"ms": tm, "bytes": bm, "GB/s": gbs(bm, tm), "vs_spmv_L": tl / tm},
        "nnz_matrix": int(A.nnz), "nnz_factors": int(LU.nnz), "n": int(n), "ordering": HEADLINE_ORDERING,
    }
    _log(f"precond c128 {t_pre:.3f} ms ({gbs(bp, t_pre):.0f} GB/s), c64 {t_pre32:.3f} ms; "
         f"spmv c128 {t128 * 1e3:.1f} us ({gbs(b128, t128):.0f} GB/s), c64 {t64 * 1e3:.1f} us "
         f"({gbs(b64, t64):.0f} GB/s)")
    # per fp64 solve: BiCGSTAB applies the preconditioner twice per iteration
    # (GMRES once per iteration plus once per restart cycle)
    its = res["fp64"]["inner_its"]
    m = HEADLINE["fp64"][1]
    applies = (its + -(-its // m)) if "gmres" in HEADLINE["fp64"][0] else 2 * its
    share = (applies * t_pre) / max(res["fp64"]["median_ms"], 1e-9)
    roof = {"bound": "hbm", "achieved": gbs(bp, t_pre), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs(bp, t_pre) / PEAK_HBM_GBS, "traffic": None,
            "kernel": "preconditioner application (ILU(0) lower + upper triangular solve, complex128, factors in "
                      "colour-class order, input and output in RCM order through the permutation): k_trsv_level, "
                      "one launch per level of each factor (about 14 each); the unit is one application",
            "bytes_per_launch": bp, "avg_launch_ms": t_pre, "unit_of_launch": "one application (all levels)",
            "applications_per_fp64_solve": applies,
            "share_of_fp64_step": share}
    tr = _traffic()
    if tr is not None:
        roof["traffic"] = tr
    return kern, roof


def counter_run(ssl, qs, torch, apps):
    """Only the dominant kernel: `apps` applications of the complex128
    preconditioner on the headline's prepared Kerr chain (for the rocprofv3
    counter runs that write profiles/traffic.json)."""
    ch = qs.config(4)
    Hd = _device_csr(ch.H, torch)
    Cd = [_device_csr(c, torch) for c in ch.c_ops]
    L = _prepared_chain(ssl, Hd, Cd)
    x = torch.ones(L.n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    try:
        for _ in range(apps):
            ssl.apply(L, ssl.SS_OP_PRECOND, x.cpu().numpy(), prec="fp64")
    finally:
        L.free()
    torch.cuda.synchronize()
    _log(f"counter run: {apps} applications of the complex128 preconditioner")


def cpu_baseline(ch, res):
    """The oracle's CPU fp64 sparse reference on the same workload, one full
    solve on one thread (BLAS limited to one thread)."""
    import threadpoolctl
    from oracle.sparse_ref import steady_state_iterative
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        rho, info = steady_state_iterative(ch.H, ch.c_ops, tol=1e-12)
        dt = time.perf_counter() - t0
    errs = {p: float(np.max(np.abs(res[p]["rho"] - rho))) for p in ("fp64", "mixed")}
    _log(f"cpu sparse reference: {dt:.1f} s, {info['iterations']} its, resid {info['resid_l2']:.1e}; "
         f"max|rho_gpu - rho_cpu| fp64 {errs['fp64']:.2e}, mixed {errs['mixed']:.2e}")
    cb = {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
          "sample": "one full solve of the same workload (kerr_chain_3x10, n = 1e6) by the oracle's fp64 "
                    "sparse reference: RCM, ILU(0) in C, BiCGSTAB with refinement to ||L rho|| <= 1e-12, "
                    "one thread",
          "seconds": dt, "iterations": info["iterations"], "resid_l2": info["resid_l2"]}
    return cb, errs


# -------------------------------------------------------------- side legs
def jc_batch(ssl, qs, torch, args):
    """B independent Jaynes-Cummings systems (cavity 40 x qubit), each with
    its own seeded parameter draw, assembled and solved together."""
    B = args.batch
    systems = [qs.jaynes_cummings(40, seed=k) for k in range(B)]
    dev = [(_device_csr(s.H, torch), [_device_csr(c, torch) for c in s.c_ops]) for s in systems]
    N = systems[0].dim
    outs = [torch.empty(N * N, dtype=torch.complex128, device="cuda") for _ in range(B)]
    torch.cuda.synchronize()
    out = {"workload": f"{B} driven Jaynes-Cummings systems, cavity 40 x qubit (n = 6400), parameters "
                       f"drawn per system from U[0.1, 2] with seeds 0..{B - 1}"}
    for prec in ("mixed", "fp64"):
        def step():
            Ls = ssl.build_liouvillian_batch(dev)
            _, infos = ssl.solve_batch(Ls, "trace_bicgstab", tol=1e-10, outs=outs, prec=prec)
            for L in Ls:
                L.free()
            return infos
        if prec == "mixed":
            step()  # warm-up (library caches, code objects)
            _log(f"jc batch {prec}: warm-up step done")
        torch.cuda.synchronize()
        # a step takes seconds: the draws ILU(0) cannot precondition are solved
        # again with iLUT and GMRES, one by one
        reps = max(1, args.batch_reps)
        infos, times = [], []
        for r in range(reps):
            ts = time.perf_counter()
            infos.append(step())
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
            _log(f"jc batch {prec}: step {r + 1}/{reps} {1e3 * times[-1]:.1f} ms")
        dt = float(np.median(times))
        last = infos[-1]
        its = [i["inner_its"] for i in last]
        # the workgroup-resident launch: the bytes of the systems it solved
        inwg = [i for i in last if not i["fell_back"]]
        alg = float(sum(i["bytes_alg"] for i in inwg))
        tk = inwg[0]["t_kernel_ms"] if inwg else float("nan")
        fb = [i for i in last if i["fell_back"]]
        out[prec] = {"solves_per_s": B / dt, "ms_per_step_median": 1e3 * dt, "t_kernel_ms": tk,
                     "fell_back": len(fb),
                     "kernel_GB/s": alg / (tk * 1e-3) / 1e9, "kernel_frac": alg / (tk * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "inner_its_min_median_max": [int(min(its)), float(np.median(its)), int(max(its))],
                     "worst_resid_l2": max(i["resid_l2"] for i in last),
                     "all_ok": all(i["status"] == 0 for i in last)}
        _log(f"jc batch {prec}: {B / dt:.0f} solves/s, kernel {tk:.2f} ms "
             f"({out[prec]['kernel_frac'] * 100:.1f} % of peak), its {out[prec]['inner_its_min_median_max']}")
    from oracle.steady import steady_state_dense
    sample = [0, B // 2, B - 1]
    errs = []
    for prec in ("mixed",):
        Ls = ssl.build_liouvillian_batch([dev[i] for i in sample])
        rhos, _ = ssl.solve_batch(Ls, "trace_bicgstab", tol=1e-10, prec=prec)
        for L in Ls:
            L.free()
        for r, i in zip(rhos, sample):
            errs.append(float(np.max(np.abs(r - steady_state_dense(systems[i].H, systems[i].c_ops)))))
    out["max_abs_err_vs_oracle_sample"] = max(errs)
    out["mixed_vs_fp64"] = out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    return out


def spin_chain_leg(ssl, qs):
    sc = qs.spin_chain(8)
    Ls = ssl.build_liouvillian(sc.H, sc.c_ops)
    out = {"workload": f"spin_chain_8 (d = {sc.dim}, n = {sc.dim ** 2})"}
    try:
        for prec in ("mixed", "fp64"):
            t0 = time.perf_counter()
            _, si = ssl.solve(Ls, "auto", tol=1e-10, prec=prec, raise_on_error=False)
            dt = time.perf_counter() - t0
            out[f"auto_{prec}"] = {"s": dt, "status": si["status"], "method": si["method"],
                                   "bandwidth": si["bandwidth"], "resid_l2": si["resid_l2"],
                                   "outer_its": si["outer_its"], "inner_its": si["inner_its"]}
            _log(f"spin chain auto {prec}: {dt:.3f} s, method {si['method']}, resid {si['resid_l2']:.2e}, "
                 f"its {si['outer_its']}/{si['inner_its']}")
    finally:
        Ls.free()
    # the chain's steady state is I / d, inverse power's default start, so the
    # solve above has nothing to do; from a random trace-1 Hermitian start it
    # iterates (five spins with iLUT: from such a start zero-fill ILU stalls,
    # and at six spins and more every ILU variant does)
    s5 = qs.spin_chain(5)
    L5 = ssl.build_liouvillian(s5.H, s5.c_ops)
    try:
        for prec in ("mixed", "fp64"):
            t0 = time.perf_counter()
            _, si = ssl.solve(L5, "invpow_bicgstab", tol=1e-10, prec=prec, raise_on_error=False, random_start=True,
                              seed=1, ilu="ilut", no_fallback=True)
            dt = time.perf_counter() - t0
            out[f"spin5_random_start_ilut_{prec}"] = {"s": dt, "status": si["status"], "resid_l2": si["resid_l2"],
                                                       "outer_its": si["outer_its"], "inner_its": si["inner_its"]}
            _log(f"spin chain 5 random start (iLUT) {prec}: {dt:.3f} s, resid {si['resid_l2']:.2e}, "
                 f"its {si['outer_its']}/{si['inner_its']}")
    finally:
        L5.free()
    return out


def _run_stream(ssl, systems, arrivals, prec):
    """Submit each request at its arrival time, poll until all are done;
    returns (wall seconds, latencies in ms, {index: (rho, info)})."""
    S = ssl.Server(hbm_budget_bytes=32 << 30, max_slots=1024)
    pending, lat, res = {}, [], {}
    nxt = 0
    try:
        t0 = time.perf_counter()
        while nxt < len(systems) or pending:
            now = time.perf_counter() - t0
            while nxt < len(systems) and arrivals[nxt] <= now:
                s = systems[nxt]
                pending[S.submit(s.H, s.c_ops, "trace_bicgstab", 1e-10, prec=prec)] = (nxt, time.perf_counter())
                nxt += 1
            for t in list(pending):
                r = S.poll(t)
                if r is not None:
                    i, ts = pending.pop(t)
                    lat.append(1e3 * (time.perf_counter() - ts))
                    res[i] = r
            time.sleep(0.0002)
        wall = time.perf_counter() - t0
    finally:
        S.close()
    return wall, np.asarray(lat), res


def serve_stream(ssl, qs, n_requests, reps=10):
    """Serving stream of Kerr requests (cutoff N ~ U{10..60}, (Delta, E) on
    a 21 x 20 grid, seed 1): burst capacity (all arrive at t = 0) in both
    precisions, then Poisson arrivals at 0.5, 1 and 2 times the mixed
    capacity; p50/p99 of submit-to-result latency; a sample checked against
    the dense oracle.  Each measurement is repeated `reps` times on a fresh
    server and its median reported, with the spread of the throughput."""
    from oracle.steady import steady_state_dense
    stream = qs.serving_stream(n_requests, rate=0.0, seed=1)
    systems = [qs.kerr(N, delta=dl, E=E) for (_, N, dl, E) in stream]
    out = {"workload": f"{n_requests} Kerr requests, N ~ U{{10..60}}, (Delta, E) on a 21 x 20 grid, seed 1",
           "method": "trace_bicgstab", "tol": 1e-10, "repetitions": reps}

    def repeated(arrivals, prec):
        runs = []
        for _ in range(reps):
            wall, lat, res = _run_stream(ssl, systems, arrivals, prec)
            runs.append((n_requests / wall, float(np.percentile(lat, 50)), float(np.percentile(lat, 99)), res))
        thr = [r[0] for r in runs]
        rec = {"solves_per_s": float(np.median(thr)), "solves_per_s_min_max": [float(min(thr)), float(max(thr))],
               "p50_ms": float(np.median([r[1] for r in runs])), "p99_ms": float(np.median([r[2] for r in runs])),
               "all_converged": all(v[1]["status"] == 0 and v[1]["resid_l2"] <= 1e-10
                                    for r in runs for v in r[3].values())}
        return rec, runs[-1][3]

    for prec in ("mixed", "fp64"):
        rec, res = repeated([0.0] * n_requests, prec)
        sample = [i for i in range(n_requests) if systems[i].dim <= 30][:8]
        err = max(float(np.max(np.abs(res[i][0] - steady_state_dense(systems[i].H, systems[i].c_ops))))
                  for i in sample) if sample else None
        rec.update({"max_abs_err_vs_oracle_sample": err, "sample_size": len(sample)})
        out[f"burst_{prec}"] = rec
        _log(f"serving burst {prec}: median {rec['solves_per_s']:.1f} solves/s over {reps} "
             f"(min {rec['solves_per_s_min_max'][0]:.0f}, max {rec['solves_per_s_min_max'][1]:.0f}), "
             f"p50 {rec['p50_ms']:.1f} ms, p99 {rec['p99_ms']:.1f} ms, err {err}")
    cap = out["burst_mixed"]["solves_per_s"]
    for f in (0.5, 1.0, 2.0):
        rate = f * cap
        pstream = qs.serving_stream(n_requests, rate=rate, seed=1)
        rec, _ = repeated([a for (a, _, _, _) in pstream], "mixed")
        rec["rate_per_s"] = rate
        out[f"poisson_mixed_{f}x"] = rec
        _log(f"serving poisson {f}x ({rate:.0f}/s): median {rec['solves_per_s']:.0f} solves/s, "
             f"p50 {rec['p50_ms']:.1f} ms, p99 {rec['p99_ms']:.1f} ms")
    out["mixed_vs_fp64_capacity"] = cap / out["burst_fp64"]["solves_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256, help="systems of the batched Jaynes-Cummings step")
    ap.add_argument("--batch-reps", type=int, default=1, help="timed repetitions of the batched step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="kernels,jc_batch,spin_chain,serving",
                    help="secondary measurements to run (comma list; empty for none)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-reps", type=int, default=10, help="repetitions of each serving measurement (median)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MB (the known-size reference for "
                         "the HBM counter runs)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write profiles/traffic.json from the rocpd databases of a FETCH_SIZE and a WRITE_SIZE "
                         "counter run (both taken with --copy-calibration-mb 256 --counter-apps N) and exit; no "
                         "GPU is used")
    ap.add_argument("--counter-apps", type=int, default=0,
                    help="run only N applications of the dominant kernel (for the counter runs) and exit; with "
                         "--traffic-from, the N those runs used")
    args = ap.parse_args()
    if args.traffic_from:
        if args.counter_apps <= 0:
            raise SystemExit("--traffic-from needs --counter-apps N (the applications the counter runs made)")
        write_traffic(*args.traffic_from, apps=args.counter_apps)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported: this build measures one "
              "MI355X (a single solve fits one GPU; independent requests would be routed to separate GPUs)",
              file=sys.stderr)
        return 2

    import torch

    import paper_1504_06768_amd as ssl
    import qsystems as qs

    torch.cuda.set_device(0)
    if args.copy_calibration_mb > 0:
        nb = args.copy_calibration_mb << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        _log(f"calibration copy: {nb} bytes read and written")
        del src, dst

    if args.counter_apps > 0:
        counter_run(ssl, qs, torch, args.counter_apps)
        return 0

    ch, Hd, Cd, res = headline(ssl, qs, torch, args)
    f64, mx = res["fp64"], res["mixed"]
    errors = {}
    line = {
        "metric": "steady-state solves/sec + SpMV HBM GB/s at ||L.rho||<=1e-10, mixed vs FP64",
        "value": f64["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "median_ms_per_step": f64["median_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "kerr_chain_3x10: three coupled driven Kerr cavities, N = 10 each, J = 0.3 "
                               "(d = 1000, Liouvillian n = 1e6, 20.7 M non-zeros); one full solve per step "
                               "(assembly, shift, RCM and the colour-class order, ILU(0), inverse power with "
                               "BiCGSTAB (fp64) or GMRES(40) (mixed) inner solves, finish)",
                   "method": {p: HEADLINE[p][0] for p in HEADLINE}, "gmres_m": HEADLINE["mixed"][1], "tol": 1e-10,
                   "ordering": HEADLINE_ORDERING, "ilu": "ilu0"},
        "worst_resid_l2": f64["worst_resid_l2"],
        "fp64": {k: v for k, v in f64.items() if k != "rho"},
        "mixed": {k: v for k, v in mx.items() if k != "rho"},
        "mixed_vs_fp64": mx["solves_per_s"] / f64["solves_per_s"],
        "rcm_order": res["rcm_order"],
    }
    legs = [x for x in args.legs.split(",") if x]
    try:
        kern, roof = dominant_kernel(ssl, ch, Hd, Cd, res)
        line["roofline"] = roof
        if "kernels" in legs:
            line["kernels"] = kern
    except Exception as e:  # recorded, never silent
        errors["roofline"] = f"{type(e).__name__}: {e}"
        traceback.print_exc()
    if not args.no_cpu_baseline:
        try:
            cb, errs = cpu_baseline(ch, res)
            line["cpu_baseline"] = cb
            line["max_abs_err_vs_oracle"] = errs["fp64"]
            line["mixed"]["max_abs_err_vs_oracle"] = errs["mixed"]
        except Exception as e:
            errors["cpu_baseline"] = f"{type(e).__name__}: {e}"
            traceback.print_exc()
    for name, fn in (("jc_batch", lambda: jc_batch(ssl, qs, torch, args)),
                     ("spin_chain", lambda: spin_chain_leg(ssl, qs)),
                     ("serving", lambda: serve_stream(ssl, qs, args.serve_requests, max(1, args.serve_reps)))):
        if name not in legs or (name == "serving" and args.serve_requests <= 0):
            continue
        try:
            line[name] = fn()
        except Exception as e:
            errors[name] = f"{type(e).__name__}: {e}"
            traceback.print_exc()
    line["errors"] = errors
    print(json.dumps(line), flush=True)
    return 3 if errors else 0


if __name__ == "__main__":
    sys.exit(main())
