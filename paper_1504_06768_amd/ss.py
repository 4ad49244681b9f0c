"""ctypes binding of libss.so (include/ss.h), same entry-point names.

Inputs are scipy sparse matrices, numpy arrays or torch tensors; host
inputs are converted to CSR with int64 row pointers, int32 column indices and
interleaved complex128 values and handed to the library, which validates and
copies them to the device.  Torch tensors on the GPU are passed as device
pointers.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libss.so")

SS_OK, SS_PENDING = 0, 1
SS_E_INVALID_ARG, SS_E_OOM, SS_E_NOT_CONVERGED, SS_E_BREAKDOWN = -1, -2, -3, -4
SS_E_ZERO_PIVOT, SS_E_HIP, SS_E_STATE, SS_E_TIMEOUT = -5, -6, -7, -8
SS_TRACE_BICGSTAB, SS_TRACE_GMRES, SS_INVPOW_BICGSTAB, SS_INVPOW_GMRES, SS_AUTO = 0, 1, 2, 3, 4
SS_FP64, SS_MIXED = 0, 1
SS_ILU0, SS_ILUT = 0, 1
SS_ORDER_RCM, SS_ORDER_NATURAL, SS_ORDER_COLOUR = 0, 1, 2
SS_FLAG_HERMITIZE, SS_FLAG_NO_FALLBACK, SS_FLAG_DEVICE_WIDE, SS_FLAG_WORKGROUP = 1, 2, 4, 8
SS_FLAG_SYNCFREE, SS_FLAG_TRSV_BLOCK, SS_FLAG_TRSV_LEVELS, SS_FLAG_COND_EST = 16, 32, 64, 128
SS_FLAG_MATRIX_FREE, SS_FLAG_FORCE_BREAKDOWN, SS_FLAG_TRSV_GROUPS, SS_FLAG_RANDOM_START = 256, 512, 1024, 2048
SS_FLAG_TRSV_CLASSES = 4096
SS_MAT_L, SS_MAT_A, SS_MAT_A_PERM, SS_MAT_LU, SS_MAT_SYM = 0, 1, 2, 3, 4
SS_OP_SPMV_L, SS_OP_SPMV_APERM, SS_OP_PRECOND, SS_OP_LSOLVE, SS_OP_USOLVE = 0, 1, 2, 3, 4
SS_OP_PRECOND_SYNCFREE, SS_OP_PRECOND_BLOCK, SS_OP_PRECOND_LEVELS, SS_OP_APPLY_L = 5, 6, 7, 8
SS_OP_PRECOND_GROUPS = 9
SS_OP_PRECOND_CLASSES = 10

METHODS = {"trace_bicgstab": 0, "trace_gmres": 1, "invpow_bicgstab": 2, "invpow_gmres": 3, "auto": 4}
PRECS = {"fp64": 0, "mixed": 1}


class SolverError(RuntimeError):
    def __init__(self, code: int, msg: str, info: Optional[dict] = None):
        super().__init__(f"[{code}] {msg}")
        self.code = code
        self.info = info


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p), ("data", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("ilu", ctypes.c_int32), ("ordering", ctypes.c_int32),
                ("gmres_m", ctypes.c_int32), ("maxiter", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("trace_row", ctypes.c_int32),
                ("drop_tol", ctypes.c_double), ("fill", ctypes.c_double), ("sigma", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("weight", ctypes.c_double), ("seed", ctypes.c_int64),
                ("ilu_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_its", ctypes.c_int32), ("inner_its", ctypes.c_int32),
                ("breakdowns", ctypes.c_int32), ("pivots_guarded", ctypes.c_int32), ("fell_back", ctypes.c_int32),
                ("bandwidth", ctypes.c_int32), ("path", ctypes.c_int32),
                ("profile", ctypes.c_int64), ("nnz_matrix", ctypes.c_int64), ("nnz_factors", ctypes.c_int64),
                ("resid_l2", ctypes.c_double), ("herm_err", ctypes.c_double), ("trace_err", ctypes.c_double),
                ("cond_est", ctypes.c_double), ("fill_factor", ctypes.c_double), ("weight", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("t_kernel_ms", ctypes.c_double), ("bytes_alg", ctypes.c_double),
                ("method", ctypes.c_int32), ("colours", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_INFO_KEYS = [name for name, _ in _Info._fields_]


def _info_dicts(infos, k: int) -> list:
    """as_dict of the first k entries of an _Info array, read in one pass."""
    if k == 0:
        return []
    rows = np.ctypeslib.as_array(infos)[:k].tolist()
    out = []
    for r in rows:
        out.append(dict(zip(_INFO_KEYS, r)))
    return out


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python paper_1504_06768_amd/build.py` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ss_options_default": (ctypes.c_int, [P]),
        "ss_build_liouvillian": (ctypes.c_int, [P, P, I32, I64, P]),
        "ss_build_liouvillian_batch": (ctypes.c_int, [ctypes.c_int32, P, P, P, P]),
        "ss_solve": (ctypes.c_int, [P, I32, D, P, P, P]),
        "ss_solve_batch": (ctypes.c_int, [P, I32, I32, D, P, P, P, P]),
        "ss_liouv_free": (None, [P]),
        "ss_liouv_shape": (ctypes.c_int, [P, P, P, P]),
        "ss_prepare": (ctypes.c_int, [P, I32, P]),
        "ss_export_csr": (ctypes.c_int, [P, I32, P, P, P, P]),
        "ss_export_perm": (ctypes.c_int, [P, P]),
        "ss_apply": (ctypes.c_int, [P, I32, I32, P, P]),
        "ss_apply_noalloc": (ctypes.c_int, [P, I32, I32, P, P]),
        "ss_bandwidth_profile": (ctypes.c_int, [P, I32, P, P]),
        "ss_time_operator": (ctypes.c_int, [P, I32, I32, I32, P]),
        "ss_server_create": (ctypes.c_int, [ctypes.c_size_t, I32, P]),
        "ss_submit": (ctypes.c_int, [P, P, P, I32, I64, I32, D, P, P]),
        "ss_poll": (ctypes.c_int, [P, ctypes.c_uint64, P, P]),
        "ss_server_drain": (ctypes.c_int, [P]),
        "ss_server_stats": (ctypes.c_int, [P, P]),
        "ss_server_destroy": (None, [P]),
        "ss_last_error": (ctypes.c_char_p, []),
        "ss_set_stream": (ctypes.c_int, [P]),
        "ss_set_allocator": (ctypes.c_int, [P, P, P]),
        "ss_trim_cache": (ctypes.c_int, []),
        "ss_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("ss_options_default", "ss_build_liouvillian", "ss_build_liouvillian_batch", "ss_solve",
            "ss_solve_batch", "ss_liouv_free", "ss_liouv_shape",
            "ss_prepare", "ss_export_csr", "ss_export_perm", "ss_apply", "ss_apply_noalloc", "ss_bandwidth_profile",
            "ss_time_operator",
            "ss_server_create", "ss_submit", "ss_poll", "ss_server_drain", "ss_server_stats", "ss_server_destroy",
            "ss_last_error", "ss_set_stream", "ss_set_allocator", "ss_trim_cache", "ss_version")


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None


def set_allocator(alloc=None, free=None):
    """ss_set_allocator: alloc(nbytes) -> device pointer (int), free(ptr);
    both None restores hipMalloc / hipFree.  The callables are kept alive
    here; they may be called from the library's set-up threads."""
    global _allocator_refs
    if (alloc is None) != (free is None):
        raise ValueError("give both callbacks or neither")
    if alloc is None:
        _check(_lib.ss_set_allocator(None, None, None), "ss_set_allocator")
        _allocator_refs = None
        return
    def _a(n, ctx):
        try:
            return int(alloc(int(n))) or None
        except Exception:  # reported to the library as an allocation failure
            return None

    def _f(p, ctx):
        try:
            free(int(p))
        except Exception:
            pass

    a = _ALLOC_T(_a)
    f = _FREE_T(_f)
    _check(_lib.ss_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None),
           "ss_set_allocator")
    _allocator_refs = (a, f)


def trim_cache():
    """ss_trim_cache: release the device blocks the library keeps for reuse."""
    _check(_lib.ss_trim_cache(), "ss_trim_cache")


def library_path() -> str:
    return _LIB_PATH


def version() -> str:
    return _lib.ss_version().decode()


def _err() -> str:
    m = _lib.ss_last_error()
    return m.decode() if m else ""


def _check(rc: int, what: str, info=None):
    if rc != SS_OK:
        raise SolverError(rc, f"{what}: {_err()}", info)


# ------------------------------------------------------------ marshalling
class _HostCsr:
    """Keeps the converted arrays alive while the library reads them."""

    def __init__(self, m):
        if _is_torch(m):
            raise TypeError("pass device CSR matrices as a tuple of torch tensors (indptr, indices, data, n)")
        if isinstance(m, tuple):
            # (indptr int64, indices int32, data complex128, n) as torch device
            # tensors or numpy host arrays, passed through unchanged
            indptr, indices, data, n = m
            self.keep = (indptr, indices, data)
            nnz = indices.numel() if _is_torch(indices) else indices.size
            self.s = _Csr(int(n), int(nnz), _ptr(indptr), _ptr(indices), _ptr(data))
            return
        A = sp.csr_matrix(m, dtype=np.complex128)
        A.sum_duplicates()
        A.sort_indices()
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.data = np.ascontiguousarray(A.data, dtype=np.complex128)
        self.s = _Csr(A.shape[0], A.nnz, self.indptr.ctypes.data, self.indices.ctypes.data,
                      self.data.ctypes.data)
        if A.shape[0] != A.shape[1]:
            raise ValueError("operators must be square")


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x) -> int:
    if _is_torch(x):
        return int(x.data_ptr())
    return int(x.ctypes.data)


def options(prec="fp64", ilu="ilu0", ordering="rcm", gmres_m=20, maxiter=1000, max_outer=20,
            drop_tol=1e-4, fill=10.0, sigma=1e-15, inner_tol=0.0, weight=0.0, hermitize=False,
            no_fallback=False, trace_row=-1, path="auto", trsv="auto", cond_est=False,
            matrix_free=False, force_breakdown=False, random_start=False, seed=0, ilu_sweeps=0) -> _Options:
    o = _Options()
    _lib.ss_options_default(ctypes.byref(o))
    o.prec = PRECS[prec] if isinstance(prec, str) else int(prec)
    o.ilu = {"ilu0": 0, "ilut": 1}[ilu] if isinstance(ilu, str) else int(ilu)
    o.ordering = {"rcm": 0, "natural": 1, "colour": 2}[ordering] if isinstance(ordering, str) else int(ordering)
    o.gmres_m, o.maxiter, o.max_outer = gmres_m, maxiter, max_outer
    o.drop_tol, o.fill, o.sigma, o.inner_tol, o.weight = drop_tol, fill, sigma, inner_tol, weight
    o.trace_row = int(trace_row)
    o.flags = (SS_FLAG_HERMITIZE if hermitize else 0) | (SS_FLAG_NO_FALLBACK if no_fallback else 0)
    o.flags |= {"auto": 0, "device": SS_FLAG_DEVICE_WIDE, "workgroup": SS_FLAG_WORKGROUP}[path]
    o.flags |= {"auto": 0, "syncfree": SS_FLAG_SYNCFREE, "block": SS_FLAG_TRSV_BLOCK,
                "levels": SS_FLAG_TRSV_LEVELS, "groups": SS_FLAG_TRSV_GROUPS,
                "classes": SS_FLAG_TRSV_CLASSES}[trsv]
    if cond_est:
        o.flags |= SS_FLAG_COND_EST
    if matrix_free:
        o.flags |= SS_FLAG_MATRIX_FREE
    if force_breakdown:
        o.flags |= SS_FLAG_FORCE_BREAKDOWN
    if random_start:
        o.flags |= SS_FLAG_RANDOM_START
    o.seed = int(seed)
    o.ilu_sweeps = int(ilu_sweeps)
    return o


def _method(m) -> int:
    return METHODS[m] if isinstance(m, str) else int(m)


# ----------------------------------------------------------- entry points
class Liouvillian:
    """Owning wrapper of an ss_liouv handle."""

    def __init__(self, handle: int, N: int):
        self.handle = ctypes.c_void_p(handle)
        self.N = N
        self.n = N * N

    def shape(self):
        N, n, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.ss_liouv_shape(self.handle, ctypes.byref(N), ctypes.byref(n), ctypes.byref(nnz)),
               "ss_liouv_shape")
        return N.value, n.value, nnz.value

    @property
    def nnz(self) -> int:
        return self.shape()[2]

    def free(self):
        if self.handle:
            _lib.ss_liouv_free(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_liouvillian(H, c_ops: Iterable = ()) -> Liouvillian:
    """ss_build_liouvillian: assemble L on the device from H and c_ops."""
    Hc = _HostCsr(H)
    cs = [_HostCsr(c) for c in c_ops]
    arr = (_Csr * max(len(cs), 1))(*[c.s for c in cs])
    N = Hc.s.n
    h = ctypes.c_void_p()
    _check(_lib.ss_build_liouvillian(ctypes.byref(Hc.s), arr if cs else None, len(cs), N, ctypes.byref(h)),
           "ss_build_liouvillian")
    return Liouvillian(h.value, N)


def build_liouvillian_batch(systems) -> list:
    """ss_build_liouvillian_batch: assemble many Liouvillians together.
    `systems` is a sequence of (H, c_ops) pairs in any form build_liouvillian
    takes; returns one Liouvillian per system."""
    systems = list(systems)
    k = len(systems)
    if k == 0:
        return []
    Hs = (_Csr * k)()
    arrs = (ctypes.c_void_p * k)()
    ncs = (ctypes.c_int32 * k)()
    # an operator object (or list of collapse operators) that appears in
    # several systems is converted once; `systems` keeps every object alive
    # for the call, so the identities stay unique
    conv, lists = {}, {}

    def host(m):
        c = conv.get(id(m))
        if c is None:
            c = conv[id(m)] = _HostCsr(m)
        return c

    for i, (H, c_ops) in enumerate(systems):
        ent = lists.get(id(c_ops))
        if ent is None:
            cs = [host(c) for c in c_ops]
            arr = (_Csr * max(len(cs), 1))(*[c.s for c in cs])
            ent = lists[id(c_ops)] = (cs, arr, ctypes.cast(arr, ctypes.c_void_p).value if cs else None, len(cs))
        Hs[i] = host(H).s
        arrs[i] = ent[2]
        ncs[i] = ent[3]
    hs = (ctypes.c_void_p * k)()
    _check(_lib.ss_build_liouvillian_batch(k, Hs, arrs, ncs, hs), "ss_build_liouvillian_batch")
    return [Liouvillian(hs[i], int(Hs[i].n)) for i in range(k)]


def solve(L: Liouvillian, method="trace_bicgstab", tol: float = 1e-10, out=None, raise_on_error=True,
          **opts):
    """ss_solve: returns (rho as an N x N complex128 array, info dict).  `out`
    may be a torch complex128 tensor on the GPU (N*N elements) to receive rho
    in column-major order; rho is then returned as that tensor."""
    o = options(**opts)
    info = _Info()
    if out is not None:
        ptr = _ptr(out)
        rho = out
    else:
        buf = np.empty(L.n, dtype=np.complex128)
        ptr = buf.ctypes.data
        rho = buf
    rc = _lib.ss_solve(L.handle, _method(method), float(tol), ctypes.byref(o), ctypes.c_void_p(ptr),
                       ctypes.byref(info))
    d = info.as_dict()
    if rc != SS_OK and raise_on_error:
        raise SolverError(rc, f"ss_solve: {_err()}", d)
    if out is None:
        rho = rho.reshape(L.N, L.N, order="F")
    return rho, d


def solve_batch(Ls, method="trace_bicgstab", tol: float = 1e-10, outs=None, raise_on_error=True, **opts):
    """ss_solve_batch: independent systems solved together, one workgroup
    each.  `outs` may be a list of torch complex128 device tensors (N_i^2
    elements each) to receive the rho's; returns (list of rho, list of info
    dicts)."""
    Ls = list(Ls)
    k = len(Ls)
    o = options(**opts)
    infos = (_Info * max(k, 1))()
    status = (ctypes.c_int32 * max(k, 1))()
    handles = (ctypes.c_void_p * max(k, 1))(*[L.handle for L in Ls])
    if outs is not None:
        rhos = list(outs)
        ptrs = [_ptr(t) for t in rhos]
    else:
        bufs = [np.empty(L.n, dtype=np.complex128) for L in Ls]
        rhos = bufs
        ptrs = [b.ctypes.data for b in bufs]
    parr = (ctypes.c_void_p * max(k, 1))(*ptrs)
    rc = _lib.ss_solve_batch(handles, k, _method(method), float(tol), ctypes.byref(o), parr, infos, status)
    ds = _info_dicts(infos, k)
    if rc != SS_OK and raise_on_error:
        raise SolverError(rc, f"ss_solve_batch: {_err()}", ds)
    if outs is None:
        rhos = [r.reshape(L.N, L.N, order="F") for r, L in zip(rhos, Ls)]
    return rhos, ds


def prepare(L: Liouvillian, method="trace_bicgstab", **opts):
    """ss_prepare: the set-up half of ss_solve (transform, ordering, ILU)."""
    o = options(**opts)
    _check(_lib.ss_prepare(L.handle, _method(method), ctypes.byref(o)), "ss_prepare")


def export_csr(L: Liouvillian, which=SS_MAT_L) -> sp.csr_matrix:
    nnz = ctypes.c_int64()
    _check(_lib.ss_export_csr(L.handle, which, ctypes.byref(nnz), None, None, None), "ss_export_csr")
    indptr = np.empty(L.n + 1, dtype=np.int64)
    indices = np.empty(nnz.value, dtype=np.int32)
    data = np.empty(nnz.value, dtype=np.complex128)
    _check(_lib.ss_export_csr(L.handle, which, None, indptr.ctypes.data, indices.ctypes.data,
                              data.ctypes.data), "ss_export_csr")
    return sp.csr_matrix((data, indices, indptr), shape=(L.n, L.n))


def export_perm(L: Liouvillian) -> np.ndarray:
    perm = np.empty(L.n, dtype=np.int32)
    _check(_lib.ss_export_perm(L.handle, perm.ctypes.data), "ss_export_perm")
    return perm


def apply(L: Liouvillian, op: int, x, prec="fp64"):
    """ss_apply: y = op(x) for a vector of n complex values."""
    xh = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty(L.n, dtype=np.complex128)
    _check(_lib.ss_apply(L.handle, op, PRECS[prec] if isinstance(prec, str) else prec, xh.ctypes.data,
                         y.ctypes.data), "ss_apply")
    return y


def apply_noalloc(L: Liouvillian, op: int, x, y, prec="fp64"):
    """ss_apply_noalloc: y = op(x) with x, y device buffers of n complex128
    values (torch tensors on the GPU); nothing is allocated."""
    _check(_lib.ss_apply_noalloc(L.handle, op, PRECS[prec] if isinstance(prec, str) else prec, _ptr(x), _ptr(y)),
           "ss_apply_noalloc")
    return y


def time_operator(L: Liouvillian, op: int, prec="fp64", reps: int = 50) -> float:
    """ss_time_operator: mean milliseconds per application (HIP events)."""
    ms = ctypes.c_double()
    _check(_lib.ss_time_operator(L.handle, op, PRECS[prec] if isinstance(prec, str) else prec, int(reps),
                                 ctypes.byref(ms)), "ss_time_operator")
    return ms.value


def bandwidth_profile(L: Liouvillian, which=SS_MAT_A_PERM):
    B, P = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.ss_bandwidth_profile(L.handle, which, ctypes.byref(B), ctypes.byref(P)), "ss_bandwidth_profile")
    return B.value, P.value


class _ServerStats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64),
                ("peak_resident_bytes", ctypes.c_uint64), ("resident", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("groups", ctypes.c_uint64), ("largest_group", ctypes.c_uint64),
                ("workers", ctypes.c_int32), ("max_group", ctypes.c_int32)]


class Server:
    """ss_server_*: continuous-batching request server."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, max_slots: int = 256):
        h = ctypes.c_void_p()
        _check(_lib.ss_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)), "ss_server_create")
        self.handle = h
        self._N = {}

    def submit(self, H, c_ops=(), method="trace_bicgstab", tol=1e-10, **opts) -> int:
        Hc = _HostCsr(H)
        cs = [_HostCsr(c) for c in c_ops]
        arr = (_Csr * max(len(cs), 1))(*[c.s for c in cs])
        o = options(**opts)
        t = ctypes.c_uint64()
        _check(_lib.ss_submit(self.handle, ctypes.byref(Hc.s), arr if cs else None, len(cs), Hc.s.n,
                              _method(method), float(tol), ctypes.byref(o), ctypes.byref(t)), "ss_submit")
        self._N[t.value] = Hc.s.n
        return t.value

    def poll(self, ticket: int):
        """Returns None while pending, else (rho, info); raises on failure."""
        N = self._N[ticket]
        rho = np.empty(N * N, dtype=np.complex128)
        info = _Info()
        rc = _lib.ss_poll(self.handle, ctypes.c_uint64(ticket), rho.ctypes.data, ctypes.byref(info))
        if rc == SS_PENDING:
            return None
        del self._N[ticket]
        d = info.as_dict()
        if rc != SS_OK:
            raise SolverError(rc, f"ss_poll: {_err()}", d)
        return rho.reshape(N, N, order="F"), d

    def drain(self):
        _check(_lib.ss_server_drain(self.handle), "ss_server_drain")

    def stats(self) -> dict:
        """ss_server_stats: budget, resident and peak footprint, counts."""
        st = _ServerStats()
        _check(_lib.ss_server_stats(self.handle, ctypes.byref(st)), "ss_server_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if self.handle:
            _lib.ss_server_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
