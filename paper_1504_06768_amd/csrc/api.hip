// extern "C" entry points of include/ss.h: argument checks, error
// translation and handle lifetime.  The work itself is in the other files.
#include <mutex>
#include <type_traits>

#include "assemble.hpp"
#include "csr_tools.hpp"
#include "handle.hpp"
#include "rcm.hpp"

namespace ss {
void set_thread_stream(hipStream_t s);
}

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

}  // namespace

namespace ss {
// The calling thread's message for ss_last_error (the server reports a
// request's failure, recorded on its scheduler thread, this way at ss_poll).
void set_last_error(const std::string &msg) { g_err = msg; }
}  // namespace ss

namespace {

template <typename F>
int guarded(F &&f) {
    // an error left by an earlier HIP call of the caller's thread is not this
    // call's: cleared, so that the launch checks inside report only their own
    (void)hipGetLastError();
    try {
        return f();
    } catch (const ss::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(SS_E_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SS_E_HIP, e.what());
    }
}

ss_options resolve(const ss_options *opt) {
    ss_options o;
    ss_options_default(&o);
    if (opt) o = *opt;
    if (o.gmres_m <= 0) o.gmres_m = 20;
    if (o.maxiter <= 0) o.maxiter = 1000;
    if (o.max_outer <= 0) o.max_outer = 20;
    if (o.fill <= 0) o.fill = 10.0;
    if (o.drop_tol < 0) o.drop_tol = 1e-4;
    return o;
}

}  // namespace

extern "C" {

const char *ss_last_error(void) { return g_err.c_str(); }

const char *ss_version(void) { return "ssolve-0.1 (gfx950)"; }

int ss_options_default(ss_options *opt) {
    if (!opt) return fail(SS_E_INVALID_ARG, "opt is NULL");
    std::memset(opt, 0, sizeof(*opt));
    opt->prec = SS_FP64;
    opt->ilu = SS_ILU0;
    opt->ordering = SS_ORDER_RCM;
    opt->gmres_m = 20;
    opt->maxiter = 1000;
    opt->max_outer = 20;
    opt->flags = 0;
    opt->trace_row = -1;
    opt->drop_tol = 1e-4;
    opt->fill = 10.0;
    opt->sigma = 1e-15;
    opt->inner_tol = 0.0;
    opt->weight = 0.0;
    return SS_OK;
}

int ss_set_allocator(ss_alloc_fn alloc, ss_free_fn free_fn, void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(SS_E_INVALID_ARG, "give both callbacks or neither");
    return guarded([&]() -> int {
        ss::set_allocator(alloc, free_fn, ctx);
        return SS_OK;
    });
}

int ss_trim_cache(void) {
    return guarded([&]() -> int {
        ss::trim_device_cache();
        return SS_OK;
    });
}

int ss_set_stream(void *hip_stream) {
    ss::set_thread_stream(reinterpret_cast<hipStream_t>(hip_stream));
    return SS_OK;
}

int ss_build_liouvillian(const ss_csr_z *H, const ss_csr_z *c_ops, int32_t n_cops, int64_t N, ss_liouv *out) {
    return guarded([&]() -> int {
        SS_REQUIRE(out != nullptr, SS_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        std::unique_ptr<ss_liouv_s> h(new ss_liouv_s());
        h->own_stream = ss::pooled_stream();
        h->N = N;
        h->d = (int)N;
        h->n = (int)(N * N);
        ss::assemble_liouvillian(H, c_ops, n_cops, N, ss::stream_of(h.get()), h->L, h->lin);
        *out = h.release();
        return SS_OK;
    });
}

int ss_build_liouvillian_batch(int32_t count, const ss_csr_z *H, const ss_csr_z *const *c_ops,
                               const int32_t *n_cops, ss_liouv *out) {
    std::vector<std::unique_ptr<ss_liouv_s>> hs;
    const int rc = guarded([&]() -> int {
        SS_REQUIRE(count >= 0, SS_E_INVALID_ARG, "negative count");
        if (count == 0) return SS_OK;
        SS_REQUIRE(out != nullptr && H != nullptr && n_cops != nullptr, SS_E_INVALID_ARG, "null argument");
        for (int k = 0; k < count; ++k) out[k] = nullptr;
        std::vector<int> batched, single;
        for (int k = 0; k < count; ++k) {
            bool dev = ss::batch_assembly_fits(H[k].n) && n_cops[k] >= 0 && n_cops[k] <= ss::MAX_COPS &&
                       (n_cops[k] == 0 || (c_ops != nullptr && c_ops[k] != nullptr));
            auto on_device = [](const ss_csr_z &m) {
                return m.indptr && ss::is_device_ptr(m.indptr) &&
                       (m.nnz == 0 || (m.indices && m.data && ss::is_device_ptr(m.indices) && ss::is_device_ptr(m.data)));
            };
            if (dev) dev = on_device(H[k]);
            for (int c = 0; dev && c < n_cops[k]; ++c) dev = on_device(c_ops[k][c]);
            (dev ? batched : single).push_back(k);
            std::unique_ptr<ss_liouv_s> h(new ss_liouv_s());
            h->own_stream = ss::pooled_stream();
            h->N = H[k].n;
            h->d = (int)H[k].n;
            h->n = (int)(H[k].n * H[k].n);
            hs.push_back(std::move(h));
        }
        if (!batched.empty()) {
            std::vector<ss_csr_z> bH;
            std::vector<const ss_csr_z *> bC;
            std::vector<int> bn;
            std::vector<ss::AsmTarget> tg;
            for (int k : batched) {
                bH.push_back(H[k]);
                bC.push_back(n_cops[k] ? c_ops[k] : nullptr);
                bn.push_back(n_cops[k]);
                ss_liouv h = hs[(size_t)k].get();
                tg.push_back(ss::AsmTarget{&h->L, &h->lin, ss::stream_of(h)});
            }
            hipStream_t s = ss::stream_of(hs[(size_t)batched[0]].get());
            ss::assemble_batch((int)batched.size(), bH.data(), bC.data(), bn.data(), tg.data(), s);
        }
        for (int k : single) {
            ss_liouv h = hs[(size_t)k].get();
            SS_REQUIRE(n_cops[k] == 0 || c_ops != nullptr, SS_E_INVALID_ARG, "c_ops is NULL");
            ss::assemble_liouvillian(&H[k], n_cops[k] ? c_ops[k] : nullptr, n_cops[k], H[k].n, ss::stream_of(h), h->L,
                                     h->lin);
        }
        for (int k = 0; k < count; ++k) out[k] = hs[(size_t)k].release();
        return SS_OK;
    });
    if (rc != SS_OK) {
        for (auto &h : hs) {
            if (h && h->own_stream) ss::set_current_stream(h->own_stream);
            h.reset();
        }
        if (out)
            for (int k = 0; k < count; ++k) out[k] = nullptr;
    }
    return rc;
}

void ss_liouv_free(ss_liouv L) {
    if (!L) return;
    // the stream belongs to the pool: its work is left to finish, and every
    // device block of the handle is released against one event on it
    if (L->own_stream) ss::set_current_stream(L->own_stream);
    ss::FreeScope scope(ss::stream_peek(L));
    delete L;
}

int ss_liouv_shape(ss_liouv L, int64_t *N, int64_t *n, int64_t *nnz) {
    if (!L) return fail(SS_E_INVALID_ARG, "null handle");
    if (N) *N = L->N;
    if (n) *n = L->n;
    if (nnz) *nnz = L->L.nnz;
    return SS_OK;
}

int ss_prepare(ss_liouv L, int32_t method, const ss_options *opt) {
    return guarded([&]() -> int {
        SS_REQUIRE(L != nullptr, SS_E_INVALID_ARG, "null handle");
        ss::prepare(L, method, resolve(opt));
        return SS_OK;
    });
}

int ss_solve(ss_liouv L, int32_t method, double tol, const ss_options *opt, double *rho_out, ss_info *info) {
    if (info) std::memset(info, 0, sizeof(*info));
    const int rc = guarded([&]() -> int {
        SS_REQUIRE(L != nullptr, SS_E_INVALID_ARG, "null handle");
        SS_REQUIRE(rho_out != nullptr, SS_E_INVALID_ARG, "rho_out is NULL");
        const int st = ss::solve(L, method, tol, resolve(opt), rho_out, info);
        if (st == SS_E_NOT_CONVERGED) g_err = "iteration limit reached before ||L rho|| <= tol";
        if (st == SS_E_BREAKDOWN) g_err = "BiCGSTAB breakdown (no fallback allowed)";
        return st;
    });
    if (info) info->status = rc;
    return rc;
}

int ss_solve_batch(ss_liouv *Ls, int32_t count, int32_t method, double tol, const ss_options *opt,
                   double **rho_out, ss_info *infos, int32_t *status) {
    if (infos && count > 0) std::memset(infos, 0, sizeof(ss_info) * (size_t)count);
    return guarded([&]() -> int {
        SS_REQUIRE(count >= 0, SS_E_INVALID_ARG, "negative count");
        if (count == 0) return SS_OK;
        SS_REQUIRE(Ls != nullptr, SS_E_INVALID_ARG, "null handle array");
        for (int i = 0; i < count; ++i) {
            SS_REQUIRE(Ls[i] != nullptr, SS_E_INVALID_ARG, "null handle in the batch");
            for (int j = 0; j < i; ++j) SS_REQUIRE(Ls[j] != Ls[i], SS_E_INVALID_ARG, "handle repeated in the batch");
        }
        const int st = ss::solve_batch(Ls, count, method, tol, resolve(opt), rho_out, infos, status);
        if (st != SS_OK) g_err = ss::batch_error().empty() ? "a system of the batch did not converge" : ss::batch_error();
        return st;
    });
}

static const ss::CsrBuf<double2> *pick(ss_liouv L, int which) {
    switch (which) {
        case SS_MAT_L: return &L->L;
        case SS_MAT_A: return L->prepared ? &L->A : nullptr;
        case SS_MAT_A_PERM: return L->prepared ? &L->Ap : nullptr;
        case SS_MAT_LU: return L->prepared ? &L->LU : nullptr;
        case SS_MAT_SYM: return L->prepared ? &L->S : nullptr;
        default: return nullptr;
    }
}

int ss_export_csr(ss_liouv L, int32_t which, int64_t *nnz, int64_t *indptr, int32_t *indices, double *data) {
    return guarded([&]() -> int {
        SS_REQUIRE(L != nullptr, SS_E_INVALID_ARG, "null handle");
        const ss::CsrBuf<double2> *m = pick(L, which);
        SS_REQUIRE(m != nullptr, which >= 0 && which <= 4 ? SS_E_STATE : SS_E_INVALID_ARG,
                   "matrix not available (unknown id, or ss_prepare not called)");
        if (nnz) *nnz = m->nnz;
        hipStream_t s = ss::stream_of(L);
        if (indptr) {
            std::vector<int> rp((size_t)m->n + 1);
            ss::d2h(rp.data(), m->rowptr.get(), rp.size(), s);
            for (size_t i = 0; i < rp.size(); ++i) indptr[i] = rp[i];
        }
        if (indices && m->nnz) ss::d2h(indices, m->col.get(), (size_t)m->nnz, s);
        if (data && m->nnz) ss::d2h(reinterpret_cast<double2 *>(data), m->val.get(), (size_t)m->nnz, s);
        return SS_OK;
    });
}

// out[q] = a[b[q]]
__global__ void k_compose(int n, const int *a, const int *b, int *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = a[b[q]];
}

int ss_export_perm(ss_liouv L, int32_t *perm) {
    return guarded([&]() -> int {
        SS_REQUIRE(L != nullptr && perm != nullptr, SS_E_INVALID_ARG, "null argument");
        SS_REQUIRE(L->prepared, SS_E_STATE, "ss_prepare not called");
        hipStream_t s = ss::stream_of(L);
        const int n = L->n;
        if (L->split && n > 0) {
            // the factors' order: RCM position cp[q] of factor row q
            ss::DevBuf<int> fp((size_t)n);
            k_compose<<<ss::div_up(n, 256), 256, 0, s>>>(n, L->perm.get(), L->cp.get(), fp.get());
            SS_HIP(hipGetLastError());
            ss::d2h(perm, fp.get(), (size_t)n, s);
        } else {
            ss::d2h(perm, L->perm.get(), (size_t)n, s);
        }
        return SS_OK;
    });
}

int ss_bandwidth_profile(ss_liouv L, int32_t which, int64_t *B, int64_t *P) {
    return guarded([&]() -> int {
        SS_REQUIRE(L != nullptr && B != nullptr && P != nullptr, SS_E_INVALID_ARG, "null argument");
        const ss::CsrBuf<double2> *m = pick(L, which);
        SS_REQUIRE(m != nullptr, SS_E_STATE, "matrix not available");
        ss::bandwidth_profile(m->n, m->rowptr.get(), m->col.get(), B, P, ss::stream_of(L));
        return SS_OK;
    });
}

static bool is_precond_op(int op) {
    return op == SS_OP_PRECOND || op == SS_OP_PRECOND_SYNCFREE || op == SS_OP_PRECOND_BLOCK ||
           op == SS_OP_PRECOND_LEVELS || op == SS_OP_PRECOND_GROUPS || op == SS_OP_PRECOND_CLASSES;
}

static int precond_mode(int op) {
    return op == SS_OP_PRECOND_BLOCK    ? ss::PRE_BLOCK
           : op == SS_OP_PRECOND_LEVELS ? ss::PRE_LEVELS
           : op == SS_OP_PRECOND_GROUPS   ? ss::PRE_GROUPS
           : op == SS_OP_PRECOND_CLASSES  ? ss::PRE_CLASSES
                                        : ss::PRE_AUTO;
}

int ss_apply(ss_liouv L, int32_t op, int32_t prec, const double *x, double *y) {
    return guarded([&]() -> int {
        SS_REQUIRE(L != nullptr && x != nullptr && y != nullptr, SS_E_INVALID_ARG, "null argument");
        SS_REQUIRE(prec == SS_FP64 || prec == SS_MIXED, SS_E_INVALID_ARG, "unknown precision");
        SS_REQUIRE(op >= 0 && op <= 10, SS_E_INVALID_ARG, "unknown operator");
        const bool pre = is_precond_op(op);
        const bool natural = (op == SS_OP_SPMV_L || op == SS_OP_APPLY_L);
        SS_REQUIRE(natural || L->prepared, SS_E_STATE, "ss_prepare not called");
        SS_REQUIRE(natural || prec == SS_FP64 || L->p_opt.prec == SS_MIXED, SS_E_STATE,
                   "complex64 operators exist only after a mixed-precision ss_prepare");
        hipStream_t s = ss::stream_of(L);
        const int n = L->n;
        ss::DevBuf<double2> xd((size_t)n), yd((size_t)n);
        SS_HIP(hipMemcpyAsync(xd.get(), x, sizeof(double2) * n,
                              ss::is_device_ptr(x) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        if (op == SS_OP_SPMV_L) {
            const ss::Csr<double2> A = L->L.view();
            ss::spmv<double2>(A, xd.get(), yd.get(), ss::spmv_group(A.n, A.nnz), s);
        } else if (op == SS_OP_APPLY_L) {
            ss::lindblad_apply(L->lin.view(), xd.get(), nullptr, 0, ss::mk(0.0, 0.0), nullptr, nullptr, yd.get(),
                               nullptr, s);
        } else if (prec == SS_FP64) {
            if (op == SS_OP_SPMV_APERM) {
                const ss::Csr<double2> A = L->Ap.view();
                ss::spmv<double2>(A, xd.get(), yd.get(), ss::spmv_group(A.n, A.nnz), s);
            } else {
                ss::Precond<double2> M;
                M.setup(&L->LU, L->lu_diag.get(), n, s);
                if (L->split) M.pin = L->cp.get();
                if (pre && op != SS_OP_PRECOND_SYNCFREE) M.use_levels(L->LU.view(), s, precond_mode(op), L->colours ? L->lorder.get() : nullptr);
                if (pre) M.apply(xd.get(), yd.get(), s);
                else if (op == SS_OP_LSOLVE) M.lower(xd.get(), yd.get(), s);
                else M.upper(xd.get(), yd.get(), s);
                SS_REQUIRE(!(M.read_status(s) & ss::STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "triangular solve timed out");
            }
        } else {
            ss::DevBuf<float2> xf((size_t)n), yf((size_t)n);
            ss::convert<float2, double2>(n, xd.get(), xf.get(), nullptr, s);
            if (op == SS_OP_SPMV_APERM) {
                const ss::Csr<float2> A = L->Ap32.view();
                ss::spmv<float2>(A, xf.get(), yf.get(), ss::spmv_group(A.n, A.nnz), s);
            } else {
                ss::Precond<float2> M;
                M.setup(&L->LU32, L->lu_diag.get(), n, s);
                if (L->split) M.pin = L->cp.get();
                if (pre && op != SS_OP_PRECOND_SYNCFREE) M.use_levels(L->LU.view(), s, precond_mode(op), L->colours ? L->lorder.get() : nullptr);
                if (pre) M.apply(xf.get(), yf.get(), s);
                else if (op == SS_OP_LSOLVE) M.lower(xf.get(), yf.get(), s);
                else M.upper(xf.get(), yf.get(), s);
                SS_REQUIRE(!(M.read_status(s) & ss::STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "triangular solve timed out");
            }
            ss::convert<double2, float2>(n, yf.get(), yd.get(), nullptr, s);
        }
        SS_HIP(hipMemcpyAsync(y, yd.get(), sizeof(double2) * n,
                              ss::is_device_ptr(y) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        SS_HIP(hipStreamSynchronize(s));
        return SS_OK;
    });
}

int ss_time_operator(ss_liouv L, int32_t op, int32_t prec, int32_t reps, double *avg_ms) {
    return guarded([&]() -> int {
        SS_REQUIRE(L != nullptr && avg_ms != nullptr && reps > 0, SS_E_INVALID_ARG, "bad argument");
        const bool pre = is_precond_op(op);
        const bool natural = (op == SS_OP_SPMV_L || op == SS_OP_APPLY_L);
        SS_REQUIRE(natural || op == SS_OP_SPMV_APERM || pre, SS_E_INVALID_ARG, "operator cannot be timed");
        SS_REQUIRE(natural || L->prepared, SS_E_STATE, "ss_prepare not called");
        SS_REQUIRE(natural || prec == SS_FP64 || L->p_opt.prec == SS_MIXED, SS_E_STATE,
                   "complex64 operators exist only after a mixed-precision ss_prepare");
        hipStream_t s = ss::stream_of(L);
        const int n = L->n;
        hipEvent_t e0, e1;
        SS_HIP(hipEventCreate(&e0));
        SS_HIP(hipEventCreate(&e1));
        float ms = 0.f;
        auto run = [&](auto zero_val) {
            using T = decltype(zero_val);
            ss::DevBuf<T> x((size_t)n), y((size_t)n);
            ss::zero<T>(n, y.get(), s);
            ss::DevBuf<double2> ones((size_t)n);
            ss::zero<double2>(n, ones.get(), s);
            ss::convert<T, double2>(n, ones.get(), x.get(), nullptr, s);
            const ss::CsrBuf<T> *A = nullptr;
            const ss::CsrBuf<T> *LU = nullptr;
            if constexpr (std::is_same<T, double2>::value) {
                A = natural ? &L->L : &L->Ap;
                LU = &L->LU;
            } else {
                A = &L->Ap32;
                LU = &L->LU32;
            }
            ss::Precond<T> M;
            if (pre) M.setup(LU, L->lu_diag.get(), n, s);
            if (pre && L->split) M.pin = L->cp.get();
            if (pre && op != SS_OP_PRECOND_SYNCFREE) M.use_levels(L->LU.view(), s, precond_mode(op), L->colours ? L->lorder.get() : nullptr);
            const ss::Csr<T> Av = A->view();
            const int g = ss::spmv_group(Av.n, Av.nnz);
            auto once = [&]() {
                if (pre) M.apply(x.get(), y.get(), s);
                else if constexpr (std::is_same<T, double2>::value) {
                    if (op == SS_OP_APPLY_L)
                        ss::lindblad_apply(L->lin.view(), x.get(), nullptr, 0, ss::mk(0.0, 0.0), nullptr, nullptr,
                                           y.get(), nullptr, s);
                    else ss::spmv<T>(Av, x.get(), y.get(), g, s);
                } else ss::spmv<T>(Av, x.get(), y.get(), g, s);
            };
            once();  // warm-up
            SS_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) once();
            SS_HIP(hipEventRecord(e1, s));
            SS_HIP(hipEventSynchronize(e1));
            SS_HIP(hipEventElapsedTime(&ms, e0, e1));
        };
        try {
            if (prec == SS_FP64 || natural) run(double2{0, 0});
            else run(float2{0, 0});
        } catch (...) {
            ss::hip_quiet(hipEventDestroy(e0));
            ss::hip_quiet(hipEventDestroy(e1));
            throw;
        }
        ss::hip_quiet(hipEventDestroy(e0));
        ss::hip_quiet(hipEventDestroy(e1));
        *avg_ms = (double)ms / reps;
        return SS_OK;
    });
}

}  // extern "C"
