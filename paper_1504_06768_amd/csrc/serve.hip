// Continuous-batching request server (ss_server_*): many small steady-state
// solves resident on the device at once.
//
// Pipeline of one request: submitted (inputs copied) -> admitted, when a slot
// is free and its predicted device footprint fits the budget -> set up by a
// worker thread on its own stream (assembly, transform, RCM, ILU, level
// schedules: the same kernels as ss_solve) -> ready -> solved together with
// every other ready request of the same precision in one launch of the
// workgroup-resident solver (one workgroup per request) -> finished
// (certificate, rho copied to the host) -> its device memory returns to the
// budget.  Requests that arrive while a batch runs are admitted and set up
// concurrently on the worker streams and join the next launch, so set-up and
// solve work of different requests overlap on the device.  Each request's
// arithmetic is confined to its own workgroup, so its result does not depend
// on what else is in the batch.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "handle.hpp"

namespace ss {

struct HostCsr {
    int64_t n = 0;
    std::vector<int64_t> indptr;
    std::vector<int32_t> indices;
    std::vector<double> data;
    ss_csr_z view() const {
        ss_csr_z c;
        c.n = n;
        c.nnz = (int64_t)indices.size();
        c.indptr = indptr.data();
        c.indices = indices.data();
        c.data = data.data();
        return c;
    }
};

static HostCsr copy_in(const ss_csr_z *m, int64_t N, const char *what) {
    SS_REQUIRE(m != nullptr && m->n == N && m->nnz >= 0 && m->indptr, SS_E_INVALID_ARG,
               std::string(what) + ": bad matrix");
    HostCsr h;
    h.n = m->n;
    h.indptr.resize((size_t)m->n + 1);
    h.indices.resize((size_t)m->nnz);
    h.data.resize(2 * (size_t)m->nnz);
    auto cp = [](void *dst, const void *src, size_t bytes) {
        if (!bytes) return;
        if (is_device_ptr(src)) SS_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        else std::memcpy(dst, src, bytes);
    };
    cp(h.indptr.data(), m->indptr, sizeof(int64_t) * h.indptr.size());
    if (m->nnz) {
        SS_REQUIRE(m->indices && m->data, SS_E_INVALID_ARG, std::string(what) + ": null arrays");
        cp(h.indices.data(), m->indices, sizeof(int32_t) * h.indices.size());
        cp(h.data.data(), m->data, sizeof(double) * h.data.size());
    }
    return h;
}

// Upper bound of the device bytes a request holds while resident: the
// Liouvillian's nnz is bounded from the operators' structure (I (x) G and
// G^T (x) I rows, plus conj(C) (x) C), times the matrices kept per nonzero.
static size_t predict_footprint(const HostCsr &H, const std::vector<HostCsr> &C, int prec) {
    const double d = (double)H.n;
    double g = (double)H.indices.size();
    double cc = 0.0;
    for (const HostCsr &c : C) {
        double rows2 = 0.0;
        for (int64_t r = 0; r < c.n; ++r) {
            const double k = (double)(c.indptr[r + 1] - c.indptr[r]);
            rows2 += k * k;
        }
        g += std::min(rows2, d * d);
        const double nz = (double)c.indices.size();
        cc += nz * nz;
    }
    const double nnz = std::min(2.0 * d * g + cc + d, d * d * d * d);
    const double n = d * d;
    // L, L~ (natural and permuted) and ILU factors in fp64, copies in c64,
    // symmetrised pattern, packed level layout, ~20 work vectors
    const double per_nz = 4 * (16 + 4) + (prec == SS_MIXED ? 2 * (8 + 4) : 0) + 8 + 8 * 12;
    return (size_t)(nnz * per_nz + n * (20 * 16 + 64)) + (1u << 20);
}

struct Request {
    uint64_t ticket = 0;
    HostCsr H;
    std::vector<HostCsr> C;
    int64_t N = 0;
    int method = 0;
    double tol = 1e-10;
    ss_options opt{};
    size_t footprint = 0;
    enum State { QUEUED, SETUP, READY, DONE } state = QUEUED;
    // device state while resident
    ss_liouv h = nullptr;
    WgBundle<double2> b64;
    WgBundle<float2> b32;
    // result
    int status = SS_OK;
    std::string error;
    std::vector<double> rho;
    ss_info info{};
};

}  // namespace ss

struct ss_server_s {
    size_t budget = 0;
    int max_slots = 0;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler and the setup workers
    std::condition_variable done_cv;  // wakes ss_server_drain
    std::deque<ss::Request *> queued, to_setup;
    std::map<uint64_t, ss::Request *> all;
    std::vector<ss::Request *> ready;
    size_t used = 0;
    int resident = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::thread scheduler;
    hipStream_t solve_stream = nullptr;
    int device = 0;
};

namespace ss {

static void set_error(Request *r, int code, const std::string &msg) {
    r->status = code;
    r->error = msg;
    r->info.status = code;
}

static void release_device(ss_server_s *S, Request *r) {
    if (r->h) ss_liouv_free(r->h);
    r->h = nullptr;
    r->b64 = WgBundle<double2>();
    r->b32 = WgBundle<float2>();
    S->used -= r->footprint;
    S->resident -= 1;
}

// Set-up worker: assembly, transform, ordering, factorisation and the
// workgroup problem of admitted requests, on the handle's own stream.
static void worker_loop(ss_server_s *S) {
    (void)hipSetDevice(S->device);
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->to_setup.empty(); });
            if (S->stop) return;
            r = S->to_setup.front();
            S->to_setup.pop_front();
        }
        int code = SS_OK;
        std::string msg;
        try {
            ss_csr_z Hv = r->H.view();
            std::vector<ss_csr_z> Cv;
            for (const HostCsr &c : r->C) Cv.push_back(c.view());
            ss_liouv h = nullptr;
            const int rc = ss_build_liouvillian(&Hv, Cv.empty() ? nullptr : Cv.data(), (int32_t)Cv.size(), r->N, &h);
            if (rc != SS_OK) throw Error(rc, ss_last_error());
            r->h = h;
            SS_REQUIRE(use_workgroup(h, r->method, r->opt), SS_E_INVALID_ARG,
                       "the server solves BiCGSTAB methods of systems that fit one workgroup");
            prepare(h, r->method, r->opt);
            hipStream_t s = stream_of(h);
            if (r->opt.prec == SS_MIXED) make_wg<float2>(h, r->method, r->tol, r->opt, h->Ap32, h->LU32, r->b32, s);
            else make_wg<double2>(h, r->method, r->tol, r->opt, h->Ap, h->LU, r->b64, s);
            SS_HIP(hipStreamSynchronize(s));
        } catch (const Error &e) {
            code = e.code;
            msg = e.what();
        } catch (const std::exception &e) {
            code = SS_E_HIP;
            msg = e.what();
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (code != SS_OK) {
            set_error(r, code, msg);
            release_device(S, r);
            r->state = Request::DONE;
            S->done_cv.notify_all();
        } else {
            r->state = Request::READY;
            S->ready.push_back(r);
        }
        S->cv.notify_all();
    }
}

template <typename T> WgBundle<T> &bundle(Request *r);
template <> WgBundle<double2> &bundle<double2>(Request *r) { return r->b64; }
template <> WgBundle<float2> &bundle<float2>(Request *r) { return r->b32; }

template <typename T>
static void solve_batch(ss_server_s *S, std::vector<Request *> &batch) {
    hipStream_t s = S->solve_stream;
    std::vector<WgProblem<T>> probs;
    int max_n = 0, max_lev = 0;
    for (Request *r : batch) {
        WgBundle<T> &B = bundle<T>(r);
        probs.push_back(B.P);
        max_n = std::max(max_n, B.P.n);
        max_lev = std::max(max_lev, B.levels);
    }
    DevBuf<WgProblem<T>> dP(probs.size());
    h2d(dP.get(), probs.data(), probs.size(), s);
    const auto t0 = std::chrono::steady_clock::now();
    wg_solve<T>(dP.get(), (int)probs.size(), max_n, max_lev, s);
    SS_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (Request *r : batch) {
        WgBundle<T> &B = bundle<T>(r);
        WgResult hr;
        d2h(&hr, B.res.get(), 1, s);
        SolveStats st;
        st.status = hr.status;
        st.outer = hr.outer;
        st.inner = hr.inner;
        st.breakdowns = hr.breakdowns;
        st.path = wg_fits_lds((size_t)max_n, sizeof(T), max_lev) ? 2 : 1;
        st.t_kernel_ms = ms;
        st.t_solve_ms = ms;
        st.elem_bytes = (double)sizeof(T);
        r->rho.resize(2 * (size_t)r->N * r->N);
        if (hr.status == SS_E_BREAKDOWN && !(r->opt.flags & SS_FLAG_NO_FALLBACK)) {
            // BiCGSTAB broke down, diverged or stalled on this request: solve it
            // again on its own with the device-wide GMRES
            ss_options od = r->opt;
            od.flags |= SS_FLAG_DEVICE_WIDE;
            const int gm = (r->method == SS_TRACE_BICGSTAB) ? SS_TRACE_GMRES : SS_INVPOW_GMRES;
            r->status = solve(r->h, gm, r->tol, od, r->rho.data(), &r->info);
            r->info.fell_back = 1;
        } else {
            r->status = finish(r->h, B.x.get(), r->opt, r->tol, st, r->rho.data(), &r->info, s);
        }
        if (r->status == SS_E_NOT_CONVERGED) r->error = "iteration limit reached before ||L rho|| <= tol";
        if (r->status == SS_E_BREAKDOWN) r->error = "BiCGSTAB breakdown";
    }
}

// Scheduler: admission by slots and footprint, then one batched launch per
// precision over every ready request.
static void scheduler_loop(ss_server_s *S) {
    (void)hipSetDevice(S->device);
    set_current_stream(S->solve_stream);
    while (true) {
        std::vector<Request *> b64, b32;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] {
                if (S->stop) return true;
                if (!S->ready.empty()) return true;
                return !S->queued.empty() && S->resident < S->max_slots &&
                       (S->resident == 0 || S->used + S->queued.front()->footprint <= S->budget);
            });
            if (S->stop) return;
            // admit in arrival order while slots and memory allow (a request
            // larger than the whole budget is admitted alone)
            while (!S->queued.empty() && S->resident < S->max_slots) {
                Request *r = S->queued.front();
                if (S->resident > 0 && S->used + r->footprint > S->budget) break;
                S->queued.pop_front();
                S->used += r->footprint;
                S->resident += 1;
                r->state = Request::SETUP;
                S->to_setup.push_back(r);
            }
            for (Request *r : S->ready) (r->opt.prec == SS_MIXED ? b32 : b64).push_back(r);
            S->ready.clear();
            S->cv.notify_all();
        }
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<Request *> &batch = pass ? b32 : b64;
            if (batch.empty()) continue;
            try {
                if (pass) solve_batch<float2>(S, batch);
                else solve_batch<double2>(S, batch);
            } catch (const Error &e) {
                for (Request *r : batch) set_error(r, e.code, e.what());
            } catch (const std::exception &e) {
                for (Request *r : batch) set_error(r, SS_E_HIP, e.what());
            }
            std::lock_guard<std::mutex> lk(S->mu);
            for (Request *r : batch) {
                release_device(S, r);
                r->state = Request::DONE;
            }
            S->done_cv.notify_all();
            S->cv.notify_all();
        }
    }
}

}  // namespace ss

namespace {
thread_local std::string s_err;
}

extern "C" {

int ss_server_create(size_t hbm_budget_bytes, int32_t max_slots, ss_server *out) {
    if (!out) return SS_E_INVALID_ARG;
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_slots <= 0) return SS_E_INVALID_ARG;
    ss_server_s *S = new (std::nothrow) ss_server_s();
    if (!S) return SS_E_OOM;
    S->budget = hbm_budget_bytes;
    S->max_slots = max_slots;
    (void)hipGetDevice(&S->device);
    if (hipStreamCreateWithFlags(&S->solve_stream, hipStreamNonBlocking) != hipSuccess) {
        delete S;
        return SS_E_HIP;
    }
    const int nworkers = 8;
    for (int i = 0; i < nworkers; ++i) S->workers.emplace_back(ss::worker_loop, S);
    S->scheduler = std::thread(ss::scheduler_loop, S);
    *out = S;
    return SS_OK;
}

int ss_submit(ss_server S, const ss_csr_z *H, const ss_csr_z *c_ops, int32_t n_cops, int64_t N, int32_t method,
              double tol, const ss_options *opt, uint64_t *ticket) {
    if (!S || !ticket || !H || N < 1 || n_cops < 0 || (n_cops > 0 && !c_ops) || !(tol > 0)) return SS_E_INVALID_ARG;
    if (method != SS_TRACE_BICGSTAB && method != SS_INVPOW_BICGSTAB) return SS_E_INVALID_ARG;
    try {
        std::unique_ptr<ss::Request> r(new ss::Request());
        r->H = ss::copy_in(H, N, "H");
        for (int k = 0; k < n_cops; ++k) r->C.push_back(ss::copy_in(&c_ops[k], N, "c_ops[k]"));
        r->N = N;
        r->method = method;
        r->tol = tol;
        ss_options_default(&r->opt);
        if (opt) r->opt = *opt;
        if (r->opt.maxiter <= 0) r->opt.maxiter = 1000;
        if (r->opt.max_outer <= 0) r->opt.max_outer = 20;
        if (r->opt.gmres_m <= 0) r->opt.gmres_m = 20;
        r->footprint = ss::predict_footprint(r->H, r->C, r->opt.prec);
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        *ticket = r->ticket;
        S->all[r->ticket] = r.get();
        S->queued.push_back(r.release());
        S->cv.notify_all();
        return SS_OK;
    } catch (const ss::Error &e) {
        return e.code;
    } catch (...) {
        return SS_E_OOM;
    }
}

int ss_poll(ss_server S, uint64_t ticket, double *rho_out, ss_info *info) {
    if (!S) return SS_E_INVALID_ARG;
    ss::Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return SS_E_INVALID_ARG;
        r = it->second;
        if (r->state != ss::Request::DONE) return SS_PENDING;
        S->all.erase(it);
    }
    const int st = r->status;
    if (info) *info = r->info;
    if (rho_out && !r->rho.empty()) {
        const size_t bytes = sizeof(double) * r->rho.size();
        if (ss::is_device_ptr(rho_out)) (void)hipMemcpy(rho_out, r->rho.data(), bytes, hipMemcpyHostToDevice);
        else std::memcpy(rho_out, r->rho.data(), bytes);
    }
    delete r;
    return st;
}

int ss_server_drain(ss_server S) {
    if (!S) return SS_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    S->done_cv.wait(lk, [&] {
        for (auto &kv : S->all)
            if (kv.second->state != ss::Request::DONE) return false;
        return true;
    });
    return SS_OK;
}

void ss_server_destroy(ss_server S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    for (std::thread &t : S->workers) t.join();
    S->scheduler.join();
    for (auto &kv : S->all) {
        ss::Request *r = kv.second;
        if (r->h) ss_liouv_free(r->h);
        delete r;
    }
    for (ss::Request *r : S->queued)
        if (S->all.find(r->ticket) == S->all.end()) delete r;
    if (S->solve_stream) (void)hipStreamDestroy(S->solve_stream);
    delete S;
}

}  // extern "C"
