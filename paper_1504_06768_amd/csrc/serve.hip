// Continuous-batching request server (ss_server_*): many small steady-state
// solves resident on the device at once.
//
// Pipeline: submitted (inputs copied to the host and validated there) ->
// admitted, in arrival order while a slot is free and the predicted device
// footprint fits the budget -> taken by one of several workers as a group of
// requests with the same method and options (at most one per compute unit):
// its inputs reach the device in one copy, the Liouvillians are assembled by
// the batched assembly, and the batched solve runs the set-up stages, one
// launch of the workgroup-resident solver (one workgroup per request) and
// the finish for all of them -> done (rho and info kept for ss_poll) -> the
// group's device memory returns to the budget.  Workers run their groups on
// their own streams side by side, so a request that arrives while a group is
// on the device is admitted as soon as slots and memory allow and its work
// overlaps the running group's.  Requests the batched path does not take
// (GMRES, SS_AUTO, sizes above the workgroup solver's default) are solved
// one by one with ss_solve's kernels.  Each request's arithmetic stays in its
// own workgroup, so its result does not depend on what else is in the group.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "assemble.hpp"
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
    // the checks of the device-side validation, on the copy, so that a bad
    // request is refused here and never reaches a group
    SS_REQUIRE(h.indptr[0] == 0 && h.indptr[(size_t)h.n] == m->nnz, SS_E_INVALID_ARG,
               std::string(what) + ": malformed indptr");
    for (int64_t r = 0; r < h.n; ++r) {
        const int64_t p = h.indptr[(size_t)r], q = h.indptr[(size_t)r + 1];
        SS_REQUIRE(p <= q && q <= m->nnz, SS_E_INVALID_ARG, std::string(what) + ": malformed indptr");
        for (int64_t e = p; e < q; ++e) {
            const int32_t c = h.indices[(size_t)e];
            SS_REQUIRE(c >= 0 && c < h.n && (e == p || c > h.indices[(size_t)e - 1]), SS_E_INVALID_ARG,
                       std::string(what) + ": column indices must be in range and strictly increasing per row");
            SS_REQUIRE(std::isfinite(h.data[2 * (size_t)e]) && std::isfinite(h.data[2 * (size_t)e + 1]),
                       SS_E_INVALID_ARG, std::string(what) + ": non-finite value");
        }
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
    std::chrono::steady_clock::time_point arrival;
    enum State { QUEUED, RUNNING, DONE } state = QUEUED;
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
    int max_group = 256;              // requests per batched launch (one per CU)
    std::mutex mu;
    std::condition_variable cv;       // wakes the workers
    std::condition_variable done_cv;  // wakes ss_server_drain
    std::deque<ss::Request *> queued;
    std::map<uint64_t, ss::Request *> all;
    size_t used = 0;
    size_t peak_used = 0;             // largest admitted footprint so far
    int resident = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    int device = 0;
    std::chrono::microseconds window{200};  // batching window (see worker_loop)
    std::chrono::steady_clock::time_point last_arrival;
    uint64_t groups = 0, max_group_seen = 0;
};

namespace ss {

static void set_error(Request *r, int code, const std::string &msg) {
    r->status = code;
    r->error = msg;
    r->info.status = code;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static size_t staged_bytes(const HostCsr &m) {
    return align256(sizeof(int64_t) * m.indptr.size()) + align256(sizeof(int32_t) * m.indices.size()) +
           align256(sizeof(double) * m.data.size());
}

// A worker's own stream (from the library's pool, never destroyed: blocks of
// the allocator cache keep events recorded on it) and page-locked staging.
struct Worker {
    hipStream_t stream = nullptr;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    ~Worker() {
        if (pinned) hip_quiet(hipHostFree(pinned));
    }
};

// Requests that the batched workgroup-resident path takes: BiCGSTAB methods,
// sizes it solves by default, operators the batched assembly accepts.
static bool batchable(const Request *r) {
    return (r->method == SS_TRACE_BICGSTAB || r->method == SS_INVPOW_BICGSTAB) &&
           use_workgroup_n(r->N * r->N, r->method, r->opt) && batch_assembly_fits(r->N) &&
           (int)r->C.size() <= MAX_COPS;
}

// A request the batched path does not take: assembled and solved on its own
// with ss_solve's kernels (device-wide or workgroup-resident, by its size).
static void run_single(Request *r) {
    std::vector<ss_csr_z> C;
    for (const HostCsr &c : r->C) C.push_back(c.view());
    const ss_csr_z H = r->H.view();
    std::unique_ptr<ss_liouv_s> h(new ss_liouv_s());
    h->own_stream = pooled_stream();
    h->N = r->N;
    h->d = (int)r->N;
    h->n = (int)(r->N * r->N);
    assemble_liouvillian(&H, C.empty() ? nullptr : C.data(), (int)C.size(), r->N, stream_of(h.get()), h->L, h->lin);
    r->rho.resize(2 * (size_t)r->N * r->N);
    std::memset(&r->info, 0, sizeof(r->info));
    r->status = solve(h.get(), r->method, r->tol, r->opt, r->rho.data(), &r->info);
    r->info.status = r->status;
    if (r->status == SS_E_NOT_CONVERGED) r->error = "iteration limit reached before ||L rho|| <= tol";
    else if (r->status == SS_E_BREAKDOWN) r->error = "BiCGSTAB breakdown";
    FreeScope fs(stream_peek(h.get()));
    h.reset();
}

// One group (same method and options): inputs to the device in one copy,
// batched assembly, batched solve; results kept in the requests.
static void run_group(Worker &W, std::vector<Request *> &g) {
    if (g.size() == 1 && !batchable(g[0])) {
        run_single(g[0]);
        return;
    }
    hipStream_t s = W.stream;
    StreamScope scope(s);
    const int m = (int)g.size();
    size_t bytes = 0;
    for (Request *r : g) {
        bytes += staged_bytes(r->H);
        for (const HostCsr &c : r->C) bytes += staged_bytes(c);
    }
    bytes = std::max<size_t>(bytes, 256);
    if (W.pinned_bytes < bytes) {
        if (W.pinned) {
            // the previous group's copy from it is complete (its solve was read back)
            SS_HIP(hipHostFree(W.pinned));
        }
        W.pinned = nullptr;
        W.pinned_bytes = 0;
        SS_HIP(hipHostMalloc(&W.pinned, bytes, hipHostMallocDefault));
        W.pinned_bytes = bytes;
    }
    DevBuf<unsigned char> dev(bytes);
    unsigned char *host = static_cast<unsigned char *>(W.pinned);
    size_t off = 0;
    auto stage = [&](const HostCsr &a) {
        ss_csr_z d;
        d.n = a.n;
        d.nnz = (int64_t)a.indices.size();
        std::memcpy(host + off, a.indptr.data(), sizeof(int64_t) * a.indptr.size());
        d.indptr = reinterpret_cast<const int64_t *>(dev.get() + off);
        off += align256(sizeof(int64_t) * a.indptr.size());
        std::memcpy(host + off, a.indices.data(), sizeof(int32_t) * a.indices.size());
        d.indices = reinterpret_cast<const int32_t *>(dev.get() + off);
        off += align256(sizeof(int32_t) * a.indices.size());
        std::memcpy(host + off, a.data.data(), sizeof(double) * a.data.size());
        d.data = reinterpret_cast<const double *>(dev.get() + off);
        off += align256(sizeof(double) * a.data.size());
        return d;
    };
    std::vector<ss_csr_z> Hd((size_t)m);
    std::vector<std::vector<ss_csr_z>> Cd((size_t)m);
    std::vector<const ss_csr_z *> Cp((size_t)m);
    std::vector<int> nc((size_t)m);
    for (int k = 0; k < m; ++k) {
        Hd[(size_t)k] = stage(g[(size_t)k]->H);
        for (const HostCsr &c : g[(size_t)k]->C) Cd[(size_t)k].push_back(stage(c));
        Cp[(size_t)k] = Cd[(size_t)k].empty() ? nullptr : Cd[(size_t)k].data();
        nc[(size_t)k] = (int)Cd[(size_t)k].size();
    }
    SS_HIP(hipMemcpyAsync(dev.get(), host, off, hipMemcpyHostToDevice, s));
    // handles and their batched assembly (the copy above is ordered before it
    // on s; assemble_batch returns with its work complete)
    std::vector<std::unique_ptr<ss_liouv_s>> hs;
    std::vector<AsmTarget> tg;
    for (Request *r : g) {
        std::unique_ptr<ss_liouv_s> h(new ss_liouv_s());
        h->own_stream = pooled_stream();
        h->N = r->N;
        h->d = (int)r->N;
        h->n = (int)(r->N * r->N);
        tg.push_back(AsmTarget{&h->L, &h->lin, stream_peek(h.get())});
        hs.push_back(std::move(h));
    }
    assemble_batch(m, Hd.data(), Cp.data(), nc.data(), tg.data(), s, true);
    // the batched solve, each request with its own tolerance
    std::vector<ss_liouv> hp;
    std::vector<double *> outs;
    std::vector<double> tols;
    for (int k = 0; k < m; ++k) {
        Request *r = g[(size_t)k];
        r->rho.resize(2 * (size_t)r->N * r->N);
        hp.push_back(hs[(size_t)k].get());
        outs.push_back(r->rho.data());
        tols.push_back(r->tol);
    }
    std::vector<ss_info> infos((size_t)m);
    std::vector<int> status((size_t)m, SS_OK);
    const ss_options o = g[0]->opt;
    ss::solve_batch(hp.data(), m, g[0]->method, tols[0], o, outs.data(), infos.data(), status.data(), tols.data());
    const std::string &first_err = batch_error();
    for (int k = 0; k < m; ++k) {
        Request *r = g[(size_t)k];
        r->info = infos[(size_t)k];
        r->status = status[(size_t)k];
        r->info.status = r->status;
        if (r->status == SS_E_NOT_CONVERGED) r->error = "iteration limit reached before ||L rho|| <= tol";
        else if (r->status == SS_E_BREAKDOWN) r->error = "BiCGSTAB breakdown";
        else if (r->status != SS_OK) r->error = first_err;
    }
    for (auto &h : hs) {
        FreeScope fs(stream_peek(h.get()));
        h.reset();
    }
}

static bool same_group(const Request *a, const Request *b) {
    return a->method == b->method && std::memcmp(&a->opt, &b->opt, sizeof(ss_options)) == 0;
}

// Whether the request at the head of the queue may start now (the lock is
// held): a free slot and room in the budget; a request larger than the whole
// budget starts alone.
static bool head_fits(const ss_server_s *S) {
    if (S->queued.empty() || S->resident >= S->max_slots) return false;
    const Request *r = S->queued.front();
    return S->resident == 0 || S->used + r->footprint <= S->budget;
}

// Worker: whenever the head of the queue fits, form a group -- the head plus
// later queued requests of the same method and options, in arrival order,
// while slots and budget allow, at most max_group -- and run it on this
// worker's stream.  Several workers run groups side by side, so a request
// that arrives while a group is on the device starts as soon as slots and
// memory allow instead of waiting for that group; its budget returns when
// its group finishes.
static void worker_loop(ss_server_s *S) {
    hip_quiet(hipSetDevice(S->device));
    Worker W;
    W.stream = pooled_stream();
    set_current_stream(W.stream);
    while (true) {
        std::vector<Request *> grp;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || head_fits(S); });
            if (S->stop) return;
            // batching window: while requests keep arriving (less than the
            // window apart) and the queue holds fewer than a full group, let
            // it fill, so that a burst forms few large groups
            while (!S->stop && head_fits(S) && (int)S->queued.size() < S->max_group) {
                const auto quiet = std::chrono::steady_clock::now() - S->last_arrival;
                if (quiet >= S->window) break;
                S->cv.wait_for(lk, S->window - quiet);
            }
            if (S->stop) return;
            if (!head_fits(S)) continue;
            Request *head = S->queued.front();
            S->queued.pop_front();
            grp.push_back(head);
            if (batchable(head)) {
                for (auto it = S->queued.begin(); it != S->queued.end() && (int)grp.size() < S->max_group;) {
                    Request *r = *it;
                    if (S->resident + (int)grp.size() >= S->max_slots) break;
                    if (same_group(head, r) && batchable(r)) {
                        size_t fp = 0;
                        for (Request *q : grp) fp += q->footprint;
                        if (S->used + fp + r->footprint > S->budget) break;
                        grp.push_back(r);
                        it = S->queued.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            for (Request *r : grp) {
                S->used += r->footprint;
                S->resident += 1;
                r->state = Request::RUNNING;
            }
            S->peak_used = std::max(S->peak_used, S->used);
            S->groups += 1;
            S->max_group_seen = std::max<uint64_t>(S->max_group_seen, grp.size());
            // another worker may take the new head
            if (head_fits(S)) S->cv.notify_one();
        }
        try {
            run_group(W, grp);
        } catch (const Error &e) {
            for (Request *r : grp) set_error(r, e.code, e.what());
        } catch (const std::exception &e) {
            for (Request *r : grp) set_error(r, SS_E_HIP, e.what());
        }
        std::lock_guard<std::mutex> lk(S->mu);
        for (Request *r : grp) {
            S->used -= r->footprint;
            S->resident -= 1;
            r->state = Request::DONE;
        }
        S->done_cv.notify_all();
        S->cv.notify_all();
    }
}

// Workers per server: SS_SERVER_WORKERS (1..16), default 4; batching window
// SS_SERVER_WINDOW_US (0..100000), default 200.
static int env_int(const char *name, int lo, int hi, int dflt) {
    const char *e = std::getenv(name);
    if (!e) return dflt;
    const int v = std::atoi(e);
    return (v >= lo && v <= hi) ? v : dflt;
}

}  // namespace ss

namespace ss {
void set_last_error(const std::string &msg);
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
    if (ss::hip_quiet(hipGetDevice(&S->device)) != hipSuccess) {
        delete S;
        return SS_E_HIP;
    }
    int cus = 0;
    if (ss::hip_quiet(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device)) == hipSuccess &&
        cus > 0)
        S->max_group = cus;
    try {
        S->window = std::chrono::microseconds(ss::env_int("SS_SERVER_WINDOW_US", 0, 100000, 200));
        const int nw = ss::env_int("SS_SERVER_WORKERS", 1, 16, 4);
        for (int k = 0; k < nw; ++k) S->workers.emplace_back(ss::worker_loop, S);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->cv.notify_all();
        }
        for (auto &t : S->workers) t.join();
        delete S;
        return SS_E_OOM;
    }
    *out = S;
    return SS_OK;
}

int ss_submit(ss_server S, const ss_csr_z *H, const ss_csr_z *c_ops, int32_t n_cops, int64_t N, int32_t method,
              double tol, const ss_options *opt, uint64_t *ticket) {
    if (!S || !ticket || !H || N < 1 || N > 46340 || n_cops < 0 || (n_cops > 0 && !c_ops) || !(tol > 0) ||
        !std::isfinite(tol))
        return SS_E_INVALID_ARG;
    if (method < SS_TRACE_BICGSTAB || method > SS_AUTO) return SS_E_INVALID_ARG;
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
        if (r->opt.fill <= 0) r->opt.fill = 10.0;
        if (r->opt.drop_tol < 0) r->opt.drop_tol = 1e-4;
        SS_REQUIRE(r->opt.prec == SS_FP64 || r->opt.prec == SS_MIXED, SS_E_INVALID_ARG, "unknown precision");
        SS_REQUIRE(r->opt.ilu == SS_ILU0 || r->opt.ilu == SS_ILUT, SS_E_INVALID_ARG, "unknown ILU kind");
        SS_REQUIRE(r->opt.ordering == SS_ORDER_RCM || r->opt.ordering == SS_ORDER_NATURAL ||
                       r->opt.ordering == SS_ORDER_COLOUR,
                   SS_E_INVALID_ARG, "unknown ordering");
        r->footprint = ss::predict_footprint(r->H, r->C, r->opt.prec);
        std::lock_guard<std::mutex> lk(S->mu);
        r->arrival = std::chrono::steady_clock::now();
        S->last_arrival = r->arrival;
        r->ticket = S->next_ticket++;
        *ticket = r->ticket;
        S->all[r->ticket] = r.get();
        S->queued.push_back(r.release());
        S->cv.notify_one();
        return SS_OK;
    } catch (const ss::Error &e) {
        ss::set_last_error(e.what());
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
    if (st != SS_OK) ss::set_last_error(r->error);
    if (info) *info = r->info;
    int rc = st;
    if (rho_out && !r->rho.empty()) {
        const size_t bytes = sizeof(double) * r->rho.size();
        if (ss::is_device_ptr(rho_out)) {
            const hipError_t e = ss::hip_quiet(hipMemcpy(rho_out, r->rho.data(), bytes, hipMemcpyHostToDevice));
            if (e != hipSuccess) {
                ss::set_last_error(std::string("ss_poll: hipMemcpy of rho to the device: ") + hipGetErrorString(e));
                rc = SS_E_HIP;
                if (info) info->status = rc;
            }
        } else {
            std::memcpy(rho_out, r->rho.data(), bytes);
        }
    }
    delete r;
    return rc;
}

int ss_server_stats(ss_server S, ss_server_stats_t *st) {
    if (!S || !st) return SS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    st->budget_bytes = S->budget;
    st->resident_bytes = S->used;
    st->peak_resident_bytes = S->peak_used;
    st->resident = S->resident;
    st->queued = (int32_t)S->queued.size();
    st->groups = S->groups;
    st->largest_group = S->max_group_seen;
    st->workers = (int32_t)S->workers.size();
    st->max_group = S->max_group;
    return SS_OK;
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
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->all) delete kv.second;
    for (ss::Request *r : S->queued)
        if (S->all.find(r->ticket) == S->all.end()) delete r;
    delete S;
}

}  // extern "C"
