// Device memory, pointer classification and the integer exclusive scan used
// to turn per-row counts into CSR row pointers.
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "ss_internal.hpp"

namespace ss {

// ------------------------------------------------------ cached allocation
// hipMalloc / hipFree cost tens to hundreds of microseconds and hipFree
// waits for the device, which would serialise the set-up of independent
// systems running on different streams.  Freed blocks (up to 64 MB, 4 GB in
// total) are therefore kept in power-of-two size classes and handed out
// again -- but only after an event, recorded at free time on the stream the
// block was allocated for, has completed, so a block is never reused while
// work queued before its release may still touch it.  Blocks are used on
// the stream that was current in the allocating thread (stream_of()), and
// the few cross-stream uses (a batched launch) are synchronised before the
// owners release their blocks.
namespace {

constexpr size_t CACHE_MAX_BLOCK = size_t(64) << 20;
constexpr size_t CACHE_MAX_TOTAL = size_t(4) << 30;

struct Cached {
    void *p;
    hipEvent_t ev;
    bool user;
};

struct Live {
    size_t cls;      // 0: not cached
    hipStream_t s;   // stream current when allocated
    bool user;       // made by the caller's allocator
};

// An event may mark the release of several blocks (all those a free scope
// releases); it returns to the pool when the last of them is reused.  Once
// seen complete it is not queried again.
struct EvState {
    int refs;
    bool done;
};

struct Cache {
    std::mutex mu;
    std::unordered_map<void *, Live> live;
    std::map<size_t, std::deque<Cached>> free_by_cls;
    std::vector<hipEvent_t> events;
    std::unordered_map<hipEvent_t, EvState> evs;
    size_t cached = 0;
};

Cache &cache() {
    static Cache *c = new Cache();  // process lifetime
    return *c;
}

thread_local hipStream_t t_current = nullptr;
thread_local hipEvent_t t_free_ev = nullptr;   // event of the open free scope
thread_local hipStream_t t_free_s = nullptr;   // its stream

// (the cache lock is held by the callers of these three)
hipEvent_t take_event(Cache &c) {
    if (!c.events.empty()) {
        hipEvent_t ev = c.events.back();
        c.events.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return ev;
}

void release_event(Cache &c, hipEvent_t ev) {
    auto it = c.evs.find(ev);
    if (it == c.evs.end()) return;
    if (--it->second.refs == 0) {
        c.evs.erase(it);
        c.events.push_back(ev);
    }
}

bool event_done(Cache &c, hipEvent_t ev) {
    auto it = c.evs.find(ev);
    if (it != c.evs.end() && it->second.done) return true;
    // hipErrorNotReady (work still queued) is also left as the thread's last
    // error: cleared here, so no later launch check reports it
    if (hip_quiet(hipEventQuery(ev)) != hipSuccess) return false;
    if (it != c.evs.end()) it->second.done = true;
    return true;
}

// optional caller allocator (ss_set_allocator)
ss_alloc_fn g_user_alloc = nullptr;
ss_free_fn g_user_free = nullptr;
void *g_user_ctx = nullptr;

void raw_free(void *p, bool user) {
    if (user) {
        if (g_user_free) g_user_free(p, g_user_ctx);
    } else {
        hip_quiet(hipFree(p));
    }
}

size_t size_class(size_t b) {
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}

void *raw_alloc(size_t bytes) {
    void *p = nullptr;
    if (g_user_alloc) {
        p = g_user_alloc(bytes, g_user_ctx);
        if (!p) {
            trim_device_cache();
            p = g_user_alloc(bytes, g_user_ctx);
        }
        if (!p) throw Error(SS_E_OOM, "caller allocator returned NULL for " + std::to_string(bytes) + " B");
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        trim_device_cache();
        e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? SS_E_OOM : SS_E_HIP,
                    "hipMalloc(" + std::to_string(bytes) + " B): " + hipGetErrorString(e));
    }
    return p;
}

}  // namespace

FreeScope::FreeScope(hipStream_t s) {
    if (!s) return;
    Cache &c = cache();
    hipEvent_t ev;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        ev = take_event(c);
        if (!ev) return;
        c.evs[ev] = EvState{1, false};  // the scope's own reference
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(c.mu);
        release_event(c, ev);
        return;
    }
    prev_ev = t_free_ev;
    prev_s = t_free_s;
    t_free_ev = ev;
    t_free_s = s;
    ev_ = ev;
}

FreeScope::~FreeScope() {
    if (!ev_) return;
    t_free_ev = prev_ev;
    t_free_s = prev_s;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    release_event(c, ev_);
}

void set_current_stream(hipStream_t s) { t_current = s; }
hipStream_t current_stream() { return t_current; }

void set_allocator(ss_alloc_fn a, ss_free_fn f, void *ctx) {
    trim_device_cache();
    g_user_alloc = a;
    g_user_free = f;
    g_user_ctx = ctx;
}

void trim_device_cache() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto &kv : c.free_by_cls) {
        for (Cached &b : kv.second) {
            hip_quiet(hipEventSynchronize(b.ev));
            raw_free(b.p, b.user);
            release_event(c, b.ev);
        }
        kv.second.clear();
    }
    c.cached = 0;
}

void *dev_alloc(size_t bytes) {
    Cache &c = cache();
    const size_t cls = bytes <= CACHE_MAX_BLOCK ? size_class(bytes) : 0;
    if (cls) {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.free_by_cls.find(cls);
        if (it != c.free_by_cls.end()) {
            std::deque<Cached> &v = it->second;
            const bool user = g_user_alloc != nullptr;
            // oldest first: those are the blocks whose last use has most
            // likely completed, so the first query usually succeeds
            for (size_t k = 0; k < v.size(); ++k) {
                if (v[k].user == user && event_done(c, v[k].ev)) {
                    void *p = v[k].p;
                    release_event(c, v[k].ev);
                    v.erase(v.begin() + (long)k);
                    c.cached -= cls;
                    c.live[p] = Live{cls, t_current, user};
                    return p;
                }
            }
        }
    }
    const bool user = g_user_alloc != nullptr;
    void *p = raw_alloc(cls ? cls : bytes);
    std::lock_guard<std::mutex> lk(c.mu);
    c.live[p] = Live{cls, t_current, user};
    return p;
}

void dev_free(void *p) {
    if (!p) return;
    Cache &c = cache();
    Live l{0, nullptr, false};
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.live.find(p);
        if (it == c.live.end()) return;  // not a block of this allocator
        l = it->second;
        c.live.erase(it);
        if (l.cls && c.cached + l.cls <= CACHE_MAX_TOTAL) {
            if (t_free_ev && l.s == t_free_s) {
                // a free scope on the block's stream: its event covers every
                // use queued before the scope opened
                c.evs[t_free_ev].refs++;
                c.free_by_cls[l.cls].push_back(Cached{p, t_free_ev, l.user});
                c.cached += l.cls;
                return;
            }
            hipEvent_t ev = take_event(c);
            if (ev) {
                // (dev_free runs in destructors: failures are cleared, never thrown)
                if (!l.s) hip_quiet(hipDeviceSynchronize());  // no stream known: wait for everything
                if (hipEventRecord(ev, l.s) == hipSuccess) {
                    c.evs[ev] = EvState{1, false};
                    c.free_by_cls[l.cls].push_back(Cached{p, ev, l.user});
                    c.cached += l.cls;
                    return;
                }
                (void)hipGetLastError();
                c.events.push_back(ev);
            }
        }
    }
    if (l.s) hip_quiet(hipStreamSynchronize(l.s));
    raw_free(p, l.user);  // uncached (hipFree also waits for the device)
}

// ------------------------------------------------------------ stream pool
// Handles take their stream from a fixed pool (created once, never
// destroyed): creating and destroying a stream per handle costs milliseconds.
hipStream_t pooled_stream() {
    static std::mutex mu;
    static std::vector<hipStream_t> pool;
    static size_t next = 0;
    constexpr size_t POOL = 16;
    std::lock_guard<std::mutex> lk(mu);
    if (pool.empty()) {
        for (size_t k = 0; k < POOL; ++k) {
            hipStream_t s = nullptr;
            SS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            pool.push_back(s);
        }
    }
    return pool[next++ % POOL];
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// -------------------------------------------------------------------- scan
// 256 threads x 4 items per block; per-block totals are scanned recursively.
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 4;
constexpr int SCAN_B = SCAN_T * SCAN_I;

__global__ void __launch_bounds__(SCAN_T) k_scan_block(const int *in, int *out, int64_t n,
                                                      int *block_sums) {
    __shared__ int s[SCAN_T];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)t * SCAN_I;
    int v[SCAN_I];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
    }
    int loc[SCAN_I];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) { loc[k] = sum; sum += v[k]; }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int x = (t >= off) ? s[t - off] : 0;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    const int excl = s[t] - sum;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = excl + loc[k];
    }
    if (t == SCAN_T - 1) block_sums[blockIdx.x] = s[SCAN_T - 1];
}

__global__ void __launch_bounds__(SCAN_T) k_scan_add(int *out, int64_t n, const int *offsets) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
    const int o = offsets[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] += o;
    }
}

__global__ void k_copy_int(int *dst, const int *src) { *dst = *src; }

// Exclusive scan: out[i] = sum_{j<i} in[j] for i < n, out[n] = total.
static void scan_rec(const int *in, int *out, int64_t n, hipStream_t s) {
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    StreamScope scope(s);  // sums is released behind the kernels that read it
    DevBuf<int> sums((size_t)nb + 1);
    k_scan_block<<<(unsigned)nb, SCAN_T, 0, s>>>(in, out, n, sums.get());
    SS_HIP(hipGetLastError());
    if (nb > 1) {
        scan_rec(sums.get(), sums.get(), nb, s);
        k_scan_add<<<(unsigned)nb, SCAN_T, 0, s>>>(out, n, sums.get());
        SS_HIP(hipGetLastError());
        k_copy_int<<<1, 1, 0, s>>>(out + n, sums.get() + nb);
    } else {
        k_copy_int<<<1, 1, 0, s>>>(out + n, sums.get());
    }
    SS_HIP(hipGetLastError());
}

int64_t scan_exclusive(const int *in, int *out, int64_t n, hipStream_t s, bool want_total) {
    if (n <= 0) {
        SS_HIP(hipMemsetAsync(out, 0, sizeof(int), s));
        return 0;
    }
    scan_rec(in, out, n, s);
    if (!want_total) return -1;
    int total = 0;
    d2h(&total, out + n, 1, s);
    return total;
}

}  // namespace ss
