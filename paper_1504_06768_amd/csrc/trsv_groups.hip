// Sync-free triangular solves over all CUs with sixteen lanes per row
// (section "Iterative Solvers": the forward and backward substitutions of
// the ILU preconditioner; section "Eigenvalue Methods": they dominate each
// inner iteration of the doubly-iterative method).
//
// In RCM order the factors of the large workloads have deep level sets
// (about 1300 lower and 900 upper levels for the Kerr chain at n = 10^6),
// so a solve costs the number of levels times the time one level takes to
// reach the next: the store of a result, its visibility at device scope,
// and the poll that sees it.  What this kernel does to keep that short:
//
//  * A row is taken by a group of 16 lanes, one factor entry each (longer
//    rows continue in chunks of 16), so one poll of a wavefront is a single
//    coherent load per lane.  With one lane per row, a wavefront's poll
//    was ~12 dependent-value loads per lane and a level took ~5 us; with 16
//    lanes per row it takes ~2 us.
//  * Complex128 values are published and polled as single 16-byte
//    device-scope accesses; each 8-byte half is compared with the sentinel,
//    so a value is taken only once both halves are written.
//  * The row's lanes multiply their entry by its dependency as soon as it
//    is seen; the lane that owns the row then subtracts the products in the
//    factor's entry order, so the result has the same bits as the other
//    triangular solves of the library (this file is compiled without
//    floating-point contraction).
//  * Tasks of 4 rows follow the level order.  Only tasks near the frontier
//    poll values: a task first waits for a gating row, the last row of the
//    level two below its first level.  The gate is a hint; each value is
//    still taken only once its own publication is seen (data-as-flag).
//  * Tasks are dealt round-robin to the wavefronts without atomics when all
//    of them are resident, which the wavefronts decide together at start:
//    the last to arrive declares the static order, and a wavefront that
//    sees no arrival for 20 us declares the dynamic one, where tasks
//    are taken in order from an atomic counter (so every task waited on
//    belongs to a running wavefront).  Every wait is bounded and reports a
//    status bit instead of hanging.
#include "ilu.hpp"

namespace ss {

namespace {

constexpr int GRP = 16;              // lanes per row
constexpr int GRP_ROWS = 64 / GRP;   // rows per wavefront task
constexpr int GRP_WPB = 4;           // wavefronts per workgroup
constexpr int GRP_LAG = 2;           // levels between a task and its gate
constexpr unsigned GRP_GATE_SPINS = 1u << 16;
constexpr long long GRP_ARRIVE_TICKS = 2000;  // 20 us of the 100 MHz clock without an arrival

enum : unsigned { CTL_ARRIVE = 0, CTL_MODE = 1, CTL_TASK = 2, CTL_EXIT = 3 };
enum : unsigned { MODE_STATIC = 1, MODE_DYNAMIC = 2 };

__device__ inline __amdgpu_buffer_rsrc_t buffer_of(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff, 0x00020000);
}

// cache policy 16: device scope (sc1), coherent across the XCDs
constexpr int CPOL_DEVICE = 16;

__device__ inline bool poll_value(__amdgpu_buffer_rsrc_t r, const double2 *base, int i, double2 &out) {
    (void)base;
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, i * 16, 0, CPOL_DEVICE);
    const unsigned long long x = ((unsigned long long)w[1] << 32) | w[0];
    const unsigned long long y = ((unsigned long long)w[3] << 32) | w[2];
    if (x == SENT_F64 || y == SENT_F64) return false;
    out.x = __longlong_as_double((long long)x);
    out.y = __longlong_as_double((long long)y);
    return true;
}
__device__ inline void publish_value(__amdgpu_buffer_rsrc_t r, double2 *base, int i, double2 v) {
    (void)base;
    const unsigned long long x = canon_bits(v.x), y = canon_bits(v.y);
    const __attribute__((ext_vector_type(4))) unsigned w = {(unsigned)x, (unsigned)(x >> 32), (unsigned)y,
                                                            (unsigned)(y >> 32)};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, i * 16, 0, CPOL_DEVICE);
}
__device__ inline bool poll_value(__amdgpu_buffer_rsrc_t, const float2 *base, int i, float2 &out) {
    return try_load(base + i, out);
}
__device__ inline void publish_value(__amdgpu_buffer_rsrc_t, float2 *base, int i, float2 v) { publish(base + i, v); }

__device__ inline unsigned ld_ctl(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_group_gate(int ntask, int nlev, const int *lptr, const int4 *lslot, int lag, int *gate) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask) return;
    const int idx = t * GRP_ROWS;
    // level of slot idx: the last l with lptr[l] <= idx
    int lo = 0, hi = nlev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lptr[mid] <= idx) lo = mid;
        else hi = mid - 1;
    }
    const int g = lo - lag;
    gate[t] = (lag > 0 && g >= 0) ? lslot[lptr[g + 1] - 1].x : -1;
}

// lslot: the level schedule's slots -- lower {row, rowptr, diag, rowptr+1},
// upper {row, diag+1, rowptr+1, 0}: the row's entries are [y, z) of the CSR
template <typename T, bool UPPER>
__global__ void __launch_bounds__(GRP_WPB * 64)
    k_trsv_groups(int n, int ntask, const int4 *lslot, const int *gate, const int *col, const T *val, T *in, T *out,
                  T *reset, unsigned *ctl, unsigned nwaves, unsigned *status, const int *skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    const int r = lane / GRP, k = lane % GRP;
    const __amdgpu_buffer_rsrc_t orsrc = buffer_of(out);

    // ---- arrival: static round-robin order only if every wavefront runs
    unsigned ticket = 0;
    if (lane == 0) {
        ticket = atomicAdd(ctl + CTL_ARRIVE, 1u);
        if (ticket == nwaves - 1) atomicCAS(ctl + CTL_MODE, 0u, (unsigned)MODE_STATIC);
    }
    ticket = __shfl(ticket, 0, 64);
    unsigned mode = 0;
    if (lane == 0) {
        // wait while wavefronts keep arriving; a stall of GRP_ARRIVE_TICKS
        // means some cannot become resident now
        long long t0 = wall_clock64();
        unsigned seen = 0;
        while ((mode = ld_ctl(ctl + CTL_MODE)) == 0) {
            const unsigned a = ld_ctl(ctl + CTL_ARRIVE);
            const long long now = wall_clock64();
            if (a != seen) {
                seen = a;
                t0 = now;
            } else if (now - t0 > GRP_ARRIVE_TICKS) {
                atomicCAS(ctl + CTL_MODE, 0u, (unsigned)MODE_DYNAMIC);
                mode = ld_ctl(ctl + CTL_MODE);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    mode = __shfl(mode, 0, 64);
    auto next_dynamic = [&]() -> unsigned {
        unsigned v = 0;
        if (lane == 0) v = atomicAdd(ctl + CTL_TASK, 1u);
        return __shfl(v, 0, 64);
    };
    unsigned t = (mode == MODE_STATIC) ? ticket : next_dynamic();

    while (t < (unsigned)ntask) {
        const int idx = (int)t * GRP_ROWS + r;
        const bool active = idx < n;
        int row = 0, start = 0, len = 0;
        if (active) {
            const int4 sl = gld(lslot + idx);
            row = sl.x;
            start = sl.y;
            len = sl.z - sl.y;
        }
        // the lanes' first chunk of entries, loaded before the gate
        int q0 = 0;  // first entry of the current chunk
        bool ok = true, gdone = !active;
        int c = 0;
        T v = czero<T>(), p = czero<T>();
        if (active && k < len) {
            ok = false;
            c = gld(col + start + k);
            v = gld(val + start + k);
        }
        T acc = czero<T>(), piv = czero<T>();
        if (active && k == 0) {
            acc = gld(in + row);
            if (UPPER) {
                piv = gld(val + start - 1);
                set_sentinel(in + row);  // the lower result goes back to the sentinel
            }
            if (reset) set_sentinel(reset + row);
        }
        const int g = gld(gate + t);
        if (g >= 0) {
            T gv;
            unsigned gs = 0;
            while (!poll_value(orsrc, out, g, gv)) {
                if (++gs > GRP_GATE_SPINS) break;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        unsigned spins = 0;
        while (true) {
            if (!ok) {
                T yv;
                if (poll_value(orsrc, out, c, yv)) {
                    ok = true;
                    p = cmul(v, yv);
                }
            }
            const unsigned long long bal = __ballot(ok || gdone);
            const bool gready = !gdone && ((bal >> (r * GRP)) & 0xffffull) == 0xffffull;
            if (__any(gready)) {
                // the owner subtracts the chunk's products in entry order
#pragma unroll
                for (int kk = 0; kk < GRP; ++kk) {
                    T q;
                    q.x = __shfl(p.x, r * GRP + kk, 64);
                    q.y = __shfl(p.y, r * GRP + kk, 64);
                    if (gready && k == 0 && q0 + kk < len) acc = csub(acc, q);
                }
                if (gready) {
                    q0 += GRP;
                    spins = 0;
                    if (q0 >= len) {
                        if (k == 0) publish_value(orsrc, out, row, UPPER ? cdiv(acc, piv) : acc);
                        gdone = true;
                    } else if (q0 + k < len) {
                        ok = false;
                        c = gld(col + start + q0 + k);
                        v = gld(val + start + q0 + k);
                    }
                }
            }
            if (__all(gdone)) break;
            if (!gdone) {
                ++spins;
                if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
                    // give up on this row: flag the failure, publish what there is
                    if (k == 0) {
                        atomicOr(status, STATUS_SPIN_TIMEOUT);
                        publish_value(orsrc, out, row, acc);
                    }
                    gdone = true;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        t = (mode == MODE_STATIC) ? t + nwaves : next_dynamic();
    }
    // the last wavefront out resets the control words for the next launch
    if (lane == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (atomicAdd(ctl + CTL_EXIT, 1u) == nwaves - 1) {
            for (int i = 0; i < 4; ++i) __hip_atomic_store(ctl + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

void group_gates(const LevelSched &ls, int n, DevBuf<int> &gate, hipStream_t s) {
    const int ntask = div_up(n, GRP_ROWS);
    gate.resize((size_t)std::max(ntask, 1));
    if (n == 0) return;
    k_group_gate<<<div_up(ntask, 256), 256, 0, s>>>(ntask, ls.nlev, ls.ptr.get(), ls.slot.get(), GRP_LAG, gate.get());
    SS_HIP(hipGetLastError());
}

template <typename T>
void trsv_groups(const LevelSched &ls, const int *gate, bool upper, const Csr<T> &LU, const T *in, T *out, T *reset,
                 unsigned *ctl, unsigned *status, const int *skip, hipStream_t s) {
    const int n = LU.n;
    if (n == 0) return;
    const int ntask = div_up(n, GRP_ROWS);
    const int waves = std::min(ntask, GROUP_WAVES);
    const unsigned blocks = (unsigned)div_up(waves, GRP_WPB);
    const unsigned nwaves = blocks * GRP_WPB;
    if (upper)
        k_trsv_groups<T, true><<<blocks, GRP_WPB * 64, 0, s>>>(n, ntask, ls.slot.get(), gate, LU.col, LU.val,
                                                                const_cast<T *>(in), out, reset, ctl, nwaves,
                                                                status, skip);
    else
        k_trsv_groups<T, false><<<blocks, GRP_WPB * 64, 0, s>>>(n, ntask, ls.slot.get(), gate, LU.col, LU.val,
                                                                 const_cast<T *>(in), out, reset, ctl, nwaves,
                                                                 status, skip);
    SS_HIP(hipGetLastError());
}
template void trsv_groups<double2>(const LevelSched &, const int *, bool, const Csr<double2> &, const double2 *,
                                   double2 *, double2 *, unsigned *, unsigned *, const int *, hipStream_t);
template void trsv_groups<float2>(const LevelSched &, const int *, bool, const Csr<float2> &, const float2 *,
                                  float2 *, float2 *, unsigned *, unsigned *, const int *, hipStream_t);

}  // namespace ss
