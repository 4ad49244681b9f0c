// Colour-class ordering on the device.
//
// Not a step of the paper.  The forward and backward substitutions of the
// ILU preconditioner (section "Iterative Solvers") in RCM order (section
// "Direct factorization") form chains of about a thousand dependent rows on
// the largest workloads, and a substitution costs the length of its chain
// times the time one row's result takes to reach the next.  Numbering the
// unknowns class by class for a proper colouring of the structure of
// A + A^T puts every off-diagonal entry between two different classes, so
// a zero-fill factor has at most as many levels as there are colours, each
// level holding a whole class.  The price is a weaker preconditioner (more
// Krylov iterations), which the much cheaper substitutions repay.
//
// The colouring is the sequential greedy one visited in RCM order: each
// vertex takes the smallest colour no earlier neighbour carries.  The
// classes then follow in increasing colour, each in RCM order.  Both steps
// give the same result as their sequential definitions, bit for bit:
//  * k_earlier lists, for each position of the RCM order, the positions of
//    its earlier neighbours; the colouring then works in position space.
//  * k_greedy_colour: sixteen lanes per vertex, persistent wavefronts taking
//    four consecutive positions at a time from an atomic counter.  A vertex
//    waits only for its earlier neighbours (data-as-flag: colours start at
//    -1).  Colours past 63 (dense rows only) go through a bitmap in LDS; up
//    to 4096 colours are supported.
//  * bucket_sort puts the positions in (colour, position) order, so the
//    order inside a class is the RCM order.
#include "bucket.hpp"
#include "rcm.hpp"
#include "syncfree.hpp"

namespace ss {

namespace {

constexpr int COL_GRP = 16;                 // lanes per vertex
constexpr int COL_VPW = 64 / COL_GRP;       // vertices per wavefront task
constexpr int COL_WAVES = 2048;             // resident wavefronts
constexpr int COL_GATE = 4096;              // positions between a task and its gate
constexpr unsigned COL_GATE_SPINS = 1u << 16;
constexpr int COL_MAX = 4096;               // colours the ordering supports

__device__ inline int ld_colour(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_colour(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fill(int n, int *p, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Earlier neighbours in position space: for the vertex at position p of the
// base order, the positions q < p of its neighbours (self-loops dropped).
// One group of 16 lanes per position, four per wavefront.
template <bool FILL>
__global__ void __launch_bounds__(256) k_earlier(int n, const int *order, const int *pos_of, const int *rowptr,
                                                 const int *col, const int *erow, int *out) {
    const int lane = threadIdx.x & 63, r = lane / COL_GRP, k = lane % COL_GRP;
    const int p = (blockIdx.x * 4 + (threadIdx.x >> 6)) * COL_VPW + r;
    const bool active = p < n;
    int e0 = 0, e1 = 0, at = 0, cnt = 0;
    if (active) {
        const int v = order[p];
        e0 = rowptr[v];
        e1 = rowptr[v + 1];
        if (FILL) at = erow[p];
    }
    const unsigned long long gmask = 0xffffull << (r * COL_GRP);
    // every group walks its row in chunks of 16; the wavefront loops while any does
    for (int base = 0;; base += COL_GRP) {
        const bool more = active && e0 + base < e1;
        if (!__any(more)) break;
        int q = -1;
        if (more && e0 + base + k < e1) {
            const int u = col[e0 + base + k];
            const int qu = pos_of[u];
            if (qu < p) q = qu;  // (a self-loop has qu == p)
        }
        const unsigned long long bal = __ballot(q >= 0) & gmask;
        if (FILL && q >= 0) out[at + cnt + __popcll(bal & ((1ull << lane) - 1ull))] = q;
        cnt += __popcll(bal);
    }
    if (!FILL && active && k == 0) out[p] = cnt;
}

// The greedy colouring over the earlier-neighbour lists (position space).
// Persistent wavefronts take tasks of four consecutive positions in order
// from an atomic counter, so every position waited on belongs to a running
// wavefront.  Each lane of a vertex's group polls one earlier neighbour's
// colour (data-as-flag, -1 until set) and keeps the colours below 64 it has
// seen as bits; when the group has seen its whole list the bits are OR-ed
// across the group and the vertex takes the lowest free colour.  Colours
// from 64 on (dense rows only) are found through a bitmap of COL_MAX colours
// in LDS.  A task first waits for the vertex COL_GATE positions before it,
// which keeps the polling near the frontier.
__global__ void __launch_bounds__(64) k_greedy_colour(int n, int ntask, const int *erow, const int *ecol, int *colour,
                                                      unsigned *ctr, unsigned *status, int *ncol) {
    __shared__ unsigned long long bm[COL_VPW][COL_MAX / 64];
    const int lane = threadIdx.x, r = lane / COL_GRP, k = lane % COL_GRP;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(ctr, 1u);
        t = __shfl(t, 0, 64);
        if (t >= (unsigned)ntask) break;
        const int p = (int)t * COL_VPW + r;
        const bool active = p < n;
        int start = 0, len = 0;
        if (active) {
            start = erow[p];
            len = erow[p + 1] - start;
        }
        const int g = (int)t * COL_VPW - COL_GATE;
        if (g >= 0) {
            for (unsigned gs = 0;; ++gs) {
                const int cg = lane == 0 ? ld_colour(colour + g) : 0;
                if (__shfl(cg, 0, 64) >= 0 || gs > COL_GATE_SPINS) break;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        unsigned long long seen = 0;  // colours < 64 seen by this lane
        int q0 = 0, c = 0;
        bool ok = true, gdone = !active;
        if (active && k < len) {
            ok = false;
            c = ecol[start + k];
        }
        unsigned spins = 0;
        for (;;) {
            if (!ok) {
                const int cc = ld_colour(colour + c);
                if (cc >= 0) {
                    ok = true;
                    if (cc < 64) seen |= 1ull << cc;
                }
            }
            const unsigned long long bal = __ballot(ok || gdone);
            const bool gready = !gdone && ((bal >> (r * COL_GRP)) & 0xffffull) == 0xffffull;
            if (__any(gready)) {
                bool fin = false;
                if (gready) {
                    q0 += COL_GRP;
                    spins = 0;
                    if (q0 >= len) {
                        fin = true;
                    } else if (q0 + k < len) {
                        ok = false;
                        c = ecol[start + q0 + k];
                    }
                }
                // the group's bits, OR-ed across its 16 lanes
                unsigned long long all = seen;
#pragma unroll
                for (int off = 1; off < COL_GRP; off <<= 1) {
                    const unsigned lo = __shfl_xor((unsigned)all, off, 64);
                    const unsigned hi = __shfl_xor((unsigned)(all >> 32), off, 64);
                    all |= ((unsigned long long)hi << 32) | lo;
                }
                if (fin && ~all) {
                    if (k == 0) {
                        const int mine = __builtin_ctzll(~all);
                        st_colour(colour + p, mine);
                        atomicMax(ncol, mine + 1);
                    }
                    gdone = true;
                } else if (fin) {
                    // colours 0..63 all taken: the whole list once more into
                    // the LDS bitmap (every entry is coloured by now)
                    for (int w = k; w < COL_MAX / 64; w += COL_GRP) bm[r][w] = 0;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    bool over = false;
                    for (int f = k; f < len; f += COL_GRP) {
                        const int cc = ld_colour(colour + ecol[start + f]);
                        if (cc >= 0 && cc < COL_MAX) atomicOr(&bm[r][cc >> 6], 1ull << (cc & 63));
                        else over = true;
                    }
                    if (over) atomicOr(status, STATUS_OVERFLOW);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (k == 0) {
                        int mine = COL_MAX;
                        for (int w = 0; w < COL_MAX / 64; ++w) {
                            const unsigned long long x = bm[r][w];
                            if (~x) {
                                mine = w * 64 + __builtin_ctzll(~x);
                                break;
                            }
                        }
                        if (mine >= COL_MAX) atomicOr(status, STATUS_OVERFLOW);  // the host rejects
                        st_colour(colour + p, mine);
                        atomicMax(ncol, mine + 1);
                    }
                    gdone = true;
                }
            }
            if (__all(gdone)) break;
            if (!gdone) {
                ++spins;
                if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
                    if (k == 0) {
                        atomicOr(status, STATUS_SPIN_TIMEOUT);  // the host rejects the result
                        st_colour(colour + p, 0);
                    }
                    gdone = true;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

}  // namespace

int colour_order(const CsrBuf<double2> &S, const DevBuf<int> &base_perm, const DevBuf<int> &base_iperm,
                 DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s) {
    const int n = S.n;
    perm.resize((size_t)std::max(n, 1));
    iperm.resize((size_t)std::max(n, 1));
    if (n == 0) return 0;
    // earlier-neighbour lists in position space
    DevBuf<int> ecnt((size_t)n + 1), erow((size_t)n + 1);
    const unsigned eb = (unsigned)div_up(div_up(n, COL_VPW), 4);
    k_earlier<false><<<eb, 256, 0, s>>>(n, base_perm.get(), base_iperm.get(), S.rowptr.get(), S.col.get(), nullptr,
                                        ecnt.get());
    SS_HIP(hipGetLastError());
    const int64_t ne = scan_exclusive(ecnt.get(), erow.get(), n, s, true);
    DevBuf<int> ecol((size_t)std::max<int64_t>(ne, 1));
    k_earlier<true><<<eb, 256, 0, s>>>(n, base_perm.get(), base_iperm.get(), S.rowptr.get(), S.col.get(), erow.get(),
                                       ecol.get());
    SS_HIP(hipGetLastError());

    DevBuf<int> colour((size_t)n), ncol(1);
    DevBuf<unsigned> status(1), ctr(1);
    k_fill<<<div_up(n, 256), 256, 0, s>>>(n, colour.get(), -1);
    k_fill<<<1, 64, 0, s>>>(1, ncol.get(), 0);
    SS_HIP(hipMemsetAsync(status.get(), 0, sizeof(unsigned), s));
    SS_HIP(hipMemsetAsync(ctr.get(), 0, sizeof(unsigned), s));
    SS_HIP(hipGetLastError());
    const int ntask = div_up(n, COL_VPW);
    k_greedy_colour<<<std::min(ntask, COL_WAVES), 64, 0, s>>>(n, ntask, erow.get(), ecol.get(), colour.get(),
                                                              ctr.get(), status.get(), ncol.get());
    SS_HIP(hipGetLastError());
    int C = 0;
    unsigned st = 0;
    d2h(&C, ncol.get(), 1, s);
    d2h(&st, status.get(), 1, s);
    SS_REQUIRE(!(st & STATUS_SPIN_TIMEOUT), SS_E_HIP, "greedy colouring: a dependency wait timed out");
    SS_REQUIRE(!(st & STATUS_OVERFLOW), SS_E_INVALID_ARG, "colour order: more than 4096 colours");
    SS_REQUIRE(C >= 1 && C <= n, SS_E_HIP, "greedy colouring: colour count out of range");

    bucket_sort(n, colour.get(), C, base_perm.get(), perm.get(), iperm.get(), nullptr, s);
    SS_HIP(hipStreamSynchronize(s));
    return C;
}

}  // namespace ss
