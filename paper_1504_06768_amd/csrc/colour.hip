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
// The colouring is the sequential greedy one visited in a seeded random
// order: vertex v has priority SplitMix64(v) (output v of the generator
// seeded with 0; ties by index), and each vertex takes the smallest colour
// that no neighbour of higher priority -- earlier in the visit -- carries.
// The classes then follow in increasing colour, each in RCM order.  Both
// steps give the same result as their sequential definitions, bit for bit:
//  * k_colour_round, repeated until every vertex is coloured: a listed
//    vertex walks its row from where it stopped, eight entries at a time,
//    collecting the colours of its earlier neighbours, and stops at the
//    first one still uncoloured (it is listed for the next round).  A vertex
//    that reaches the end of its row is final.  The priority graph of a
//    random order is shallow (62 levels on the Kerr chain at n = 10^6,
//    against ~4000 for the RCM order), so the rounds are few.  Colours past
//    63 (dense rows only) are found by the wavefront together through a
//    bitmap in LDS; up to 4096 colours are supported.
//  * bucket_sort puts the vertices in (colour, RCM position) order.
#include "bucket.hpp"
#include "rcm.hpp"
#include "start.hpp"
#include "syncfree.hpp"

namespace ss {

namespace {

constexpr int COL_PASS = 8;      // row entries examined per pass
constexpr int COL_MAX = 4096;    // colours the ordering supports
constexpr int COL_BS = 256;

__device__ inline int ld_colour(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_colour(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// visit priority of vertex v: output v of SplitMix64 seeded with 0
__global__ void k_priorities(int n, const int *rowptr, uint64_t *key, int *colour, int *cursor,
                             unsigned long long *taken) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = splitmix64((uint64_t)v * 0x9E3779B97F4A7C15ull);
    colour[v] = -1;
    cursor[v] = rowptr[v];
    taken[v] = 0;
}

// orders the LDS accesses of one wavefront (no other wavefront takes part)
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One round over the m listed vertices (list == nullptr: all vertices).
// cursor[v] / taken[v] keep where a vertex stopped and the colours below 64
// its earlier neighbours carry, so a row is read once over all rounds.
__global__ void __launch_bounds__(COL_BS) k_colour_round(int m, const int *list, const int *rowptr, const int *col,
                                                         const uint64_t *key, int *colour, int *cursor,
                                                         unsigned long long *taken, int *next, int *nnext,
                                                         int *ncol, unsigned *status) {
    __shared__ unsigned long long bm[COL_BS / 64][COL_MAX / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.x * COL_BS + threadIdx.x;
    const bool active = t < m;
    int v = 0, e = 0, e1 = 0;
    uint64_t kv = 0;
    unsigned long long tk = 0;
    if (active) {
        v = list ? list[t] : t;
        kv = key[v];
        e = cursor[v];
        e1 = rowptr[v + 1];
        tk = taken[v];
    }
    bool blocked = false;
    // a vertex listed again first looks only at the neighbour that stopped it
    if (list && active && e < e1 && ld_colour(colour + col[e]) < 0) blocked = true;
    while (active && !blocked && e < e1) {
        int c[COL_PASS];
#pragma unroll
        for (int q = 0; q < COL_PASS; ++q) {
            c[q] = 0x7fffffff;  // later in the visit, or v itself: no constraint
            if (e + q < e1) {
                const int u = col[e + q];
                if (u != v) {
                    const uint64_t ku = key[u];
                    if (ku < kv || (ku == kv && u < v)) c[q] = ld_colour(colour + u);
                }
            }
        }
        int used = 0;
#pragma unroll
        for (int q = 0; q < COL_PASS; ++q) {
            if (!blocked && e + q < e1) {
                if (c[q] < 0) {
                    blocked = true;
                } else {
                    if (c[q] < 64) tk |= 1ull << c[q];
                    ++used;
                }
            }
        }
        e += used;
    }
    // blocked vertices go to the next round's list: one atomic per wavefront
    const unsigned long long bl = __ballot(blocked);
    int at = 0;
    if (lane == 0 && bl) at = atomicAdd(nnext, __popcll(bl));
    at = __shfl(at, 0, 64) + __popcll(bl & ((1ull << lane) - 1ull));
    if (blocked) {
        cursor[v] = e;
        taken[v] = tk;
        next[at] = v;
    } else if (active && ~tk) {
        const int mine = __builtin_ctzll(~tk);
        st_colour(colour + v, mine);
        atomicMax(ncol, mine + 1);
    }
    // colours 0..63 all taken: the wavefront scans each such row into a
    // bitmap of COL_MAX colours (every earlier neighbour is coloured)
    unsigned long long slow = __ballot(active && !blocked && !~tk);
    while (slow) {
        const int L = __ffsll((long long)slow) - 1;
        slow &= slow - 1;
        const int vv = __shfl(v, L, 64);
        const uint64_t kk = ((uint64_t)__shfl((unsigned)(kv >> 32), L, 64) << 32) | (unsigned)__shfl((unsigned)kv, L, 64);
        const int a = rowptr[vv], b = rowptr[vv + 1];
        bm[wave][lane] = 0;
        wave_sync();
        bool over = false;
        for (int f = a + lane; f < b; f += 64) {
            const int u = col[f];
            if (u == vv) continue;
            const uint64_t ku = key[u];
            if (!(ku < kk || (ku == kk && u < vv))) continue;
            const int cc = ld_colour(colour + u);
            if (cc >= 0 && cc < COL_MAX) atomicOr(&bm[wave][cc >> 6], 1ull << (cc & 63));
            else over = true;
        }
        wave_sync();
        const unsigned long long w = bm[wave][lane];
        const unsigned long long open = __ballot(~w != 0);
        const bool overflow = __any(over) || open == 0;
        if (lane == L) {
            if (overflow) {
                atomicOr(status, STATUS_OVERFLOW);  // more colours than supported: the host rejects
                st_colour(colour + v, COL_MAX);
            } else {
                const int word = __ffsll((long long)open) - 1;
                const int mine = word * 64 + __builtin_ctzll(~bm[wave][word]);
                st_colour(colour + v, mine);
                atomicMax(ncol, mine + 1);
            }
        }
        wave_sync();
    }
}

__global__ void k_gather_int(int n, const int *idx, const int *in, int *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[p] = in[idx[p]];
}

}  // namespace

int colour_order(const CsrBuf<double2> &S, const DevBuf<int> &base_perm, const DevBuf<int> &base_iperm,
                 DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s) {
    (void)base_iperm;
    const int n = S.n;
    perm.resize((size_t)std::max(n, 1));
    iperm.resize((size_t)std::max(n, 1));
    if (n == 0) return 0;
    DevBuf<uint64_t> key((size_t)n);
    DevBuf<unsigned long long> taken((size_t)n);
    DevBuf<int> colour((size_t)n), cursor((size_t)n), la((size_t)n), lb((size_t)n), cnt(2);
    DevBuf<unsigned> status(1);
    k_priorities<<<div_up(n, 256), 256, 0, s>>>(n, S.rowptr.get(), key.get(), colour.get(), cursor.get(),
                                                taken.get());
    SS_HIP(hipMemsetAsync(cnt.get(), 0, 2 * sizeof(int), s));  // [0] listed for the next round, [1] colours
    SS_HIP(hipMemsetAsync(status.get(), 0, sizeof(unsigned), s));
    SS_HIP(hipGetLastError());
    // every round colours at least the listed vertex of highest priority
    int m = n;
    const int *list = nullptr;
    int *out = la.get(), *spare = lb.get();
    for (int round = 0; m > 0; ++round) {
        SS_REQUIRE(round <= n, SS_E_HIP, "greedy colouring: no progress");
        k_colour_round<<<div_up(m, COL_BS), COL_BS, 0, s>>>(m, list, S.rowptr.get(), S.col.get(), key.get(),
                                                           colour.get(), cursor.get(), taken.get(), out, cnt.get(),
                                                           cnt.get() + 1, status.get());
        SS_HIP(hipGetLastError());
        int left = 0;
        d2h(&left, cnt.get(), 1, s);
        SS_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int), s));
        m = left;
        list = out;
        std::swap(out, spare);
    }
    int C = 0;
    unsigned st = 0;
    d2h(&C, cnt.get() + 1, 1, s);
    d2h(&st, status.get(), 1, s);
    SS_REQUIRE(!(st & STATUS_OVERFLOW), SS_E_INVALID_ARG, "colour order: more than 4096 colours");
    SS_REQUIRE(C >= 1 && C <= n, SS_E_HIP, "greedy colouring: colour count out of range");
    // colours by RCM position, then the classes in RCM order
    DevBuf<int> cpos((size_t)n);
    k_gather_int<<<div_up(n, 256), 256, 0, s>>>(n, base_perm.get(), colour.get(), cpos.get());
    SS_HIP(hipGetLastError());
    bucket_sort(n, cpos.get(), C, base_perm.get(), perm.get(), iperm.get(), nullptr, s);
    return C;
}

}  // namespace ss
