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
//  * The visit's dependency graph (each vertex after its earlier
//    neighbours) is walked frontier by frontier: k_colour_init counts each
//    vertex's earlier neighbours; k_colour_front colours a frontier (every
//    earlier neighbour done) and counts each vertex off at its later
//    neighbours, those reaching zero forming the next frontier.  Each edge
//    is looked at a bounded number of times, and the frontiers are few: the
//    graph of a random order is shallow (62 levels on the Kerr chain at
//    n = 10^6, against ~4000 for the RCM order).  Colours past 63 (dense
//    rows only) are found by the wavefront together through a bitmap in
//    LDS; up to 4096 colours are supported.  The frontier launches have a
//    fixed grid and read their frontier's size on the device, so the host
//    queues them in batches and reads one count per batch.
//  * bucket_sort puts the vertices in (colour, RCM position) order.
#include "bucket.hpp"
#include "rcm.hpp"
#include "start.hpp"
#include "syncfree.hpp"

namespace ss {

namespace {

constexpr int COL_MAX = 4096;    // colours the ordering supports
constexpr int COL_BS = 256;
constexpr int FRONT_G = 4;       // lanes per vertex in a frontier launch (1 to 32 measured: 4 best)
constexpr int FRONT_GRID = 2048;  // workgroups of a frontier launch (grid-stride over the frontier)
constexpr int FRONT_BATCH = 16;   // frontier launches queued per host read

__device__ inline int ld_colour(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// visit priority of vertex v: output v of SplitMix64 seeded with 0; u comes
// before v in the visit when (priority, index) is smaller
__device__ inline uint64_t priority(int v) { return splitmix64((uint64_t)v * 0x9E3779B97F4A7C15ull); }
__device__ inline bool visits_before(int u, uint64_t ku, int v, uint64_t kv) {
    return ku < kv || (ku == kv && u < v);
}

// orders the LDS accesses of one wavefront (no other wavefront takes part)
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// appends the lanes with `take` set to list[*count ...] (one atomic per
// wavefront); an append past cap entries is dropped and flagged
__device__ inline void append(bool take, int v, int *list, int *count, int cap, unsigned *status) {
    const int lane = threadIdx.x & 63;
    const unsigned long long b = __ballot(take);
    int at = 0;
    if (lane == 0 && b) at = atomicAdd(count, __popcll(b));
    at = __shfl(at, 0, 64) + __popcll(b & ((1ull << lane) - 1ull));
    if (take) {
        if (at < cap) list[at] = v;
        else atomicOr(status, STATUS_OVERFLOW);
    }
}

// largest value over the wavefront
__device__ inline int wave_max(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}

// cnt[v] = neighbours visited before v; vertices with none start the frontier
__global__ void __launch_bounds__(COL_BS) k_colour_init(int n, const int *rowptr, const int *col, int *colour,
                                                        int *cnt, int *front, int *nfront, unsigned *status) {
    const int v = blockIdx.x * COL_BS + threadIdx.x;
    int c = 0;
    if (v < n) {
        const uint64_t kv = priority(v);
        for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            const int u = col[e];
            if (u != v && visits_before(u, priority(u), v, kv)) ++c;
        }
        cnt[v] = c;
        colour[v] = -1;
    }
    append(v < n && c == 0, v, front, nfront, n, status);
}

// Frontier k of the walk: every listed vertex has all its earlier
// neighbours coloured (in earlier launches).  It takes the lowest colour none
// of them carries, then counts itself off at each later neighbour; a
// neighbour whose count reaches zero joins the next frontier.  A group of
// FRONT_G lanes takes one vertex, its row entries dealt out over the lanes,
// so that several count-off atomics of a row are in flight together (they,
// not the row walks, bound the launch); colours from 64 on
// (dense rows only) are found by the wavefront together through a bitmap in
// LDS.  The frontier sizes rotate through three counters: launch k reads
// counter k mod 3, appends to counter k+1 mod 3 and clears counter k+2 mod 3
// (read by no launch before k+2 appends to it); the lists alternate between
// two buffers.  A launch whose frontier is empty does nothing, so the host
// may queue more launches than there are frontiers.
__global__ void __launch_bounds__(COL_BS) k_colour_front(int k, int n, int *list_a, int *list_b, const int *rowptr,
                                                         const int *col, int *colour, int *cnt, int *ctr,
                                                         unsigned *status) {
    __shared__ unsigned long long bm[COL_BS / 64][COL_MAX / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane & (FRONT_G - 1);
    const int m = ctr[k % 3];
    const int *front = (k & 1) ? list_b : list_a;
    int *next = (k & 1) ? list_a : list_b;
    int *nnext = ctr + (k + 1) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctr[(k + 2) % 3] = 0;
        ctr[3] += m;  // vertices listed so far (one writer per launch, launches in stream order)
    }
    constexpr int ROWS = COL_BS / FRONT_G;  // vertices per workgroup and pass
    for (int base = blockIdx.x * ROWS; base < m; base += gridDim.x * ROWS) {
        const int t = base + (int)threadIdx.x / FRONT_G;
        const bool active = t < m;  // (the whole group)
        int v = 0, e0 = 0, e1 = 0;
        uint64_t kv = 0;
        if (active) {
            v = front[t];
            kv = priority(v);
            e0 = rowptr[v];
            e1 = rowptr[v + 1];
        }
        // colours of the earlier neighbours below 64, OR-ed over the group
        unsigned long long taken = 0;
        for (int c0 = 0;; c0 += FRONT_G) {
            const bool more = active && e0 + c0 < e1;
            if (!__any(more)) break;
            const int e = e0 + c0 + g;
            if (more && e < e1) {
                const int u = col[e];
                if (u != v && visits_before(u, priority(u), v, kv)) {
                    const int c = colour[u];
                    if (c < 64) taken |= 1ull << c;
                }
            }
        }
        for (int o = FRONT_G / 2; o > 0; o >>= 1) taken |= __shfl_xor(taken, o, 64);
        int mine = (active && ~taken) ? __builtin_ctzll(~taken) : -1;
        // colours 0..63 all taken: the wavefront scans each such row into a
        // bitmap of COL_MAX colours (the group's first lane keeps the result)
        unsigned long long slow = __ballot(active && g == 0 && !~taken);
        while (slow) {
            const int L = __ffsll((long long)slow) - 1;
            slow &= slow - 1;
            const int vv = __shfl(v, L, 64);
            const uint64_t kk = priority(vv);
            const int a = rowptr[vv], b = rowptr[vv + 1];
            bm[wave][lane] = 0;
            wave_sync();
            bool over = false;
            for (int f = a + lane; f < b; f += 64) {
                const int u = col[f];
                if (u == vv || !visits_before(u, priority(u), vv, kk)) continue;
                const int cc = colour[u];
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
                    mine = COL_MAX;
                } else {
                    const int word = __ffsll((long long)open) - 1;
                    mine = word * 64 + __builtin_ctzll(~bm[wave][word]);
                }
            }
            wave_sync();
        }
        if (active && g == 0) colour[v] = mine;
        // one atomic per wavefront for the colour count
        const int top = wave_max(g == 0 ? mine : -1);
        if (lane == 0 && top >= 0) atomicMax(ctr + 4, top + 1);
        // count off at the later neighbours, one row entry per lane
        for (int c0 = 0;; c0 += FRONT_G) {
            const bool more = active && e0 + c0 < e1;
            if (!__any(more)) break;
            const int e = e0 + c0 + g;
            bool ready = false;
            int w = 0;
            if (more && e < e1) {
                w = col[e];
                if (w != v && visits_before(v, kv, w, priority(w))) ready = atomicSub(cnt + w, 1) == 1;
            }
            append(ready, w, next, nnext, n, status);
        }
    }
}

__global__ void k_gather_int(int n, const int *idx, const int *in, int *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[p] = in[idx[p]];
}

}  // namespace

int colour_order(const CsrBuf<double2> &S, const DevBuf<int> &base_perm, const DevBuf<int> &base_iperm,
                 DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s, std::vector<int> *class_ptr) {
    (void)base_iperm;
    const int n = S.n;
    perm.resize((size_t)std::max(n, 1));
    iperm.resize((size_t)std::max(n, 1));
    if (n == 0) return 0;
    DevBuf<int> colour((size_t)n), cnt((size_t)n), la((size_t)n), lb((size_t)n), ctr(5);
    DevBuf<unsigned> status(1);
    // [0..2] frontier sizes (rotating), [3] vertices listed, [4] colours
    SS_HIP(hipMemsetAsync(ctr.get(), 0, 5 * sizeof(int), s));
    SS_HIP(hipMemsetAsync(status.get(), 0, sizeof(unsigned), s));
    k_colour_init<<<div_up(n, COL_BS), COL_BS, 0, s>>>(n, S.rowptr.get(), S.col.get(), colour.get(), cnt.get(),
                                                       la.get(), ctr.get(), status.get());
    SS_HIP(hipGetLastError());
    // each frontier is one level of the visit's dependency graph; the
    // launches are queued FRONT_BATCH at a time and the host reads the size
    // of the next frontier after each batch
    const int grid = std::min(div_up((int64_t)n * FRONT_G, COL_BS), FRONT_GRID);
    int k = 0, m = 0;
    for (;;) {
        for (int b = 0; b < FRONT_BATCH; ++b, ++k) {
            k_colour_front<<<grid, COL_BS, 0, s>>>(k, n, la.get(), lb.get(), S.rowptr.get(), S.col.get(),
                                                   colour.get(), cnt.get(), ctr.get(), status.get());
            SS_HIP(hipGetLastError());
        }
        d2h(&m, ctr.get() + k % 3, 1, s);
        if (m == 0) break;
        // every non-empty frontier colours at least one vertex
        SS_REQUIRE(k <= n, SS_E_HIP, "greedy colouring: the frontier walk did not end");
    }
    int listed = 0, C = 0;
    unsigned st = 0;
    d2h(&listed, ctr.get() + 3, 1, s);
    d2h(&C, ctr.get() + 4, 1, s);
    d2h(&st, status.get(), 1, s);
    SS_REQUIRE(!(st & STATUS_OVERFLOW), SS_E_INVALID_ARG, "colour order: more than 4096 colours");
    SS_REQUIRE(listed == n, SS_E_HIP, "greedy colouring: vertices left uncoloured or listed twice");
    SS_REQUIRE(C >= 1 && C <= n, SS_E_HIP, "greedy colouring: colour count out of range");
    // colours by RCM position, then the classes in RCM order
    DevBuf<int> cpos((size_t)n);
    k_gather_int<<<div_up(n, 256), 256, 0, s>>>(n, base_perm.get(), colour.get(), cpos.get());
    SS_HIP(hipGetLastError());
    DevBuf<int> starts((size_t)C + 1);
    bucket_sort(n, cpos.get(), C, base_perm.get(), perm.get(), iperm.get(), starts.get(), s);
    if (class_ptr) {
        class_ptr->resize((size_t)C + 1);
        d2h(class_ptr->data(), starts.get(), (size_t)C + 1, s);
    }
    return C;
}

}  // namespace ss
