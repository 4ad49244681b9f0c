// Reverse Cuthill-McKee ordering on the device (section "Direct
// factorization": BFS from a node of lowest degree, neighbours visited in
// increasing degree, per connected component, order reversed; computed on the
// structure of A + A^T and applied to rows and columns alike).
//
// The sequential queue search is reformulated level by level, which gives
// the same order: a node first reached from level k is queued by the
// frontier node that was dequeued first, i.e. the one at the lowest position
// in the order, and the children of one frontier node are queued by
// (degree, index).  So level k+1 is sorted by (parent position, degree,
// index) -- each frontier node claims its unvisited neighbours with an
// atomicMin on the position, counts and ranks the ones it owns, and an
// exclusive scan over the frontier gives every node its slot.
//
// Tie-breaks where the paper is silent: degree = graph degree in the
// symmetric pattern (stored row entries, a diagonal entry counted twice); a
// component starts at the unvisited node of lowest degree and highest index;
// equal-degree neighbours are queued in increasing index.
#include <climits>

#include "csr_tools.hpp"
#include "rcm.hpp"
#include "rowops.hpp"

namespace ss {

// --------------------------------------------------- symmetrised pattern
// One row per group of UNION_G lanes (union by shuffles); a row of A or A^T
// longer than that is merged by the group's first lane.
constexpr int UNION_G = 32;

template <bool FILL>
__global__ void __launch_bounds__(256) k_union_rows(int n, const int *ar, const int *ac, const int *br,
                                                    const int *bc, const int *orow, int *ocol, double2 *oval,
                                                    int *cnt) {
    const int r = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) / UNION_G);
    const int t = threadIdx.x & (UNION_G - 1);
    if (r >= n) return;  // (the whole group)
    const int as = ar[r], na = ar[r + 1] - as, bs = br[r], nb = br[r + 1] - bs;
    int *oc = nullptr;
    double2 *ov = nullptr;
    if (FILL) {
        oc = ocol + orow[r];
        ov = oval ? oval + orow[r] : nullptr;
    }
    int len = 0;
    if (na <= UNION_G && nb <= UNION_G) len = union_row_group<FILL, UNION_G>(as, na, bs, nb, ac, bc, oc, ov);
    else if (t == 0) len = union_row<FILL>(r, ar, ac, br, bc, oc, ov);
    if (!FILL && t == 0) cnt[r] = len;
}

void symmetrize_pattern(const CsrBuf<double2> &A, CsrBuf<double2> &S, hipStream_t s) {
    CsrBuf<double2> At;
    transpose(A, At, s, false);
    const int n = A.n;
    DevBuf<int> cnt((size_t)n + 1);
    const int grid = div_up((int64_t)n * UNION_G, 256);
    if (n) {
        k_union_rows<false><<<grid, 256, 0, s>>>(n, A.rowptr.get(), A.col.get(), At.rowptr.get(), At.col.get(),
                                                 nullptr, nullptr, nullptr, cnt.get());
        SS_HIP(hipGetLastError());
    }
    S.rowptr.resize((size_t)n + 1);
    const int64_t nnz = scan_exclusive(cnt.get(), S.rowptr.get(), n, s, true);
    SS_REQUIRE(nnz < (int64_t(1) << 31), SS_E_INVALID_ARG, "symmetrised pattern too large");
    S.n = n;
    S.nnz = (int)nnz;
    S.col.resize((size_t)nnz);
    S.val.resize((size_t)nnz);
    if (n) {
        k_union_rows<true><<<grid, 256, 0, s>>>(n, A.rowptr.get(), A.col.get(), At.rowptr.get(), At.col.get(),
                                                S.rowptr.get(), S.col.get(), S.val.get(), nullptr);
        SS_HIP(hipGetLastError());
    }
}

// ------------------------------------------------------------------ degree
__global__ void k_degree(int n, const int *rowptr, const int *col, int *deg) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int dg = rowptr[r + 1] - rowptr[r];
    int lo = rowptr[r], hi = rowptr[r + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = col[mid];
        if (c == r) { ++dg; break; }
        if (c < r) lo = mid + 1; else hi = mid - 1;
    }
    deg[r] = dg;
}

// start node: minimum of (degree, -index) over unvisited nodes
__global__ void k_pick_start(int n, const int *deg, const int *pos_of, unsigned long long *best) {
    unsigned long long b = ~0ull;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        if (pos_of[r] < 0) {
            const unsigned long long key = ((unsigned long long)(unsigned)deg[r] << 32) |
                                           (unsigned long long)(0xffffffffu - (unsigned)r);
            b = key < b ? key : b;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_down(b, off, 64);
        b = o < b ? o : b;
    }
    if ((threadIdx.x & 63) == 0 && b != ~0ull) atomicMin(best, b);
}

__global__ void k_place_start(unsigned long long *best, int *order, int *pos_of, int at) {
    const unsigned long long b = *best;
    const int r = (int)(0xffffffffu - (unsigned)(b & 0xffffffffull));
    order[at] = r;
    pos_of[r] = at;
    *best = ~0ull;
}

// one wavefront per frontier node
__global__ void __launch_bounds__(256) k_claim(int lo, int hi, const int *order, const int *rowptr, const int *col,
                                               const int *pos_of, int *owner) {
    const int lane = threadIdx.x & 63;
    const int p = lo + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= hi) return;
    const int u = order[p];
    for (int e = rowptr[u] + lane; e < rowptr[u + 1]; e += 64) {
        const int v = col[e];
        if (pos_of[v] < 0) atomicMin(&owner[v], p);
    }
}

__global__ void __launch_bounds__(256) k_count_owned(int lo, int hi, const int *order, const int *rowptr,
                                                     const int *col, const int *pos_of, const int *owner, int *cnt) {
    const int lane = threadIdx.x & 63;
    const int p = lo + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= hi) return;
    const int u = order[p];
    int c = 0;
    for (int e = rowptr[u] + lane; e < rowptr[u + 1]; e += 64) {
        const int v = col[e];
        c += (pos_of[v] < 0 && owner[v] == p);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if (lane == 0) cnt[p - lo] = c;
}

// Place the children a frontier node p owns (its unvisited neighbours whose
// claim it won), ordered by (degree, index), at order_out[base ...].  One
// wavefront per frontier node: each lane holds one row entry, and the rank
// of an owned entry is counted against the owned entries of every chunk of
// the row through cross-lane shuffles instead of re-reading the row.
template <bool ATOMIC_OWNER>
__device__ __forceinline__ void place_owned(int p, int rs, int re, int base, const int *col, const int *pos_of,
                                            const int *owner, const int *deg, int *order_out) {
    const int lane = threadIdx.x & 63;
    for (int c0 = rs; c0 < re; c0 += 64) {
        const int e = c0 + lane;
        int v = 0x7fffffff, dv = 0x7fffffff;
        bool own = false;
        if (e < re) {
            v = gld(col + e);
            const int ow = ATOMIC_OWNER ? __hip_atomic_load(owner + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                        : owner[v];
            own = pos_of[v] < 0 && ow == p;
            dv = deg[v];
        }
        if (__ballot(own) == 0) continue;  // nothing of this chunk to place
        int rank = 0;
        for (int c1 = rs; c1 < re; c1 += 64) {
            const int f = c1 + lane;
            int w = 0x7fffffff, dw = 0x7fffffff;
            bool ownw = false;
            if (c1 == c0) {
                w = v;
                dw = dv;
                ownw = own;
            } else if (f < re) {
                w = gld(col + f);
                const int ow = ATOMIC_OWNER
                                   ? __hip_atomic_load(owner + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                   : owner[w];
                ownw = pos_of[w] < 0 && ow == p;
                dw = deg[w];
            }
            if (!ownw) dw = 0x7fffffff;  // never ranks before anything
            const int cnt = min(64, re - c1);
            for (int k = 0; k < cnt; ++k) {
                const int wk = __shfl(w, k, 64);
                const int dk = __shfl(dw, k, 64);
                rank += (dk < dv) || (dk == dv && dk != 0x7fffffff && wk < v);
            }
        }
        if (own) order_out[base + rank] = v;
    }
}

__global__ void __launch_bounds__(256) k_place_children(int lo, int hi, int next, const int *order_in,
                                                        const int *rowptr, const int *col, const int *pos_of,
                                                        const int *owner, const int *deg, const int *offs,
                                                        int *order_out) {
    const int p = lo + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= hi) return;
    const int u = order_in[p];
    place_owned<false>(p, rowptr[u], rowptr[u + 1], next + offs[p - lo], col, pos_of, owner, deg, order_out);
}

__global__ void k_mark_level(int from, int to, const int *order, int *pos_of) {
    const int q = from + blockIdx.x * blockDim.x + threadIdx.x;
    if (q < to) pos_of[order[q]] = q;
}

__global__ void k_reverse(int n, const int *order, int *perm, int *iperm) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int v = order[n - 1 - q];
    perm[q] = v;
    iperm[v] = q;
}

__global__ void k_identity(int n, int *perm, int *iperm) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) { perm[q] = q; iperm[q] = q; }
}

__global__ void k_fill_int(int n, int *p, int v) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = v;
}

// ------------------------------------------------- single-workgroup form
// The same level-by-level search inside one workgroup (16 wavefronts, a
// barrier between the claim / count / scan / place / mark phases), for
// graphs small enough that launch and host round-trip latency would
// dominate the multi-kernel form.  owner[] is only changed by atomics and is
// read back with device-scope atomic loads.  With LDS set, the search state
// (degrees, positions, owners, the order and the frontier offsets: 5n + 1
// ints) lives in LDS and only the graph and the result are in memory; the
// graph is read with global loads, so that waiting for an LDS access never
// waits for them.
constexpr int RCM_BLOCK_T = 1024;

__device__ __forceinline__ int ld_owner(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
__global__ void __launch_bounds__(RCM_BLOCK_T) k_rcm_block(const RcmJob *jobs) {
    constexpr int NW = RCM_BLOCK_T / 64;
    extern __shared__ int rcm_lds[];
    const RcmJob &J = jobs[blockIdx.x];
    const int n = J.n;
    const int *rowptr = J.rowptr, *col = J.col;
    int *deg, *pos_of, *owner, *order, *offs;
    if (LDS) {
        deg = rcm_lds;
        pos_of = deg + n;
        owner = pos_of + n;
        order = owner + n;
        offs = order + n;
    } else {
        deg = J.deg;
        pos_of = J.pos_of;
        owner = J.owner;
        order = J.order;
        offs = J.offs;
    }
    int *perm = J.perm, *iperm = J.iperm;
    __shared__ unsigned long long sbest[NW];
    __shared__ int wsum[NW];
    __shared__ int s_total;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int r = tid; r < n; r += RCM_BLOCK_T) {
        pos_of[r] = -1;
        owner[r] = 0x7fffffff;
        const int rs = gld(rowptr + r), re = gld(rowptr + r + 1);
        int dg = re - rs;
        for (int e = rs; e < re; ++e) dg += (gld(col + e) == r);  // a self-loop counts twice
        deg[r] = dg;
    }
    __syncthreads();
    int visited = 0;
    while (visited < n) {
        // start node: minimum of (degree, -index) over the unvisited nodes
        unsigned long long key = ~0ull;
        for (int r = tid; r < n; r += RCM_BLOCK_T) {
            if (pos_of[r] < 0) {
                const unsigned long long k = ((unsigned long long)(unsigned)deg[r] << 32) |
                                             (unsigned long long)(0xffffffffu - (unsigned)r);
                key = k < key ? k : key;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_down(key, off, 64);
            key = o < key ? o : key;
        }
        if (lane == 0) sbest[wave] = key;
        __syncthreads();
        if (tid == 0) {
            unsigned long long b = sbest[0];
            for (int w = 1; w < NW; ++w) b = sbest[w] < b ? sbest[w] : b;
            const int r = (int)(0xffffffffu - (unsigned)(b & 0xffffffffull));
            order[visited] = r;
            pos_of[r] = visited;
        }
        __syncthreads();
        int lo = visited, hi = visited + 1;
        visited += 1;
        while (lo < hi) {
            const int width = hi - lo;
            // claim: each unvisited neighbour goes to the frontier node of lowest position
            for (int p = lo + wave; p < hi; p += NW) {
                const int u = order[p];
                const int ue = gld(rowptr + u + 1);
                for (int e = gld(rowptr + u) + lane; e < ue; e += 64) {
                    const int v = gld(col + e);
                    if (pos_of[v] < 0) atomicMin(&owner[v], p);
                }
            }
            __syncthreads();
            // count the children each frontier node owns
            for (int p = lo + wave; p < hi; p += NW) {
                const int u = order[p];
                const int ue = gld(rowptr + u + 1);
                int c = 0;
                for (int e = gld(rowptr + u) + lane; e < ue; e += 64) {
                    const int v = gld(col + e);
                    c += (pos_of[v] < 0 && ld_owner(owner + v) == p);
                }
                for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
                if (lane == 0) offs[p - lo] = c;
            }
            __syncthreads();
            // exclusive scan of the counts, in chunks of the workgroup size
            int carry = 0;
            for (int c0 = 0; c0 < width; c0 += RCM_BLOCK_T) {
                const int i = c0 + tid;
                const int v = (i < width) ? offs[i] : 0;
                int x = v;
                for (int off = 1; off < 64; off <<= 1) {
                    const int y = __shfl_up(x, off, 64);
                    if (lane >= off) x += y;
                }
                if (lane == 63) wsum[wave] = x;
                __syncthreads();
                int before = 0;
                for (int w = 0; w < wave; ++w) before += wsum[w];
                int chunk = 0;
                for (int w = 0; w < NW; ++w) chunk += wsum[w];
                if (i < width) offs[i] = carry + before + x - v;
                carry += chunk;
                __syncthreads();
            }
            if (tid == 0) s_total = carry;
            __syncthreads();
            const int total = s_total;
            // place the children of each frontier node by (degree, index)
            for (int p = lo + wave; p < hi; p += NW) {
                const int u = order[p];
                place_owned<true>(p, gld(rowptr + u), gld(rowptr + u + 1), hi + offs[p - lo], col, pos_of, owner, deg,
                                  order);
            }
            __syncthreads();
            for (int q = hi + tid; q < hi + total; q += RCM_BLOCK_T) pos_of[order[q]] = q;
            __syncthreads();
            lo = hi;
            hi += total;
            visited += total;
        }
    }
    for (int q = tid; q < n; q += RCM_BLOCK_T) {
        const int v = order[n - 1 - q];
        perm[q] = v;
        iperm[v] = q;
    }
}

bool rcm_batchable(int n) { return n <= RCM_BLOCK_MAX_N; }

void RcmScratch::alloc(int n) {
    const size_t m = (size_t)std::max(n, 1);
    deg.resize(m);
    pos_of.resize(m);
    owner.resize(m);
    order.resize(m);
    offs.resize(m + 1);
}

RcmJob RcmScratch::job(const CsrBuf<double2> &S, int *perm, int *iperm) const {
    RcmJob j;
    j.n = S.n;
    j.rowptr = S.rowptr.get();
    j.col = S.col.get();
    j.deg = deg.get();
    j.pos_of = pos_of.get();
    j.owner = owner.get();
    j.order = order.get();
    j.offs = offs.get();
    j.perm = perm;
    j.iperm = iperm;
    return j;
}

// LDS a workgroup may take (the kernel's static LDS is below 1 KB)
static size_t rcm_lds_budget() {
    static const size_t cached = []() -> size_t {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hip_quiet(hipGetDevice(&dev)) == hipSuccess && hip_quiet(hipGetDeviceProperties(&prop, dev)) == hipSuccess)
            return prop.sharedMemPerBlock > 2048 ? prop.sharedMemPerBlock - 2048 : 0;
        return 64 * 1024 - 2048;
    }();
    return cached;
}

void rcm_batch(const RcmJob *jobs, int count, hipStream_t s) {
    if (count <= 0) return;
    int max_n = 0;
    for (int k = 0; k < count; ++k) max_n = std::max(max_n, jobs[k].n);
    DevBuf<RcmJob> dj((size_t)count);
    h2d(dj.get(), jobs, (size_t)count, s);
    const size_t lds = sizeof(int) * (5 * (size_t)max_n + 1);
    if (lds <= rcm_lds_budget()) {
        hip_quiet(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rcm_block<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)rcm_lds_budget()));
        k_rcm_block<true><<<count, RCM_BLOCK_T, lds, s>>>(dj.get());
    } else {
        k_rcm_block<false><<<count, RCM_BLOCK_T, 0, s>>>(dj.get());
    }
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s));  // the job array is released on return
}

void rcm_order(const CsrBuf<double2> &S, DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s) {
    const int n = S.n;
    perm.resize((size_t)n);
    iperm.resize((size_t)n);
    if (n == 0) return;
    if (n <= RCM_BLOCK_MAX_N) {
        RcmScratch w;
        w.alloc(n);
        RcmJob j = w.job(S, perm.get(), iperm.get());
        rcm_batch(&j, 1, s);  // synchronises before the scratch is released
        return;
    }
    DevBuf<int> deg((size_t)n), pos_of((size_t)n), owner((size_t)n), order((size_t)n);
    DevBuf<int> cnt((size_t)n + 1), offs((size_t)n + 1);
    DevBuf<unsigned long long> best(1);
    k_degree<<<div_up(n, 256), 256, 0, s>>>(n, S.rowptr.get(), S.col.get(), deg.get());
    k_fill_int<<<div_up(n, 256), 256, 0, s>>>(n, pos_of.get(), -1);
    k_fill_int<<<div_up(n, 256), 256, 0, s>>>(n, owner.get(), 0x7fffffff);
    SS_HIP(hipMemsetAsync(best.get(), 0xff, sizeof(unsigned long long), s));
    SS_HIP(hipGetLastError());
    int visited = 0;
    while (visited < n) {
        k_pick_start<<<std::min(div_up(n, 256), 1024), 256, 0, s>>>(n, deg.get(), pos_of.get(), best.get());
        k_place_start<<<1, 1, 0, s>>>(best.get(), order.get(), pos_of.get(), visited);
        SS_HIP(hipGetLastError());
        int lo = visited, hi = visited + 1;
        visited += 1;
        while (lo < hi) {
            const int width = hi - lo;
            const int nb = div_up(width, 4);
            k_claim<<<nb, 256, 0, s>>>(lo, hi, order.get(), S.rowptr.get(), S.col.get(), pos_of.get(),
                                       owner.get());
            k_count_owned<<<nb, 256, 0, s>>>(lo, hi, order.get(), S.rowptr.get(), S.col.get(), pos_of.get(),
                                             owner.get(), cnt.get());
            SS_HIP(hipGetLastError());
            const int total = (int)scan_exclusive(cnt.get(), offs.get(), width, s, true);
            if (total > 0) {
                k_place_children<<<nb, 256, 0, s>>>(lo, hi, hi, order.get(), S.rowptr.get(), S.col.get(),
                                                    pos_of.get(), owner.get(), deg.get(), offs.get(), order.get());
                k_mark_level<<<div_up(total, 256), 256, 0, s>>>(hi, hi + total, order.get(), pos_of.get());
                SS_HIP(hipGetLastError());
            }
            lo = hi;
            hi += total;
            visited += total;
        }
    }
    k_reverse<<<div_up(n, 256), 256, 0, s>>>(n, order.get(), perm.get(), iperm.get());
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s));
}

void identity_order(int n, DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s) {
    perm.resize((size_t)n);
    iperm.resize((size_t)n);
    if (n) {
        k_identity<<<div_up(n, 256), 256, 0, s>>>(n, perm.get(), iperm.get());
        SS_HIP(hipGetLastError());
    }
}

// ----------------------------------------------------------- P A P^T
__global__ void k_perm_count(int n, const int *perm, const int *rowptr, int *cnt) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) cnt[q] = rowptr[perm[q] + 1] - rowptr[perm[q]];
}

// PERM_G lanes per output row: each lane maps one column through iperm and
// finds its place in the sorted row by counting the smaller columns of the
// row (shuffles within the lane group; a row's columns are distinct).  Rows
// longer than PERM_G are listed for k_perm_fill_long.
constexpr int PERM_G = 32;
constexpr int PERM_LONG_LDS = 8192;  // columns of a long row ranked from LDS

__global__ void __launch_bounds__(256) k_perm_fill(int n, const int *perm, const int *iperm, const int *rowptr,
                                                   const int *col, const double2 *val, const int *orow, int *ocol,
                                                   double2 *oval, int *longq, int *nlong) {
    const int lane = threadIdx.x & 63, g = lane & (PERM_G - 1), gb = lane - g;
    const int q = (blockIdx.x * 256 + threadIdx.x) / PERM_G;
    int rs = 0, len = 0, c = INT_MAX;
    double2 v = make_double2(0.0, 0.0);
    if (q < n) {
        const int r = perm[q];
        rs = rowptr[r];
        len = rowptr[r + 1] - rs;
        if (g < len) {
            c = iperm[col[rs + g]];
            v = val[rs + g];
        }
    }
    int rank = 0;
    for (int f = 0; f < PERM_G; ++f) rank += (__shfl(c, gb + f, 64) < c);
    if (q >= n) return;
    if (len > PERM_G) {
        if (g == 0) longq[atomicAdd(nlong, 1)] = q;
        return;
    }
    if (g < len) {
        const int o = orow[q];
        ocol[o + rank] = c;
        oval[o + rank] = v;
    }
}

// the listed long rows, one workgroup per row at a time
__global__ void __launch_bounds__(256) k_perm_fill_long(const int *longq, const int *nlong, const int *perm,
                                                        const int *iperm, const int *rowptr, const int *col,
                                                        const double2 *val, const int *orow, int *ocol,
                                                        double2 *oval) {
    __shared__ int lc[PERM_LONG_LDS];
    const int m = *nlong;
    for (int k = blockIdx.x; k < m; k += gridDim.x) {
        const int q = longq[k], r = perm[q];
        const int rs = rowptr[r], len = rowptr[r + 1] - rs, o = orow[q];
        const bool in_lds = len <= PERM_LONG_LDS;
        __syncthreads();
        if (in_lds)
            for (int f = threadIdx.x; f < len; f += 256) lc[f] = iperm[col[rs + f]];
        __syncthreads();
        for (int e = threadIdx.x; e < len; e += 256) {
            const int c = iperm[col[rs + e]];
            int rank = 0;
            if (in_lds) {
                for (int f = 0; f < len; ++f) rank += (lc[f] < c);
            } else {
                for (int f = 0; f < len; ++f) rank += (iperm[col[rs + f]] < c);
            }
            ocol[o + rank] = c;
            oval[o + rank] = val[rs + e];
        }
    }
}

void permute_matrix(const CsrBuf<double2> &A, const int *perm, const int *iperm, CsrBuf<double2> &B, hipStream_t s) {
    const int n = A.n;
    DevBuf<int> cnt((size_t)n + 1), longq((size_t)std::max(n, 1)), nlong(1);
    B.alloc(n, A.nnz);
    if (n) {
        k_perm_count<<<div_up(n, 256), 256, 0, s>>>(n, perm, A.rowptr.get(), cnt.get());
        SS_HIP(hipGetLastError());
    }
    scan_exclusive(cnt.get(), B.rowptr.get(), n, s, false);
    if (n) {
        SS_HIP(hipMemsetAsync(nlong.get(), 0, sizeof(int), s));
        k_perm_fill<<<div_up((int64_t)n * PERM_G, 256), 256, 0, s>>>(n, perm, iperm, A.rowptr.get(), A.col.get(),
                                                                      A.val.get(), B.rowptr.get(), B.col.get(),
                                                                      B.val.get(), longq.get(), nlong.get());
        SS_HIP(hipGetLastError());
        k_perm_fill_long<<<256, 256, 0, s>>>(longq.get(), nlong.get(), perm, iperm, A.rowptr.get(), A.col.get(),
                                             A.val.get(), B.rowptr.get(), B.col.get(), B.val.get());
        SS_HIP(hipGetLastError());
    }
}

// ------------------------------------------------------ vector permutes
__global__ void k_gather_c128(int n, const int *idx, const double2 *x, double2 *y) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = x[idx[q]];
}

void gather(int n, const int *idx, const double2 *x, double2 *y, hipStream_t s) {
    if (n) {
        k_gather_c128<<<div_up(n, 256), 256, 0, s>>>(n, idx, x, y);
        SS_HIP(hipGetLastError());
    }
}

}  // namespace ss
