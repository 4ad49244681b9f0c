// Workgroup-resident steady-state solve for small systems.
//
// One workgroup owns one system for the whole solve: the fp64 refinement or
// inverse-power outer loop, right-preconditioned BiCGSTAB, the CSR SpMV and
// the ILU(0) triangular solves all run between workgroup barriers, with no
// kernel launch or host round trip per iteration.  The triangular solves are
// level scheduled (section "Iterative Solvers": forward and backward
// substitution with the iLU factors): rows of one level are independent, a
// barrier separates levels, and the solution vector lives in LDS so that
// every dependency read is an LDS access.  Many systems launch together, one
// workgroup each, which is how the request server batches small solves.
#include "bucket.hpp"
#include "syncfree.hpp"
#include "wgsolve.hpp"

namespace ss {

// ================================================= level-set analysis
__device__ __forceinline__ int ld_int(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void st_int(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Sync-free level computation (thread per row, ordered workgroups):
// forward  lvl[i] = 1 + max lvl[k], k in [rowptr[i], diag[i])
// backward lvl[i] = 1 + max lvl[j], j in (diag[i], rowptr[i+1])
template <bool UPPER>
__global__ void __launch_bounds__(256) k_levels(int n, const int *rowptr, const int *col, const int *diag, int *lvl,
                                                unsigned *ctr, unsigned base, unsigned *status, int *maxlvl) {
    const unsigned bid = ordered_block(ctr, base);
    const int lin = (int)bid * 256 + threadIdx.x;
    const bool active = lin < n;
    const int row = UPPER ? n - 1 - lin : lin;
    int e = 0, ee = 0, m = -1;
    if (active) {
        e = UPPER ? diag[row] + 1 : rowptr[row];
        ee = UPPER ? rowptr[row + 1] : diag[row];
    }
    bool done = !active;
    unsigned spins = 0;
    while (true) {
        if (!done) {
            int v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (e + q < ee) ? ld_int(lvl + col[e + q]) : -1;
            int used = 0;
            bool run = true;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (run && e + q < ee && v[q] >= 0) {
                    m = max(m, v[q]);
                    ++used;
                } else {
                    run = false;
                }
            }
            e += used;
            if (used) {
                spins = 0;
            } else if (e < ee) {
                ++spins;
                if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
                    atomicOr(status, STATUS_SPIN_TIMEOUT);
                    e = ee;
                }
            }
            if (e >= ee) {
                st_int(lvl + row, m + 1);
                atomicMax(maxlvl, m + 1);
                done = true;
            }
        }
        if (__all(done)) break;
    }
}

// Levels of one class of rows [lo, hi) whose dependencies all lie in
// earlier classes (lower) or later ones (upper), whose levels are final:
// no waits.  An entry inside the class sets STATUS_CLASS_EDGE.
constexpr unsigned STATUS_CLASS_EDGE = 1u << 8;

template <bool UPPER>
__global__ void __launch_bounds__(256) k_levels_class(int lo, int hi, const int *rowptr, const int *col,
                                                      const int *diag, int *lvl, unsigned *status, int *maxlvl) {
    const int row = lo + blockIdx.x * 256 + threadIdx.x;
    int m = -1;
    if (row < hi) {
        const int e0 = UPPER ? diag[row] + 1 : rowptr[row];
        const int e1 = UPPER ? rowptr[row + 1] : diag[row];
        bool inside = false;
        for (int e = e0; e < e1; ++e) {
            const int c = col[e];
            if (UPPER ? c < hi : c >= lo) inside = true;
            else m = max(m, lvl[c]);
        }
        if (inside) atomicOr(status, STATUS_CLASS_EDGE);
        lvl[row] = m + 1;
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m >= 0) atomicMax(maxlvl, m + 1);
}

// Many systems at once, one workgroup each: its threads take the rows in
// chunks of the workgroup size, in order, so every dependency lies in an
// earlier chunk (finished) or earlier in the same chunk.
template <bool UPPER>
__global__ void __launch_bounds__(1024) k_levels_batch(const LevelJob *jobs) {
    const LevelJob &J = jobs[blockIdx.x];
    const int n = J.n;
    for (int c0 = 0; c0 < n; c0 += 1024) {
        const int lin = c0 + (int)threadIdx.x;
        const bool active = lin < n;
        const int row = UPPER ? n - 1 - lin : lin;
        int e = 0, ee = 0, m = -1;
        if (active) {
            e = UPPER ? J.diag[row] + 1 : J.rowptr[row];
            ee = UPPER ? J.rowptr[row + 1] : J.diag[row];
        }
        bool done = !active;
        unsigned spins = 0;
        while (true) {
            if (!done) {
                int v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = (e + q < ee) ? ld_int(J.lvl + J.col[e + q]) : -1;
                int used = 0;
                bool run = true;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (run && e + q < ee && v[q] >= 0) {
                        m = max(m, v[q]);
                        ++used;
                    } else {
                        run = false;
                    }
                }
                e += used;
                if (used) {
                    spins = 0;
                } else if (e < ee) {
                    ++spins;
                    if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(J.status))) {
                        atomicOr(J.status, STATUS_SPIN_TIMEOUT);
                        e = ee;
                    }
                }
                if (e >= ee) {
                    st_int(J.lvl + row, m + 1);
                    atomicMax(J.maxlvl, m + 1);
                    done = true;
                }
            }
            if (__all(done)) break;
        }
        __syncthreads();
    }
}

// The same analysis with the levels of the system in LDS (systems up to
// LEVELS_LDS_MAX rows): a dependency check is an LDS read, each row's columns
// come from memory once (eight at a time, kept in registers), and the
// largest level is reduced in the workgroup before one atomic.  As above, a
// lane never blocks: every pass over the wavefront consumes the dependencies
// that are ready and publishes the rows that are complete, so a lane waiting
// on a row held by another lane of its own wavefront cannot stall it.
constexpr int LEVELS_LDS_MAX = 16384;

template <bool UPPER>
__global__ void __launch_bounds__(1024) k_levels_batch_lds(const LevelJob *jobs) {
    extern __shared__ int slvl[];
    __shared__ int smax;
    const LevelJob &J = jobs[blockIdx.x];
    const int n = J.n;
    for (int i = threadIdx.x; i < n; i += 1024) slvl[i] = -1;
    if (threadIdx.x == 0) smax = -1;
    __syncthreads();
    int mymax = -1;
    for (int c0 = 0; c0 < n; c0 += 1024) {
        const int lin = c0 + (int)threadIdx.x;
        const bool active = lin < n;
        const int row = UPPER ? n - 1 - lin : lin;
        int e = 0, ee = 0, m = -1;
        if (active) {
            e = UPPER ? gld(J.diag + row) + 1 : gld(J.rowptr + row);
            ee = UPPER ? gld(J.rowptr + row + 1) : gld(J.diag + row);
        }
        bool done = !active;
        int c[8];
        unsigned pend = 0;  // dependencies among c[] not yet seen complete
        unsigned spins = 0;
        while (true) {
            if (!done) {
                if (pend == 0 && e < ee) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        c[q] = (e + q < ee) ? gld(J.col + e + q) : 0;
                        if (e + q < ee) pend |= 1u << q;
                    }
                    e += 8;
                }
                const unsigned before = pend;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (pend & (1u << q)) {
                        const int v = __hip_atomic_load(slvl + c[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (v >= 0) {
                            m = max(m, v);
                            pend &= ~(1u << q);
                        }
                    }
                }
                if (pend != before) {
                    spins = 0;
                } else if (pend) {
                    ++spins;
                    if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(J.status))) {
                        atomicOr(J.status, STATUS_SPIN_TIMEOUT);
                        pend = 0;
                        e = ee;
                    }
                }
                if (pend == 0 && e >= ee) {
                    __hip_atomic_store(slvl + row, m + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    gst(J.lvl + row, m + 1);
                    mymax = max(mymax, m + 1);
                    done = true;
                }
            }
            if (__all(done)) break;
        }
    }
    for (int off = 32; off > 0; off >>= 1) mymax = max(mymax, __shfl_xor(mymax, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&smax, mymax);
    __syncthreads();
    if (threadIdx.x == 0 && smax >= 0) atomicMax(J.maxlvl, smax);
}

// out[p] = in[idx[p]]
__global__ void k_gather_i32(int n, const int *idx, const int *in, int *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[p] = in[idx[p]];
}

// slot[q] for the q-th row in level order
template <bool UPPER>
__global__ void k_level_slots(int n, const int *rows, const int *rowptr, const int *diag, int4 *slot) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int i = rows[q];
    slot[q] = UPPER ? make_int4(i, diag[i] + 1, rowptr[i + 1], 0) : make_int4(i, rowptr[i], diag[i], rowptr[i + 1]);
}

__global__ void k_fill_i32(int n, int *p, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

LevelJob LevelBuild::job(const Csr<double2> &LU, const int *diag, hipStream_t s) {
    const int n = LU.n;
    lvl.resize((size_t)std::max(n, 1));
    misc.resize(2);
    status.resize(1);
    SS_HIP(hipMemsetAsync(misc.get(), 0, 2 * sizeof(int), s));
    SS_HIP(hipMemsetAsync(status.get(), 0, sizeof(unsigned), s));
    if (n) {
        k_fill_i32<<<div_up(n, 256), 256, 0, s>>>(n, lvl.get(), -1);
        SS_HIP(hipGetLastError());
    }
    LevelJob j;
    j.n = n;
    j.rowptr = LU.rowptr;
    j.col = LU.col;
    j.diag = diag;
    j.lvl = lvl.get();
    j.status = status.get();
    j.maxlvl = misc.get();
    return j;
}

template <bool UPPER>
void LevelBuild::finish(const Csr<double2> &LU, const int *diag, LevelSched &ls, hipStream_t s, const int *order) {
    const int n = LU.n;
    int maxl = 0;
    unsigned st = 0;
    d2h(&maxl, misc.get(), 1, s);
    d2h(&st, status.get(), 1, s);
    SS_REQUIRE(!(st & STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "level analysis: dependency wait timed out");
    SS_REQUIRE(!(st & STATUS_CLASS_EDGE), SS_E_HIP, "level analysis: an entry between two rows of one class");
    ls.nlev = n ? maxl + 1 : 0;
    ls.ptr.resize((size_t)ls.nlev + 1);
    ls.slot.resize((size_t)std::max(n, 1));
    // rows in (level, row) order, then their slots
    DevBuf<int> rows((size_t)std::max(n, 1));
    if (order && n) {
        DevBuf<int> key((size_t)n);
        k_gather_i32<<<div_up(n, 256), 256, 0, s>>>(n, order, lvl.get(), key.get());
        SS_HIP(hipGetLastError());
        bucket_sort(n, key.get(), ls.nlev, order, rows.get(), nullptr, ls.ptr.get(), s);
    } else {
        bucket_sort(n, lvl.get(), ls.nlev, nullptr, rows.get(), nullptr, ls.ptr.get(), s);
    }
    if (n) {
        k_level_slots<UPPER><<<div_up(n, 256), 256, 0, s>>>(n, rows.get(), LU.rowptr, diag, ls.slot.get());
        SS_HIP(hipGetLastError());
    }
    ls.hptr.resize((size_t)ls.nlev + 1);
    d2h(ls.hptr.data(), ls.ptr.get(), (size_t)ls.nlev + 1, s);  // (synchronises)
}
template void LevelBuild::finish<false>(const Csr<double2> &, const int *, LevelSched &, hipStream_t, const int *);
template void LevelBuild::finish<true>(const Csr<double2> &, const int *, LevelSched &, hipStream_t, const int *);

template <bool UPPER>
void levels_batch(const LevelJob *jobs, int count, hipStream_t s) {
    if (count <= 0) return;
    StreamScope scope(s);
    int max_n = 0;
    for (int k = 0; k < count; ++k) max_n = std::max(max_n, jobs[k].n);
    DevBuf<LevelJob> dj((size_t)count);
    h2d(dj.get(), jobs, (size_t)count, s);
    if (max_n <= LEVELS_LDS_MAX) {
        const size_t bytes = sizeof(int) * (size_t)std::max(max_n, 1);
        // the attribute is the largest size any call uses, so that a launch
        // from another thread never meets a smaller limit set in between
        hip_quiet(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_levels_batch_lds<UPPER>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(int) * LEVELS_LDS_MAX)));
        k_levels_batch_lds<UPPER><<<count, 1024, bytes, s>>>(dj.get());
    } else {
        k_levels_batch<UPPER><<<count, 1024, 0, s>>>(dj.get());
    }
    SS_HIP(hipGetLastError());
}
template void levels_batch<false>(const LevelJob *, int, hipStream_t);
template void levels_batch<true>(const LevelJob *, int, hipStream_t);

template <bool UPPER>
static void one_side(const Csr<double2> &LU, const int *diag, LevelSched &ls, hipStream_t s, const int *order,
                     const std::vector<int> *classes) {
    const int n = LU.n;
    LevelBuild lb;
    LevelJob j = lb.job(LU, diag, s);
    if (n && classes) {
        const std::vector<int> &cp = *classes;
        SS_REQUIRE(cp.size() >= 2 && cp.front() == 0 && cp.back() == n, SS_E_INVALID_ARG,
                   "level analysis: class boundaries do not cover the rows");
        const int C = (int)cp.size() - 1;
        for (int k = 0; k < C; ++k) {
            const int c = UPPER ? C - 1 - k : k;
            const int lo = cp[(size_t)c], hi = cp[(size_t)c + 1];
            SS_REQUIRE(lo <= hi, SS_E_INVALID_ARG, "level analysis: class boundaries out of order");
            if (hi == lo) continue;
            k_levels_class<UPPER><<<div_up(hi - lo, 256), 256, 0, s>>>(lo, hi, LU.rowptr, LU.col, diag, j.lvl,
                                                                      j.status, j.maxlvl);
            SS_HIP(hipGetLastError());
        }
    } else if (n) {
        BlockCounter bc;
        bc.init(s);
        const unsigned grid = (unsigned)div_up(n, 256);
        k_levels<UPPER><<<grid, 256, 0, s>>>(n, LU.rowptr, LU.col, diag, j.lvl, bc.ctr.get(), bc.take(grid),
                                             j.status, j.maxlvl);
        SS_HIP(hipGetLastError());
    }
    lb.finish<UPPER>(LU, diag, ls, s, order);
}

void build_levels(const Csr<double2> &LU, const int *diag, LevelSched &lo, LevelSched &up, hipStream_t s,
                  const int *order, const std::vector<int> *classes) {
    one_side<false>(LU, diag, lo, s, order, classes);
    one_side<true>(LU, diag, up, s, order, classes);
}

template <typename T>
__global__ void k_pack_side(int n, const int4 *in, const int *col, const T *val, bool upper, int4 *slot, int *pcol,
                            T *pval, T *aux) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int4 sl = in[idx];
    const int len = sl.z - sl.y;
    slot[idx] = make_int4(sl.x, sl.y, len, 0);
    constexpr int WG_K = WgK<T>::value;
#pragma unroll
    for (int k = 0; k < WG_K; ++k) {
        pcol[(size_t)k * n + idx] = (k < len) ? col[sl.y + k] : 0;
        pval[(size_t)k * n + idx] = (k < len) ? val[sl.y + k] : czero<T>();
    }
    aux[idx] = upper ? val[sl.y - 1] : czero<T>();
}

template <typename T>
void pack_side(const LevelSched &ls, const Csr<T> &LU, bool upper, PackedSide<T> &out, hipStream_t s) {
    const int n = LU.n;
    const size_t nn = (size_t)std::max(n, 1);
    out.slot.resize(nn);
    out.col.resize(nn * WgK<T>::value);
    out.val.resize(nn * WgK<T>::value);
    out.aux.resize(nn);
    if (n) {
        k_pack_side<T><<<div_up(n, 256), 256, 0, s>>>(n, ls.slot.get(), LU.col, LU.val, upper, out.slot.get(),
                                                       out.col.get(), out.val.get(), out.aux.get());
        SS_HIP(hipGetLastError());
    }
}
template void pack_side<double2>(const LevelSched &, const Csr<double2> &, bool, PackedSide<double2> &, hipStream_t);
template void pack_side<float2>(const LevelSched &, const Csr<float2> &, bool, PackedSide<float2> &, hipStream_t);

// ============================================== block-level primitives
// Barrier that orders only LDS traffic: unlike __syncthreads() it does not
// wait for outstanding global loads, so loads issued for the next level stay
// in flight across it.  Used where threads communicate through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int BS, int K>
__device__ __forceinline__ void blk_sum(double2 (&v)[K], double2 (*sh)[BS / 64 + 1]) {
    constexpr int NW = BS / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k].x, y = v[k].y;
        for (int off = 32; off > 0; off >>= 1) {
            x += __shfl_down(x, off, 64);
            y += __shfl_down(y, off, 64);
        }
        if (lane == 0) sh[k][wave] = mk(x, y);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double2 acc = sh[k][0];
            for (int w = 1; w < NW; ++w) acc = cadd(acc, sh[k][w]);
            sh[k][NW] = acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = sh[k][NW];
    __syncthreads();
}

constexpr int WG_G = 4;  // lanes per row in the workgroup SpMV

// y = A x (accumulated in V); returns conj(u1).y and, if u2 != null,
// conj(u2).y (or |y|^2 when u2 == y) in d0, d1 (fp64, per thread; the
// caller reduces them).  Each lane group works on WG_U rows at once so that
// the row-pointer, index/value and gather loads of several rows are in
// flight together.
constexpr int WG_U = 8;
// entries per lane and row whose loads are issued up front (rows up to
// WgE * WG_G long), bounded by the registers they hold
template <typename V> struct WgE { static constexpr int value = sizeof(V) == 16 ? 2 : 3; };

template <typename V, int BS>
__device__ __forceinline__ void blk_spmv(const Csr<V> &A, const V *x, V *y, const V *u1, const V *u2, double2 &d0,
                                double2 &d1) {
    const int l = threadIdx.x & (WG_G - 1);
    const bool u2y = (u2 == y);
    constexpr int R = BS / WG_G;  // rows per pass
    for (int base = threadIdx.x / WG_G; base < A.n; base += R * WG_U) {
        int rs[WG_U], re[WG_U];
#pragma unroll
        for (int u = 0; u < WG_U; ++u) {
            const int row = base + u * R;
            rs[u] = (row < A.n) ? gld(A.rowptr + row) : 0;
            re[u] = (row < A.n) ? gld(A.rowptr + row + 1) : 0;
        }
        V acc[WG_U];
#pragma unroll
        for (int u = 0; u < WG_U; ++u) acc[u] = czero<V>();
        int mx = 0;
#pragma unroll
        for (int u = 0; u < WG_U; ++u) mx = max(mx, re[u] - rs[u]);
        // the first WG_E entries of every row of the group: all loads issued
        // before any is used (one memory round trip instead of one per step)
        constexpr int WG_E = WgE<V>::value;
        {
            int cc[WG_U][WG_E];
            V vv[WG_U][WG_E];
#pragma unroll
            for (int u = 0; u < WG_U; ++u)
#pragma unroll
                for (int t = 0; t < WG_E; ++t) {
                    const int e = rs[u] + l + t * WG_G;
                    const bool ok = e < re[u];
                    cc[u][t] = ok ? gld(A.col + e) : -1;
                    vv[u][t] = ok ? gld(A.val + e) : czero<V>();
                }
#pragma unroll
            for (int u = 0; u < WG_U; ++u)
#pragma unroll
                for (int t = 0; t < WG_E; ++t)
                    if (cc[u][t] >= 0) acc[u] = cadd(acc[u], cmul(vv[u][t], x[cc[u][t]]));
        }
        for (int k = l + WG_E * WG_G; k < mx; k += WG_G) {
#pragma unroll
            for (int u = 0; u < WG_U; ++u) {
                const int e = rs[u] + k;
                if (e < re[u]) acc[u] = cadd(acc[u], cmul(gld(A.val + e), x[gld(A.col + e)]));
            }
        }
#pragma unroll
        for (int u = 0; u < WG_U; ++u) {
#pragma unroll
            for (int off = WG_G / 2; off > 0; off >>= 1) {
                acc[u].x += __shfl_xor(acc[u].x, off, WG_G);
                acc[u].y += __shfl_xor(acc[u].y, off, WG_G);
            }
            const int row = base + u * R;
            if (l == 0 && row < A.n) {
                gst(y + row, acc[u]);
                const double2 yy = widen(acc[u]);
                if (u1) d0 = cadd(d0, cmulc(widen(gld(u1 + row)), yy));
                if (u2y) d1.x += yy.x * yy.x + yy.y * yy.y;
                else if (u2) d1 = cadd(d1, cmulc(widen(gld(u2 + row)), yy));
            }
        }
    }
}

// One slot of a level held in registers: its packed entries are fetched a
// few levels before they are used.
template <typename T>
struct SlotRegs {
    static constexpr int WG_K = WgK<T>::value;
    int4 sl;  // {row, first CSR entry, length, 0}
    int ok;   // the slot is in the level (a register of its own: writing a
              // lane of sl would wait for its load)
    int c[WG_K];
    T v[WG_K];
    T aux;    // lower: right-hand side (level order); upper: pivot
};

// Issue the loads of slot idx (all addressed by idx: none waits on another).
// Branch-free: an index past the level end is clamped to a valid slot and
// marked invalid, so the loads stay unconditional and in flight.
template <typename T, bool UPPER>
__device__ __forceinline__ void fetch_slot(SlotRegs<T> &q, int idx, int end, int n, const int4 *slot,
                                           const int *pcol, const T *pval, const T *aux) {
    constexpr int WG_K = WgK<T>::value;
    const int j = min(idx, n - 1);
    q.sl = gld(slot + j);
#pragma unroll
    for (int k = 0; k < WG_K; ++k) {
        q.c[k] = gld(pcol + (size_t)k * n + j);
        q.v[k] = gld(pval + (size_t)k * n + j);
    }
    q.aux = gld(aux + j);
    q.ok = idx < end;
}

template <typename T, bool UPPER>
__device__ __forceinline__ void solve_regs(const SlotRegs<T> &q, const int *col, const T *val, T *Y) {
    constexpr int WG_K = WgK<T>::value;
    // the record's last field is 0; adding it keeps all four loaded
    // registers live until here, so none is reused (which would wait for
    // the load) while the ring's loads are in flight
    const int len = q.sl.z + q.sl.w;
    T acc = UPPER ? Y[q.sl.x] : q.aux;
#pragma unroll
    for (int k = 0; k < WG_K; ++k) {
        const T y = Y[q.c[k]];
        const T t = csub(acc, cmul(q.v[k], y));
        // select component-wise: a select of the whole vector type is lowered
        // through private (scratch) memory
        const bool take = k < len;
        acc.x = take ? t.x : acc.x;
        acc.y = take ? t.y : acc.y;
    }
    if (len > WG_K && q.ok) {
        for (int e = q.sl.y + WG_K; e < q.sl.y + len; ++e) acc = csub(acc, cmul(gld(val + e), Y[gld(col + e)]));
    }
    const T res = UPPER ? cdiv(acc, q.aux) : acc;
    if (q.ok) Y[q.sl.x] = res;
}

// Slots of a level beyond the first 64: fetched and solved directly.
template <typename T, bool UPPER>
__device__ __forceinline__ void solve_rest(int p0, int p1, int n, const int4 *slot, const int *pcol, const T *pval,
                                           const T *aux, const int *col, const T *val, T *Y) {
    for (int idx = p0 + 64 + (int)(threadIdx.x & 63); idx < p1; idx += 64) {
        SlotRegs<T> q;
        fetch_slot<T, UPPER>(q, idx, p1, n, slot, pcol, pval, aux);
        solve_regs<T, UPPER>(q, col, val, Y);
    }
}

// One triangular sweep over the level schedule, run by a single wavefront.
// The instructions of one wavefront reach LDS in program order, so a level
// reads the values the previous level wrote without any barrier; with Y in
// global memory a wavefront-scope fence orders the accesses instead.  A
// three-deep register ring keeps the packed slots of the next levels in
// flight while a level is solved.
template <typename T, bool UPPER, bool LDSY>
__device__ __forceinline__ void wave_sweep(int nlev, int n, const int *ptr, const int4 *slot, const int *pcol,
                                           const T *pval, const T *aux, const int *col, const T *val, T *Y) {
    // ptr holds nlev + 5 entries: the last ones repeat ptr[nlev] (empty levels)
    if (nlev <= 0) return;
    const int lane = threadIdx.x & 63;
    SlotRegs<T> r0, r1, r2;
    fetch_slot<T, UPPER>(r0, ptr[0] + lane, ptr[1], n, slot, pcol, pval, aux);
    fetch_slot<T, UPPER>(r1, ptr[1] + lane, ptr[2], n, slot, pcol, pval, aux);
    fetch_slot<T, UPPER>(r2, ptr[2] + lane, ptr[3], n, slot, pcol, pval, aux);
    for (int lev = 0; lev < nlev; lev += 3) {
#define SS_SWEEP_STEP(R, L)                                                                             \
        {                                                                                               \
            const int a0 = ptr[(L)], a1 = ptr[(L) + 1], a3 = ptr[(L) + 3], a4 = ptr[(L) + 4];           \
            solve_regs<T, UPPER>(R, col, val, Y);                                                       \
            if (a1 - a0 > 64) solve_rest<T, UPPER>(a0, a1, n, slot, pcol, pval, aux, col, val, Y);      \
            fetch_slot<T, UPPER>(R, a3 + lane, a4, n, slot, pcol, pval, aux);                           \
            if (!LDSY) {                                                                                \
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");                                  \
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");                                  \
            }                                                                                           \
        }
        SS_SWEEP_STEP(r0, lev)
        SS_SWEEP_STEP(r1, lev + 1)
        SS_SWEEP_STEP(r2, lev + 2)
#undef SS_SWEEP_STEP
    }
}

// The sweeps' level pointers as the solve kernel keeps them in LDS: every
// level split into runs of at most 64 slots, so that a single wavefront's
// register ring prefetches every slot (the rows of one level are
// independent, so any split of a level is a valid schedule).
struct WgSched {
    const int *lptr, *uptr;
    int nl, nu;
};
constexpr int WG_SPLIT_PAD = 6;  // the sweep reads up to five pointers past the last run
// LDS ints of one side's split pointers
__host__ __device__ constexpr int wg_split_ints(int nlev, int n) { return nlev + n / 64 + WG_SPLIT_PAD + 1; }

// Writes the split pointers of g[0 .. nlev] to out (one wavefront): out[s]
// is the first slot of run s; the count of runs is returned and out[count ..
// count + 5] repeat the end (room for WG_SPLIT_PAD entries past the runs).
// At most nlev + n / 64 runs.
__device__ __forceinline__ int split_levels(const int *g, int nlev, int *out) {
    const int lane = threadIdx.x & 63;
    int base = 0;
    for (int l0 = 0; l0 < nlev; l0 += 64) {
        const int l = l0 + lane;
        int a = 0, cnt = 0;
        if (l < nlev) {
            a = g[l];
            cnt = (g[l + 1] - a + 63) >> 6;
        }
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        for (int q = 0; q < cnt; ++q) out[base + incl - cnt + q] = a + 64 * q;
        base += __shfl(incl, 63, 64);
    }
    const int end = g[nlev];
    if (lane < WG_SPLIT_PAD) out[base + lane] = end;
    return base;
}

template <typename T, int BS, bool LDSY>
__device__ __forceinline__ void blk_precond(const WgProblem<T> &P, const WgSched &S, const T *b, T *out, T *Y) {
    const int n = P.n;
    // right-hand side in the forward sweep's level order, so the sweep reads
    // it by slot index
    T *bl = P.work + 10 * (size_t)n;
    for (int idx = threadIdx.x; idx < n; idx += BS) gst(bl + idx, gld(b + gld(P.lslot + idx).x));
    __syncthreads();
    if (threadIdx.x < 64) {
        wave_sweep<T, false, LDSY>(S.nl, n, S.lptr, P.lslot, P.lcol, P.lval, bl, P.LU.col, P.LU.val, Y);
        wave_sweep<T, true, LDSY>(S.nu, n, S.uptr, P.uslot, P.ucol, P.uval, P.uaux, P.LU.col, P.LU.val, Y);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += BS) gst(out + i, Y[i]);
    __syncthreads();
}

struct InnerStats {
    int its;
    int converged;
    int breakdowns;
    long long t_pre;
    long long t_spmv;
};

// relative residual growth (squared) at which an inner solve counts as
// diverged: the preconditioner does not make BiCGSTAB work on this system
constexpr double WG_DIVERGED2 = 1e8;

// Right-preconditioned BiCGSTAB (van der Vorst) on A d = b from d = 0, to
// ||r|| <= rtol ||b||; breakdown (r^ orthogonal to r, or omega = 0) restarts
// with r^ = r up to three times.
template <typename T, int BS, bool LDSY>
__device__ __forceinline__ InnerStats blk_bicgstab(const WgProblem<T> &P, const WgSched &S, const T *b, T *x,
                                                   double rtol, T *Y,
                                                   double2 (*red)[BS / 64 + 1]) {
    const int n = P.n;
    T *r = P.work, *rh = r + n, *p = rh + n, *v = p + n, *sv = v + n, *t = sv + n, *ph = t + n, *sh = ph + n;
    // (a threshold whose square overflows makes every breakdown test fire)
    const double bd_eps = P.force_breakdown ? 1e300 : (sizeof(typename RealOf<T>::type) == 8 ? 1e-30 : 1e-14);
    InnerStats st = {0, 0, 0, 0, 0};
    double2 q1[1] = {mk(0.0, 0.0)};
    for (int i = threadIdx.x; i < n; i += BS) {
        const T bi = gld(b + i);
        gst(r + i, bi);
        gst(rh + i, bi);
        gst(p + i, czero<T>());
        gst(v + i, czero<T>());
        gst(x + i, czero<T>());
        const double2 w = widen(bi);
        q1[0].x += w.x * w.x + w.y * w.y;
    }
    blk_sum<BS, 1>(q1, red);
    const double b2 = q1[0].x;
    if (b2 == 0.0) {
        st.converged = 1;
        return st;
    }
    const double tol2 = rtol * rtol * b2;
    double rhat2 = b2;
    double2 rho = mk(b2, 0.0), rho_old = mk(1.0, 0.0), alpha = mk(1.0, 0.0), omega = mk(1.0, 0.0);
    while (st.its < P.maxiter) {
        const double2 beta = cmul(cdiv(rho, rho_old), cdiv(alpha, omega));
        for (int i = threadIdx.x; i < n; i += BS) {
            const double2 q = csub(widen(gld(p + i)), cmul(omega, widen(gld(v + i))));
            gst(p + i, from_c128<T>(cadd(widen(gld(r + i)), cmul(beta, q))));
        }
        __syncthreads();
        long long c0 = wall_clock64();
        blk_precond<T, BS, LDSY>(P, S, p, ph, Y);
        long long c1 = wall_clock64();
        double2 q2[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
        blk_spmv<T, BS>(P.A, LDSY ? Y : ph, v, rh, v, q2[0], q2[1]);
        blk_sum<BS, 2>(q2, red);
        long long c2 = wall_clock64();
        st.t_pre += c1 - c0;
        st.t_spmv += c2 - c1;
        const double2 rv = q2[0];
        bool breakdown = !((rv.x * rv.x + rv.y * rv.y) > bd_eps * bd_eps * rhat2 * q2[1].x);
        if (!breakdown) {
            alpha = cdiv(rho, rv);
            double2 q3[1] = {mk(0.0, 0.0)};
            for (int i = threadIdx.x; i < n; i += BS) {
                const T si = from_c128<T>(csub(widen(gld(r + i)), cmul(alpha, widen(gld(v + i)))));
                gst(sv + i, si);
                const double2 w = widen(si);
                q3[0].x += w.x * w.x + w.y * w.y;
            }
            blk_sum<BS, 1>(q3, red);
            if (q3[0].x <= tol2) {
                for (int i = threadIdx.x; i < n; i += BS)
                    gst(x + i, from_c128<T>(cadd(widen(gld(x + i)), cmul(alpha, widen(gld(ph + i))))));
                __syncthreads();
                st.its += 1;
                st.converged = 1;
                return st;
            }
            c0 = wall_clock64();
            blk_precond<T, BS, LDSY>(P, S, sv, sh, Y);
            c1 = wall_clock64();
            double2 q4[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
            blk_spmv<T, BS>(P.A, LDSY ? Y : sh, t, sv, t, q4[0], q4[1]);
            blk_sum<BS, 2>(q4, red);
            c2 = wall_clock64();
            st.t_pre += c1 - c0;
            st.t_spmv += c2 - c1;
            // omega = (t, s) / (t, t) = conj(s^H t) / |t|^2
            omega = (q4[1].x > 0.0) ? cscale(cconj(q4[0]), 1.0 / q4[1].x) : mk(0.0, 0.0);
            double2 q5[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
            for (int i = threadIdx.x; i < n; i += BS) {
                const double2 xi =
                    cadd(cadd(widen(gld(x + i)), cmul(alpha, widen(gld(ph + i)))), cmul(omega, widen(gld(sh + i))));
                gst(x + i, from_c128<T>(xi));
                const T ri = from_c128<T>(csub(widen(gld(sv + i)), cmul(omega, widen(gld(t + i)))));
                gst(r + i, ri);
                const double2 rw = widen(ri);
                q5[0] = cadd(q5[0], cmulc(widen(gld(rh + i)), rw));
                q5[1].x += rw.x * rw.x + rw.y * rw.y;
            }
            blk_sum<BS, 2>(q5, red);
            st.its += 1;
            rho_old = rho;
            rho = q5[0];
            const double r2 = q5[1].x;
            if (r2 <= tol2) {
                st.converged = 1;
                return st;
            }
            if (!(r2 <= WG_DIVERGED2 * b2)) {
                st.breakdowns = 3 + 1;  // diverged (or NaN): give up like an unrecoverable breakdown
                return st;
            }
            breakdown = !(omega.x != 0.0 || omega.y != 0.0) ||
                        !((rho.x * rho.x + rho.y * rho.y) > bd_eps * bd_eps * rhat2 * r2);
        }
        if (breakdown) {
            if (st.breakdowns >= 3) return st;
            st.breakdowns += 1;
            double2 q6[1] = {mk(0.0, 0.0)};
            for (int i = threadIdx.x; i < n; i += BS) {
                const T ri = gld(r + i);
                gst(rh + i, ri);
                gst(p + i, czero<T>());
                gst(v + i, czero<T>());
                const double2 w = widen(ri);
                q6[0].x += w.x * w.x + w.y * w.y;
            }
            blk_sum<BS, 1>(q6, red);
            rhat2 = q6[0].x;
            rho = mk(rhat2, 0.0);
            rho_old = mk(1.0, 0.0);
            alpha = mk(1.0, 0.0);
            omega = mk(1.0, 0.0);
        }
    }
    return st;
}

// ============================================ single-workgroup (L U)^-1
// Triangular solve pair of a large system in one workgroup: levels are
// separated by workgroup barriers and the solution vector stays in global
// memory (cache resident), so a level costs a barrier plus an L2 round trip
// instead of the cross-device handshakes of the sync-free kernels.
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_precond_block(int n, int nlev_l, const int *lptr, const int4 *lslot,
                                                      const int *lcol, const T *lval, int nlev_u, const int *uptr,
                                                      const int4 *uslot, const int *ucol, const T *uval,
                                                      const T *uaux, const int *col, const T *val, const T *b,
                                                      T *bl, T *out, const int *skip) {
    if (skip && *skip) return;
    for (int idx = threadIdx.x; idx < n; idx += BS) bl[idx] = b[lslot[idx].x];
    __syncthreads();
    for (int lev = 0; lev < nlev_l; ++lev) {
        const int p0 = lptr[lev], p1 = lptr[lev + 1];
        for (int idx = p0 + threadIdx.x; idx < p1; idx += BS) {
            SlotRegs<T> q;
            fetch_slot<T, false>(q, idx, p1, n, lslot, lcol, lval, bl);
            solve_regs<T, false>(q, col, val, out);
        }
        __syncthreads();
    }
    for (int lev = 0; lev < nlev_u; ++lev) {
        const int p0 = uptr[lev], p1 = uptr[lev + 1];
        for (int idx = p0 + threadIdx.x; idx < p1; idx += BS) {
            SlotRegs<T> q;
            fetch_slot<T, true>(q, idx, p1, n, uslot, ucol, uval, uaux);
            solve_regs<T, true>(q, col, val, out);
        }
        __syncthreads();
    }
}

template <typename T>
void precond_block(const BlockPrecond<T> &B, const Csr<T> &LU, const T *b, T *out, T *bl, hipStream_t s,
                   const int *skip) {
    if (LU.n == 0) return;
    k_precond_block<T, 1024><<<1, 1024, 0, s>>>(LU.n, B.lo->nlev, B.lo->ptr.get(), B.pl->slot.get(),
                                                  B.pl->col.get(), B.pl->val.get(), B.up->nlev, B.up->ptr.get(),
                                                  B.pu->slot.get(), B.pu->col.get(), B.pu->val.get(),
                                                  B.pu->aux.get(), LU.col, LU.val, b, bl, out, skip);
    SS_HIP(hipGetLastError());
}
template void precond_block<double2>(const BlockPrecond<double2> &, const Csr<double2> &, const double2 *,
                                     double2 *, double2 *, hipStream_t, const int *);
template void precond_block<float2>(const BlockPrecond<float2> &, const Csr<float2> &, const float2 *, float2 *,
                                    float2 *, hipStream_t, const int *);

// ================================================== the solve kernel
template <typename T, int BS, bool LDSY>
__global__ void __launch_bounds__(BS) k_wg_solve(const WgProblem<T> *probs) {
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    __shared__ double2 red[3][BS / 64 + 1];
    const WgProblem<T> &P = probs[blockIdx.x];
    T *Y = LDSY ? reinterpret_cast<T *>(dyn_lds) : P.ysc;
    const int n = P.n;
    // level pointers in LDS next to Y (reading them is then an LDS access,
    // ordered with the other LDS traffic of the sweeps), split into runs of
    // at most 64 slots and padded with repeats of the end so the sweeps can
    // read ahead without bounds checks
    __shared__ int nsplit[2];
    WgSched S;
    {
        int *lp = reinterpret_cast<int *>(dyn_lds + (LDSY ? (size_t)n * sizeof(T) : 0));
        int *up = lp + wg_split_ints(P.nlev_l, n);
        const int wave = threadIdx.x >> 6;
        if (wave < 2) {
            const int c = wave == 0 ? split_levels(P.lptr, P.nlev_l, lp) : split_levels(P.uptr, P.nlev_u, up);
            if ((threadIdx.x & 63) == 0) nsplit[wave] = c;
        }
        __syncthreads();
        S = WgSched{lp, up, nsplit[0], nsplit[1]};
    }
    T *bT = P.work + 8 * (size_t)n, *dT = bT + n;
    int status = SS_E_NOT_CONVERGED, inner = 0, breakdowns = 0, outer = 0;
    double resid = INFINITY;
    const long long t_start = wall_clock64();
    long long t_pre = 0, t_spmv = 0;
    for (outer = 0; outer <= P.max_outer; ++outer) {
        // fp64 residual: trace row  r = b - A x;  inverse power  r = A x + sigma x = L x
        double2 q[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
        double2 dummy = mk(0.0, 0.0), dummy2 = mk(0.0, 0.0);
        blk_spmv<double2, BS>(P.A64, P.x64, P.r64, nullptr, nullptr, dummy, dummy2);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += BS) {
            const double2 ax = P.r64[i];
            const double2 ri = P.trace ? csub(P.b64[i], ax) : cadd(ax, cscale(P.x64[i], P.sigma));
            P.r64[i] = ri;
            q[0].x += ri.x * ri.x + ri.y * ri.y;
        }
        for (int k = threadIdx.x; k < P.d; k += BS) q[1] = cadd(q[1], P.x64[P.tpos[k]]);
        __syncthreads();
        if (threadIdx.x == 0 && P.trace) q[2] = P.r64[P.q0];
        blk_sum<BS, 3>(q, red);
        const double r2 = q[0].x;
        const double2 tr = q[1];
        const double trm = sqrt(tr.x * tr.x + tr.y * tr.y);
        double lx2 = r2;
        if (P.trace) {
            // L x = -r + w (1 - Tr x) e_q0 (the permuted row q0 carries T)
            const double2 rq = q[2];
            const double2 e0 = csub(cmul(P.w, mk(1.0 - tr.x, -tr.y)), rq);
            lx2 = fmax(r2 - (rq.x * rq.x + rq.y * rq.y), 0.0) + e0.x * e0.x + e0.y * e0.y;
        }
        resid = (trm > 0.0) ? sqrt(lx2) / trm : INFINITY;
        if ((P.trace == 0 || outer > 0) && resid <= P.tol) { status = SS_OK; break; }
        if (outer == P.max_outer) break;
        const double rn = sqrt(r2);
        if (rn == 0.0) { status = SS_OK; break; }
        const double rtol = (P.rtol_in > 0.0) ? P.rtol_in : fmax(0.1 * P.tol / rn, 1e-13);
        const double inv = 1.0 / rn;
        for (int i = threadIdx.x; i < n; i += BS) bT[i] = from_c128<T>(cscale(P.r64[i], inv));
        __syncthreads();
        const InnerStats is = blk_bicgstab<T, BS, LDSY>(P, S, bT, dT, fmin(rtol, 0.5), Y, red);
        inner += is.its;
        breakdowns += is.breakdowns;
        t_pre += is.t_pre;
        t_spmv += is.t_spmv;
        if (!is.converged && (is.breakdowns >= 3 || is.its >= P.maxiter)) {
            // unrecoverable breakdown, divergence or stagnation of the inner
            // solve: report it so the caller can switch to GMRES
            status = SS_E_BREAKDOWN;
            break;
        }
        const double sc = P.trace ? rn : -rn;
        for (int i = threadIdx.x; i < n; i += BS) P.x64[i] = cadd(P.x64[i], cscale(widen(dT[i]), sc));
        __syncthreads();
        if (!P.trace) {
            double2 qt[1] = {mk(0.0, 0.0)};
            for (int k = threadIdx.x; k < P.d; k += BS) qt[0] = cadd(qt[0], P.x64[P.tpos[k]]);
            blk_sum<BS, 1>(qt, red);
            const double2 invt = cdiv(mk(1.0, 0.0), qt[0]);
            for (int i = threadIdx.x; i < n; i += BS) P.x64[i] = cmul(P.x64[i], invt);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        P.res->status = status;
        P.res->outer = outer;
        P.res->inner = inner;
        P.res->breakdowns = breakdowns;
        P.res->resid = resid;
        P.res->ticks_precond = t_pre;
        P.res->ticks_spmv = t_spmv;
        P.res->ticks_total = wall_clock64() - t_start;
    }
}

static size_t lds_budget() {
    // (initialised once, thread-safe: servers set up groups from several threads)
    static const size_t cached = []() -> size_t {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hip_quiet(hipGetDevice(&dev)) == hipSuccess && hip_quiet(hipGetDeviceProperties(&prop, dev)) == hipSuccess) {
            const size_t b = prop.sharedMemPerBlock;
            // static LDS of the kernel (reduction scratch) stays below 1 KB
            return b > 2048 ? b - 2048 : 0;
        }
        return 64 * 1024 - 2048;
    }();
    return cached;
}

template <typename T>
int wg_lds_capacity() {
    return (int)(lds_budget() / sizeof(T));
}
template int wg_lds_capacity<double2>();
template int wg_lds_capacity<float2>();

// LDS ints of both sides' split level pointers (at most nlev + n / 64 runs
// per side, plus the padding)
static size_t wg_ptr_ints(size_t n, int levels) { return (size_t)levels + 2 * (n / 64) + 2 * WG_SPLIT_PAD + 2; }

bool wg_fits_lds(size_t n, size_t elem, int levels) {
    return n * elem + sizeof(int) * wg_ptr_ints(n, levels) <= lds_budget();
}

template <typename T>
void wg_solve(const WgProblem<T> *probs, int count, int max_n, int max_levels, hipStream_t s) {
    if (count <= 0) return;
    const size_t ptr_bytes = sizeof(int) * wg_ptr_ints((size_t)max_n, max_levels);
    const size_t bytes = (size_t)max_n * sizeof(T) + ptr_bytes;
    if (bytes <= lds_budget()) {
        hip_quiet(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wg_solve<T, WG_BS, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_budget()));
        k_wg_solve<T, WG_BS, true><<<count, WG_BS, bytes, s>>>(probs);
    } else {
        SS_REQUIRE(ptr_bytes <= lds_budget(), SS_E_INVALID_ARG, "too many levels for the workgroup solver");
        hip_quiet(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wg_solve<T, WG_BS, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_budget()));
        k_wg_solve<T, WG_BS, false><<<count, WG_BS, ptr_bytes, s>>>(probs);
    }
    SS_HIP(hipGetLastError());
}
template void wg_solve<double2>(const WgProblem<double2> *, int, int, int, hipStream_t);
template void wg_solve<float2>(const WgProblem<float2> *, int, int, int, hipStream_t);

}  // namespace ss
