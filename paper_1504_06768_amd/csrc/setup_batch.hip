// Batched set-up stages: the transform of eq. (linear) or eq. (inverse) and
// the symmetrised pattern for every system of a batch, in a fixed number of
// launches (flattened over the systems' rows) and one host wait.
//
// Output sizes are bounded before anything runs -- nnz(A) <= nnz(L) + d for
// the trace row (d trace columns), <= nnz(L) + n for the shift (a diagonal
// per row), nnz(S) <= 2 nnz(A) -- so every buffer is allocated up front and
// the exact sizes are read back once at the end.  The row functions and the
// summation order are those of the one-system kernels, so each handle gets
// the same A, w, trace row and S as ss_prepare computes.
#include <cstring>

#include "start.hpp"
#include "batch.hpp"
#include "handle.hpp"
#include "rowops.hpp"
#include "setup_batch.hpp"
#include "syncfree.hpp"

namespace ss {

struct ScalarJob {
    int n, d;
    Csr<double2> L;
    int forced;     // trace row requested (-1: choose)
    double weight;  // trace-row weight requested (0: mean diagonal)
    double2 *w;     // out: the weight (the handle's device copy)
    double2 *wcopy; // out: the weight again, for the host
    int *trow;      // out: the trace row
};

// One block per trace-row system.  The mean diagonal is summed in the order
// of the one-system reduction (256 partial sums over rows b 256 + t + k 65536,
// each reduced as a tree, then added in block order).
__global__ void __launch_bounds__(256) k_bt_scalars(const ScalarJob *jobs) {
    __shared__ double sx[256], sy[256], px[256], py[256];
    const ScalarJob J = jobs[blockIdx.x];
    const int t = threadIdx.x;
    double2 w = mk(J.weight, 0.0);
    if (J.weight == 0.0) {
        for (int b = 0; b < 256; ++b) {
            if (b * 256 >= J.n) {
                // no row falls to this partial: its sum is +0.0, as computed
                if (t == 0) {
                    px[b] = 0.0;
                    py[b] = 0.0;
                }
                continue;
            }
            double ax = 0, ay = 0;
            for (int r = b * 256 + t; r < J.n; r += 256 * 256) {
                int lo = J.L.rowptr[r], hi = J.L.rowptr[r + 1] - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int c = J.L.col[mid];
                    if (c == r) { ax += J.L.val[mid].x; ay += J.L.val[mid].y; break; }
                    if (c < r) lo = mid + 1; else hi = mid - 1;
                }
            }
            sx[t] = ax;
            sy[t] = ay;
            __syncthreads();
            for (int off = 128; off > 0; off >>= 1) {
                if (t < off) {
                    sx[t] += sx[t + off];
                    sy[t] += sy[t + off];
                }
                __syncthreads();
            }
            if (t == 0) {
                px[b] = sx[0];
                py[b] = sy[0];
            }
            __syncthreads();
        }
        if (t == 0) {
            double ax = 0, ay = 0;
            for (int b = 0; b < 256; ++b) { ax += px[b]; ay += py[b]; }
            w = mk(ax / J.n, ay / J.n);
            // zero mean diagonal: any nonzero weight gives the same rho
            if (w.x == 0.0 && w.y == 0.0) w = mk(1.0, 0.0);
        }
    }
    const int r = pick_trace_row_block(J.d, J.L.rowptr, J.L.col, J.L.val, J.forced);
    if (t == 0) {
        *J.w = w;
        *J.wcopy = w;
        *J.trow = r;
    }
}

struct ModJob {
    int n, d;
    Csr<double2> L;
    int trace;
    double sigma;
    const double2 *w;
    const int *trow;
    int *rowptr;  // counts, then row pointers of A
    int *col;
    double2 *val;
};

template <bool FILL>
__global__ void __launch_bounds__(256) k_bt_modify(const ModJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const ModJob &J = jobs[jb];
    const int r = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (r >= J.n) return;
    const int *rp = J.L.rowptr;
    if (!J.trace) {
        if (FILL) shift_row<true>(r, rp, J.L.col, J.L.val, J.sigma, J.col + J.rowptr[r], J.val + J.rowptr[r]);
        else J.rowptr[r] = shift_row<false>(r, rp, J.L.col, J.L.val, J.sigma, nullptr, nullptr);
        return;
    }
    // trace-row transform: row lengths only (k_bt_trace_row and k_bt_copy fill)
    if (FILL) return;
    const int rt = *J.trow;
    J.rowptr[r] = (r == rt) ? trace_row0<false>(J.d, rt, rp, J.L.col, J.L.val, *J.w, nullptr, nullptr)
                            : rp[r + 1] - rp[r];
}

// Trace-row transform, fill, of the trace row itself (one thread per system;
// a trace row index outside the matrix leaves every row as it is).
__global__ void __launch_bounds__(256) k_bt_trace_row(const ModJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const ModJob &J = jobs[jb];
    if (threadIdx.x != 0 || J.n == 0) return;
    const int rt = *J.trow;
    if (rt < 0 || rt >= J.n) return;
    trace_row0<true>(J.d, rt, J.L.rowptr, J.L.col, J.L.val, *J.w, J.col + J.rowptr[rt], J.val + J.rowptr[rt]);
}

// Trace-row transform, fill, of every other row: an unchanged copy, one
// thread per entry (coalesced).  Rows before the trace row keep their
// positions; rows after it move by the trace row's change of length.
__global__ void __launch_bounds__(256) k_bt_copy(const ModJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const ModJob &J = jobs[jb];
    const int e = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (e >= J.L.nnz) return;
    const int rt = *J.trow;
    int dest = e;
    if (rt >= 0 && rt < J.n) {
        const int a = J.L.rowptr[rt], b = J.L.rowptr[rt + 1];
        if (e >= a && e < b) return;
        if (e >= b) dest = e + (J.rowptr[rt + 1] - J.rowptr[rt]) - (b - a);
    }
    J.col[dest] = J.L.col[e];
    J.val[dest] = J.L.val[e];
}

struct PatJob {
    int n;
    const int *arow;  // A (pattern)
    const int *acol;
    int *trow;        // A^T: counts, then row pointers
    int *cursor;      // scatter cursors (a copy of the row pointers)
    int *tcol_raw;    // scattered columns of A^T (unsorted rows)
    int *tcol;        // sorted
    int *srow;        // S: counts, then row pointers
    int *scol;
    double2 *sval;
};

// STEP 0: count the columns of A; 1: scatter A^T; 2: sort the rows of A^T
// (a wavefront per row); 3: count S rows; 4: fill S.
template <int STEP>
__global__ void __launch_bounds__(256) k_bt_pattern(const PatJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const PatJob &J = jobs[jb];
    if (STEP == 2) {
        // 16 lanes per row of A^T (rows up to 16 entries sorted in one pass)
        const int row = (blockIdx.x - bstart[jb]) * 16 + (int)(threadIdx.x >> 4);
        if (row < J.n) sort_row_wave<int, 16>(J.trow[row], J.trow[row + 1], J.tcol_raw, nullptr, J.tcol, nullptr);
        return;
    }
    if (STEP == 4) {
        // S = A + A^T filled row by row: 16 lanes per row, rows of up to 16
        // entries on both sides merged by shuffle, longer ones by one lane
        // (the counting pass stays one thread per row: it writes one value)
        const int r = (blockIdx.x - bstart[jb]) * 16 + (int)(threadIdx.x >> 4);
        if (r >= J.n) return;  // (uniform over the row's lanes)
        const int as = J.arow[r], na = J.arow[r + 1] - as, bs = J.trow[r], nb = J.trow[r + 1] - bs;
        if (na <= 16 && nb <= 16)
            union_row_group<true, 16>(as, na, bs, nb, J.acol, J.tcol, J.scol + J.srow[r], J.sval + J.srow[r]);
        else if ((threadIdx.x & 15) == 0)
            union_row<true>(r, J.arow, J.acol, J.trow, J.tcol, J.scol + J.srow[r], J.sval + J.srow[r]);
        return;
    }
    const int r = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (r >= J.n) return;
    if (STEP == 0) {
        for (int e = J.arow[r]; e < J.arow[r + 1]; ++e) atomicAdd(&J.trow[J.acol[e]], 1);
    } else if (STEP == 1) {
        for (int e = J.arow[r]; e < J.arow[r + 1]; ++e) J.tcol_raw[atomicAdd(&J.cursor[J.acol[e]], 1)] = r;
    } else {
        J.srow[r] = union_row<false>(r, J.arow, J.acol, J.trow, J.tcol, nullptr, nullptr);
    }
}

template <typename Job>
static void launch_rows(void (*kernel)(const Job *, const int *, int), const std::vector<Job> &jobs,
                        const std::vector<int> &blocks, hipStream_t s) {
    std::vector<int> pre;
    const int nb = block_prefix(blocks, pre);
    if (nb == 0) return;
    DevBuf<int> dpre = upload(pre, s);
    DevBuf<Job> dj = upload(jobs, s);
    kernel<<<(unsigned)nb, 256, 0, s>>>(dj.get(), dpre.get(), (int)jobs.size());
    SS_HIP(hipGetLastError());
}

void transform_batch(ss_liouv *hs, int count, bool trace, const ss_options &o, hipStream_t s) {
    if (count == 0) return;
    StreamScope scope(s);
    // per-system outputs, allocated up front with the size bounds
    std::vector<int64_t> boundA((size_t)count);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        StreamScope own(stream_peek(h));
        h->prepared = false;
        h->d_w.resize(1);
        const int64_t bA = (int64_t)h->L.nnz + (trace ? h->d : h->n);
        SS_REQUIRE(2 * bA < (int64_t(1) << 31), SS_E_INVALID_ARG, "transformed matrix too large for a batch");
        boundA[(size_t)k] = bA;
        h->A.rowptr.resize((size_t)h->n + 1);
        h->A.col.resize((size_t)bA);
        h->A.val.resize((size_t)bA);
        h->S.rowptr.resize((size_t)h->n + 1);
        h->S.col.resize((size_t)(2 * bA));
        h->S.val.resize((size_t)(2 * bA));
        h->perm.resize((size_t)h->n);
        h->iperm.resize((size_t)h->n);
    }
    // meta: trace row, nnz(A), nnz(S) per system; the weights
    DevBuf<int> meta((size_t)3 * count);
    DevBuf<double2> wmeta((size_t)count);
    SS_HIP(hipMemsetAsync(meta.get(), 0, meta.bytes(), s));
    int *m_trow = meta.get(), *m_nnzA = meta.get() + count, *m_nnzS = meta.get() + 2 * count;

    if (trace) {
        std::vector<ScalarJob> sj((size_t)count);
        for (int k = 0; k < count; ++k) {
            ss_liouv h = hs[k];
            sj[(size_t)k] =
                ScalarJob{h->n, h->d, h->L.view(), o.trace_row, o.weight, h->d_w.get(), wmeta.get() + k, m_trow + k};
        }
        DevBuf<ScalarJob> dsj = upload(sj, s);
        k_bt_scalars<<<(unsigned)count, 256, 0, s>>>(dsj.get());
        SS_HIP(hipGetLastError());
    }

    std::vector<ModJob> mj((size_t)count);
    std::vector<int> rblocks((size_t)count), wblocks((size_t)count);
    std::vector<ScanJob> scA((size_t)count);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        mj[(size_t)k] = ModJob{h->n, h->d, h->L.view(), trace ? 1 : 0, o.sigma, h->d_w.get(), m_trow + k,
                               h->A.rowptr.get(), h->A.col.get(), h->A.val.get()};
        rblocks[(size_t)k] = div_up(h->n, 256);
        wblocks[(size_t)k] = div_up(h->n, 16);
        scA[(size_t)k] = ScanJob{h->A.rowptr.get(), h->n, m_nnzA + k, nullptr};
    }
    launch_rows(k_bt_modify<false>, mj, rblocks, s);
    seg_scan(scA, s);
    if (trace) {
        std::vector<int> one((size_t)count, 1), eblocks((size_t)count);
        for (int k = 0; k < count; ++k) eblocks[(size_t)k] = div_up(hs[k]->L.nnz, 256);
        launch_rows(k_bt_trace_row, mj, one, s);
        launch_rows(k_bt_copy, mj, eblocks, s);
    } else {
        launch_rows(k_bt_modify<true>, mj, rblocks, s);
    }

    // A^T (pattern) in one arena, then S = A + A^T
    std::vector<size_t> off((size_t)count + 1, 0);
    for (int k = 0; k < count; ++k)
        off[(size_t)k + 1] = off[(size_t)k] + 2 * ((size_t)hs[k]->n + 1) + 2 * (size_t)boundA[(size_t)k];
    DevBuf<int> arena(off[(size_t)count]);
    SS_HIP(hipMemsetAsync(arena.get(), 0, arena.bytes(), s));
    std::vector<PatJob> pj((size_t)count);
    std::vector<ScanJob> scT((size_t)count), scS((size_t)count);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        int *base = arena.get() + off[(size_t)k];
        PatJob &p = pj[(size_t)k];
        p.n = h->n;
        p.arow = h->A.rowptr.get();
        p.acol = h->A.col.get();
        p.trow = base;
        p.cursor = base + h->n + 1;
        p.tcol_raw = base + 2 * (h->n + 1);
        p.tcol = p.tcol_raw + boundA[(size_t)k];
        p.srow = h->S.rowptr.get();
        p.scol = h->S.col.get();
        p.sval = h->S.val.get();
        scT[(size_t)k] = ScanJob{p.trow, h->n, nullptr, p.cursor};
        scS[(size_t)k] = ScanJob{p.srow, h->n, m_nnzS + k, nullptr};
    }
    launch_rows(k_bt_pattern<0>, pj, rblocks, s);
    seg_scan(scT, s);
    launch_rows(k_bt_pattern<1>, pj, rblocks, s);
    launch_rows(k_bt_pattern<2>, pj, wblocks, s);
    launch_rows(k_bt_pattern<3>, pj, rblocks, s);
    seg_scan(scS, s);
    launch_rows(k_bt_pattern<4>, pj, wblocks, s);

    // the one host wait: sizes, trace rows and weights
    std::vector<int> hm((size_t)3 * count);
    std::vector<double2> hw((size_t)count);
    SS_HIP(hipMemcpyAsync(hw.data(), wmeta.get(), sizeof(double2) * count, hipMemcpyDeviceToHost, s));
    d2h(hm.data(), meta.get(), hm.size(), s);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        h->A.n = h->n;
        h->A.nnz = hm[(size_t)count + k];
        h->S.n = h->n;
        h->S.nnz = hm[(size_t)2 * count + k];
        if (trace) {
            h->trow = hm[(size_t)k];
            h->w = hw[(size_t)k];
        } else {
            h->trow = 0;
            h->w = mk(0.0, 0.0);
        }
    }
}


// ------------------------------------------------------------ P A P^T
struct PermJob {
    int n, d;
    const int *perm, *iperm;
    Csr<double2> A;
    int *prow;        // P A P^T: counts, then row pointers
    int *pcol;
    double2 *pval;
    int *lucol;       // ILU(0) factor: pattern of P A P^T, values at the sentinel
    double2 *luval;   // (null when the factor is not ILU(0))
    int *diag;        // diagonal positions in P A P^T
    int *lu_diag;     // the same for the factor (null: not ILU(0))
    int *tpos;        // permuted positions of the diagonal of rho
    int trow;
    int *missing;     // rows without a diagonal entry
    int *q0;          // permuted position of the trace row
};

// STEP 0: row lengths; 1: rows (a wavefront each, columns mapped through
// iperm and rank-sorted as in k_perm_fill); 2: diagonal positions, trace
// positions and q0.
constexpr int PERM_G = 16;  // lanes per row in the permutation's fill (rows up to 16 entries in one pass)

template <int STEP>
__global__ void __launch_bounds__(256) k_bt_permute(const PermJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const PermJob &J = jobs[jb];
    if (STEP == 1) {
        // PERM_G lanes per row, 256 / PERM_G rows per workgroup
        const int lane = threadIdx.x & (PERM_G - 1);
        const int q = (blockIdx.x - bstart[jb]) * (256 / PERM_G) + (int)(threadIdx.x / PERM_G);
        if (q >= J.n) return;  // (uniform over the row's lanes)
        const int r = gld(J.perm + q);
        const int rs = gld(J.A.rowptr + r), re = gld(J.A.rowptr + r + 1);
        const int o = gld(J.prow + q);
        if (re - rs <= PERM_G) {
            // the whole row in one pass: each lane maps its own column, the
            // ranks come from the other lanes' values by shuffle (the trip
            // count is the same for all lanes of the row)
            const int e = rs + lane;
            const int c = (e < re) ? gld(J.iperm + gld(J.A.col + e)) : 0x7fffffff;
            int rank = 0;
            for (int f = 0; f < re - rs; ++f) rank += (__shfl(c, f, PERM_G) < c);
            if (e < re) {
                J.pcol[o + rank] = c;
                J.pval[o + rank] = gld(J.A.val + e);
                if (J.lucol) {
                    J.lucol[o + rank] = c;
                    set_sentinel(J.luval + o + rank);
                }
            }
            return;
        }
        for (int e = rs + lane; e < re; e += PERM_G) {
            const int c = gld(J.iperm + gld(J.A.col + e));
            int rank = 0;
            for (int f = rs; f < re; ++f) rank += (gld(J.iperm + gld(J.A.col + f)) < c);
            J.pcol[o + rank] = c;
            J.pval[o + rank] = J.A.val[e];
            if (J.lucol) {
                J.lucol[o + rank] = c;
                set_sentinel(J.luval + o + rank);
            }
        }
        return;
    }
    const int r = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (r >= J.n) return;
    if (STEP == 0) {
        const int a = J.perm[r];
        J.prow[r] = J.A.rowptr[a + 1] - J.A.rowptr[a];
        return;
    }
    int lo = J.prow[r], hi = J.prow[r + 1] - 1, pos = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = J.pcol[mid];
        if (c == r) { pos = mid; break; }
        if (c < r) lo = mid + 1; else hi = mid - 1;
    }
    J.diag[r] = pos;
    if (J.lu_diag) J.lu_diag[r] = pos;
    if (pos < 0) atomicAdd(J.missing, 1);
    if (r < J.d) J.tpos[r] = J.iperm[(int64_t)r * (J.d + 1)];
    if (r == 0) *J.q0 = J.iperm[J.trow];
}

void permute_batch(ss_liouv *hs, int count, bool ilu0, hipStream_t s, std::vector<PermResult> &res) {
    res.assign((size_t)count, PermResult{});
    if (count == 0) return;
    StreamScope scope(s);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        StreamScope own(stream_peek(h));
        h->Ap.alloc(h->n, h->A.nnz);
        h->diag.resize((size_t)h->n);
        h->tpos.resize((size_t)h->d);
        if (ilu0) {
            h->LU.alloc(h->n, h->A.nnz);
            h->lu_diag.resize((size_t)h->n);
        }
    }
    DevBuf<int> meta((size_t)2 * count);
    SS_HIP(hipMemsetAsync(meta.get(), 0, meta.bytes(), s));
    std::vector<PermJob> pj((size_t)count);
    std::vector<int> rblocks((size_t)count), wblocks((size_t)count);
    std::vector<ScanJob> sc((size_t)count);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        PermJob &p = pj[(size_t)k];
        p.n = h->n;
        p.d = h->d;
        p.perm = h->perm.get();
        p.iperm = h->iperm.get();
        p.A = h->A.view();
        p.prow = h->Ap.rowptr.get();
        p.pcol = h->Ap.col.get();
        p.pval = h->Ap.val.get();
        p.lucol = ilu0 ? h->LU.col.get() : nullptr;
        p.luval = ilu0 ? h->LU.val.get() : nullptr;
        p.diag = h->diag.get();
        p.lu_diag = ilu0 ? h->lu_diag.get() : nullptr;
        p.tpos = h->tpos.get();
        p.trow = h->trow;
        p.missing = meta.get() + k;
        p.q0 = meta.get() + count + k;
        rblocks[(size_t)k] = div_up(h->n, 256);
        wblocks[(size_t)k] = div_up(h->n, 256 / PERM_G);
        sc[(size_t)k] = ScanJob{p.prow, h->n, nullptr, ilu0 ? h->LU.rowptr.get() : nullptr};
    }
    launch_rows(k_bt_permute<0>, pj, rblocks, s);
    seg_scan(sc, s);
    launch_rows(k_bt_permute<1>, pj, wblocks, s);
    launch_rows(k_bt_permute<2>, pj, rblocks, s);
    std::vector<int> hm((size_t)2 * count);
    d2h(hm.data(), meta.get(), hm.size(), s);
    for (int k = 0; k < count; ++k) {
        res[(size_t)k].missing = hm[(size_t)k];
        hs[k]->q0 = hm[(size_t)count + k];
        hs[k]->diag_added = hm[(size_t)k];
    }
}


// ------------------------------------------- workgroup-resident problems
struct SideJob {
    int n, upper;
    const int *lvl;     // level of each row
    int *cnt;           // nlev + 1 counts, then scatter cursors
    int *ptr;           // level pointers
    int4 *slot;         // level-ordered slots {row, first, end, 0}
    const int *rowptr;  // factor pattern
    const int *diag;
};

// STEP 0: rows per level; 1: scatter the rows into level order (the order
// inside a level does not matter: its rows are independent).
// atomicAdd(cnt + key, 1) for every active lane of the wavefront, with one
// atomic per distinct key: the lanes sharing a key take consecutive values in
// lane order (rows of one level sit close together in the ordering, so a
// wavefront holds few distinct levels).
__device__ inline int wave_claim(int *cnt, int key) {
    const int lane = threadIdx.x & 63;
    int pos = 0;
    unsigned long long todo = __ballot(1);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, leader, 64);
        const unsigned long long m = __ballot(key == k) & todo;
        int base = 0;
        if (lane == leader) base = atomicAdd(cnt + k, __popcll(m));
        base = __shfl(base, leader, 64);
        if ((m >> lane) & 1ull) pos = base + __popcll(m & ((1ull << lane) - 1ull));
        todo &= ~m;
    }
    return pos;
}

template <int STEP>
__global__ void __launch_bounds__(256) k_bt_levels(const SideJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const SideJob &J = jobs[jb];
    const int i = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (i >= J.n) return;
    const int pos = wave_claim(J.cnt, J.lvl[i]);
    if (STEP == 0) return;
    J.slot[pos] = J.upper ? make_int4(i, J.diag[i] + 1, J.rowptr[i + 1], 0)
                          : make_int4(i, J.rowptr[i], J.diag[i], J.rowptr[i + 1]);
}

template <typename T>
struct PackJob {
    int n, upper;
    const int4 *in;  // level-ordered slots
    const int *col;  // factor (precision T)
    const T *val;
    int4 *slot;
    int *pcol;
    T *pval, *aux;
};

// The packed level-order layout of one factor side (see PackedSide).
template <typename T>
__global__ void __launch_bounds__(256) k_bt_pack(const PackJob<T> *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const PackJob<T> &J = jobs[jb];
    const int idx = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (idx >= J.n) return;
    const int4 sl = J.in[idx];
    const int len = sl.z - sl.y;
    J.slot[idx] = make_int4(sl.x, sl.y, len, 0);
    constexpr int K = WgK<T>::value;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        J.pcol[(size_t)k * J.n + idx] = (k < len) ? J.col[sl.y + k] : 0;
        J.pval[(size_t)k * J.n + idx] = (k < len) ? J.val[sl.y + k] : czero<T>();
    }
    J.aux[idx] = J.upper ? J.val[sl.y - 1] : czero<T>();
}

struct StartJob {
    int n, d, trace, trow;
    double2 w;
    const int *perm;
    double2 *x, *b;  // zeroed
    int random;      // SS_FLAG_RANDOM_START (inverse power)
    uint64_t seed;
};

// Start vector and right-hand side in the permuted order: trace row
// b = w e_trow, x = 0; inverse power x = vec(I / d).
__global__ void __launch_bounds__(256) k_bt_start(const StartJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const StartJob &J = jobs[jb];
    const int q = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (q >= J.n) return;
    const int r = J.perm[q];
    if (J.trace) {
        if (r == J.trow) J.b[q] = J.w;
    } else if (J.random) {
        J.x[q] = random_start_value(J.d, r, J.seed);
    } else if (r % (J.d + 1) == 0) {
        J.x[q] = mk(1.0 / J.d, 0.0);
    }
}

// Carves aligned pieces out of one allocation.
struct Carver {
    size_t off = 0;
    template <typename U>
    size_t take(size_t count) {
        const size_t at = (off + 255) & ~size_t(255);
        off = at + sizeof(U) * std::max<size_t>(count, 1);
        return at;
    }
};

void levels_setup_batch(ss_liouv *hs, int count, hipStream_t s, LevelBatch &out) {
    out = LevelBatch();
    out.hs.assign(hs, hs + count);
    if (count == 0) return;
    StreamScope scope(s);
    for (int k = 0; k < count; ++k) out.pos[hs[k]] = k;
    // level analysis of both sides of every factor: levels at -1, one launch per side
    std::vector<size_t> loff((size_t)count + 1, 0);
    for (int k = 0; k < count; ++k) loff[(size_t)k + 1] = loff[(size_t)k] + 2 * (size_t)std::max(hs[k]->n, 1);
    DevBuf<int> lvl(loff[(size_t)count]);
    DevBuf<unsigned> meta((size_t)4 * count);  // per side: status, max level
    SS_HIP(hipMemsetAsync(lvl.get(), 0xff, lvl.bytes(), s));
    SS_HIP(hipMemsetAsync(meta.get(), 0, meta.bytes(), s));
    std::vector<LevelJob> jl((size_t)count), ju((size_t)count);
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        for (int side = 0; side < 2; ++side) {
            LevelJob &j = side ? ju[(size_t)k] : jl[(size_t)k];
            j.n = h->n;
            j.rowptr = h->LU.rowptr.get();
            j.col = h->LU.col.get();
            j.diag = h->lu_diag.get();
            j.lvl = lvl.get() + loff[(size_t)k] + (size_t)side * std::max(h->n, 1);
            j.status = meta.get() + 4 * k + 2 * side;
            j.maxlvl = reinterpret_cast<int *>(meta.get() + 4 * k + 2 * side + 1);
        }
    }
    levels_batch<false>(jl.data(), count, s);
    levels_batch<true>(ju.data(), count, s);
    std::vector<unsigned> hm((size_t)4 * count);
    d2h(hm.data(), meta.get(), hm.size(), s);
    out.nl.resize((size_t)count);
    out.nu.resize((size_t)count);
    for (int k = 0; k < count; ++k) {
        SS_REQUIRE(!(hm[4 * (size_t)k] & STATUS_SPIN_TIMEOUT) && !(hm[4 * (size_t)k + 2] & STATUS_SPIN_TIMEOUT),
                   SS_E_TIMEOUT, "level analysis: dependency wait timed out");
        out.nl[(size_t)k] = hs[k]->n ? (int)hm[4 * (size_t)k + 1] + 1 : 0;
        out.nu[(size_t)k] = hs[k]->n ? (int)hm[4 * (size_t)k + 3] + 1 : 0;
    }
    // schedules of both sides in one arena: counts, scan, scatter
    struct Lay {
        size_t lptr, uptr, lcnt, ucnt, lslot, uslot;
    };
    std::vector<Lay> lay((size_t)count);
    Carver cv;
    for (int k = 0; k < count; ++k) {
        const size_t n = (size_t)std::max(hs[k]->n, 1);
        Lay &L = lay[(size_t)k];
        L.lptr = cv.take<int>((size_t)out.nl[(size_t)k] + 1);
        L.uptr = cv.take<int>((size_t)out.nu[(size_t)k] + 1);
        L.lcnt = cv.take<int>((size_t)out.nl[(size_t)k] + 1);
        L.ucnt = cv.take<int>((size_t)out.nu[(size_t)k] + 1);
        L.lslot = cv.take<int4>(n);
        L.uslot = cv.take<int4>(n);
    }
    out.arena.resize(cv.off);
    SS_HIP(hipMemsetAsync(out.arena.get(), 0, out.arena.bytes(), s));
    unsigned char *base = out.arena.get();
    std::vector<SideJob> sj;
    std::vector<ScanJob> sc;
    std::vector<int> sblocks;
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        const Lay &L = lay[(size_t)k];
        for (int side = 0; side < 2; ++side) {
            SideJob j;
            j.n = h->n;
            j.upper = side;
            j.lvl = (side ? ju : jl)[(size_t)k].lvl;
            j.cnt = (int *)(base + (side ? L.ucnt : L.lcnt));
            j.ptr = (int *)(base + (side ? L.uptr : L.lptr));
            j.slot = (int4 *)(base + (side ? L.uslot : L.lslot));
            j.rowptr = h->LU.rowptr.get();
            j.diag = h->lu_diag.get();
            sj.push_back(j);
            sblocks.push_back(div_up(h->n, 256));
            sc.push_back(ScanJob{j.cnt, side ? out.nu[(size_t)k] : out.nl[(size_t)k], nullptr, j.ptr});
        }
        out.lptr.push_back((const int *)(base + L.lptr));
        out.uptr.push_back((const int *)(base + L.uptr));
        out.lslot.push_back((const int4 *)(base + L.lslot));
        out.uslot.push_back((const int4 *)(base + L.uslot));
    }
    launch_rows(k_bt_levels<0>, sj, sblocks, s);
    seg_scan(sc, s);
    launch_rows(k_bt_levels<1>, sj, sblocks, s);
    SS_HIP(hipStreamSynchronize(s));  // lvl is released on return
}

template <typename T>
void wg_setup_batch(ss_liouv *hs, int count, int method, const double *tols, const ss_options &o,
                    const LevelBatch &lb, hipStream_t s, WgBatch<T> &out) {
    out.probs.assign((size_t)count, WgProblem<T>{});
    out.levels.assign((size_t)count, 0);
    if (count == 0) return;
    StreamScope scope(s);
    const bool trace = (method == SS_TRACE_BICGSTAB || method == SS_TRACE_GMRES);
    // one arena for every system's packed factors, vectors and scratch
    constexpr int K = WgK<T>::value;
    struct Lay {
        size_t pls, pus, plc, puc, plv, puv, pla, pua, work, ysc, x, r, b, res;
    };
    std::vector<Lay> lay((size_t)count);
    std::vector<int> li((size_t)count);
    Carver cv;
    for (int k = 0; k < count; ++k) {
        auto it = lb.pos.find(hs[k]);
        SS_REQUIRE(it != lb.pos.end(), SS_E_STATE, "no level schedule for a system of the batch");
        li[(size_t)k] = it->second;
        const size_t n = (size_t)std::max(hs[k]->n, 1);
        Lay &L = lay[(size_t)k];
        L.pls = cv.take<int4>(n);
        L.pus = cv.take<int4>(n);
        L.plc = cv.take<int>(n * K);
        L.puc = cv.take<int>(n * K);
        L.plv = cv.take<T>(n * K);
        L.puv = cv.take<T>(n * K);
        L.pla = cv.take<T>(n);
        L.pua = cv.take<T>(n);
        L.work = cv.take<T>(11 * n);
        L.ysc = cv.take<T>(n);
        L.x = cv.take<double2>(n);
        L.r = cv.take<double2>(n);
        L.b = cv.take<double2>(n);
        L.res = cv.take<WgResult>(1);
    }
    out.arena.resize(cv.off);
    SS_HIP(hipMemsetAsync(out.arena.get(), 0, out.arena.bytes(), s));
    unsigned char *base = out.arena.get();
    auto at = [&](size_t off) { return base + off; };

    std::vector<PackJob<T>> pj;
    std::vector<StartJob> st;
    std::vector<int> pblocks, stblocks;
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        const Lay &L = lay[(size_t)k];
        const int q = li[(size_t)k];
        const CsrBuf<T> &LUin = lu_of<T>(h);
        for (int side = 0; side < 2; ++side) {
            PackJob<T> p;
            p.n = h->n;
            p.upper = side;
            p.in = side ? lb.uslot[(size_t)q] : lb.lslot[(size_t)q];
            p.col = LUin.col.get();
            p.val = LUin.val.get();
            p.slot = (int4 *)at(side ? L.pus : L.pls);
            p.pcol = (int *)at(side ? L.puc : L.plc);
            p.pval = (T *)at(side ? L.puv : L.plv);
            p.aux = (T *)at(side ? L.pua : L.pla);
            pj.push_back(p);
            pblocks.push_back(div_up(h->n, 256));
        }
        st.push_back(StartJob{h->n, h->d, trace ? 1 : 0, h->trow, h->w, h->perm.get(), (double2 *)at(L.x),
                              (double2 *)at(L.b), (o.flags & SS_FLAG_RANDOM_START) ? 1 : 0, (uint64_t)o.seed});
        stblocks.push_back(div_up(h->n, 256));
    }
    launch_rows(k_bt_pack<T>, pj, pblocks, s);
    launch_rows(k_bt_start, st, stblocks, s);

    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        const Lay &L = lay[(size_t)k];
        const int q = li[(size_t)k];
        WgProblem<T> &P = out.probs[(size_t)k];
        std::memset(&P, 0, sizeof(P));
        P.n = h->n;
        P.d = h->d;
        P.q0 = h->q0;
        P.trace = trace ? 1 : 0;
        P.nlev_l = lb.nl[(size_t)q];
        P.nlev_u = lb.nu[(size_t)q];
        P.maxiter = o.maxiter;
        P.max_outer = o.max_outer > 0 ? o.max_outer : 20;
        P.tol = tols[k];
        P.rtol_in = (o.inner_tol > 0) ? o.inner_tol : (o.prec == SS_MIXED ? 1e-4 : 0.0);
        P.force_breakdown = (o.flags & SS_FLAG_FORCE_BREAKDOWN) ? 1 : 0;
        P.sigma = o.sigma;
        P.w = h->w;
        P.A = ap_of<T>(h).view();
        P.A64 = h->Ap.view();
        P.LU = lu_of<T>(h).view();
        P.diag = h->lu_diag.get();
        P.lptr = lb.lptr[(size_t)q];
        P.lslot = (const int4 *)at(L.pls);
        P.lcol = (const int *)at(L.plc);
        P.lval = (const T *)at(L.plv);
        P.uptr = lb.uptr[(size_t)q];
        P.uslot = (const int4 *)at(L.pus);
        P.ucol = (const int *)at(L.puc);
        P.uval = (const T *)at(L.puv);
        P.uaux = (const T *)at(L.pua);
        P.tpos = h->tpos.get();
        P.b64 = trace ? (const double2 *)at(L.b) : nullptr;
        P.x64 = (double2 *)at(L.x);
        P.r64 = (double2 *)at(L.r);
        P.work = (T *)at(L.work);
        P.ysc = (T *)at(L.ysc);
        P.res = (WgResult *)at(L.res);
        out.levels[(size_t)k] = P.nlev_l + P.nlev_u;
    }
}
template void wg_setup_batch<float2>(ss_liouv *, int, int, const double *, const ss_options &, const LevelBatch &,
                                     hipStream_t, WgBatch<float2> &);
template void wg_setup_batch<double2>(ss_liouv *, int, int, const double *, const ss_options &, const LevelBatch &,
                                      hipStream_t, WgBatch<double2> &);


// --------------------------------------------------------------- finish
struct FinishJob {
    int n, d, hermitize;
    const double2 *x;  // solution, permuted
    const int *perm, *tpos;
    Csr<double2> L;    // assembled L (certificate)
    const int *prow, *pcol;  // P A P^T pattern (bandwidth, profile)
    int *colmax;       // n scratch, zeroed
    double2 *tmp;      // n scratch (before the Hermitian part is taken)
    double2 *rho;      // the result, natural order (the caller's device buffer or staging)
    double *out;       // tr.x, tr.y, ||L rho||^2, herm err, ub, lb, up, lp
};

constexpr int FIN_BS = 512;

template <typename V, typename Op>
__device__ inline V fin_reduce(V v, V *sh, Op op) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = FIN_BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    const V r = sh[0];
    __syncthreads();
    return r;
}

// One block per system: the steps of finish() with the same formulas; the
// trace is summed in the order of the one-system kernel (256 strided partial
// sums and a tree), so rho itself is identical; the certificate's sums run
// in another order than the device-wide SpMV and norm.
__global__ void __launch_bounds__(FIN_BS) k_bt_finish(const FinishJob *jobs) {
    __shared__ double sx[FIN_BS], sy[FIN_BS];
    __shared__ long long sl[FIN_BS];
    const FinishJob &J = jobs[blockIdx.x];
    const int t = threadIdx.x, n = J.n, d = J.d;
    // trace of the permuted solution
    double ax = 0, ay = 0;
    if (t < 256)
        for (int k = t; k < d; k += 256) {
            const double2 v = J.x[J.tpos[k]];
            ax += v.x;
            ay += v.y;
        }
    sx[t] = ax;
    sy[t] = ay;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            sx[t] += sx[t + off];
            sy[t] += sy[t + off];
        }
        __syncthreads();
    }
    const double2 tr = mk(sx[0], sy[0]);
    __syncthreads();
    const double2 inv = cdiv(mk(1.0, 0.0), tr);
    double2 *r1 = J.hermitize ? J.tmp : J.rho;
    for (int q = t; q < n; q += FIN_BS) r1[J.perm[q]] = cmul(J.x[q], inv);
    __syncthreads();
    if (J.hermitize) {
        for (int q = t; q < n; q += FIN_BS) {
            const int i = q % d, j = q / d;
            const double2 a = J.tmp[q], b = J.tmp[(int64_t)i * d + j];
            J.rho[q] = mk(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        }
        __syncthreads();
    }
    // certificate, Hermiticity error, bandwidth and profile
    double r2 = 0, herm = 0;
    long long ub = 0, lb = 0, up = 0;
    for (int r = t; r < n; r += FIN_BS) {
        double2 acc = mk(0.0, 0.0);
        for (int e = J.L.rowptr[r]; e < J.L.rowptr[r + 1]; ++e) acc = cadd(acc, cmul(J.L.val[e], J.rho[J.L.col[e]]));
        r2 += acc.x * acc.x + acc.y * acc.y;
        const int i = r % d, j = r / d;
        const double2 a = J.rho[r], b = J.rho[(int64_t)i * d + j];
        const double dx = a.x - b.x, dy = a.y + b.y;
        herm = fmax(herm, sqrt(dx * dx + dy * dy));
        const int rs = J.prow[r], re = J.prow[r + 1];
        if (re > rs) {
            const int cmin = J.pcol[rs], cmax = J.pcol[re - 1];
            ub = max(ub, (long long)(cmax - r));
            lb = max(lb, (long long)(r - cmin));
            if (cmax > r) up += cmax - r;
            for (int e = rs; e < re; ++e) {
                const int c = J.pcol[e];
                if (r > c) atomicMax(&J.colmax[c], r - c);
            }
        }
    }
    r2 = fin_reduce(r2, sx, [](double p, double q) { return p + q; });
    herm = fin_reduce(herm, sx, [](double p, double q) { return fmax(p, q); });
    ub = fin_reduce(ub, sl, [](long long p, long long q) { return max(p, q); });
    lb = fin_reduce(lb, sl, [](long long p, long long q) { return max(p, q); });
    up = fin_reduce(up, sl, [](long long p, long long q) { return p + q; });
    __syncthreads();
    long long lp = 0;
    for (int c = t; c < n; c += FIN_BS) lp += J.colmax[c];
    lp = fin_reduce(lp, sl, [](long long p, long long q) { return p + q; });
    if (t == 0) {
        J.out[0] = tr.x;
        J.out[1] = tr.y;
        J.out[2] = r2;
        J.out[3] = herm;
        J.out[4] = (double)ub;
        J.out[5] = (double)lb;
        J.out[6] = (double)up;
        J.out[7] = (double)lp;
    }
}

void finish_batch(ss_liouv *hs, int count, const double2 *const *xs, const ss_options &o, const double *tols,
                  const SolveStats *st, double *const *rho_out, ss_info *const *infos, int *status, hipStream_t s) {
    if (count == 0) return;
    StreamScope scope(s);
    const bool herm = (o.flags & SS_FLAG_HERMITIZE) != 0;
    std::vector<char> on_dev((size_t)count, 0);
    std::vector<size_t> off((size_t)count + 1, 0), soff((size_t)count + 1, 0);
    for (int k = 0; k < count; ++k) {
        const size_t n = (size_t)hs[k]->n;
        on_dev[(size_t)k] = rho_out[k] && is_device_ptr(rho_out[k]);
        off[(size_t)k + 1] = off[(size_t)k] + (herm ? n : 0);
        soff[(size_t)k + 1] = soff[(size_t)k] + (on_dev[(size_t)k] ? 0 : n);
    }
    size_t nint = 0;
    for (int k = 0; k < count; ++k) nint += (size_t)hs[k]->n;
    DevBuf<int> colmax(nint);
    DevBuf<double2> tmp(off[(size_t)count]), stage(soff[(size_t)count]);
    DevBuf<double> out((size_t)8 * count);
    SS_HIP(hipMemsetAsync(colmax.get(), 0, colmax.bytes(), s));
    std::vector<FinishJob> fj((size_t)count);
    size_t ci = 0;
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        FinishJob &j = fj[(size_t)k];
        j.n = h->n;
        j.d = h->d;
        j.hermitize = herm ? 1 : 0;
        j.x = xs[k];
        j.perm = h->perm.get();
        j.tpos = h->tpos.get();
        j.L = h->L.view();
        j.prow = h->Ap.rowptr.get();
        j.pcol = h->Ap.col.get();
        j.colmax = colmax.get() + ci;
        ci += (size_t)h->n;
        j.tmp = tmp.get() + off[(size_t)k];
        j.rho = on_dev[(size_t)k] ? reinterpret_cast<double2 *>(rho_out[k]) : stage.get() + soff[(size_t)k];
        j.out = out.get() + 8 * (size_t)k;
    }
    DevBuf<FinishJob> dj = upload(fj, s);
    k_bt_finish<<<(unsigned)count, FIN_BS, 0, s>>>(dj.get());
    SS_HIP(hipGetLastError());
    std::vector<double> ho((size_t)8 * count);
    d2h(ho.data(), out.get(), ho.size(), s);
    if (soff[(size_t)count]) {
        std::vector<double2> hr(soff[(size_t)count]);
        d2h(hr.data(), stage.get(), hr.size(), s);
        for (int k = 0; k < count; ++k)
            if (rho_out[k] && !on_dev[(size_t)k])
                std::memcpy(rho_out[k], hr.data() + soff[(size_t)k], sizeof(double2) * hs[k]->n);
    }
    for (int k = 0; k < count; ++k) {
        const double *v = ho.data() + 8 * (size_t)k;
        const int64_t bw = (int64_t)v[4] + (int64_t)v[5] + 1;
        const int64_t pf = (int64_t)v[6] + (int64_t)v[7];
        status[k] = fill_info(hs[k], o, tols[k], st[k], sqrt(v[2]), v[3], mk(v[0], v[1]), bw, pf, infos[k],
                              stream_peek(hs[k]));
    }
}


__global__ void k_bt_results(const WgResult *const *src, int count, WgResult *dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[k] = *src[k];
}

void read_results(const std::vector<const WgResult *> &src, std::vector<WgResult> &out, hipStream_t s) {
    out.resize(src.size());
    if (src.empty()) return;
    StreamScope scope(s);
    DevBuf<const WgResult *> dsrc = upload(src, s);
    DevBuf<WgResult> dst(src.size());
    k_bt_results<<<div_up((int64_t)src.size(), 256), 256, 0, s>>>(dsrc.get(), (int)src.size(), dst.get());
    SS_HIP(hipGetLastError());
    d2h(out.data(), dst.get(), out.size(), s);
}


// ------------------------------------------------------ complex64 copies
struct C64Job {
    int n, nnz;
    const int *rowptr, *col;
    const double2 *val;
    int *rowptr32, *col32;
    float2 *val32;
};

// One job per matrix: pattern copied, values rounded to complex64 (as
// copy_pattern_c64 does for one matrix).
__global__ void __launch_bounds__(256) k_bt_c64(const C64Job *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const C64Job &J = jobs[jb];
    const int i = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (i <= J.n) J.rowptr32[i] = J.rowptr[i];
    if (i < J.nnz) {
        J.col32[i] = J.col[i];
        J.val32[i] = from_c128<float2>(J.val[i]);
    }
}

void c64_copies_batch(ss_liouv *hs, int count, hipStream_t s) {
    if (count == 0) return;
    StreamScope scope(s);
    std::vector<C64Job> jobs;
    std::vector<int> blocks;
    for (int k = 0; k < count; ++k) {
        ss_liouv h = hs[k];
        StreamScope own(stream_peek(h));
        h->Ap32.alloc(h->Ap.n, h->Ap.nnz);
        h->LU32.alloc(h->LU.n, h->LU.nnz);
        for (int m = 0; m < 2; ++m) {
            const CsrBuf<double2> &a = m ? h->LU : h->Ap;
            CsrBuf<float2> &b = m ? h->LU32 : h->Ap32;
            jobs.push_back(C64Job{a.n, a.nnz, a.rowptr.get(), a.col.get(), a.val.get(), b.rowptr.get(), b.col.get(),
                                  b.val.get()});
            blocks.push_back(div_up((int64_t)std::max(a.n + 1, a.nnz), 256));
        }
    }
    launch_rows(k_bt_c64, jobs, blocks, s);
    SS_HIP(hipStreamSynchronize(s));
}

}  // namespace ss
