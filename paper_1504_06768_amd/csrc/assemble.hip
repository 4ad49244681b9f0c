// Liouvillian assembly on the device (section "Steady-state density matrix",
// eq. lindblad, column stacking of eq. eigval).
//
// With vec(A rho B) = (B^T (x) A) vec(rho), the Lindblad generator is
//   L = I (x) Gpre + Gpost (x) I + sum_k conj(C_k) (x) C_k,
//   Gpre  = -i H - 1/2 D,        D = sum_k C_k^+ C_k,
//   Gpost = (i H - 1/2 D)^T.
// Row r = i + d j of L therefore holds
//   columns k + d j     with Gpre[i, k]                    (I (x) Gpre)
//   columns i + d l     with Gpost[j, l]                   (Gpost (x) I)
//   columns k + d l     with conj(C[j, l]) C[i, k]         (conj(C) (x) C)
// and is produced directly, sorted and with duplicates summed in a fixed
// order, by one thread; no global sort is needed.
#include <cstdlib>
#include <cstring>

#include "assemble.hpp"
#include "batch.hpp"
#include "csr_tools.hpp"

namespace ss {

// ---------------------------------------------------- d x d coefficient rows
// One workgroup per row i.  Terms are added one sparse row at a time with a
// barrier in between, so every dense entry receives its contributions in the
// same order on every run.
__global__ void __launch_bounds__(64) k_gterms(int d, Csr<double2> H, Csr<double2> Ht, const OpPair *ops,
                                               int nops, double2 *Gpre, double2 *Gpost) {
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    double2 *pre = Gpre + (size_t)i * d;
    double2 *post = Gpost + (size_t)i * d;
    // -i H[i, :]  and  +i H^T[i, :]
    for (int e = H.rowptr[i] + t; e < H.rowptr[i + 1]; e += 64) {
        const double2 h = H.val[e];
        pre[H.col[e]] = cadd(pre[H.col[e]], mk(h.y, -h.x));
    }
    for (int e = Ht.rowptr[i] + t; e < Ht.rowptr[i + 1]; e += 64) {
        const double2 h = Ht.val[e];
        post[Ht.col[e]] = cadd(post[Ht.col[e]], mk(-h.y, h.x));
    }
    __syncthreads();
    for (int k = 0; k < nops; ++k) {
        const Csr<double2> C = ops[k].C, Ct = ops[k].Ct;
        // m runs over the non-zeros of column i of C (row i of C^T)
        for (int em = Ct.rowptr[i]; em < Ct.rowptr[i + 1]; ++em) {
            const int m = Ct.col[em];
            const double2 cmi = Ct.val[em];  // C[m, i]
            for (int e = C.rowptr[m] + t; e < C.rowptr[m + 1]; e += 64) {
                const int c = C.col[e];
                const double2 cmc = C.val[e];                        // C[m, c]
                const double2 dpre = cmulc(cmi, cmc);                // conj(C[m,i]) C[m,c]
                const double2 dpost = cmulc(cmc, cmi);               // C[m,i] conj(C[m,c])
                pre[c] = csub(pre[c], cscale(dpre, 0.5));
                post[c] = csub(post[c], cscale(dpost, 0.5));
            }
            __syncthreads();
        }
    }
}

// Dense rows -> CSR with exact zeros dropped (one wavefront per row).
__global__ void __launch_bounds__(256) k_dense_count(int d, const double2 *G, int *cnt) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= d) return;
    int c = 0;
    for (int j = lane; j < d; j += 64) {
        const double2 v = G[(size_t)row * d + j];
        c += (v.x != 0.0 || v.y != 0.0);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if (lane == 0) cnt[row] = c;
}

__global__ void __launch_bounds__(256) k_dense_fill(int d, const double2 *G, const int *rowptr, int *col,
                                                    double2 *val) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= d) return;
    int pos = rowptr[row];
    for (int j0 = 0; j0 < d; j0 += 64) {
        const int j = j0 + lane;
        double2 v = mk(0.0, 0.0);
        if (j < d) v = G[(size_t)row * d + j];
        const bool nz = (j < d) && (v.x != 0.0 || v.y != 0.0);
        const unsigned long long mask = __ballot(nz);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (nz) {
            col[pos + before] = j;
            val[pos + before] = v;
        }
        pos += __popcll(mask);
    }
}

static void dense_to_csr(int d, const double2 *G, CsrBuf<double2> &out, hipStream_t s) {
    DevBuf<int> cnt((size_t)d + 1);
    k_dense_count<<<div_up(d, 4), 256, 0, s>>>(d, G, cnt.get());
    SS_HIP(hipGetLastError());
    out.rowptr.resize((size_t)d + 1);
    const int64_t nnz = scan_exclusive(cnt.get(), out.rowptr.get(), d, s, true);
    out.n = d;
    out.nnz = (int)nnz;
    out.col.resize((size_t)nnz);
    out.val.resize((size_t)nnz);
    k_dense_fill<<<div_up(d, 4), 256, 0, s>>>(d, G, out.rowptr.get(), out.col.get(), out.val.get());
    SS_HIP(hipGetLastError());
}

// -------------------------------------------------------- Liouvillian rows
struct RowSources {
    int d;
    Csr<double2> Gp;  // Gpre
    Csr<double2> Gq;  // Gpost
    const OpPair *ops;
    int nops;
};

constexpr int BIG = 0x7fffffff;

// Walks row r = i + d j of L in increasing column order; emits every non-zero
// (column, value).  Returns the number emitted.
template <bool FILL>
__device__ int liouvillian_row(const RowSources &S, int r, int *out_col, double2 *out_val) {
    const int d = S.d;
    const int i = r % d, j = r / d;
    int oc[MAX_COPS], oce[MAX_COPS];
    for (int k = 0; k < S.nops; ++k) {
        oc[k] = S.ops[k].C.rowptr[j];
        oce[k] = S.ops[k].C.rowptr[j + 1];
    }
    int bq = S.Gq.rowptr[j];
    const int bqe = S.Gq.rowptr[j + 1];
    bool a_pending = true;
    int cnt = 0;
    while (true) {
        // next column block l
        int l = a_pending ? j : BIG;
        if (bq < bqe) l = min(l, S.Gq.col[bq]);
        for (int k = 0; k < S.nops; ++k)
            if (oc[k] < oce[k]) l = min(l, S.ops[k].C.col[oc[k]]);
        if (l == BIG) break;
        const bool useA = a_pending && (l == j);
        const bool useB = (bq < bqe) && (S.Gq.col[bq] == l);
        const double2 bval = useB ? S.Gq.val[bq] : mk(0.0, 0.0);
        // inner cursors over k
        int ka = useA ? S.Gp.rowptr[i] : 0;
        const int kae = useA ? S.Gp.rowptr[i + 1] : 0;
        bool bpend = useB;
        int ki[MAX_COPS], kie[MAX_COPS];
        double2 coef[MAX_COPS];
        for (int k = 0; k < S.nops; ++k) {
            const bool use = (oc[k] < oce[k]) && (S.ops[k].C.col[oc[k]] == l);
            ki[k] = use ? S.ops[k].C.rowptr[i] : 0;
            kie[k] = use ? S.ops[k].C.rowptr[i + 1] : 0;
            coef[k] = use ? cconj(S.ops[k].C.val[oc[k]]) : mk(0.0, 0.0);
        }
        while (true) {
            int kk = (ka < kae) ? S.Gp.col[ka] : BIG;
            if (bpend) kk = min(kk, i);
            for (int k = 0; k < S.nops; ++k)
                if (ki[k] < kie[k]) kk = min(kk, S.ops[k].C.col[ki[k]]);
            if (kk == BIG) break;
            double2 v = mk(0.0, 0.0);
            if (ka < kae && S.Gp.col[ka] == kk) { v = cadd(v, S.Gp.val[ka]); ++ka; }
            if (bpend && kk == i) { v = cadd(v, bval); bpend = false; }
            for (int k = 0; k < S.nops; ++k) {
                if (ki[k] < kie[k] && S.ops[k].C.col[ki[k]] == kk) {
                    v = cadd(v, cmul(coef[k], S.ops[k].C.val[ki[k]]));
                    ++ki[k];
                }
            }
            if (v.x != 0.0 || v.y != 0.0) {
                if (FILL) {
                    out_col[cnt] = kk + d * l;
                    out_val[cnt] = v;
                }
                ++cnt;
            }
        }
        if (useA) a_pending = false;
        if (useB) ++bq;
        for (int k = 0; k < S.nops; ++k)
            if (oc[k] < oce[k] && S.ops[k].C.col[oc[k]] == l) ++oc[k];
    }
    return cnt;
}

__global__ void __launch_bounds__(256) k_l_count(RowSources S, int n, int *cnt) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) cnt[r] = liouvillian_row<false>(S, r, nullptr, nullptr);
}

__global__ void __launch_bounds__(256) k_l_fill(RowSources S, int n, const int *rowptr, int *col, double2 *val) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) liouvillian_row<true>(S, r, col + rowptr[r], val + rowptr[r]);
}

void assemble_liouvillian(const ss_csr_z *H, const ss_csr_z *c_ops, int n_cops, int64_t N, hipStream_t s,
                          CsrBuf<double2> &L, LindbladBuf &ops) {
    SS_REQUIRE(N >= 1 && N <= 46340, SS_E_INVALID_ARG, "N must be in [1, 46340] so that N^2 < 2^31");
    SS_REQUIRE(n_cops >= 0 && n_cops <= MAX_COPS, SS_E_INVALID_ARG,
               "n_cops must be in [0, " + std::to_string(MAX_COPS) + "]");
    SS_REQUIRE(n_cops == 0 || c_ops != nullptr, SS_E_INVALID_ARG, "c_ops is NULL");
    const int d = (int)N;
    const int64_t n = (int64_t)N * N;
    StreamScope scope(s);

    CsrBuf<double2> Hd, Htd;
    upload_csr(H, N, Hd, s, "H");
    transpose(Hd, Htd, s, true);
    std::vector<CsrBuf<double2>> C(n_cops), Ct(n_cops);
    std::vector<OpPair> hops(n_cops);
    for (int k = 0; k < n_cops; ++k) {
        upload_csr(&c_ops[k], N, C[k], s, "c_ops[k]");
        transpose(C[k], Ct[k], s, true);
        hops[k].C = C[k].view();
        hops[k].Ct = Ct[k].view();
    }
    DevBuf<OpPair> dops((size_t)std::max(n_cops, 1));
    if (n_cops) h2d(dops.get(), hops.data(), n_cops, s);

    // dense d x d staging of Gpre and Gpost, then compaction
    CsrBuf<double2> Gp, Gq;
    {
        DevBuf<double2> Gpre((size_t)d * d), Gpost((size_t)d * d);
        SS_HIP(hipMemsetAsync(Gpre.get(), 0, Gpre.bytes(), s));
        SS_HIP(hipMemsetAsync(Gpost.get(), 0, Gpost.bytes(), s));
        k_gterms<<<d, 64, 0, s>>>(d, Hd.view(), Htd.view(), dops.get(), n_cops, Gpre.get(), Gpost.get());
        SS_HIP(hipGetLastError());
        dense_to_csr(d, Gpre.get(), Gp, s);
        dense_to_csr(d, Gpost.get(), Gq, s);
    }

    RowSources S;
    S.d = d;
    S.Gp = Gp.view();
    S.Gq = Gq.view();
    S.ops = dops.get();
    S.nops = n_cops;
    DevBuf<int> cnt((size_t)n + 1);
    k_l_count<<<div_up(n, 256), 256, 0, s>>>(S, (int)n, cnt.get());
    SS_HIP(hipGetLastError());
    L.rowptr.resize((size_t)n + 1);
    const int64_t nnz = scan_exclusive(cnt.get(), L.rowptr.get(), n, s, true);
    SS_REQUIRE(nnz >= 0 && nnz < (int64_t(1) << 31), SS_E_INVALID_ARG, "nnz(L) exceeds 2^31 - 1");
    L.n = (int)n;
    L.nnz = (int)nnz;
    L.col.resize((size_t)nnz);
    L.val.resize((size_t)nnz);
    k_l_fill<<<div_up(n, 256), 256, 0, s>>>(S, (int)n, L.rowptr.get(), L.col.get(), L.val.get());
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s));
    ops.d = d;
    ops.Gp = std::move(Gp);
    ops.Gq = std::move(Gq);
    ops.C = std::move(C);
}


// ------------------------------------------------------------ batches
// Many systems assembled together: every step above runs once for the whole
// batch (flattened grids, one job per system or matrix), temporaries live in
// one arena per batch, and the host waits twice (for the sizes of Gpre/Gpost
// with the validation flags, then for nnz(L)).  Each entry receives its
// terms in the same order as in assemble_liouvillian, so a handle built in a
// batch holds the same L as one built on its own.

struct IngestJob {  // one input matrix: validated, then copied
    const int64_t *indptr;
    const int32_t *indices;
    const double *data;
    int64_t nnz;
    int n;
    int sys;
    int *rowptr;
    int *col;
    double2 *val;
};

// One block per matrix, one thread per row (strided): the checks of
// k_validate_csr, then the row is copied with int32 row pointers.  A matrix
// with any error gets all-zero row pointers (every row empty), so the kernels
// that follow before the host reads the flags never see its entries.
__global__ void __launch_bounds__(256) k_asm_ingest(const IngestJob *jobs, unsigned *flags) {
    __shared__ unsigned bad;
    const IngestJob J = jobs[blockIdx.x];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    unsigned err = 0;
    for (int64_t i = threadIdx.x; i <= J.n; i += 256) {
        const int64_t p = J.indptr[i];
        unsigned e = 0;
        if (i == 0 && p != 0) e |= 1;
        if (i == J.n && p != J.nnz) e |= 1;
        if (p < 0 || p > J.nnz) e |= 1;
        if (i < J.n && !e) {
            const int64_t q = J.indptr[i + 1];
            if (q < p || q > J.nnz) {
                e |= 1;
            } else {
                int prev = -1;
                for (int64_t k = p; k < q; ++k) {
                    const int c = J.indices[k];
                    const double re = J.data[2 * k], im = J.data[2 * k + 1];
                    if (c < 0 || c >= J.n || c <= prev) { e |= 2; break; }
                    if (!isfinite(re) || !isfinite(im)) { e |= 4; break; }
                    prev = c;
                    J.col[k] = c;
                    J.val[k] = mk(re, im);
                }
            }
        }
        J.rowptr[i] = e ? 0 : (int)p;
        err |= e;
    }
    if (err) atomicOr(&bad, err);
    __syncthreads();
    if (bad) {
        for (int64_t i = threadIdx.x; i <= J.n; i += 256) J.rowptr[i] = 0;
        if (threadIdx.x == 0) atomicOr(&flags[J.sys], bad);
    }
}

struct GtermJob {  // one system: dense Gpre / Gpost staging
    int d;
    int nops;
    Csr<double2> H;
    Csr<double2> C[MAX_COPS];
    double2 *Gpre, *Gpost;  // d x d each, zeroed
};

// One block per system.  -i H and +i H^T go in first (distinct entries, all
// in parallel), then -1/2 D row by row of each C_k: row m adds
// conj(C[m,i]) C[m,c] to D[i,c] for every pair of its non-zeros, and a
// barrier separates rows, so each entry sees its terms in the order
// (k, m ascending), as in k_gterms.
__global__ void __launch_bounds__(256) k_asm_gterms(const GtermJob *jobs) {
    const GtermJob &J = jobs[blockIdx.x];
    const int d = J.d;
    for (int a = threadIdx.x; a < d; a += 256) {
        for (int e = J.H.rowptr[a]; e < J.H.rowptr[a + 1]; ++e) {
            const int b = J.H.col[e];
            const double2 h = J.H.val[e];
            double2 *pre = J.Gpre + (size_t)a * d + b;
            double2 *post = J.Gpost + (size_t)b * d + a;
            *pre = cadd(*pre, mk(h.y, -h.x));
            *post = cadd(*post, mk(-h.y, h.x));
        }
    }
    __syncthreads();
    for (int k = 0; k < J.nops; ++k) {
        const Csr<double2> C = J.C[k];
        for (int m = 0; m < d; ++m) {
            const int e0 = C.rowptr[m], nz = C.rowptr[m + 1] - e0;
            if (nz == 0) continue;
            for (int p = threadIdx.x; p < nz * nz; p += 256) {
                const int u = p / nz, v = p - u * nz;
                const int i = C.col[e0 + u], c = C.col[e0 + v];
                const double2 cmi = C.val[e0 + u], cmc = C.val[e0 + v];
                double2 *pre = J.Gpre + (size_t)i * d + c;
                double2 *post = J.Gpost + (size_t)i * d + c;
                *pre = csub(*pre, cscale(cmulc(cmi, cmc), 0.5));
                *post = csub(*post, cscale(cmulc(cmc, cmi), 0.5));
            }
            __syncthreads();
        }
    }
}

struct DenseJob {  // one dense d x d matrix -> CSR
    int d;
    const double2 *G;
    int *rowptr;  // counts, then (after the scan) row pointers
    int *col;
    double2 *val;
};

// One wavefront per row (4 per block); FILL writes the row's non-zeros.
template <bool FILL>
__global__ void __launch_bounds__(256) k_asm_dense(const DenseJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const DenseJob J = jobs[jb];
    const int lane = threadIdx.x & 63;
    const int row = (blockIdx.x - bstart[jb]) * 4 + (threadIdx.x >> 6);
    if (row >= J.d) return;
    const double2 *g = J.G + (size_t)row * J.d;
    if (!FILL) {
        int c = 0;
        for (int j = lane; j < J.d; j += 64) c += (g[j].x != 0.0 || g[j].y != 0.0);
        for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
        if (lane == 0) J.rowptr[row] = c;
        return;
    }
    int pos = J.rowptr[row];
    for (int j0 = 0; j0 < J.d; j0 += 64) {
        const int j = j0 + lane;
        double2 v = mk(0.0, 0.0);
        if (j < J.d) v = g[j];
        const bool nz = (j < J.d) && (v.x != 0.0 || v.y != 0.0);
        const unsigned long long mask = __ballot(nz);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (nz) {
            J.col[pos + before] = j;
            J.val[pos + before] = v;
        }
        pos += __popcll(mask);
    }
}

struct RowJob {  // one system's rows of L
    RowSources S;
    int n;
    int *rowptr;
    int *col;
    double2 *val;
};

template <bool FILL>
__global__ void __launch_bounds__(256) k_asm_rows(const RowJob *jobs, const int *bstart, int njobs) {
    const int jb = job_of_block(bstart, njobs, blockIdx.x);
    const RowJob &J = jobs[jb];
    const int r = (blockIdx.x - bstart[jb]) * 256 + threadIdx.x;
    if (r >= J.n) return;
    if (FILL) liouvillian_row<true>(J.S, r, J.col + J.rowptr[r], J.val + J.rowptr[r]);
    else J.rowptr[r] = liouvillian_row<false>(J.S, r, nullptr, nullptr);
}

static void check_matrix(const ss_csr_z *m, int64_t N, int sys, const char *what, bool on_device) {
    const std::string w = "system " + std::to_string(sys) + ", " + what;
    SS_REQUIRE(m != nullptr, SS_E_INVALID_ARG, w + ": null matrix");
    SS_REQUIRE(m->n == N, SS_E_INVALID_ARG, w + ": dimension " + std::to_string(m->n) + " != N = " + std::to_string(N));
    SS_REQUIRE(m->nnz >= 0 && m->nnz < (int64_t(1) << 31), SS_E_INVALID_ARG, w + ": bad nnz");
    SS_REQUIRE(m->indptr != nullptr, SS_E_INVALID_ARG, w + ": null indptr");
    SS_REQUIRE(m->nnz == 0 || (m->indices && m->data), SS_E_INVALID_ARG, w + ": null arrays");
    SS_REQUIRE(on_device ||
                   (is_device_ptr(m->indptr) && (m->nnz == 0 || (is_device_ptr(m->indices) && is_device_ptr(m->data)))),
               SS_E_INVALID_ARG, w + ": batched assembly takes device arrays only");
}

bool batch_assembly_fits(int64_t N) { return N >= 1 && N <= ASM_BATCH_MAX_N; }

// One chunk of systems [k0, k1) (the dense staging of the chunk fits the cap).
static void assemble_chunk(int k0, int k1, const ss_csr_z *H, const ss_csr_z *const *c_ops, const int *n_cops,
                           const AsmTarget *out, hipStream_t s) {
    const int m = k1 - k0;
    StreamScope scope(s);
    // staging of H (not kept) and every handle's buffers
    std::vector<CsrBuf<double2>> Hs((size_t)m);
    std::vector<IngestJob> ing;
    for (int q = 0; q < m; ++q) {
        const int k = k0 + q;
        const int d = (int)H[k].n;
        Hs[(size_t)q].alloc(d, (int)H[k].nnz);
        ing.push_back(IngestJob{H[k].indptr, H[k].indices, H[k].data, H[k].nnz, d, q, Hs[(size_t)q].rowptr.get(),
                                Hs[(size_t)q].col.get(), Hs[(size_t)q].val.get()});
        LindbladBuf &lin = *out[k].lin;
        {
            StreamScope own(out[k].tag);
            lin.d = d;
            lin.C.clear();
            lin.C.resize((size_t)n_cops[k]);
            for (int c = 0; c < n_cops[k]; ++c) lin.C[(size_t)c].alloc(d, (int)c_ops[k][c].nnz);
            lin.Gp.rowptr.resize((size_t)d + 1);
            lin.Gq.rowptr.resize((size_t)d + 1);
            out[k].L->rowptr.resize((size_t)d * d + 1);
        }
        for (int c = 0; c < n_cops[k]; ++c) {
            const ss_csr_z &C = c_ops[k][c];
            ing.push_back(IngestJob{C.indptr, C.indices, C.data, C.nnz, d, q, lin.C[(size_t)c].rowptr.get(),
                                    lin.C[(size_t)c].col.get(), lin.C[(size_t)c].val.get()});
        }
    }
    // dense staging offsets
    std::vector<size_t> goff((size_t)m + 1, 0);
    for (int q = 0; q < m; ++q) {
        const size_t d = (size_t)H[k0 + q].n;
        goff[(size_t)q + 1] = goff[(size_t)q] + 2 * d * d;
    }
    DevBuf<double2> stage(goff[(size_t)m]);
    SS_HIP(hipMemsetAsync(stage.get(), 0, stage.bytes(), s));
    // meta: flags[m], Gp/Gq totals [2m], L totals [m]
    DevBuf<unsigned> meta((size_t)4 * m);
    SS_HIP(hipMemsetAsync(meta.get(), 0, meta.bytes(), s));
    unsigned *flags = meta.get();
    int *gtot = reinterpret_cast<int *>(meta.get() + m);
    int *ltot = reinterpret_cast<int *>(meta.get() + 3 * m);

    DevBuf<IngestJob> d_ing(ing.size());
    h2d(d_ing.get(), ing.data(), ing.size(), s);
    k_asm_ingest<<<(unsigned)ing.size(), 256, 0, s>>>(d_ing.get(), flags);
    SS_HIP(hipGetLastError());

    std::vector<GtermJob> gj((size_t)m);
    std::vector<DenseJob> dj;
    std::vector<int> dblocks;
    std::vector<ScanJob> sj;
    for (int q = 0; q < m; ++q) {
        const int k = k0 + q;
        const int d = (int)H[k].n;
        GtermJob &g = gj[(size_t)q];
        std::memset(&g, 0, sizeof(g));
        g.d = d;
        g.nops = n_cops[k];
        g.H = Hs[(size_t)q].view();
        for (int c = 0; c < n_cops[k]; ++c) g.C[c] = out[k].lin->C[(size_t)c].view();
        g.Gpre = stage.get() + goff[(size_t)q];
        g.Gpost = g.Gpre + (size_t)d * d;
        LindbladBuf &lin = *out[k].lin;
        dj.push_back(DenseJob{d, g.Gpre, lin.Gp.rowptr.get(), nullptr, nullptr});
        dj.push_back(DenseJob{d, g.Gpost, lin.Gq.rowptr.get(), nullptr, nullptr});
        dblocks.push_back(div_up(d, 4));
        dblocks.push_back(div_up(d, 4));
        sj.push_back(ScanJob{lin.Gp.rowptr.get(), d, gtot + 2 * q, nullptr});
        sj.push_back(ScanJob{lin.Gq.rowptr.get(), d, gtot + 2 * q + 1, nullptr});
    }
    DevBuf<GtermJob> d_gj((size_t)m);
    h2d(d_gj.get(), gj.data(), (size_t)m, s);
    k_asm_gterms<<<(unsigned)m, 256, 0, s>>>(d_gj.get());
    SS_HIP(hipGetLastError());

    std::vector<int> dpre;
    const int dnb = block_prefix(dblocks, dpre);
    DevBuf<int> d_dpre(dpre.size());
    h2d(d_dpre.get(), dpre.data(), dpre.size(), s);
    DevBuf<DenseJob> d_dj(dj.size());
    h2d(d_dj.get(), dj.data(), dj.size(), s);
    k_asm_dense<false><<<(unsigned)dnb, 256, 0, s>>>(d_dj.get(), d_dpre.get(), (int)dj.size());
    SS_HIP(hipGetLastError());
    seg_scan(sj, s);

    // host wait 1: validation flags and the sizes of Gpre / Gpost
    std::vector<unsigned> hmeta((size_t)3 * m);
    d2h(hmeta.data(), meta.get(), hmeta.size(), s);
    for (int q = 0; q < m; ++q) {
        const unsigned f = hmeta[(size_t)q];
        const std::string w = "system " + std::to_string(k0 + q);
        SS_REQUIRE(!(f & 1), SS_E_INVALID_ARG, w + ": malformed indptr");
        SS_REQUIRE(!(f & 2), SS_E_INVALID_ARG, w + ": column indices must be in range and strictly increasing per row");
        SS_REQUIRE(!(f & 4), SS_E_INVALID_ARG, w + ": non-finite value");
    }
    for (int q = 0; q < m; ++q) {
        const int k = k0 + q;
        const int d = (int)H[k].n;
        LindbladBuf &lin = *out[k].lin;
        StreamScope own(out[k].tag);
        const int np = (int)hmeta[(size_t)m + 2 * q], nq = (int)hmeta[(size_t)m + 2 * q + 1];
        lin.Gp.n = d;
        lin.Gp.nnz = np;
        lin.Gp.col.resize((size_t)np);
        lin.Gp.val.resize((size_t)np);
        lin.Gq.n = d;
        lin.Gq.nnz = nq;
        lin.Gq.col.resize((size_t)nq);
        lin.Gq.val.resize((size_t)nq);
        dj[(size_t)2 * q].col = lin.Gp.col.get();
        dj[(size_t)2 * q].val = lin.Gp.val.get();
        dj[(size_t)2 * q + 1].col = lin.Gq.col.get();
        dj[(size_t)2 * q + 1].val = lin.Gq.val.get();
    }
    h2d(d_dj.get(), dj.data(), dj.size(), s);
    k_asm_dense<true><<<(unsigned)dnb, 256, 0, s>>>(d_dj.get(), d_dpre.get(), (int)dj.size());
    SS_HIP(hipGetLastError());

    // rows of L
    std::vector<OpPair> ops;
    std::vector<int> opoff((size_t)m + 1, 0);
    for (int q = 0; q < m; ++q) {
        const int k = k0 + q;
        for (int c = 0; c < n_cops[k]; ++c) {
            OpPair op;
            op.C = out[k].lin->C[(size_t)c].view();
            op.Ct = Csr<double2>();
            ops.push_back(op);
        }
        opoff[(size_t)q + 1] = (int)ops.size();
    }
    DevBuf<OpPair> d_ops(std::max<size_t>(ops.size(), 1));
    if (!ops.empty()) h2d(d_ops.get(), ops.data(), ops.size(), s);
    std::vector<RowJob> rj((size_t)m);
    std::vector<int> rblocks((size_t)m);
    std::vector<ScanJob> lsj((size_t)m);
    for (int q = 0; q < m; ++q) {
        const int k = k0 + q;
        const int d = (int)H[k].n;
        RowJob &r = rj[(size_t)q];
        r.S.d = d;
        r.S.Gp = out[k].lin->Gp.view();
        r.S.Gq = out[k].lin->Gq.view();
        r.S.ops = d_ops.get() + opoff[(size_t)q];
        r.S.nops = n_cops[k];
        r.n = d * d;
        r.rowptr = out[k].L->rowptr.get();
        r.col = nullptr;
        r.val = nullptr;
        rblocks[(size_t)q] = div_up(r.n, 256);
        lsj[(size_t)q] = ScanJob{r.rowptr, r.n, ltot + q, nullptr};
    }
    std::vector<int> rpre;
    const int rnb = block_prefix(rblocks, rpre);
    DevBuf<int> d_rpre(rpre.size());
    h2d(d_rpre.get(), rpre.data(), rpre.size(), s);
    DevBuf<RowJob> d_rj((size_t)m);
    h2d(d_rj.get(), rj.data(), (size_t)m, s);
    k_asm_rows<false><<<(unsigned)rnb, 256, 0, s>>>(d_rj.get(), d_rpre.get(), m);
    SS_HIP(hipGetLastError());
    seg_scan(lsj, s);

    // host wait 2: nnz(L)
    std::vector<int> lnnz((size_t)m);
    d2h(lnnz.data(), ltot, (size_t)m, s);
    for (int q = 0; q < m; ++q) {
        const int k = k0 + q;
        CsrBuf<double2> &L = *out[k].L;
        StreamScope own(out[k].tag);
        L.n = rj[(size_t)q].n;
        L.nnz = lnnz[(size_t)q];
        L.col.resize((size_t)L.nnz);
        L.val.resize((size_t)L.nnz);
        rj[(size_t)q].col = L.col.get();
        rj[(size_t)q].val = L.val.get();
    }
    h2d(d_rj.get(), rj.data(), (size_t)m, s);
    k_asm_rows<true><<<(unsigned)rnb, 256, 0, s>>>(d_rj.get(), d_rpre.get(), m);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s));
    FreeScope fs(s);  // the staged copies of H: one release event for all
    Hs.clear();
}

void assemble_batch(int count, const ss_csr_z *H, const ss_csr_z *const *c_ops, const int *n_cops,
                    const AsmTarget *out, hipStream_t s, bool on_device) {
    for (int k = 0; k < count; ++k) {
        check_matrix(&H[k], H[k].n, k, "H", on_device);
        const int64_t N = H[k].n;
        SS_REQUIRE(batch_assembly_fits(N), SS_E_INVALID_ARG,
                   "system " + std::to_string(k) + ": batched assembly takes N in [1, " +
                       std::to_string(ASM_BATCH_MAX_N) + "]");
        SS_REQUIRE(n_cops[k] >= 0 && n_cops[k] <= MAX_COPS, SS_E_INVALID_ARG,
                   "system " + std::to_string(k) + ": n_cops must be in [0, " + std::to_string(MAX_COPS) + "]");
        SS_REQUIRE(n_cops[k] == 0 || c_ops[k] != nullptr, SS_E_INVALID_ARG,
                   "system " + std::to_string(k) + ": c_ops is NULL");
        for (int c = 0; c < n_cops[k]; ++c) check_matrix(&c_ops[k][c], N, k, "c_ops[k]", on_device);
    }
    // chunks whose dense staging stays under the cap (SS_ASM_STAGE_MB
    // lowers it, so that small batches can exercise the chunking)
    size_t cap = ASM_BATCH_STAGE_BYTES;
    if (const char *e = std::getenv("SS_ASM_STAGE_MB")) {
        const long mb = std::atol(e);
        if (mb > 0) cap = std::min(cap, (size_t)mb << 20);
    }
    int k0 = 0;
    while (k0 < count) {
        size_t bytes = 0;
        int k1 = k0;
        while (k1 < count) {
            const size_t d = (size_t)H[k1].n;
            const size_t b = 2 * d * d * sizeof(double2);
            if (k1 > k0 && bytes + b > cap) break;
            bytes += b;
            ++k1;
        }
        assemble_chunk(k0, k1, H, c_ops, n_cops, out, s);
        k0 = k1;
    }
}

}  // namespace ss
