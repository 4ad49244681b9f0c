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
#include "assemble.hpp"
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
        SS_HIP(hipStreamSynchronize(s));
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

}  // namespace ss
