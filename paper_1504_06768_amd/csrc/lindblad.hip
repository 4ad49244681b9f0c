// Matrix-free application of the Lindblad generator (eq. lindblad, column
// stacking as in eq. eigval).
//
// Element r = i + d j of L vec(rho), with rho stored column-major:
//   sum_k Gpre[i, k] rho[k, j]                         (I (x) Gpre)
// + sum_l Gpost[j, l] rho[i, l]                        (Gpost (x) I)
// + sum_c sum_l conj(C_c[j, l]) sum_k C_c[i, k] rho[k, l]   (conj(C) (x) C)
// These are the same three groups of terms the assembly merges into row r of
// L, so the result equals the assembled SpMV up to the rounding order.
//
// One thread per output element, a wavefront per 64 rows of one column j:
// the Gpost and collapse terms read rho coalesced with their row-j
// coefficients in scalar registers, and the Gpre term gathers within column
// j.  The d x d operators are small and stay in the caches, so HBM traffic is
// rho and the result (plus the ordering, b and the scattered output of the
// residual form) instead of the n x n complex128 matrix.
#include "blas.hpp"
#include "lindblad.hpp"

namespace ss {

LindbladOp LindbladBuf::view() const {
    LindbladOp v;
    v.d = d;
    v.nops = (int)C.size();
    v.Gp = Gp.view();
    v.Gq = Gq.view();
    for (int k = 0; k < v.nops && k < MAX_COPS; ++k) v.C[k] = C[(size_t)k].view();
    return v;
}

size_t LindbladBuf::bytes() const {
    size_t b = Gp.bytes() + Gq.bytes();
    for (const auto &c : C) b += c.bytes();
    return b;
}

// acc + sum_{e0 <= e < e1} val[e] x[col[e]], added in order of e; four
// indices are fetched before their gathers so that the loads overlap.
__device__ inline double2 row_gather(double2 acc, const int *col, const double2 *val, int e0, int e1,
                                     const double2 *x) {
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        const int c0 = col[e], c1 = col[e + 1], c2 = col[e + 2], c3 = col[e + 3];
        const double2 x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
        acc = cadd(acc, cmul(val[e], x0));
        acc = cadd(acc, cmul(val[e + 1], x1));
        acc = cadd(acc, cmul(val[e + 2], x2));
        acc = cadd(acc, cmul(val[e + 3], x3));
    }
    for (; e < e1; ++e) acc = cadd(acc, cmul(val[e], x[col[e]]));
    return acc;
}

// acc + sum_{e0 <= e < e1} val[e] x[d col[e]], in order of e (the
// coefficients are wave-uniform; the gathers are coalesced across lanes).
__device__ inline double2 col_gather(double2 acc, const int *col, const double2 *val, int e0, int e1,
                                     const double2 *x, int64_t d) {
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        const double2 x0 = x[d * col[e]], x1 = x[d * col[e + 1]], x2 = x[d * col[e + 2]], x3 = x[d * col[e + 3]];
        acc = cadd(acc, cmul(val[e], x0));
        acc = cadd(acc, cmul(val[e + 1], x1));
        acc = cadd(acc, cmul(val[e + 2], x2));
        acc = cadd(acc, cmul(val[e + 3], x3));
    }
    for (; e < e1; ++e) acc = cadd(acc, cmul(val[e], x[d * col[e]]));
    return acc;
}

// Element (i, j); j is the same for the whole wavefront, so the loops over
// row j of Gpost and of every C_k run on scalar loads.
__device__ inline double2 lindblad_element(const LindbladOp &A, const double2 *rho, int i, int j) {
    const int64_t d = A.d;
    double2 acc = row_gather(mk(0.0, 0.0), A.Gp.col, A.Gp.val, A.Gp.rowptr[i], A.Gp.rowptr[i + 1], rho + d * j);
    acc = col_gather(acc, A.Gq.col, A.Gq.val, A.Gq.rowptr[j], A.Gq.rowptr[j + 1], rho + i, d);
    for (int c = 0; c < A.nops; ++c) {
        const int *rp = A.C[c].rowptr;
        const int *cc = A.C[c].col;
        const double2 *cv = A.C[c].val;
        const int a0 = rp[i], a1 = rp[i + 1];
        for (int el = rp[j]; el < rp[j + 1]; ++el) {
            const double2 t = row_gather(mk(0.0, 0.0), cc, cv, a0, a1, rho + d * cc[el]);
            acc = cadd(acc, cmulc(cv[el], t));  // conj(C[j, l]) t
        }
    }
    return acc;
}

// Wavefront task t covers rows i = 64 (t mod tiles) + lane of column
// j = t / tiles (tiles = ceil(d / 64)).  The element r = i + d j goes to
// position o = iperm ? iperm[r] : r of the output.
template <bool PARTIALS>
__global__ void __launch_bounds__(VEC_BS) k_lindblad(LindbladOp A, int tiles, const int *__restrict__ iperm,
                                                     const double2 *__restrict__ rho, int trow, double2 w,
                                                     const double2 *__restrict__ trace,
                                                     const double2 *__restrict__ b, double2 *__restrict__ y,
                                                     double2 *__restrict__ partials) {
    double2 acc[1] = {mk(0.0, 0.0)};
    const int d = A.d;
    const int lane = threadIdx.x & 63;
    const int64_t ntasks = (int64_t)tiles * d;
    const int64_t nwaves = (int64_t)gridDim.x * (VEC_BS / 64);
    for (int64_t t = (int64_t)blockIdx.x * (VEC_BS / 64) + (threadIdx.x >> 6); t < ntasks; t += nwaves) {
        const int j = __builtin_amdgcn_readfirstlane((int)(t / tiles));
        const int i = (int)(t - (int64_t)j * tiles) * 64 + lane;
        if (i < d) {
            const int r = i + d * j;
            double2 v = lindblad_element(A, rho, i, j);
            if (trace && r == trow) v = cadd(v, cmul(w, *trace));
            const int o = iperm ? iperm[r] : r;
            const double2 out = b ? csub(b[o], v) : v;
            y[o] = out;
            if (PARTIALS) acc[0].x += out.x * out.x + out.y * out.y;
        }
    }
    if (PARTIALS) block_partials<1>(acc, partials);
}

int lindblad_blocks(int d) {
    const int64_t tasks = (int64_t)div_up(d, 64) * d;
    return (int)std::max<int64_t>(1, std::min<int64_t>(div_up(tasks, VEC_BS / 64), VEC_MAX_BLOCKS));
}

void lindblad_apply(const LindbladOp &A, const double2 *rho, const int *iperm, int trow, double2 w,
                    const double2 *trace, const double2 *b, double2 *y, double2 *partials, hipStream_t s) {
    if (A.d == 0) return;
    const int tiles = div_up(A.d, 64);
    const int nb = lindblad_blocks(A.d);
    if (partials)
        k_lindblad<true><<<nb, VEC_BS, 0, s>>>(A, tiles, iperm, rho, trow, w, trace, b, y, partials);
    else
        k_lindblad<false><<<nb, VEC_BS, 0, s>>>(A, tiles, iperm, rho, trow, w, trace, b, y, nullptr);
    SS_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(256) k_unpermute(int n, const int *iperm, const double2 *x, double2 *rho) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < n) rho[r] = x[iperm[r]];
}

void unpermute(int n, const int *iperm, const double2 *x, double2 *rho, hipStream_t s) {
    if (n == 0) return;
    k_unpermute<<<div_up(n, 256), 256, 0, s>>>(n, iperm, x, rho);
    SS_HIP(hipGetLastError());
}

}  // namespace ss
