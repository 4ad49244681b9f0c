// Sparse matrix-vector product (section "Iterative Solvers": each Krylov
// iteration needs matrix-vector products with the permuted Liouvillian) and
// the vector kernels around it.
//
// CSR SpMV: a group of G lanes (G = 4..32, from the mean row length) per row,
// so consecutive lanes read consecutive values/indices of a row (coalesced
// streams) while x is gathered through the caches; the group reduces with
// cross-lane shuffles.  Reductions are deterministic: per-block partials in a
// fixed order, then one block sums the partials in a fixed order.
#include "blas.hpp"

namespace ss {

int spmv_group(int n, int nnz) {
    const double mean = n ? (double)nnz / n : 0.0;
    if (mean <= 6) return 4;
    if (mean <= 12) return 8;
    if (mean <= 24) return 16;
    return 32;
}

// ---------------------------------------------------- block partial sums
// One workgroup per group of partials (sum_partials_block): 256 threads up to
// 4096 partials, 1024 above (the fused SpMV's up to 16384).
template <int BS>
__global__ void __launch_bounds__(BS) k_sum_partials(const double2 *partials, int nb, double2 *out) {
    const int k = blockIdx.x;
    const double2 v = sum_partials_block<BS>(partials + (int64_t)k * nb, nb);
    if (threadIdx.x == 0) out[k] = v;
}

void sum_partials(const double2 *partials, int nb, int k, double2 *out, hipStream_t s) {
    if (nb <= 4096) k_sum_partials<256><<<k, 256, 0, s>>>(partials, nb, out);
    else k_sum_partials<SUM_BS><<<k, SUM_BS, 0, s>>>(partials, nb, out);
    SS_HIP(hipGetLastError());
}

// --------------------------------------------------------------- SpMV
// G lanes per row, up to U entries per lane per round with every load of a
// round issued before its products are formed.  The matrix is streamed once,
// so its values and indices are read non-temporally (NT) when that pays,
// leaving the caches to the gathered x.  Measured on the Kerr chain's
// P A P^T (n = 10^6, 20.7 M entries, 512 MB of other data written between
// repetitions so that nothing of the matrix is cached): complex128 138 us
// with one entry per lane per round (G = 16) -> 109 us with G = 16, U = 2,
// NT; complex64 108 us -> 79 us with G = 8, U = 3 (NT slower there).
// One row's sum of products, split over the G lanes of its group (each
// lane's share; the caller reduces across the group).
template <typename T, int G, int U, bool NT>
__device__ __forceinline__ T row_products(int rb, int re, int l, const int *col, const T *val, const T *x) {
    T acc = czero<T>();
    for (int e0 = rb; e0 < re; e0 += G * U) {
        int c[U];
        T v[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * G + l;
            if (e < re) {
                if (NT) {
                    c[u] = __builtin_nontemporal_load(col + e);
                    v[u].x = __builtin_nontemporal_load(&val[e].x);
                    v[u].y = __builtin_nontemporal_load(&val[e].y);
                } else {
                    c[u] = col[e];
                    v[u] = val[e];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * G + l < re) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * G + l < re) acc = cadd(acc, cmul(v[u], xv[u]));
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, G);
        acc.y += __shfl_xor(acc.y, off, G);
    }
    return acc;
}

template <typename T, int G, int U, bool NT>
__global__ void __launch_bounds__(256) k_spmv(int n, const int *rowptr, const int *col, const T *val, const T *x,
                                              T *y, const int *skip) {
    if (skip && *skip) return;
    const int groups = gridDim.x * (256 / G);
    const int l = threadIdx.x & (G - 1);
    for (int row = blockIdx.x * (256 / G) + threadIdx.x / G; row < n; row += groups) {
        const T acc = row_products<T, G, U, NT>(rowptr[row], rowptr[row + 1], l, col, val, x);
        if (l == 0) y[row] = acc;
    }
}

// y = A x with u1^H y and u2^H y (or y^H y) accumulated per block
template <typename T, int G, int U, bool NT>
__global__ void __launch_bounds__(256) k_spmv_dots(int n, const int *rowptr, const int *col, const T *val,
                                                   const T *x, T *y, const T *u1, const T *u2, bool u2_is_y,
                                                   double2 *partials, const int *skip) {
    if (skip && *skip) return;
    const int groups = gridDim.x * (256 / G);
    const int l = threadIdx.x & (G - 1);
    double2 d[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int row = blockIdx.x * (256 / G) + threadIdx.x / G; row < n; row += groups) {
        const T acc = row_products<T, G, U, NT>(rowptr[row], rowptr[row + 1], l, col, val, x);
        if (l == 0) {
            y[row] = acc;
            const double2 yy = widen(acc);
            d[0] = cadd(d[0], cmulc(widen(u1[row]), yy));
            if (u2_is_y) d[1].x += yy.x * yy.x + yy.y * yy.y;
            else if (u2) d[1] = cadd(d[1], cmulc(widen(u2[row]), yy));
        }
    }
    block_partials<2>(d, partials);
}

template <typename T>
void spmv(const Csr<T> &A, const T *x, T *y, int group, hipStream_t s, const int *skip) {
    if (A.n == 0) return;
    const bool c128 = sizeof(T) == 16;
    // rows 17..32 entries long (the Kerr chain): the measured best shapes
    if (group == 16) {
        if (c128) {
            const int nb = div_up(A.n, 256 / 16);
            k_spmv<T, 16, 2, true><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, skip);
        } else {
            const int nb = div_up(A.n, 256 / 8);
            k_spmv<T, 8, 3, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, skip);
        }
        SS_HIP(hipGetLastError());
        return;
    }
    const int rows_per_block = 256 / group;
    const int nb = (int)std::min<int64_t>(div_up(A.n, rows_per_block), 8192);
    switch (group) {
        case 4: k_spmv<T, 4, 1, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, skip); break;
        case 8: k_spmv<T, 8, 1, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, skip); break;
        default: k_spmv<T, 32, 1, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, skip); break;
    }
    SS_HIP(hipGetLastError());
}

template <typename T>
int spmv_dots(const Csr<T> &A, const T *x, T *y, const T *u1, const T *u2, double2 *partials, int group,
              hipStream_t s, const int *skip) {
    const bool u2y = (u2 == y);
    // the shapes of spmv() for rows of 17..32 entries
    const bool c128 = sizeof(T) == 16;
    const int g = (group == 16 && !c128) ? 8 : group;
    // enough workgroups that most rows' loads are in flight at once (each
    // group takes a few rows in turn), capped for the partial sums
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(div_up(A.n, 256 / g), SPMV_DOTS_MAX_BLOCKS));
    switch (group) {
        case 4: k_spmv_dots<T, 4, 1, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, u1, u2, u2y, partials, skip); break;
        case 8: k_spmv_dots<T, 8, 1, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, u1, u2, u2y, partials, skip); break;
        case 16:
            if (c128) k_spmv_dots<T, 16, 2, true><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, u1, u2, u2y, partials, skip);
            else k_spmv_dots<T, 8, 3, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, u1, u2, u2y, partials, skip);
            break;
        default: k_spmv_dots<T, 32, 1, false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, x, y, u1, u2, u2y, partials, skip); break;
    }
    SS_HIP(hipGetLastError());
    return nb;
}

template void spmv<double2>(const Csr<double2> &, const double2 *, double2 *, int, hipStream_t, const int *);
template void spmv<float2>(const Csr<float2> &, const float2 *, float2 *, int, hipStream_t, const int *);
template int spmv_dots<double2>(const Csr<double2> &, const double2 *, double2 *, const double2 *, const double2 *,
                                double2 *, int, hipStream_t, const int *);
template int spmv_dots<float2>(const Csr<float2> &, const float2 *, float2 *, const float2 *, const float2 *,
                               double2 *, int, hipStream_t, const int *);

template <int G>
__global__ void __launch_bounds__(256) k_spmv_residual(int n, const int *rowptr, const int *col, const double2 *val,
                                                       const double2 *b, const double2 *x, double2 *r,
                                                       double2 *partials) {
    const int groups = gridDim.x * (256 / G);
    const int l = threadIdx.x & (G - 1);
    double2 d[1] = {mk(0.0, 0.0)};
    for (int row = blockIdx.x * (256 / G) + threadIdx.x / G; row < n; row += groups) {
        double2 acc = mk(0.0, 0.0);
        const int re = rowptr[row + 1];
        for (int e = rowptr[row] + l; e < re; e += G) acc = cadd(acc, cmul(val[e], x[col[e]]));
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off, G);
            acc.y += __shfl_xor(acc.y, off, G);
        }
        if (l == 0) {
            const double2 rr = b ? csub(b[row], acc) : acc;
            r[row] = rr;
            d[0].x += rr.x * rr.x + rr.y * rr.y;
        }
    }
    block_partials<1>(d, partials);
}

void spmv_residual(const Csr<double2> &A, const double2 *b, const double2 *x, double2 *r, double2 *partials,
                   int group, hipStream_t s) {
    const int nb = vec_blocks(A.n);
    switch (group) {
        case 4: k_spmv_residual<4><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, b, x, r, partials); break;
        case 8: k_spmv_residual<8><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, b, x, r, partials); break;
        case 16: k_spmv_residual<16><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, b, x, r, partials); break;
        default: k_spmv_residual<32><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, A.val, b, x, r, partials); break;
    }
    SS_HIP(hipGetLastError());
}

// ------------------------------------------------------------- norms
template <typename T>
__global__ void __launch_bounds__(256) k_norm2(int64_t n, const T *x, double2 *partials) {
    double2 d[1] = {mk(0.0, 0.0)};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 v = widen(x[i]);
        d[0].x += v.x * v.x + v.y * v.y;
    }
    block_partials<1>(d, partials);
}

template <typename T>
void norm2(int64_t n, const T *x, double2 *partials, double2 *out, hipStream_t s) {
    const int nb = vec_blocks(n);
    k_norm2<T><<<nb, 256, 0, s>>>(n, x, partials);
    SS_HIP(hipGetLastError());
    sum_partials(partials, nb, 1, out, s);
}
template void norm2<double2>(int64_t, const double2 *, double2 *, double2 *, hipStream_t);
template void norm2<float2>(int64_t, const float2 *, double2 *, double2 *, hipStream_t);

template <typename T>
__global__ void __launch_bounds__(256) k_norm_inf(int64_t n, const T *x, double2 *partials) {
    __shared__ double sh[256];
    double m = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 v = widen(x[i]);
        m = fmax(m, sqrt(v.x * v.x + v.y * v.y));
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = mk(sh[0], 0.0);
}

__global__ void k_max_partials(const double2 *partials, int nb, double2 *out) {
    if (threadIdx.x != 0) return;
    double m = 0;
    for (int b = 0; b < nb; ++b) m = fmax(m, partials[b].x);
    *out = mk(m, 0.0);
}

template <typename T>
void norm_inf(int64_t n, const T *x, double2 *partials, double2 *out, hipStream_t s) {
    const int nb = vec_blocks(n);
    k_norm_inf<T><<<nb, 256, 0, s>>>(n, x, partials);
    k_max_partials<<<1, 64, 0, s>>>(partials, nb, out);
    SS_HIP(hipGetLastError());
}
template void norm_inf<double2>(int64_t, const double2 *, double2 *, double2 *, hipStream_t);
template void norm_inf<float2>(int64_t, const float2 *, double2 *, double2 *, hipStream_t);

__global__ void k_gather_sum(int m, const int *idx, const double2 *x, double2 *out) {
    __shared__ double sx[256], sy[256];
    double ax = 0, ay = 0;
    for (int k = threadIdx.x; k < m; k += 256) {
        const double2 v = x[idx[k]];
        ax += v.x;
        ay += v.y;
    }
    sx[threadIdx.x] = ax;
    sy[threadIdx.x] = ay;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sx[threadIdx.x] += sx[threadIdx.x + off];
            sy[threadIdx.x] += sy[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = mk(sx[0], sy[0]);
}

void gather_sum(int m, const int *idx, const double2 *x, double2 *out, hipStream_t s) {
    k_gather_sum<<<1, 256, 0, s>>>(m, idx, x, out);
    SS_HIP(hipGetLastError());
}

// -------------------------------------------------- conversions / axpy
template <typename TD, typename TS>
__global__ void k_convert(int64_t n, const TS *src, TD *dst, const double2 *scale_den) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double2 v = widen(src[i]);
    if (scale_den) {
        const double sc = 1.0 / scale_den->x;
        v.x *= sc;
        v.y *= sc;
    }
    dst[i] = from_c128<TD>(v);
}

template <typename TD, typename TS>
void convert(int64_t n, const TS *src, TD *dst, const double2 *scale_den, hipStream_t s) {
    if (n <= 0) return;
    k_convert<TD, TS><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, src, dst, scale_den);
    SS_HIP(hipGetLastError());
}
template void convert<double2, double2>(int64_t, const double2 *, double2 *, const double2 *, hipStream_t);
template void convert<float2, double2>(int64_t, const double2 *, float2 *, const double2 *, hipStream_t);
template void convert<double2, float2>(int64_t, const float2 *, double2 *, const double2 *, hipStream_t);

template <typename T>
__global__ void k_axpy_widen(int64_t n, const double2 *alpha_src, const T *d, double2 *x) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double a = alpha_src->x;
    const double2 v = widen(d[i]);
    x[i] = mk(x[i].x + a * v.x, x[i].y + a * v.y);
}

template <typename T>
void axpy_widen(int64_t n, const double2 *alpha_src, const T *d, double2 *x, hipStream_t s) {
    if (n <= 0) return;
    k_axpy_widen<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, alpha_src, d, x);
    SS_HIP(hipGetLastError());
}
template void axpy_widen<double2>(int64_t, const double2 *, const double2 *, double2 *, hipStream_t);
template void axpy_widen<float2>(int64_t, const double2 *, const float2 *, double2 *, hipStream_t);

template <typename T>
__global__ void k_zero(int64_t n, T *x) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = czero<T>();
}

template <typename T>
void zero(int64_t n, T *x, hipStream_t s) {
    if (n <= 0) return;
    k_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x);
    SS_HIP(hipGetLastError());
}
template void zero<double2>(int64_t, double2 *, hipStream_t);
template void zero<float2>(int64_t, float2 *, hipStream_t);

}  // namespace ss
