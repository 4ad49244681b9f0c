// Sparse matrix-vector products, vector kernels and deterministic reductions
// (blas.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

constexpr int VEC_BS = 256;
constexpr int VEC_MAX_BLOCKS = 1024;

inline int vec_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(div_up(n, VEC_BS), VEC_MAX_BLOCKS)); }

// Per-block sums of K complex values over a VEC_BS-thread block, written to
// partials[k * gridDim.x + blockIdx.x] in a fixed order (deterministic).
template <int K>
__device__ inline void block_partials(double2 (&v)[K], double2 *partials) {
    __shared__ double2 sh[K][VEC_BS / 64];
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
            for (int w = 1; w < VEC_BS / 64; ++w) acc = cadd(acc, sh[k][w]);
            partials[k * gridDim.x + blockIdx.x] = acc;
        }
    }
}

// Sum of nb partials by a workgroup of BS threads: thread t adds partials
// t, t + BS, ... in order, then a fixed tree; the result is valid in
// thread 0.  Every thread of the workgroup must call it.
constexpr int SUM_BS = 1024;
template <int BS = SUM_BS>
__device__ inline double2 sum_partials_block(const double2 *p, int nb) {
    __shared__ double sx[BS], sy[BS];
    const int t = threadIdx.x;
    double x = 0, y = 0;
    for (int b = t; b < nb; b += BS) {
        x += p[b].x;
        y += p[b].y;
    }
    __syncthreads();  // (the arrays may still be read by a previous call)
    sx[t] = x;
    sy[t] = y;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (t < off) {
            sx[t] += sx[t + off];
            sy[t] += sy[t + off];
        }
        __syncthreads();
    }
    return make_double2(sx[0], sy[0]);
}

// lanes per row for the CSR SpMV, from the mean row length
int spmv_group(int n, int nnz);

// y = A x
template <typename T>
void spmv(const Csr<T> &A, const T *x, T *y, int group, hipStream_t s, const int *skip = nullptr);

// y = A x and block partials of conj(u1).y and (if u2 != null) conj(u2).y;
// u2 == y requests y^H y.  Returns the number of workgroups nb (at most
// SPMV_DOTS_MAX_BLOCKS); partials: 2 * nb entries, the second group at nb.
constexpr int SPMV_DOTS_MAX_BLOCKS = 16384;
template <typename T>
int spmv_dots(const Csr<T> &A, const T *x, T *y, const T *u1, const T *u2, double2 *partials, int group,
              hipStream_t s, const int *skip);

// r = b - A x in fp64 plus block partials of ||r||^2 (partials[0 .. nb))
void spmv_residual(const Csr<double2> &A, const double2 *b, const double2 *x, double2 *r, double2 *partials,
                   int group, hipStream_t s);

// sum of the first nb partials of each of k groups (group stride nb) into
// out[0..k) on the device, in a fixed order
void sum_partials(const double2 *partials, int nb, int k, double2 *out, hipStream_t s);

// ||x||^2 of a complex vector (fp64 accumulation) into *out (device)
template <typename T>
void norm2(int64_t n, const T *x, double2 *partials, double2 *out, hipStream_t s);

// max_i |x_i| into *out (device, .x)
template <typename T>
void norm_inf(int64_t n, const T *x, double2 *partials, double2 *out, hipStream_t s);

// sum_k x[idx[k]] for k < m (fp64), into *out (device)
void gather_sum(int m, const int *idx, const double2 *x, double2 *out, hipStream_t s);

// dst = src (widening / rounding between precisions), with an optional
// device-side scale factor 1 / *scale_den (.x) when scale_den != null
template <typename TD, typename TS>
void convert(int64_t n, const TS *src, TD *dst, const double2 *scale_den, hipStream_t s);

// x += alpha * d with alpha = *alpha_src (device, real part .x), x fp64
template <typename T>
void axpy_widen(int64_t n, const double2 *alpha_src, const T *d, double2 *x, hipStream_t s);

// x[i] = 0
template <typename T>
void zero(int64_t n, T *x, hipStream_t s);

}  // namespace ss
