// Generic CSR kernels: input validation/upload, transpose, row sorting and
// per-row structural queries.  Used by assembly, transforms and ordering.
#include "csr_tools.hpp"
#include "rowops.hpp"

namespace ss {

// ------------------------------------------------------------- validation
// One thread per row: checks monotone indptr, strictly increasing in-range
// column indices and finite values; converts indptr to int32.
__global__ void k_validate_csr(int64_t n, int64_t nnz, const int64_t *indptr, const int32_t *indices,
                               const double *data, int *rowptr32, unsigned *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t p = indptr[i];
    unsigned err = 0;
    if (i == 0 && p != 0) err |= 1;
    if (i == n && p != nnz) err |= 1;
    if (p < 0 || p > nnz) err |= 1;
    if (i < n && !err) {
        const int64_t q = indptr[i + 1];
        if (q < p || q > nnz) {
            err |= 1;
        } else {
            int prev = -1;
            for (int64_t e = p; e < q; ++e) {
                const int c = indices[e];
                if (c < 0 || c >= n || c <= prev) { err |= 2; break; }
                prev = c;
                const double re = data[2 * e], im = data[2 * e + 1];
                if (!isfinite(re) || !isfinite(im)) { err |= 4; break; }
            }
        }
    }
    rowptr32[i] = (int)p;
    if (err) atomicOr(bad, err);
}

void upload_csr(const ss_csr_z *in, int64_t N, CsrBuf<double2> &out, hipStream_t s, const char *what) {
    SS_REQUIRE(in != nullptr, SS_E_INVALID_ARG, std::string(what) + ": null matrix");
    SS_REQUIRE(in->n == N, SS_E_INVALID_ARG,
               std::string(what) + ": dimension " + std::to_string(in->n) + " != N = " + std::to_string(N));
    SS_REQUIRE(in->nnz >= 0 && in->nnz < (int64_t(1) << 31), SS_E_INVALID_ARG, std::string(what) + ": bad nnz");
    SS_REQUIRE(in->indptr != nullptr, SS_E_INVALID_ARG, std::string(what) + ": null indptr");
    SS_REQUIRE(in->nnz == 0 || (in->indices && in->data), SS_E_INVALID_ARG, std::string(what) + ": null arrays");
    const int64_t n = in->n, nnz = in->nnz;
    out.alloc((int)n, (int)nnz);
    // stage raw arrays on the device (a device-to-device copy when the caller's
    // arrays are already resident)
    DevBuf<int64_t> ip((size_t)n + 1);
    DevBuf<int32_t> ix((size_t)nnz);
    DevBuf<double2> dv((size_t)nnz);
    const hipMemcpyKind k1 = is_device_ptr(in->indptr) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    SS_HIP(hipMemcpyAsync(ip.get(), in->indptr, sizeof(int64_t) * (n + 1), k1, s));
    if (nnz) {
        const hipMemcpyKind k2 = is_device_ptr(in->indices) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        const hipMemcpyKind k3 = is_device_ptr(in->data) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        SS_HIP(hipMemcpyAsync(ix.get(), in->indices, sizeof(int32_t) * nnz, k2, s));
        SS_HIP(hipMemcpyAsync(dv.get(), in->data, sizeof(double2) * nnz, k3, s));
    }
    DevBuf<unsigned> bad(1);
    SS_HIP(hipMemsetAsync(bad.get(), 0, sizeof(unsigned), s));
    k_validate_csr<<<div_up(n + 1, 256), 256, 0, s>>>(n, nnz, ip.get(), ix.get(), (const double *)dv.get(),
                                                      out.rowptr.get(), bad.get());
    SS_HIP(hipGetLastError());
    if (nnz) {
        SS_HIP(hipMemcpyAsync(out.col.get(), ix.get(), sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
        SS_HIP(hipMemcpyAsync(out.val.get(), dv.get(), sizeof(double2) * nnz, hipMemcpyDeviceToDevice, s));
    }
    unsigned hbad = 0;
    d2h(&hbad, bad.get(), 1, s);
    SS_REQUIRE(!(hbad & 1), SS_E_INVALID_ARG, std::string(what) + ": malformed indptr");
    SS_REQUIRE(!(hbad & 2), SS_E_INVALID_ARG,
               std::string(what) + ": column indices must be in range and strictly increasing per row");
    SS_REQUIRE(!(hbad & 4), SS_E_INVALID_ARG, std::string(what) + ": non-finite value");
}

// ------------------------------------------------------------- row sorting
// One wavefront per row: rank sort by column (columns are unique within a
// row), so the result does not depend on the order entries were scattered in.
template <typename T>
__global__ void __launch_bounds__(256) k_sort_rows(int n, const int *rowptr, const int *col_in, const T *val_in,
                                                   int *col_out, T *val_out) {
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row < n) sort_row_wave<T>(rowptr[row], rowptr[row + 1], col_in, val_in, col_out, val_out);
}

template <typename T>
void sort_rows(int n, const int *rowptr, const int *col_in, const T *val_in, int *col_out, T *val_out,
               hipStream_t s) {
    if (n <= 0) return;
    k_sort_rows<T><<<div_up(n, 4), 256, 0, s>>>(n, rowptr, col_in, val_in, col_out, val_out);
    SS_HIP(hipGetLastError());
}
template void sort_rows<double2>(int, const int *, const int *, const double2 *, int *, double2 *, hipStream_t);
template void sort_rows<float2>(int, const int *, const int *, const float2 *, int *, float2 *, hipStream_t);

// --------------------------------------------------------------- transpose
__global__ void k_count_cols(int nnz, const int *col, int *cnt) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[col[e]], 1);
}

template <typename T>
__global__ void k_scatter_transpose(int n, const int *rowptr, const int *col, const T *val, int *cursor,
                                    int *tcol, T *tval) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int pos = atomicAdd(&cursor[col[e]], 1);
        tcol[pos] = r;
        if (val) tval[pos] = val[e];
    }
}

template <typename T>
void transpose(const CsrBuf<T> &A, CsrBuf<T> &At, hipStream_t s, bool with_values) {
    const int n = A.n, nnz = A.nnz;
    StreamScope scope(s);
    At.alloc(n, nnz);
    DevBuf<int> cnt((size_t)n + 1);
    SS_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int) * (n + 1), s));
    if (nnz) {
        k_count_cols<<<div_up(nnz, 256), 256, 0, s>>>(nnz, A.col.get(), cnt.get());
        SS_HIP(hipGetLastError());
    }
    scan_exclusive(cnt.get(), At.rowptr.get(), n, s, false);
    SS_HIP(hipMemcpyAsync(cnt.get(), At.rowptr.get(), sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    DevBuf<int> tcol((size_t)nnz);
    DevBuf<T> tval(with_values ? (size_t)nnz : 1);
    if (n) {
        k_scatter_transpose<T><<<div_up(n, 256), 256, 0, s>>>(n, A.rowptr.get(), A.col.get(),
                                                               with_values ? A.val.get() : nullptr, cnt.get(),
                                                               tcol.get(), tval.get());
        SS_HIP(hipGetLastError());
    }
    sort_rows<T>(n, At.rowptr.get(), tcol.get(), with_values ? tval.get() : nullptr, At.col.get(),
                 with_values ? At.val.get() : nullptr, s);
}
template void transpose<double2>(const CsrBuf<double2> &, CsrBuf<double2> &, hipStream_t, bool);

// ----------------------------------------------------------- diagonal find
template <typename T>
__global__ void k_find_diag(int n, const int *rowptr, const int *col, int *diag, unsigned *missing) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int lo = rowptr[r], hi = rowptr[r + 1] - 1, pos = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = col[mid];
        if (c == r) { pos = mid; break; }
        if (c < r) lo = mid + 1; else hi = mid - 1;
    }
    diag[r] = pos;
    if (pos < 0 && missing) atomicAdd(missing, 1u);
}

int find_diagonal(int n, const int *rowptr, const int *col, int *diag, hipStream_t s) {
    DevBuf<unsigned> miss(1);
    SS_HIP(hipMemsetAsync(miss.get(), 0, sizeof(unsigned), s));
    if (n) {
        k_find_diag<double2><<<div_up(n, 256), 256, 0, s>>>(n, rowptr, col, diag, miss.get());
        SS_HIP(hipGetLastError());
    }
    unsigned h = 0;
    d2h(&h, miss.get(), 1, s);
    return (int)h;
}

// ------------------------------------------------- bandwidth and profile
// Section "Direct factorization": ub = max (j - i), lb = max (i - j) over
// non-zeros; up = sum_i max_j (j - i), lp = sum_j max_i (i - j), each per-row
// (per-column) maximum clamped at zero.
__global__ void k_band_rows(int n, const int *rowptr, const int *col, int *ub, int *lb, unsigned long long *up,
                            int *colmax) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int rs = rowptr[r], re = rowptr[r + 1];
    if (re > rs) {
        const int cmin = col[rs], cmax = col[re - 1];
        atomicMax(ub, cmax - r);
        atomicMax(lb, r - cmin);
        if (cmax > r) atomicAdd(up, (unsigned long long)(cmax - r));
        for (int e = rs; e < re; ++e) {
            const int c = col[e];
            if (r > c) atomicMax(&colmax[c], r - c);
        }
    }
}

__global__ void k_sum_int(int n, const int *v, unsigned long long *out) {
    unsigned long long acc = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += (unsigned)v[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

void bandwidth_profile(int n, const int *rowptr, const int *col, int64_t *B, int64_t *P, hipStream_t s) {
    DevBuf<int> bands(2), colmax((size_t)n + 1);
    DevBuf<unsigned long long> sums(2);
    const int init[2] = {0, 0};
    SS_HIP(hipMemcpyAsync(bands.get(), init, sizeof(init), hipMemcpyHostToDevice, s));
    SS_HIP(hipMemsetAsync(sums.get(), 0, 2 * sizeof(unsigned long long), s));
    SS_HIP(hipMemsetAsync(colmax.get(), 0, sizeof(int) * (n + 1), s));
    if (n) {
        k_band_rows<<<div_up(n, 256), 256, 0, s>>>(n, rowptr, col, bands.get(), bands.get() + 1, sums.get(),
                                                   colmax.get());
        SS_HIP(hipGetLastError());
        k_sum_int<<<256, 256, 0, s>>>(n, colmax.get(), sums.get() + 1);
        SS_HIP(hipGetLastError());
    }
    int hb[2];
    unsigned long long hs[2];
    d2h(hb, bands.get(), 2, s);
    d2h(hs, sums.get(), 2, s);
    *B = (int64_t)hb[0] + hb[1] + 1;
    *P = (int64_t)hs[0] + (int64_t)hs[1];
}

}  // namespace ss
