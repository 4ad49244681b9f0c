// Device memory, pointer classification and the integer exclusive scan used
// to turn per-row counts into CSR row pointers.
#include "ss_internal.hpp"

namespace ss {

void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? SS_E_OOM : SS_E_HIP,
                    "hipMalloc(" + std::to_string(bytes) + " B): " + hipGetErrorString(e));
    }
    return p;
}

void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// -------------------------------------------------------------------- scan
// 256 threads x 4 items per block; per-block totals are scanned recursively.
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 4;
constexpr int SCAN_B = SCAN_T * SCAN_I;

__global__ void __launch_bounds__(SCAN_T) k_scan_block(const int *in, int *out, int64_t n,
                                                      int *block_sums) {
    __shared__ int s[SCAN_T];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)t * SCAN_I;
    int v[SCAN_I];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
    }
    int loc[SCAN_I];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) { loc[k] = sum; sum += v[k]; }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int x = (t >= off) ? s[t - off] : 0;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    const int excl = s[t] - sum;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = excl + loc[k];
    }
    if (t == SCAN_T - 1) block_sums[blockIdx.x] = s[SCAN_T - 1];
}

__global__ void __launch_bounds__(SCAN_T) k_scan_add(int *out, int64_t n, const int *offsets) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
    const int o = offsets[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] += o;
    }
}

__global__ void k_copy_int(int *dst, const int *src) { *dst = *src; }

// Exclusive scan: out[i] = sum_{j<i} in[j] for i < n, out[n] = total.
static void scan_rec(const int *in, int *out, int64_t n, hipStream_t s) {
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    DevBuf<int> sums((size_t)nb + 1);
    k_scan_block<<<(unsigned)nb, SCAN_T, 0, s>>>(in, out, n, sums.get());
    SS_HIP(hipGetLastError());
    if (nb > 1) {
        scan_rec(sums.get(), sums.get(), nb, s);
        k_scan_add<<<(unsigned)nb, SCAN_T, 0, s>>>(out, n, sums.get());
        SS_HIP(hipGetLastError());
        k_copy_int<<<1, 1, 0, s>>>(out + n, sums.get() + nb);
    } else {
        k_copy_int<<<1, 1, 0, s>>>(out + n, sums.get());
    }
    SS_HIP(hipGetLastError());
    // sums must outlive the kernels that read it
    SS_HIP(hipStreamSynchronize(s));
}

int64_t scan_exclusive(const int *in, int *out, int64_t n, hipStream_t s, bool want_total) {
    if (n <= 0) {
        SS_HIP(hipMemsetAsync(out, 0, sizeof(int), s));
        return 0;
    }
    scan_rec(in, out, n, s);
    if (!want_total) return -1;
    int total = 0;
    d2h(&total, out + n, 1, s);
    return total;
}

}  // namespace ss
