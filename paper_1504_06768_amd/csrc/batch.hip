// Batched set-up helpers: a segmented scan with one block per system.
#include "batch.hpp"

namespace ss {

// One 1024-thread block per segment: each thread scans a contiguous chunk,
// the chunk sums are scanned in shared memory (fixed order).
__global__ void __launch_bounds__(1024) k_seg_scan(const ScanJob *jobs) {
    __shared__ int sh[1024];
    const ScanJob J = jobs[blockIdx.x];
    const int t = threadIdx.x;
    const int chunk = (J.len + 1023) / 1024;
    const int b = min(J.len, t * chunk), e = min(J.len, b + chunk);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += J.a[i];
    sh[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int run = sh[t] - sum;
    for (int i = b; i < e; ++i) {
        const int c = J.a[i];
        J.a[i] = run;
        if (J.copy) J.copy[i] = run;
        run += c;
    }
    if (t == 1023) {
        J.a[J.len] = sh[1023];
        if (J.copy) J.copy[J.len] = sh[1023];
        if (J.total) *J.total = sh[1023];
    }
}

void seg_scan(const std::vector<ScanJob> &jobs, hipStream_t s) {
    if (jobs.empty()) return;
    DevBuf<ScanJob> d = upload(jobs, s);
    k_seg_scan<<<(unsigned)jobs.size(), 1024, 0, s>>>(d.get());
    SS_HIP(hipGetLastError());
}

int block_prefix(const std::vector<int> &blocks, std::vector<int> &pre) {
    pre.assign(blocks.size() + 1, 0);
    for (size_t j = 0; j < blocks.size(); ++j) pre[j + 1] = pre[j] + blocks[j];
    return pre.back();
}

}  // namespace ss
