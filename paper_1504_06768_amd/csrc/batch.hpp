// Helpers of the batched set-up kernels (batch.hip): many systems handled by
// one launch, each system a job owning a contiguous range of blocks.
#pragma once
#include <vector>

#include "ss_internal.hpp"

namespace ss {

// Job index of block b from the exclusive block prefix bstart[0..njobs].
__device__ inline int job_of_block(const int *bstart, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bstart[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// In-place exclusive scan of a[0..len): a[i] = sum of the counts before i,
// a[len] = *total = the sum of all; with copy != null, copy[0..len] = a too.
struct ScanJob {
    int *a;
    int len;
    int *total;
    int *copy;
};

// One launch for every job (one 1024-thread block each); the job array is
// uploaded from `jobs` and released behind the launch on s.
void seg_scan(const std::vector<ScanJob> &jobs, hipStream_t s);

// pre = exclusive prefix of blocks; returns the total.
int block_prefix(const std::vector<int> &blocks, std::vector<int> &pre);

// Device copy of a host vector, released behind the work queued on s.
template <typename T>
DevBuf<T> upload(const std::vector<T> &v, hipStream_t s) {
    StreamScope scope(s);
    DevBuf<T> d(std::max<size_t>(v.size(), 1));
    if (!v.empty()) h2d(d.get(), v.data(), v.size(), s);
    return d;
}

}  // namespace ss
