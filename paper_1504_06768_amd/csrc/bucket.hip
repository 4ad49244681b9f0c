// Stable bucket sort of positions by small integer keys: the colour classes
// of the colour-class ordering and the level sets of the triangular-solve
// schedules.
//
// The positions are cut into chunks, one wavefront each.  A first pass
// counts every key in every chunk; an exclusive scan of those counts in
// (key, chunk) order gives each (key, chunk) pair its first output slot; a
// second pass walks the chunk again in order and hands out the slots.  In
// both passes the lanes of one 64-position round that hold the same key find
// each other with one ballot per key bit, and a running count per key sits
// in LDS, so the order inside a key is the position order and no global
// counter is contended.  Keys are taken in windows of BKT_WIN (one LDS
// counter each); the chunk length grows with the number of keys so that a
// window's counters stay within BKT_COUNTERS_MAX.
#include "bucket.hpp"

namespace ss {

namespace {

constexpr int BKT_WIN = 1024;       // keys per window
constexpr int BKT_BITS = 10;        // log2(BKT_WIN)
constexpr int BKT_CHUNK_MIN = 1024;  // positions per chunk, at least
constexpr int64_t BKT_COUNTERS_MAX = int64_t(1) << 22;

// lanes of this wavefront whose key equals this lane's (keys < BKT_WIN;
// lanes with in = false take part in the ballots only)
__device__ inline unsigned long long same_key(bool in, int key) {
    unsigned long long m = __ballot(in);
#pragma unroll
    for (int b = 0; b < BKT_BITS; ++b) {
        const bool bit = (key >> b) & 1;
        const unsigned long long bb = __ballot(in && bit);
        m &= bit ? bb : ~bb;
    }
    return in ? m : 0ull;
}

// cnt[(k - k0) * nb + b] = positions of chunk b with key k (k0 <= k < k0 + kw)
__global__ void __launch_bounds__(64) k_bucket_count(int n, int chunk, int nb, int k0, int kw, const int *key,
                                                     int *cnt) {
    __shared__ int sc[BKT_WIN];
    const int lane = threadIdx.x, b = blockIdx.x;
    for (int k = lane; k < kw; k += 64) sc[k] = 0;
    __syncthreads();
    const int p0 = b * chunk, p1 = min(n, p0 + chunk);
    for (int r = p0; r < p1; r += 64) {
        const int p = r + lane;
        const int k = p < p1 ? key[p] - k0 : -1;
        const bool in = k >= 0 && k < kw;
        const unsigned long long m = same_key(in, in ? k : 0);
        if (in && lane == __ffsll((long long)m) - 1) sc[k] += __popcll(m);
        __syncthreads();
    }
    for (int k = lane; k < kw; k += 64) cnt[(size_t)k * nb + b] = sc[k];
}

// offs: exclusive scan of cnt; before: positions with keys below k0
__global__ void __launch_bounds__(64) k_bucket_scatter(int n, int chunk, int nb, int k0, int kw, int before,
                                                       const int *key, const int *items, const int *offs, int *out,
                                                       int *inv) {
    __shared__ int sc[BKT_WIN];
    const int lane = threadIdx.x, b = blockIdx.x;
    for (int k = lane; k < kw; k += 64) sc[k] = before + offs[(size_t)k * nb + b];
    __syncthreads();
    const int p0 = b * chunk, p1 = min(n, p0 + chunk);
    for (int r = p0; r < p1; r += 64) {
        const int p = r + lane;
        const int k = p < p1 ? key[p] - k0 : -1;
        const bool in = k >= 0 && k < kw;
        const unsigned long long m = same_key(in, in ? k : 0);
        const int lead = in ? __ffsll((long long)m) - 1 : 0;
        const int at = in ? sc[k] : 0;  // read by every lane of the key before the leader moves it on
        __syncthreads();
        if (in) {
            const int q = at + __popcll(m & ((1ull << lane) - 1ull));
            const int v = items ? items[p] : p;
            out[q] = v;
            if (inv) inv[v] = q;
            if (lane == lead) sc[k] = at + __popcll(m);
        }
        __syncthreads();
    }
}

// starts[k0 + k] = before + offs[k * nb] (first slot of key k0 + k)
__global__ void k_bucket_starts(int kw, int nb, int before, const int *offs, int *starts) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kw) starts[k] = before + offs[(size_t)k * nb];
}

__global__ void k_bucket_end(int nkeys, int n, int *starts) { starts[nkeys] = n; }

}  // namespace

void bucket_sort(int n, const int *key, int nkeys, const int *items, int *out, int *inv, int *starts,
                 hipStream_t s) {
    SS_REQUIRE(n >= 0 && nkeys >= 0, SS_E_INVALID_ARG, "bucket sort: bad sizes");
    if (starts) {
        k_bucket_end<<<1, 1, 0, s>>>(nkeys, n, starts);
        SS_HIP(hipGetLastError());
    }
    if (n == 0 || nkeys == 0) return;
    const int kw_max = std::min(nkeys, BKT_WIN);
    int64_t chunk = std::max<int64_t>(BKT_CHUNK_MIN, ((int64_t)n * kw_max + BKT_COUNTERS_MAX - 1) / BKT_COUNTERS_MAX);
    chunk = (chunk + 63) / 64 * 64;
    const int nb = (int)(((int64_t)n + chunk - 1) / chunk);
    DevBuf<int> cnt((size_t)kw_max * nb + 1), offs((size_t)kw_max * nb + 1);
    int before = 0;  // positions whose keys lie in lower windows
    for (int k0 = 0; k0 < nkeys; k0 += BKT_WIN) {
        const int kw = std::min(BKT_WIN, nkeys - k0);
        k_bucket_count<<<nb, 64, 0, s>>>(n, (int)chunk, nb, k0, kw, key, cnt.get());
        SS_HIP(hipGetLastError());
        const int64_t total = scan_exclusive(cnt.get(), offs.get(), (int64_t)kw * nb, s, true);
        k_bucket_scatter<<<nb, 64, 0, s>>>(n, (int)chunk, nb, k0, kw, before, key, items, offs.get(), out, inv);
        if (starts) k_bucket_starts<<<div_up(kw, 256), 256, 0, s>>>(kw, nb, before, offs.get(), starts + k0);
        SS_HIP(hipGetLastError());
        before += (int)total;
    }
    SS_REQUIRE(before == n, SS_E_INVALID_ARG, "bucket sort: a key lies outside [0, nkeys)");
    // the scratch buffers are released on return
    SS_HIP(hipStreamSynchronize(s));
}

}  // namespace ss
