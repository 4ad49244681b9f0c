// Level-synchronous triangular solves for shallow level schedules (section
// "Iterative Solvers": the forward and backward substitutions of the ILU
// preconditioner).
//
// In the colour-class ordering a zero-fill factor has about ten levels of
// ~10^5 rows each.  A substitution is then bound by memory bandwidth, not by
// the time a result takes to reach the rows that need it, so each level is
// one plain launch: every value a row needs was written by an earlier
// launch, and nothing is polled.  CLS_G lanes take a row's entries in turn,
// a butterfly sums their products, and the first lane writes the row.  The
// products are summed in a tree instead of in entry order, so the results
// agree with the sync-free solves to rounding, not bit for bit.
#include "ilu.hpp"

namespace ss {

namespace {

constexpr int CLS_G = 8;      // lanes per row
constexpr int CLS_BS = 256;   // threads per workgroup

// slot {row, first entry, end entry, .}: lower rows subtract entries
// [first, end) of L (unit diagonal); upper rows those of U and divide by the
// pivot just before them
template <typename T, bool UPPER>
__global__ void __launch_bounds__(CLS_BS) k_trsv_level(int lo, int hi, const int4 *slot, const int *col,
                                                        const T *val, const T *in, T *out, const int *skip) {
    if (skip && *skip) return;
    const int t = blockIdx.x * CLS_BS + threadIdx.x;
    const int idx = lo + t / CLS_G, k = t % CLS_G;
    const bool active = idx < hi;
    int4 sl = make_int4(0, 0, 0, 0);
    T acc = czero<T>();
    if (active) {
        sl = slot[idx];
        for (int e = sl.y + k; e < sl.z; e += CLS_G) acc = cadd(acc, cmul(val[e], out[col[e]]));
    }
#pragma unroll
    for (int off = CLS_G / 2; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, 64);
        acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (active && k == 0) {
        T r = csub(in[sl.x], acc);
        if (UPPER) r = cdiv(r, val[sl.y - 1]);
        out[sl.x] = r;
    }
}

}  // namespace

template <typename T>
void trsv_classes(const LevelSched &ls, bool upper, const Csr<T> &LU, const T *in, T *out, const int *skip,
                  hipStream_t s) {
    SS_REQUIRE((int)ls.hptr.size() == ls.nlev + 1, SS_E_STATE, "level schedule without its host copy");
    for (int l = 0; l < ls.nlev; ++l) {
        const int lo = ls.hptr[(size_t)l], hi = ls.hptr[(size_t)l + 1];
        if (hi <= lo) continue;
        const unsigned grid = (unsigned)div_up((int64_t)(hi - lo) * CLS_G, CLS_BS);
        if (upper)
            k_trsv_level<T, true><<<grid, CLS_BS, 0, s>>>(lo, hi, ls.slot.get(), LU.col, LU.val, in, out, skip);
        else
            k_trsv_level<T, false><<<grid, CLS_BS, 0, s>>>(lo, hi, ls.slot.get(), LU.col, LU.val, in, out, skip);
    }
    SS_HIP(hipGetLastError());
}
template void trsv_classes<double2>(const LevelSched &, bool, const Csr<double2> &, const double2 *, double2 *,
                                    const int *, hipStream_t);
template void trsv_classes<float2>(const LevelSched &, bool, const Csr<float2> &, const float2 *, float2 *,
                                   const int *, hipStream_t);

}  // namespace ss
