// Level-synchronous triangular solves for shallow level schedules (section
// "Iterative Solvers": the forward and backward substitutions of the ILU
// preconditioner).
//
// In the colour-class ordering a zero-fill factor has about ten levels of
// ~10^5 rows each.  A substitution is then bound by memory bandwidth, not by
// the time a result takes to reach the rows that need it, so each level is
// one plain launch: every value a row needs was written by an earlier
// launch, and nothing is polled.  A group of lanes takes a row's entries, a
// butterfly sums their products, and the first lane writes the row.  The
// products are summed in a tree instead of in entry order, so the results
// agree with the sync-free solves to rounding, not bit for bit.
#include "ilu.hpp"

namespace ss {

namespace {

constexpr int CLS_BS = 256;  // threads per workgroup

// slot {row, first entry, end entry, .}: lower rows subtract entries
// [first, end) of L (unit diagonal); upper rows those of U and divide by the
// pivot just before them.  G lanes per row take up to U entries each per
// round, with every load of a round issued before its products are formed;
// a level then needs few enough threads to be resident at once, and each
// thread's memory latencies overlap.
template <typename T, bool UPPER, int G, int U>
__global__ void __launch_bounds__(CLS_BS) k_trsv_level(int lo, int hi, const int4 *slot, const int *col,
                                                       const T *val, const T *in, T *out, const int *pin, T *outp,
                                                       const int *skip) {
    if (skip && *skip) return;
    // workgroups go round-robin to the eight XCDs (b -> b % 8); renumbered
    // so that each XCD takes a contiguous eighth of the level, whose rows
    // gather from a narrower part of the vector through that XCD's L2
    const unsigned g = gridDim.x, bx = blockIdx.x;
    const unsigned lb = (g % 8) ? bx : (bx % 8) * (g / 8) + bx / 8;
    const int t = (int)lb * CLS_BS + threadIdx.x;
    const int idx = lo + t / G, l = t % G;
    const bool active = idx < hi;
    int4 sl = make_int4(0, 0, 0, 0);
    T acc = czero<T>(), b = czero<T>(), piv = czero<T>();
    if (active) {
        sl = slot[idx];
        if (l == 0) {
            b = in[(!UPPER && pin) ? pin[sl.x] : sl.x];
            if (UPPER) piv = val[sl.y - 1];
        }
        for (int e0 = sl.y; e0 < sl.z; e0 += G * U) {
            int c[U];
            T v[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * G + l;
                if (e < sl.z) {
                    c[u] = col[e];
                    v[u] = val[e];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e0 + u * G + l < sl.z) xv[u] = out[c[u]];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e0 + u * G + l < sl.z) acc = cadd(acc, cmul(v[u], xv[u]));
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, G);
        acc.y += __shfl_xor(acc.y, off, G);
    }
    if (active && l == 0) {
        T r = csub(b, acc);
        if (UPPER) r = cdiv(r, piv);
        out[sl.x] = r;
        if (UPPER && pin) outp[pin[sl.x]] = r;
    }
}

template <typename T, bool UPPER, int G, int U>
void levels_launch(const LevelSched &ls, const Csr<T> &LU, const T *in, T *out, const int *pin, T *outp,
                   const int *skip, hipStream_t s) {
    for (int l = 0; l < ls.nlev; ++l) {
        const int lo = ls.hptr[(size_t)l], hi = ls.hptr[(size_t)l + 1];
        if (hi <= lo) continue;
        const unsigned grid = (unsigned)((div_up((int64_t)(hi - lo) * G, CLS_BS) + 7) / 8 * 8);  // a multiple of 8
        k_trsv_level<T, UPPER, G, U><<<grid, CLS_BS, 0, s>>>(lo, hi, ls.slot.get(), LU.col, LU.val, in, out, pin,
                                                             outp, skip);
    }
}

}  // namespace

template <typename T>
void trsv_classes(const LevelSched &ls, bool upper, const Csr<T> &LU, const T *in, T *out, const int *skip,
                  hipStream_t s, const int *pin, T *outp) {
    SS_REQUIRE((int)ls.hptr.size() == ls.nlev + 1, SS_E_STATE, "level schedule without its host copy");
    if (LU.n == 0) return;
    // mean entries per row of one triangle (the other's are about as many).
    // Kerr chain in the colour-class order (~10 per triangle), per complex128
    // application: 8 lanes x 3 entries 0.345 ms; 8 x 4 0.346, 8 x 2 0.352,
    // 8 x 6 0.356, 4 x 4 0.368, 4 x 3 0.372, 4 x 2 0.374, 8 x 1 0.379,
    // 16 x 2 0.383, 16 x 1 0.402, 2 x 6 0.446 ms
    const double mean = std::max(0.0, (double)(LU.nnz - LU.n) / (2.0 * LU.n));
    if (mean <= 12) {
        if (upper) levels_launch<T, true, 8, 3>(ls, LU, in, out, pin, outp, skip, s);
        else levels_launch<T, false, 8, 3>(ls, LU, in, out, pin, outp, skip, s);
    } else if (mean <= 32) {
        if (upper) levels_launch<T, true, 8, 4>(ls, LU, in, out, pin, outp, skip, s);
        else levels_launch<T, false, 8, 4>(ls, LU, in, out, pin, outp, skip, s);
    } else {
        if (upper) levels_launch<T, true, 32, 2>(ls, LU, in, out, pin, outp, skip, s);
        else levels_launch<T, false, 32, 2>(ls, LU, in, out, pin, outp, skip, s);
    }
    SS_HIP(hipGetLastError());
}
template void trsv_classes<double2>(const LevelSched &, bool, const Csr<double2> &, const double2 *, double2 *,
                                    const int *, hipStream_t, const int *, double2 *);
template void trsv_classes<float2>(const LevelSched &, bool, const Csr<float2> &, const float2 *, float2 *,
                                   const int *, hipStream_t, const int *, float2 *);

}  // namespace ss
