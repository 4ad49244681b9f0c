// Problem transforms of the Liouvillian (a2):
//   modified  L~ = L + w T  (section "Direct factorization", eq. linear), T
//             with ones at the columns k (d + 1) of the diagonal of rho in one
//             population row (the paper's row 0 on request, by default the
//             population row with the smallest |L_rr|), w = mean of the
//             diagonal of L unless given;
//   shifted   L - sigma I   (section "Eigenvalue Methods", eq. inverse).
#include "csr_tools.hpp"
#include "rowops.hpp"
#include "transform.hpp"

namespace ss {

// Sum of the diagonal of a CSR matrix (binary search per row), reduced in a
// fixed order: per-block partial sums, then one block adds them in order.
__global__ void __launch_bounds__(256) k_diag_partial(int n, const int *rowptr, const int *col, const double2 *val,
                                                      double2 *partial) {
    __shared__ double sx[256], sy[256];
    double ax = 0, ay = 0;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
        int lo = rowptr[r], hi = rowptr[r + 1] - 1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int c = col[mid];
            if (c == r) { ax += val[mid].x; ay += val[mid].y; break; }
            if (c < r) lo = mid + 1; else hi = mid - 1;
        }
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
    if (threadIdx.x == 0) partial[blockIdx.x] = mk(sx[0], sy[0]);
}

__global__ void k_mean_finish(int nparts, const double2 *partial, int n, double2 *out) {
    if (threadIdx.x != 0) return;
    double ax = 0, ay = 0;
    for (int b = 0; b < nparts; ++b) { ax += partial[b].x; ay += partial[b].y; }
    *out = mk(ax / n, ay / n);
}

void mean_diagonal(const CsrBuf<double2> &L, double2 *d_out, hipStream_t s) {
    constexpr int NB = 256;
    StreamScope scope(s);
    DevBuf<double2> part(NB);
    k_diag_partial<<<NB, 256, 0, s>>>(L.n, L.rowptr.get(), L.col.get(), L.val.get(), part.get());
    SS_HIP(hipGetLastError());
    k_mean_finish<<<1, 64, 0, s>>>(NB, part.get(), L.n, d_out);
    SS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- modified
// The row carrying T: any population row k (d + 1) may take it, because the
// population rows of L sum to zero (trace preservation); the one with the
// smallest |L_rr| is taken so that a structurally zero diagonal (a state no
// channel leaves, e.g. a ground state) gets the trace entry as its pivot.
__global__ void k_pick_trace_row(int d, const int *rowptr, const int *col, const double2 *val, int forced,
                                 int *row_out) {
    const int r = pick_trace_row_block(d, rowptr, col, val, forced);
    if (threadIdx.x == 0) *row_out = r;
}

int pick_trace_row(const CsrBuf<double2> &L, int d, int forced, hipStream_t s) {
    DevBuf<int> r(1);
    k_pick_trace_row<<<1, 256, 0, s>>>(d, L.rowptr.get(), L.col.get(), L.val.get(), forced, r.get());
    SS_HIP(hipGetLastError());
    int h = 0;
    d2h(&h, r.get(), 1, s);
    return h;
}

__global__ void k_mod_count(int n, int d, int rt, const int *rowptr, const int *col, const double2 *val,
                            const double2 *w, int *cnt) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (r == rt) cnt[r] = trace_row0<false>(d, rt, rowptr, col, val, *w, nullptr, nullptr);
    else cnt[r] = rowptr[r + 1] - rowptr[r];
}

// MOD_G lanes per row: every row but the trace row is copied (coalesced);
// the trace row is merged with T by the group's first lane
constexpr int MOD_G = 32;

__global__ void __launch_bounds__(256) k_mod_fill(int n, int d, int rt, const int *rowptr, const int *col,
                                                  const double2 *val, const double2 *w, const int *orow, int *ocol,
                                                  double2 *oval) {
    const int r = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) / MOD_G);
    const int g = threadIdx.x & (MOD_G - 1);
    if (r >= n) return;
    if (r == rt) {
        if (g == 0) trace_row0<true>(d, rt, rowptr, col, val, *w, ocol + orow[r], oval + orow[r]);
    } else {
        const int o = orow[r], rs = rowptr[r], re = rowptr[r + 1];
        for (int e = rs + g; e < re; e += MOD_G) {
            ocol[o + e - rs] = col[e];
            oval[o + e - rs] = val[e];
        }
    }
}

// ----------------------------------------------------------------- shifted
// One row per group of SHIFT_G lanes, its entries in chunks of SHIFT_G:
// the same output as shift_row (diagonal shifted, entries that become or are
// zero dropped, a diagonal -sigma inserted where the row has none), written
// coalesced.  The entries' places come from ballots over the group: kept
// entries before a lane, and the insertion point (the first column past the
// diagonal when no diagonal entry has been met).
constexpr int SHIFT_G = 32;

template <bool FILL>
__global__ void __launch_bounds__(256) k_shift_rows(int n, const int *rowptr, const int *col, const double2 *val,
                                                    double sigma, const int *orow, int *ocol, double2 *oval,
                                                    int *cnt) {
    const int lane = threadIdx.x & 63, g = lane & (SHIFT_G - 1);
    const unsigned long long gmask = 0xffffffffull << (lane & 32);
    const unsigned long long below = gmask & ((1ull << lane) - 1ull);
    const int r = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) / SHIFT_G);
    const bool row_ok = r < n;
    int rs = 0, re = 0, o = 0;
    if (row_ok) {
        rs = rowptr[r];
        re = rowptr[r + 1];
        if (FILL) o = orow[r];
    }
    int at = 0;
    bool placed = false;
    for (int base = rs;; base += SHIFT_G) {
        const bool more = row_ok && base < re;
        if (!__any(more)) break;
        const int e = base + g;
        const bool has = more && e < re;
        int c = 0;
        double2 v = mk(0.0, 0.0);
        if (has) {
            c = col[e];
            v = val[e];
            if (c == r) v.x -= sigma;
        }
        const bool keep = has && (v.x != 0.0 || v.y != 0.0);
        const unsigned long long kp = __ballot(keep) & gmask;
        const unsigned long long eq = __ballot(has && c == r) & gmask;
        const unsigned long long gt = __ballot(has && c > r) & gmask;
        int ins_lane = 64;  // (none)
        if (!placed && !eq && gt) ins_lane = __ffsll((long long)gt) - 1;
        const bool ins = ins_lane < 64;
        if (FILL) {
            if (keep) {
                const int p = at + __popcll(kp & below) + ((ins && lane >= ins_lane) ? 1 : 0);
                ocol[o + p] = c;
                oval[o + p] = v;
            }
            if (ins && lane == ins_lane) {
                const int p = at + __popcll(kp & below);
                ocol[o + p] = r;
                oval[o + p] = mk(-sigma, 0.0);
            }
        }
        at += __popcll(kp) + (ins ? 1 : 0);
        placed = placed || eq || ins;
    }
    if (!row_ok) return;
    if (!placed) {
        if (FILL && g == 0) {
            ocol[o + at] = r;
            oval[o + at] = mk(-sigma, 0.0);
        }
        ++at;
    }
    if (!FILL && g == 0) cnt[r] = at;
}

static void finish_rows(CsrBuf<double2> &A, int n, DevBuf<int> &cnt, hipStream_t s) {
    A.rowptr.resize((size_t)n + 1);
    const int64_t nnz = scan_exclusive(cnt.get(), A.rowptr.get(), n, s, true);
    SS_REQUIRE(nnz < (int64_t(1) << 31), SS_E_INVALID_ARG, "transformed matrix too large");
    A.n = n;
    A.nnz = (int)nnz;
    A.col.resize((size_t)nnz);
    A.val.resize((size_t)nnz);
}

void make_modified(const CsrBuf<double2> &L, int d, int rt, const double2 *d_w, CsrBuf<double2> &A, hipStream_t s) {
    const int n = L.n;
    StreamScope scope(s);
    DevBuf<int> cnt((size_t)n + 1);
    k_mod_count<<<div_up(n, 256), 256, 0, s>>>(n, d, rt, L.rowptr.get(), L.col.get(), L.val.get(), d_w, cnt.get());
    SS_HIP(hipGetLastError());
    finish_rows(A, n, cnt, s);
    k_mod_fill<<<div_up((int64_t)n * MOD_G, 256), 256, 0, s>>>(n, d, rt, L.rowptr.get(), L.col.get(), L.val.get(),
                                                               d_w, A.rowptr.get(), A.col.get(), A.val.get());
    SS_HIP(hipGetLastError());
}

void make_shifted(const CsrBuf<double2> &L, double sigma, CsrBuf<double2> &A, hipStream_t s) {
    const int n = L.n;
    StreamScope scope(s);
    DevBuf<int> cnt((size_t)n + 1);
    const int grid = div_up((int64_t)n * SHIFT_G, 256);
    if (n) {
        k_shift_rows<false><<<grid, 256, 0, s>>>(n, L.rowptr.get(), L.col.get(), L.val.get(), sigma, nullptr,
                                                 nullptr, nullptr, cnt.get());
        SS_HIP(hipGetLastError());
    }
    finish_rows(A, n, cnt, s);
    if (n) {
        k_shift_rows<true><<<grid, 256, 0, s>>>(n, L.rowptr.get(), L.col.get(), L.val.get(), sigma, A.rowptr.get(),
                                                A.col.get(), A.val.get(), nullptr);
        SS_HIP(hipGetLastError());
    }
}

}  // namespace ss
