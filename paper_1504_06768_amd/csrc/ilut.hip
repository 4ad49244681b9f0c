// Dual-threshold incomplete LU without pivoting, ILUT(drop_tol, fill)
// (section "Iterative Solvers": the iLU preconditioner with a drop tolerance
// and a fill limit; section "Numerical Simulations": the fill-factor study).
//
// Row i is eliminated in increasing column order (row-wise IKJ form):
//   w = a_i, tau = drop_tol * ||a_i||_inf, keep = ceil(fill * nnz(a_i));
//   for each k < i present in w, smallest first:
//       l = w_k / u_kk; drop it when |l| < tau, otherwise keep it as the
//       multiplier and apply w_j -= l u_kj for every stored u_kj, j > k
//       (entries not yet in w are fill);
//   then the strict upper part keeps the entries with |w_j| >= tau, and each
//   strict part keeps at most `keep` entries, largest magnitude first, ties
//   to the lower column; the diagonal is always kept and the pivot boost of
//   ILU(0) applies.
// Complex products and Smith's quotient are written out and the file is
// compiled without floating-point contraction, so each step rounds like a
// plain sequential implementation of these rules.
//
// GPU layout.  One wavefront per row, rows taken in increasing order from an
// atomic counter by a persistent set of wavefronts (so every row a wavefront
// waits on has already been taken by a running one).  A finished row is
// written into a per-row slot of capacity min(keep, bw_lower) + 1 +
// min(keep, bw_upper), then published by a done flag (release / acquire at
// device scope); the slots are compacted into CSR at the end.  In RCM order
// every entry of row i, fill included, lies in the window
// [i - bw_lower, i + bw_upper] of the input's bandwidths, so each wavefront
// keeps its working row dense over that window in device memory, a bitmap of
// the present columns in LDS (to walk the lower part in column order and to
// emit the upper part sorted), and a list of the touched columns (to clear
// the window for the next row).  The `keep` largest entries are found by a
// radix select on the magnitudes' bit patterns.
#include <climits>

#include "ilu.hpp"
#include "syncfree.hpp"

namespace ss {

namespace {

constexpr int ILUT_HIST = 256;
constexpr long long ILUT_WAIT_TICKS = 2000000000ll;  // 20 s of the 100 MHz clock

__device__ __forceinline__ double2 t_mul(double2 a, double2 b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 t_sub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
// Smith's method (R. L. Smith, CACM 5 (1962) 435)
__device__ __forceinline__ double2 t_div(double2 a, double2 b) {
    if (fabs(b.x) >= fabs(b.y)) {
        const double ratio = b.y / b.x, den = b.x + b.y * ratio;
        return mk((a.x + a.y * ratio) / den, (a.y - a.x * ratio) / den);
    }
    const double ratio = b.x / b.y, den = b.x * ratio + b.y;
    return mk((a.x * ratio + a.y) / den, (a.y * ratio - a.x) / den);
}
__device__ __forceinline__ double t_abs(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ unsigned long long mag_bits(double m) {
    return (unsigned long long)__double_as_longlong(m);
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) { return (1ull << lane) - 1ull; }

__device__ __forceinline__ int wave_sum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
// exclusive prefix sum over the lanes
__device__ __forceinline__ int wave_excl(int v, int lane) {
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x - v;
}

// First set bit of the LDS bitmap at a position in [p, lim), or -1.
__device__ int next_bit(const unsigned *bits, int p, int lim, int lane) {
    if (p >= lim) return -1;
    const int wl = (lim - 1) >> 5;
    for (int w0 = p >> 5; w0 <= wl; w0 += 64) {
        const int w = w0 + lane;
        unsigned v = 0;
        if (w <= wl) {
            v = bits[w];
            if (w == (p >> 5)) v &= ~0u << (p & 31);
            if (w == wl) {
                const int r = lim - (wl << 5);
                if (r < 32) v &= (1u << r) - 1u;
            }
        }
        const unsigned long long m = __ballot(v != 0);
        if (m) {
            const int L = __ffsll((long long)m) - 1;
            const unsigned vv = __shfl(v, L, 64);
            return ((w0 + L) << 5) + __ffs(vv) - 1;
        }
    }
    return -1;
}

// Radix select over a candidate set given by get(idx, bits, col) -> valid:
// on return every candidate with (bits > T) or (bits == T and col <= cstar)
// is one of the `keep` largest (ties to the lower column), and those are
// exactly `keep` candidates.  Requires keep >= 1 and more than keep
// candidates.
template <class Get>
__device__ void select_top(Get get, int count, int keep, unsigned *hist, int lane, unsigned long long &T,
                           int &cstar) {
    unsigned long long prefix = 0, pmask = 0;
    int need = keep;  // rank wanted inside the current prefix class, from the top
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = lane; b < ILUT_HIST; b += 64) hist[b] = 0;
        for (int c = 0; c < count; c += 64) {
            const int idx = c + lane;
            unsigned long long bits = 0;
            int col = 0;
            if (idx < count && get(idx, bits, col) && (bits & pmask) == prefix)
                atomicAdd(&hist[(bits >> shift) & 255u], 1u);
        }
        // digit d, scanning from the top, where the cumulative count reaches need
        int h[4], s4 = 0;
        for (int q = 0; q < 4; ++q) {
            h[q] = (int)hist[255 - (4 * lane + q)];
            s4 += h[q];
        }
        const int above = wave_excl(s4, lane);  // count in bins above this lane's four
        int dsel = -1, before = 0;
        if (above < need && above + s4 >= need) {
            int acc = above;
            for (int q = 0; q < 4; ++q) {
                if (acc + h[q] >= need) {
                    dsel = 255 - (4 * lane + q);
                    before = acc;
                    break;
                }
                acc += h[q];
            }
        }
        const unsigned long long owner = __ballot(dsel >= 0);
        const int L = __ffsll((long long)owner) - 1;
        dsel = __shfl(dsel, L, 64);
        before = __shfl(before, L, 64);
        need -= before;
        prefix |= (unsigned long long)dsel << shift;
        pmask |= 255ull << shift;
    }
    T = prefix;
    // ties at T: the need-th smallest column among them
    unsigned cp = 0, cm = 0;
    int needc = need;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = lane; b < ILUT_HIST; b += 64) hist[b] = 0;
        for (int c = 0; c < count; c += 64) {
            const int idx = c + lane;
            unsigned long long bits = 0;
            int col = 0;
            if (idx < count && get(idx, bits, col) && bits == T && ((unsigned)col & cm) == cp)
                atomicAdd(&hist[((unsigned)col >> shift) & 255u], 1u);
        }
        int h[4], s4 = 0;
        for (int q = 0; q < 4; ++q) {
            h[q] = (int)hist[4 * lane + q];
            s4 += h[q];
        }
        const int below = wave_excl(s4, lane);
        int dsel = -1, before = 0;
        if (below < needc && below + s4 >= needc) {
            int acc = below;
            for (int q = 0; q < 4; ++q) {
                if (acc + h[q] >= needc) {
                    dsel = 4 * lane + q;
                    before = acc;
                    break;
                }
                acc += h[q];
            }
        }
        const unsigned long long owner = __ballot(dsel >= 0);
        const int L = __ffsll((long long)owner) - 1;
        dsel = __shfl(dsel, L, 64);
        before = __shfl(before, L, 64);
        needc -= before;
        cp |= (unsigned)dsel << shift;
        cm |= 255u << shift;
    }
    cstar = (int)cp;
}

struct IlutArgs {
    int n;
    const int *rowptr;
    const int *col;
    const double2 *a;
    int bwl, bwu, ws, nwords;  // window [i - bwl, i + bwu], ws = bwl + bwu + 1 entries
    double drop, fill, detect, boost;
    const long long *soff;     // slot offsets (n + 1)
    int *scol;
    double2 *sval;
    int2 *meta;                // {lower count, upper count} of each finished row
    unsigned *done;
    double2 *win;              // per wavefront: ws entries
    int *touched;              // per wavefront: ws entries
    int *mcol;                 // per wavefront: bwl + 1 entries
    double2 *mval;
    unsigned *next_row;
    unsigned *status;
    int *nguard;
};

__device__ __forceinline__ int keep_of(double fill, int nz) {
    const double k = ceil(fill * (double)nz);
    return k > (double)INT_MAX ? INT_MAX : (int)k;
}

}  // namespace

__global__ void __launch_bounds__(256) k_ilut(IlutArgs g, int wpb) {
    extern __shared__ unsigned lds[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    if (wib >= wpb) return;
    const long long wid = (long long)blockIdx.x * wpb + wib;
    unsigned *bits = lds + (size_t)wib * (g.nwords + ILUT_HIST);
    unsigned *hist = bits + g.nwords;
    double2 *W = g.win + wid * g.ws;
    int *touched = g.touched + wid * g.ws;
    int *mcol = g.mcol + wid * (g.bwl + 1);
    double2 *mval = g.mval + wid * (g.bwl + 1);
    for (int w = lane; w < g.nwords; w += 64) bits[w] = 0;

    for (;;) {
        int i = 0, stop = 0;
        if (lane == 0) {
            i = (int)atomicAdd(g.next_row, 1u);
            stop = aborted(g.status) ? 1 : 0;
        }
        i = __shfl(i, 0, 64);
        stop = __shfl(stop, 0, 64);
        if (i >= g.n || stop) break;
        const int rs = g.rowptr[i], re = g.rowptr[i + 1], nz = re - rs;
        const int base = i - g.bwl;
        // scatter a_i into the window
        int nt = 0;
        double rn = 0.0;
        for (int c = rs; c < re; c += 64) {
            const int e = c + lane;
            bool add = false;
            int idx = 0;
            if (e < re) {
                const double2 v = g.a[e];
                idx = g.col[e] - base;
                W[idx] = v;
                atomicOr(&bits[idx >> 5], 1u << (idx & 31));
                rn = fmax(rn, t_abs(v));
                add = true;
            }
            const unsigned long long m = __ballot(add);
            if (add) touched[nt + __popcll(m & lanes_below(lane))] = idx;
            nt += __popcll(m);
        }
        rn = wave_max(rn);
        const double tau = g.drop * rn;
        const int keep = keep_of(g.fill, nz);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");

        // lower part in increasing column order
        int nm = 0, maxidx = 0;
        int cursor = (nz > 0) ? g.col[rs] - base : g.bwl;
        bool failed = false;
        for (;;) {
            const int kidx = next_bit(bits, cursor, g.bwl, lane);
            if (kidx < 0) break;
            cursor = kidx + 1;
            const int k = kidx + base;
            // wait for row k
            int ok = 1;
            if (lane == 0) {
                if (__hip_atomic_load(g.done + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                    const long long t0 = wall_clock64();
                    unsigned spins = 0;
                    while (__hip_atomic_load(g.done + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                        __builtin_amdgcn_s_sleep(2);
                        if ((++spins & 255u) == 0 &&
                            (aborted(g.status) || wall_clock64() - t0 > ILUT_WAIT_TICKS)) {
                            atomicOr(g.status, STATUS_SPIN_TIMEOUT);
                            ok = 0;
                            break;
                        }
                    }
                }
            }
            ok = __shfl(ok, 0, 64);
            if (!ok) {
                failed = true;
                break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int2 mk_ = g.meta[k];
            const long long ok0 = g.soff[k] + mk_.x;  // slot position of u_kk
            const double2 ukk = g.sval[ok0];
            const double2 l = t_div(W[kidx], ukk);
            if (t_abs(l) < tau) {
                if (lane == 0) W[kidx] = mk(0.0, 0.0);
                continue;
            }
            if (lane == 0) {
                mcol[nm] = k;
                mval[nm] = l;
            }
            ++nm;
            for (int c = 0; c < mk_.y; c += 64) {
                const int f = c + lane;
                bool add = false;
                int idx = 0;
                if (f < mk_.y) {
                    const long long p = ok0 + 1 + f;
                    idx = g.scol[p] - base;
                    const double2 t = t_mul(l, g.sval[p]);
                    const unsigned bit = 1u << (idx & 31);
                    const unsigned old = atomicOr(&bits[idx >> 5], bit);
                    if (old & bit) {
                        W[idx] = t_sub(W[idx], t);
                    } else {
                        W[idx] = t_sub(mk(0.0, 0.0), t);
                        add = true;
                    }
                }
                const unsigned long long m = __ballot(add);
                if (add) touched[nt + __popcll(m & lanes_below(lane))] = idx;
                nt += __popcll(m);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        }
        if (failed) break;

        // upper candidates: |w_j| >= tau, j > i
        int mu = 0;
        for (int c = 0; c < nt; c += 64) {
            const int t = c + lane;
            int cnt = 0;
            if (t < nt) {
                const int idx = touched[t];
                maxidx = max(maxidx, idx);
                if (idx > g.bwl && t_abs(W[idx]) >= tau) cnt = 1;
            }
            mu += wave_sum(cnt);
        }
        maxidx = wave_max(maxidx);

        // thresholds of the fill cap
        unsigned long long Tl = 0, Tu = 0;
        int cl = INT_MAX, cu = INT_MAX;
        const bool cap_l = nm > keep, cap_u = mu > keep;
        if (keep > 0 && cap_l) {
            auto getl = [&](int idx, unsigned long long &b, int &col) {
                b = mag_bits(t_abs(mval[idx]));
                col = mcol[idx];
                return true;
            };
            select_top(getl, nm, keep, hist, lane, Tl, cl);
        }
        if (keep > 0 && cap_u) {
            auto getu = [&](int t, unsigned long long &b, int &col) {
                const int idx = touched[t];
                if (idx <= g.bwl) return false;
                const double m = t_abs(W[idx]);
                if (!(m >= tau)) return false;
                b = mag_bits(m);
                col = idx + base;
                return true;
            };
            select_top(getu, nt, keep, hist, lane, Tu, cu);
        }

        // write the slot: kept multipliers (already in column order), pivot,
        // kept upper entries in column order (walk of the bitmap)
        const long long o = g.soff[i], o_end = g.soff[i + 1];
        int lc = 0;
        if (keep > 0) {
            for (int c = 0; c < nm; c += 64) {
                const int t = c + lane;
                bool kp = false;
                int col = 0;
                double2 v = mk(0.0, 0.0);
                if (t < nm) {
                    col = mcol[t];
                    v = mval[t];
                    if (!cap_l) {
                        kp = true;
                    } else {
                        const unsigned long long b = mag_bits(t_abs(v));
                        kp = (b > Tl) || (b == Tl && col <= cl);
                    }
                }
                const unsigned long long m = __ballot(kp);
                if (kp) {
                    const long long p = o + lc + __popcll(m & lanes_below(lane));
                    if (p < o_end) {
                        g.scol[p] = col;
                        g.sval[p] = v;
                    } else {
                        atomicOr(g.status, STATUS_OVERFLOW);
                    }
                }
                lc += __popcll(m);
            }
        }
        if (lane == 0) {
            const bool present = (bits[g.bwl >> 5] >> (g.bwl & 31)) & 1u;
            double2 piv = present ? W[g.bwl] : mk(0.0, 0.0);
            if (g.detect > 0.0) {
                const double bound = g.detect * rn;
                double value = g.boost * rn;
                const double m = t_abs(piv);
                if (!(m >= bound)) {
                    if (value <= 0.0) value = 1.0;
                    if (piv.x == 0.0 && piv.y == 0.0) piv = mk(value, 0.0);
                    else piv = mk(piv.x / m * value, piv.y / m * value);
                    atomicAdd(g.nguard, 1);
                }
            } else if (piv.x == 0.0 && piv.y == 0.0) {
                atomicOr(g.status, STATUS_ZERO_PIVOT);
            }
            if (o + lc < o_end) {
                g.scol[o + lc] = i;
                g.sval[o + lc] = piv;
            } else {
                atomicOr(g.status, STATUS_OVERFLOW);
            }
        }
        int uc = 0;
        if (keep > 0 && maxidx > g.bwl) {
            const int w_first = (g.bwl + 1) >> 5, w_last = maxidx >> 5;
            for (int w0 = w_first; w0 <= w_last; w0 += 64) {
                const int w = w0 + lane;
                unsigned v = 0;
                if (w <= w_last) {
                    v = bits[w];
                    if (w == w_first) v &= ~0u << ((g.bwl + 1) & 31);
                }
                int cnt = 0;
                for (unsigned x = v; x; x &= x - 1) {
                    const int idx = (w << 5) + __ffs(x) - 1;
                    const double m = t_abs(W[idx]);
                    bool kp = m >= tau;
                    if (kp && cap_u) {
                        const unsigned long long b = mag_bits(m);
                        kp = (b > Tu) || (b == Tu && idx + base <= cu);
                    }
                    cnt += kp;
                }
                int p = wave_excl(cnt, lane);
                const int tot = wave_sum(cnt);
                for (unsigned x = v; x; x &= x - 1) {
                    const int idx = (w << 5) + __ffs(x) - 1;
                    const double2 val = W[idx];
                    const double m = t_abs(val);
                    bool kp = m >= tau;
                    if (kp && cap_u) {
                        const unsigned long long b = mag_bits(m);
                        kp = (b > Tu) || (b == Tu && idx + base <= cu);
                    }
                    if (kp) {
                        const long long q = o + lc + 1 + uc + p;
                        if (q < o_end) {
                            g.scol[q] = idx + base;
                            g.sval[q] = val;
                        } else {
                            atomicOr(g.status, STATUS_OVERFLOW);
                        }
                        ++p;
                    }
                }
                uc += tot;
            }
        }
        if (lane == 0) {
            if (o + lc + 1 + uc > o_end) {
                // cannot happen when the selection is exact; keep the slot readable
                lc = min(lc, (int)(o_end - o - 1));
                uc = (int)(o_end - o - 1) - lc;
            }
            g.meta[i] = make_int2(lc, uc);
        }
        // publish: slot and meta visible device-wide before the flag
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(g.done + i, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        // clear the window and the bitmap for the next row
        for (int c = 0; c < nt; c += 64) {
            const int t = c + lane;
            if (t < nt) {
                const int idx = touched[t];
                W[idx] = mk(0.0, 0.0);
                bits[idx >> 5] = 0u;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
}

namespace {

__global__ void k_lu_bandwidths(int n, const int *rowptr, const int *col, int *bw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int rs = rowptr[i], re = rowptr[i + 1];
    if (re > rs) {
        atomicMax(bw, i - col[rs]);
        atomicMax(bw + 1, col[re - 1] - i);
    }
}

__global__ void k_slot_caps(int n, const int *rowptr, double fill, int bwl, int bwu, long long *cap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int keep = keep_of(fill, rowptr[i + 1] - rowptr[i]);
    cap[i] = (long long)min(keep, bwl) + 1 + (long long)min(keep, bwu);
}

// serial-in-chunks exclusive scan of n int64 values by one workgroup
__global__ void __launch_bounds__(1024) k_scan64(int n, const long long *in, long long *out) {
    __shared__ long long part[1024];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c = 0; c < n; c += 1024) {
        const int i = c + (int)threadIdx.x;
        const long long v = (i < n) ? in[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const long long y = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < n) out[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_row_lengths(int n, const int2 *meta, long long *len) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) len[i] = (long long)meta[i].x + 1 + meta[i].y;
}

// wavefront per row: slot -> CSR row, row pointers narrowed to int, diagonal
// positions
__global__ void k_compact(int n, const long long *soff, const int *scol, const double2 *sval, const int2 *meta,
                          const long long *rp64, int *rowptr, int *col, double2 *val, int *diag) {
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const long long o = soff[i];
    const long long r = rp64[i];
    const int len = (int)(rp64[i + 1] - r);
    for (int e = lane; e < len; e += 64) {
        col[r + e] = scol[o + e];
        val[r + e] = sval[o + e];
    }
    if (lane == 0) {
        rowptr[i] = (int)r;
        diag[i] = (int)r + meta[i].x;
        if (i == n - 1) rowptr[n] = (int)rp64[n];
    }
}

}  // namespace

IluResult ilut_factor(const CsrBuf<double2> &A, const int *diag, double drop_tol, double fill, double detect,
                      double boost, CsrBuf<double2> &LU, DevBuf<int> &lu_diag, hipStream_t s) {
    (void)diag;
    SS_REQUIRE(drop_tol >= 0.0 && fill >= 0.0, SS_E_INVALID_ARG, "ILUT needs drop_tol >= 0 and fill >= 0");
    const int n = A.n;
    IluResult res;
    if (n == 0) {
        LU.alloc(0, 0);
        SS_HIP(hipMemsetAsync(LU.rowptr.get(), 0, sizeof(int), s));
        lu_diag.resize(1);
        return res;
    }
    DevBuf<int> bw(2);
    SS_HIP(hipMemsetAsync(bw.get(), 0, 2 * sizeof(int), s));
    k_lu_bandwidths<<<div_up(n, 256), 256, 0, s>>>(n, A.rowptr.get(), A.col.get(), bw.get());
    SS_HIP(hipGetLastError());
    int hb[2];
    d2h(hb, bw.get(), 2, s);
    const int bwl = hb[0], bwu = hb[1];
    const int ws = bwl + bwu + 1;
    const int nwords = (ws + 31) / 32;
    const size_t lds_wave = sizeof(unsigned) * ((size_t)nwords + ILUT_HIST);
    SS_REQUIRE(lds_wave <= 65536, SS_E_INVALID_ARG,
               "ILUT: bandwidth of the ordered matrix too large for the working-row window");
    const int wpb = (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / lds_wave));

    // slots
    DevBuf<long long> cap((size_t)n), soff((size_t)n + 1);
    k_slot_caps<<<div_up(n, 256), 256, 0, s>>>(n, A.rowptr.get(), fill, bwl, bwu, cap.get());
    k_scan64<<<1, 1024, 0, s>>>(n, cap.get(), soff.get());
    SS_HIP(hipGetLastError());
    long long slots = 0;
    d2h(&slots, soff.get() + n, 1, s);
    DevBuf<int> scol((size_t)slots);
    DevBuf<double2> sval((size_t)slots);
    DevBuf<int2> meta((size_t)n);
    DevBuf<unsigned> done((size_t)n);
    SS_HIP(hipMemsetAsync(done.get(), 0, sizeof(unsigned) * n, s));

    // persistent wavefronts, each with its window (bounded to ~4 GB of scratch)
    const size_t per_wave = (size_t)ws * (sizeof(double2) + sizeof(int)) + (size_t)(bwl + 1) * (sizeof(int) + sizeof(double2));
    const size_t budget = (size_t)4 << 30;
    int nw = (int)std::min<size_t>((size_t)2048, std::max<size_t>(64, budget / per_wave));
    nw = std::min(nw, n);
    nw = div_up(nw, wpb) * wpb;
    DevBuf<double2> win((size_t)nw * ws), mval((size_t)nw * (bwl + 1));
    DevBuf<int> touched((size_t)nw * ws), mcol((size_t)nw * (bwl + 1));
    SS_HIP(hipMemsetAsync(win.get(), 0, sizeof(double2) * (size_t)nw * ws, s));
    DevBuf<unsigned> ctr(2);
    DevBuf<int> nguard(1);
    SS_HIP(hipMemsetAsync(ctr.get(), 0, 2 * sizeof(unsigned), s));
    SS_HIP(hipMemsetAsync(nguard.get(), 0, sizeof(int), s));

    IlutArgs g;
    g.n = n;
    g.rowptr = A.rowptr.get();
    g.col = A.col.get();
    g.a = A.val.get();
    g.bwl = bwl;
    g.bwu = bwu;
    g.ws = ws;
    g.nwords = nwords;
    g.drop = drop_tol;
    g.fill = fill;
    g.detect = detect;
    g.boost = boost;
    g.soff = soff.get();
    g.scol = scol.get();
    g.sval = sval.get();
    g.meta = meta.get();
    g.done = done.get();
    g.win = win.get();
    g.touched = touched.get();
    g.mcol = mcol.get();
    g.mval = mval.get();
    g.next_row = ctr.get();
    g.status = ctr.get() + 1;
    g.nguard = nguard.get();
    k_ilut<<<nw / wpb, wpb * 64, wpb * lds_wave, s>>>(g, wpb);
    SS_HIP(hipGetLastError());
    unsigned st = 0;
    d2h(&st, ctr.get() + 1, 1, s);
    SS_REQUIRE(!(st & STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "ILUT: a row dependency wait timed out");
    SS_REQUIRE(!(st & STATUS_ZERO_PIVOT), SS_E_ZERO_PIVOT, "ILUT: zero pivot");
    SS_REQUIRE(!(st & STATUS_OVERFLOW), SS_E_HIP, "ILUT: a row exceeded its slot (internal error)");

    // compact the slots into CSR
    DevBuf<long long> len((size_t)n), rp64((size_t)n + 1);
    k_row_lengths<<<div_up(n, 256), 256, 0, s>>>(n, meta.get(), len.get());
    k_scan64<<<1, 1024, 0, s>>>(n, len.get(), rp64.get());
    SS_HIP(hipGetLastError());
    long long total = 0;
    d2h(&total, rp64.get() + n, 1, s);
    SS_REQUIRE(total >= 0 && total <= INT_MAX, SS_E_OOM, "ILUT factors exceed 2^31 entries");
    LU.alloc(n, (int)total);
    lu_diag.resize((size_t)n);
    k_compact<<<div_up(n, 4), 256, 0, s>>>(n, soff.get(), scol.get(), sval.get(), meta.get(), rp64.get(),
                                           LU.rowptr.get(), LU.col.get(), LU.val.get(), lu_diag.get());
    SS_HIP(hipGetLastError());
    d2h(&res.guarded, nguard.get(), 1, s);
    return res;
}

}  // namespace ss
