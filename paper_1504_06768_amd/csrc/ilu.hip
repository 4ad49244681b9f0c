// Incomplete LU factorisation with zero fill, ILU(0) (section "Iterative
// Solvers": iLU preconditioner of the permuted modified Liouvillian), and the
// sync-free sparse triangular solves that apply it.
//
// Factorisation: row-wise (IKJ) elimination, one wavefront per row, rows in
// increasing order.  For every k < i with a_ik != 0 (increasing k): wait for
// row k's published U part, l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for the
// j > k present in both row i and row k.  This is the serial ILU(0) order,
// and every product and difference is rounded on its own (the file is built
// without floating-point contraction), so all the ILU(0) kernels here give
// the same factors.  Done in fp64 for both precisions; the mixed path rounds the
// finished factors to complex64.
//
// Pivot boost: a pivot with |u_ii| < detect * ||a_i||_inf is replaced by
// boost * ||a_i||_inf times the pivot's phase (or by that value when the pivot
// is 0) and counted.  Tiny pivots come from states no channel leaves (a
// structurally zero diagonal of L) and from the shift sigma of L - sigma I;
// without pivoting, a pivot boosted to a fraction of the row norm keeps the
// preconditioner bounded, and the Krylov iteration on the exact matrix
// absorbs the rank-one difference.
#include <climits>

#include "csr_tools.hpp"
#include "ilu.hpp"
#include "ilu_fp.hpp"
#include "syncfree.hpp"

namespace ss {

constexpr int ILU_WPB = 4;  // wavefronts (rows) per workgroup

// One row of the ILU(0) elimination, by one wavefront (see the file header).
__device__ __forceinline__ void ilu0_row(int row, const int *rowptr, const int *col, const int *diag,
                                         const double2 *a, double2 *w, double2 *out, double detect, double boost,
                                         unsigned *status, int *nguard) {
    const int lane = threadIdx.x & 63;
    const int rs = rowptr[row], re = rowptr[row + 1], dg = diag[row];
    double rn = 0.0;
    for (int e = rs + lane; e < re; e += 64) {
        const double2 v = a[e];
        w[e] = v;
        rn = fmax(rn, sqrt(v.x * v.x + v.y * v.y));
    }
    for (int off = 32; off > 0; off >>= 1) rn = fmax(rn, __shfl_xor(rn, off, 64));

    for (int ek = rs; ek < dg; ++ek) {
        const int k = col[ek];
        const int dk = diag[k];
        const int ke = rowptr[k + 1];
        double2 ukk = mk(0.0, 0.0);
        if (lane == 0) ukk = wait_load(out + dk, status);
        ukk.x = __shfl(ukk.x, 0, 64);
        ukk.y = __shfl(ukk.y, 0, 64);
        const int owner = (ek - rs) & 63;
        double2 l = mk(0.0, 0.0);
        if (lane == owner) {
            l = cdiv(w[ek], ukk);
            w[ek] = l;
        }
        l.x = __shfl(l.x, owner, 64);
        l.y = __shfl(l.y, owner, 64);
        for (int e = rs + lane; e < re; e += 64) {
            if (e <= ek) continue;
            const int j = col[e];
            int lo = dk + 1, hi = ke - 1, f = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = col[mid];
                if (c == j) { f = mid; break; }
                if (c < j) lo = mid + 1; else hi = mid - 1;
            }
            if (f >= 0) {
                const double2 u = wait_load(out + f, status);
                w[e] = csub(w[e], cmul(l, u));
            }
        }
    }
    if (lane == ((dg - rs) & 63)) {
        const double2 p = w[dg];
        const double mag = sqrt(p.x * p.x + p.y * p.y);
        const double bound = detect * rn;
        if (!(mag >= bound)) {
            const double b = (rn > 0.0) ? boost * rn : 1.0;
            w[dg] = (mag > 0.0) ? cscale(p, b / mag) : mk(b, 0.0);
            atomicAdd(nguard, 1);
        }
    }
    for (int e = rs + lane; e < re; e += 64) publish(out + e, w[e]);
}

__global__ void __launch_bounds__(ILU_WPB * 64) k_ilu0(int n, const int *rowptr, const int *col, const int *diag,
                                                       const double2 *a, double2 *w, double2 *out, unsigned *ctr,
                                                       unsigned base, double detect, double boost,
                                                       unsigned *status, int *nguard) {
    const unsigned bid = ordered_block(ctr, base);
    const int row = (int)bid * ILU_WPB + (int)(threadIdx.x >> 6);
    if (row >= n) return;
    ilu0_row(row, rowptr, col, diag, a, w, out, detect, boost, status, nguard);
}

// Many systems at once, one workgroup each: its wavefronts take the rows in
// increasing order (wavefront k: rows k, k + 16, ...), so the lowest
// unfinished row always belongs to a wavefront that is working on it and
// whose dependencies are done.
constexpr int ILU_BATCH_WAVES = 16;

__global__ void __launch_bounds__(ILU_BATCH_WAVES * 64) k_ilu0_batch(const Ilu0Job *jobs, double detect,
                                                                     double boost) {
    const Ilu0Job &J = jobs[blockIdx.x];
    for (int row = (int)(threadIdx.x >> 6); row < J.n; row += ILU_BATCH_WAVES)
        ilu0_row(row, J.rowptr, J.col, J.diag, J.a, J.w, J.out, detect, boost, J.status, J.nguard);
}

template <typename T>
__global__ void k_fill_sentinel(int64_t n, T *p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) set_sentinel(p + i);
}

template <typename T>
void fill_sentinel(int64_t n, T *p, hipStream_t s) {
    if (n > 0) {
        k_fill_sentinel<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, p);
        SS_HIP(hipGetLastError());
    }
}
template void fill_sentinel<double2>(int64_t, double2 *, hipStream_t);
template void fill_sentinel<float2>(int64_t, float2 *, hipStream_t);

__global__ void k_round_c64(int64_t n, const double2 *a, float2 *b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = to_c64(a[i]);
}

void round_to_c64(int64_t n, const double2 *a, float2 *b, hipStream_t s) {
    if (n > 0) {
        k_round_c64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, b);
        SS_HIP(hipGetLastError());
    }
}

Ilu0Job Ilu0Batch::prepare(const CsrBuf<double2> &A, const int *diag, CsrBuf<double2> &LU, hipStream_t s) {
    const int n = A.n, nnz = A.nnz;
    LU.alloc(n, nnz);
    SS_HIP(hipMemcpyAsync(LU.rowptr.get(), A.rowptr.get(), sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) SS_HIP(hipMemcpyAsync(LU.col.get(), A.col.get(), sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
    work.resize((size_t)std::max(nnz, 1));
    fill_sentinel<double2>(nnz, LU.val.get(), s);
    flags.resize(2);
    SS_HIP(hipMemsetAsync(flags.get(), 0, 2 * sizeof(unsigned), s));
    Ilu0Job j;
    j.n = n;
    j.rowptr = A.rowptr.get();
    j.col = A.col.get();
    j.diag = diag;
    j.a = A.val.get();
    j.w = work.get();
    j.out = LU.val.get();
    j.status = flags.get();
    j.nguard = reinterpret_cast<int *>(flags.get() + 1);
    return j;
}

IluResult Ilu0Batch::result(hipStream_t s) {
    unsigned f[2] = {0, 0};
    d2h(f, flags.get(), 2, s);
    SS_REQUIRE(!(f[0] & STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "ILU(0): dependency wait timed out");
    IluResult r;
    r.guarded = (int)f[1];
    return r;
}

void ilu0_batch(const Ilu0Job *jobs, int count, double detect, double boost, hipStream_t s) {
    if (count <= 0) return;
    DevBuf<Ilu0Job> dj((size_t)count);
    h2d(dj.get(), jobs, (size_t)count, s);
    k_ilu0_batch<<<count, ILU_BATCH_WAVES * 64, 0, s>>>(dj.get(), detect, boost);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s));  // the job array is released on return
}

// Many systems at once with their level schedules (the level sets of the
// strict lower part: row i depends exactly on the rows k < i it holds).  One
// workgroup per system walks the levels with a barrier in between; inside a
// level, groups of ILU_LG lanes take one row each.  No row waits for
// another, so the factor is read with plain loads.  Each row takes the steps
// of ilu0_row in the same order with the same arithmetic, so the factors are
// the same.
//
// Short rows (the common case) take a register path: the row's entries stay
// in registers (ILU_FM per lane), the structure of every row k it holds is
// fetched at once, and the U part of each such row (up to ILU_LG entries
// after the pivot, one per lane) is read in one pass and matched against the
// row's columns by shuffles.  That is a handful of dependent memory rounds
// per row instead of several per eliminated entry.  Other rows (the trace
// row, rows that hold it) take the general loop through the work array.
constexpr int ILU_LG = 8;
constexpr int ILU_LVL_BS = 1024;
constexpr int ILU_FM = 2;       // row entries per lane on the register path

// The general loop: one row by one group of LG lanes, the working row in J.w.
template <int LG>
__device__ __forceinline__ void ilu0_row_group(const Ilu0Job &J, int row, int rs, int re, int dg, int lane,
                                               double detect, double boost) {
    double rn = 0.0;
    for (int e = rs + lane; e < re; e += LG) {
        const double2 v = gld(J.a + e);
        gst(J.w + e, v);
        rn = fmax(rn, sqrt(v.x * v.x + v.y * v.y));
    }
    for (int off = LG / 2; off > 0; off >>= 1) rn = fmax(rn, __shfl_xor(rn, off, LG));
    for (int ek = rs; ek < dg; ++ek) {
        const int k = gld(J.col + ek);
        const int dk = gld(J.diag + k);
        const int ke = gld(J.rowptr + k + 1);
        const double2 ukk = gld(J.out + dk);
        const int owner = (ek - rs) % LG;
        double2 l = mk(0.0, 0.0);
        if (lane == owner) {
            l = cdiv(gld(J.w + ek), ukk);
            gst(J.w + ek, l);
        }
        l.x = __shfl(l.x, owner, LG);
        l.y = __shfl(l.y, owner, LG);
        for (int e = rs + lane; e < re; e += LG) {
            if (e <= ek) continue;
            const int j = gld(J.col + e);
            int lo = dk + 1, hi = ke - 1, f = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = gld(J.col + mid);
                if (c == j) { f = mid; break; }
                if (c < j) lo = mid + 1; else hi = mid - 1;
            }
            if (f >= 0) gst(J.w + e, csub(gld(J.w + e), cmul(l, gld(J.out + f))));
        }
    }
    if (lane == (dg - rs) % LG) {
        const double2 p = gld(J.w + dg);
        const double mag = sqrt(p.x * p.x + p.y * p.y);
        const double bound = detect * rn;
        if (!(mag >= bound)) {
            const double b = (rn > 0.0) ? boost * rn : 1.0;
            gst(J.w + dg, (mag > 0.0) ? cscale(p, b / mag) : mk(b, 0.0));
            atomicAdd(J.nguard, 1);
        }
    }
    for (int e = rs + lane; e < re; e += LG) gst(J.out + e, gld(J.w + e));
}

// One row of a level, by the LG lanes of its group (slot = {row, row start,
// pivot position, row end}; every row it depends on is final).  The
// register path takes rows of up to LG * FM entries with at most LG entries
// before the pivot, each of whose rows k has at most LG entries after its
// pivot.
template <int LG, int FM>
__device__ __forceinline__ void ilu0_slot(const Ilu0Job &J, int4 slot, int lane, double detect, double boost) {
    constexpr int FK = LG;
    const int row = slot.x, rs = slot.y, dg = slot.z, re = slot.w;
    const int nl = dg - rs;  // entries before the pivot: the rows k this row eliminates with
    bool fast = (re - rs <= LG * FM) && nl <= FK;
    // the row in registers: entry rs + lane + LG m in slot m
    int cj[FM];
    double2 wv[FM];
    double rn = 0.0;
    int dk0 = 0, ke0 = 0;  // structure of row k = col[rs + lane] (lane < nl)
    if (fast) {
#pragma unroll
        for (int m = 0; m < FM; ++m) {
            const int e = rs + lane + LG * m;
            cj[m] = -1;
            wv[m] = mk(0.0, 0.0);
            if (e < re) {
                cj[m] = gld(J.col + e);
                wv[m] = gld(J.a + e);
            }
        }
        if (lane < nl) {
            dk0 = gld(J.diag + cj[0]);
            ke0 = gld(J.rowptr + cj[0] + 1);
        }
#pragma unroll
        for (int m = 0; m < FM; ++m)
            if (rs + lane + LG * m < re) rn = fmax(rn, sqrt(wv[m].x * wv[m].x + wv[m].y * wv[m].y));
        // every U part must fit one entry per lane
        int wide = (lane < nl && ke0 - dk0 - 1 > LG) ? 1 : 0;
        for (int off = LG / 2; off > 0; off >>= 1) wide |= __shfl_xor(wide, off, LG);
        fast = !wide;
    }
    if (!fast) {
        ilu0_row_group<LG>(J, row, rs, re, dg, lane, detect, boost);
        return;
    }
    for (int off = LG / 2; off > 0; off >>= 1) rn = fmax(rn, __shfl_xor(rn, off, LG));
    // U parts: for lower entry p, lane t holds entry dk + 1 + t of row k
    int uc[FK];
    double2 uv[FK], ukk[FK];
#pragma unroll
    for (int p = 0; p < FK; ++p) {
        const int dk = __shfl(dk0, p, LG), ke = __shfl(ke0, p, LG);
        uc[p] = -1;
        uv[p] = mk(0.0, 0.0);
        ukk[p] = mk(1.0, 0.0);
        if (p < nl) {
            ukk[p] = gld(J.out + dk);
            const int f = dk + 1 + lane;
            if (f < ke) {
                uc[p] = gld(J.col + f);
                uv[p] = gld(J.out + f);
            }
        }
    }
    // eliminate with rows k in increasing order (the lower entries
    // are sorted): l = a_ik / u_kk, then a_ij -= l u_kj on the
    // columns j > k the two rows share
#pragma unroll
    for (int p = 0; p < FK; ++p) {
        if (p < nl) {
            double2 l = mk(0.0, 0.0);
            if (lane == p) {
                l = cdiv(wv[0], ukk[p]);
                wv[0] = l;
            }
            l.x = __shfl(l.x, p, LG);
            l.y = __shfl(l.y, p, LG);
            int sm[FM];
#pragma unroll
            for (int m = 0; m < FM; ++m) sm[m] = -1;
            for (int t = 0; t < LG; ++t) {
                const int c = __shfl(uc[p], t, LG);
#pragma unroll
                for (int m = 0; m < FM; ++m)
                    if (c >= 0 && c == cj[m]) sm[m] = t;
            }
#pragma unroll
            for (int m = 0; m < FM; ++m) {
                double2 u;
                u.x = __shfl(uv[p].x, sm[m] < 0 ? 0 : sm[m], LG);
                u.y = __shfl(uv[p].y, sm[m] < 0 ? 0 : sm[m], LG);
                if (sm[m] >= 0) wv[m] = csub(wv[m], cmul(l, u));
            }
        }
    }
    // pivot guard on the lane holding the diagonal entry
#pragma unroll
    for (int m = 0; m < FM; ++m) {
        if (nl == lane + LG * m) {
            const double2 p = wv[m];
            const double mag = sqrt(p.x * p.x + p.y * p.y);
            const double bound = detect * rn;
            if (!(mag >= bound)) {
                const double b = (rn > 0.0) ? boost * rn : 1.0;
                wv[m] = (mag > 0.0) ? cscale(p, b / mag) : mk(b, 0.0);
                atomicAdd(J.nguard, 1);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < FM; ++m) {
        const int e = rs + lane + LG * m;
        if (e < re) gst(J.out + e, wv[m]);
    }
}

__global__ void __launch_bounds__(ILU_LVL_BS) k_ilu0_levels(const Ilu0Job *jobs, double detect, double boost) {
    const Ilu0Job &J = jobs[blockIdx.x];
    const int g = threadIdx.x / ILU_LG, lane = threadIdx.x % ILU_LG;
    constexpr int NG = ILU_LVL_BS / ILU_LG;
    // the next level's end is fetched a level ahead
    int s0 = J.nlev > 0 ? gld(J.lptr) : 0, s1 = J.nlev > 0 ? gld(J.lptr + 1) : 0;
    for (int lv = 0; lv < J.nlev; ++lv) {
        const int s2 = (lv + 2 <= J.nlev) ? gld(J.lptr + lv + 2) : 0;
        for (int sl = s0 + g; sl < s1; sl += NG) ilu0_slot<ILU_LG, ILU_FM>(J, gld(J.lslot + sl), lane, detect, boost);
        __syncthreads();
        s0 = s1;
        s1 = s2;
    }
}

// One system, one launch per level of its lower schedule: a group of LG
// lanes per row, every dependency finished by an earlier launch.  A row of
// up to LG entries (at most LG of them before the pivot, and every row k it
// eliminates with holding at most LG entries after its pivot) stays in
// registers, one entry per lane; the U parts of the rows k are fetched eight
// at a time (one entry per lane each), each entry finds its column among the
// row's (kept sorted in LDS) by binary search, and a matched u_kj goes to the
// lane holding column j through LDS.  Other rows take the general loop.  The
// steps and their arithmetic are those of ilu0_row, so the factors are the
// same.
constexpr int ILU_LEVEL_BS = 256;
constexpr int ILU_WIDE_LG = 32;
constexpr int ILU_LONG_BS = 256;     // threads of k_ilu0_long
constexpr int ILU_LONG_MAX = 2048;   // entries of a row k_ilu0_long holds in LDS
constexpr int ILU_WIDE_PF = 8;  // U parts fetched per memory round

// orders the LDS accesses of one wavefront (the lane group lies in one)
__device__ __forceinline__ void ilu_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// scol, su, stag: the group's LG entries of LDS
template <int LG>
__device__ __forceinline__ void ilu0_slot_wide(const Ilu0Job &J, int4 slot, int lane, double detect,
                                               double boost, int *scol, double2 *su, int *stag) {
    const int row = slot.x, rs = slot.y, dg = slot.z, re = slot.w;
    const int nl = dg - rs;  // entries before the pivot: the rows k this row eliminates with
    const bool in = rs + lane < re;
    const int cj = in ? gld(J.col + rs + lane) : -1;
    double2 wv = in ? gld(J.a + rs + lane) : mk(0.0, 0.0);
    double rn = in ? sqrt(wv.x * wv.x + wv.y * wv.y) : 0.0;
    int dk0 = 0, ke0 = 0;
    double2 ukk0 = mk(1.0, 0.0);
    if (lane < nl && lane < LG) {
        dk0 = gld(J.diag + cj);
        ke0 = gld(J.rowptr + cj + 1);
    }
    int wide = (re - rs > LG || nl > LG || (lane < nl && ke0 - dk0 - 1 > LG)) ? 1 : 0;
    for (int off = LG / 2; off > 0; off >>= 1) {
        wide |= __shfl_xor(wide, off, LG);
        rn = fmax(rn, __shfl_xor(rn, off, LG));
    }
    if (wide) {
        ilu0_row_group<LG>(J, row, rs, re, dg, lane, detect, boost);
        return;
    }
    if (lane < nl) ukk0 = gld(J.out + dk0);
    // the row's columns, sorted, padded past its end
    scol[lane] = in ? cj : INT_MAX;
    stag[lane] = -1;
    ilu_wave_sync();
    for (int p0 = 0; p0 < nl; p0 += ILU_WIDE_PF) {
        int uc[ILU_WIDE_PF];
        double2 uv[ILU_WIDE_PF];
#pragma unroll
        for (int q = 0; q < ILU_WIDE_PF; ++q) {
            const int p = p0 + q;
            const int dk = __shfl(dk0, p < nl ? p : 0, LG), ke = __shfl(ke0, p < nl ? p : 0, LG);
            uc[q] = -1;
            uv[q] = mk(0.0, 0.0);
            const int f = dk + 1 + lane;
            if (p < nl && f < ke) {
                uc[q] = gld(J.col + f);
                uv[q] = gld(J.out + f);
            }
        }
        // where each fetched u_kj's column sits in the row (-1: not there)
        int hit[ILU_WIDE_PF];
#pragma unroll
        for (int q = 0; q < ILU_WIDE_PF; ++q) {
            hit[q] = -1;
            if (uc[q] >= 0) {
                int pos = 0;
                for (int st = LG / 2; st > 0; st >>= 1)
                    if (scol[pos + st - 1] < uc[q]) pos += st;
                if (scol[pos] < uc[q]) ++pos;
                if (pos < LG && scol[pos] == uc[q]) hit[q] = pos;
            }
        }
#pragma unroll
        for (int q = 0; q < ILU_WIDE_PF; ++q) {
            const int p = p0 + q;
            if (p < nl) {
                // l = a_ik / u_kk on the lane holding lower entry p
                double2 ukk;
                ukk.x = __shfl(ukk0.x, p, LG);
                ukk.y = __shfl(ukk0.y, p, LG);
                double2 l = mk(0.0, 0.0);
                if (lane == p) {
                    l = cdiv(wv, ukk);
                    wv = l;
                }
                l.x = __shfl(l.x, p, LG);
                l.y = __shfl(l.y, p, LG);
                // a_ij -= l u_kj where row k's U part holds column j
                if (hit[q] >= 0) {
                    su[hit[q]] = uv[q];
                    stag[hit[q]] = p;
                }
                ilu_wave_sync();
                if (stag[lane] == p) wv = csub(wv, cmul(l, su[lane]));
                ilu_wave_sync();
            }
        }
    }
    // pivot guard on the lane holding the diagonal entry
    if (lane == nl) {
        const double mag = sqrt(wv.x * wv.x + wv.y * wv.y);
        const double bound = detect * rn;
        if (!(mag >= bound)) {
            const double b = (rn > 0.0) ? boost * rn : 1.0;
            wv = (mag > 0.0) ? cscale(wv, b / mag) : mk(b, 0.0);
            atomicAdd(J.nguard, 1);
        }
    }
    if (in) gst(J.out + rs + lane, wv);
}

// Rows longer than LG entries and at most ILU_LONG_MAX (a trace row) are
// listed in longq for k_ilu0_long when longq is given.
template <int LG>
__global__ void __launch_bounds__(ILU_LEVEL_BS) k_ilu0_level(Ilu0Job J, int lo, int hi, double detect, double boost,
                                                             int *longq, int *nlong) {
    __shared__ int scol[ILU_LEVEL_BS], stag[ILU_LEVEL_BS];
    __shared__ double2 su[ILU_LEVEL_BS];
    const int t = blockIdx.x * ILU_LEVEL_BS + threadIdx.x;
    const int sl = lo + t / LG, lane = t % LG;
    if (sl >= hi) return;  // (whole groups)
    const int gb = (int)threadIdx.x - lane;
    const int4 slot = gld(J.lslot + sl);
    const int len = slot.w - slot.y;
    if (longq && len > LG && len <= ILU_LONG_MAX) {
        if (lane == 0) longq[atomicAdd(nlong, 1)] = sl;
        return;
    }
    ilu0_slot_wide<LG>(J, slot, lane, detect, boost, scol + gb, su + gb, stag + gb);
}

// The listed long rows of one level, one workgroup per row at a time: the
// row's columns and values in LDS; for each entry k before the pivot, in
// order, one thread forms l_ik = w_ik / u_kk and the workgroup subtracts
// l_ik u_kj from the row's entry of column j for every j of row k's U part
// (found by binary search over the row's columns in LDS).  The steps and
// their arithmetic are those of ilu0_row_group, so the factors are the same.
__global__ void __launch_bounds__(ILU_LONG_BS) k_ilu0_long(Ilu0Job J, const int *longq, const int *nlong,
                                                           double detect, double boost) {
    __shared__ int scol[ILU_LONG_MAX];
    __shared__ double2 sw[ILU_LONG_MAX];
    __shared__ double srn[ILU_LONG_BS / 64];
    __shared__ int sdk, ske;
    __shared__ double2 sl;
    const int m = *nlong;
    for (int q = blockIdx.x; q < m; q += gridDim.x) {
        const int4 slot = gld(J.lslot + longq[q]);
        const int rs = slot.y, dg = slot.z, re = slot.w;
        const int len = re - rs, nl = dg - rs;
        __syncthreads();  // (the previous row's LDS reads are done)
        double rn = 0.0;
        for (int t = threadIdx.x; t < len; t += ILU_LONG_BS) {
            scol[t] = gld(J.col + rs + t);
            const double2 v = gld(J.a + rs + t);
            sw[t] = v;
            rn = fmax(rn, sqrt(v.x * v.x + v.y * v.y));
        }
        for (int off = 32; off > 0; off >>= 1) rn = fmax(rn, __shfl_xor(rn, off, 64));
        if ((threadIdx.x & 63) == 0) srn[threadIdx.x >> 6] = rn;
        __syncthreads();
        rn = srn[0];
        for (int w = 1; w < ILU_LONG_BS / 64; ++w) rn = fmax(rn, srn[w]);
        for (int p = 0; p < nl; ++p) {
            if (threadIdx.x == 0) {
                const int k = scol[p];
                const int dk = gld(J.diag + k);
                sdk = dk;
                ske = gld(J.rowptr + k + 1);
                const double2 l = cdiv(sw[p], gld(J.out + dk));
                sw[p] = l;
                sl = l;
            }
            __syncthreads();
            const int dk = sdk, ke = ske;
            const double2 l = sl;
            for (int f = dk + 1 + threadIdx.x; f < ke; f += ILU_LONG_BS) {
                const int c = gld(J.col + f);
                int lo = p + 1, hi = len - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int cm = scol[mid];
                    if (cm == c) {
                        sw[mid] = csub(sw[mid], cmul(l, gld(J.out + f)));
                        break;
                    }
                    if (cm < c) lo = mid + 1; else hi = mid - 1;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double2 pv = sw[nl];
            const double mag = sqrt(pv.x * pv.x + pv.y * pv.y);
            const double bound = detect * rn;
            if (!(mag >= bound)) {
                const double b = (rn > 0.0) ? boost * rn : 1.0;
                sw[nl] = (mag > 0.0) ? cscale(pv, b / mag) : mk(b, 0.0);
                atomicAdd(J.nguard, 1);
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < len; t += ILU_LONG_BS) gst(J.out + rs + t, sw[t]);
    }
}

// the longest row (one atomic per wavefront)
__global__ void k_ilu_max_row(int n, const int *rowptr, int *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    int len = (r < n) ? rowptr[r + 1] - rowptr[r] : 0;
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, len);
}

void ilu0_levels_batch(const Ilu0Job *jobs, int count, double detect, double boost, hipStream_t s) {
    if (count <= 0) return;
    StreamScope scope(s);
    DevBuf<Ilu0Job> dj((size_t)count);
    h2d(dj.get(), jobs, (size_t)count, s);
    k_ilu0_levels<<<count, ILU_LVL_BS, 0, s>>>(dj.get(), detect, boost);
    SS_HIP(hipGetLastError());
}

IluResult ilu0_factor_levels(const CsrBuf<double2> &A, const int *diag, const LevelSched &lo, double detect,
                             double boost, CsrBuf<double2> &LU, hipStream_t s) {
    SS_REQUIRE((int)lo.hptr.size() == lo.nlev + 1, SS_E_STATE, "level schedule without its host copy");
    const int n = A.n, nnz = A.nnz;
    LU.alloc(n, nnz);
    SS_HIP(hipMemcpyAsync(LU.rowptr.get(), A.rowptr.get(), sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) SS_HIP(hipMemcpyAsync(LU.col.get(), A.col.get(), sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
    DevBuf<double2> work((size_t)std::max(nnz, 1));
    DevBuf<int> nguard(1);
    SS_HIP(hipMemsetAsync(nguard.get(), 0, sizeof(int), s));
    Ilu0Job j;
    j.n = n;
    j.rowptr = A.rowptr.get();
    j.col = A.col.get();
    j.diag = diag;
    j.a = A.val.get();
    j.w = work.get();
    j.out = LU.val.get();
    j.status = nullptr;
    j.nguard = nguard.get();
    j.nlev = lo.nlev;
    j.lptr = lo.ptr.get();
    j.lslot = lo.slot.get();
    // rows longer than a lane group (a trace row) go to k_ilu0_long, level by
    // level after the level's other rows
    int maxlen = 0;
    DevBuf<int> mx(1), longq, nlong(1);
    if (n) {
        SS_HIP(hipMemsetAsync(mx.get(), 0, sizeof(int), s));
        k_ilu_max_row<<<div_up(n, 256), 256, 0, s>>>(n, A.rowptr.get(), mx.get());
        SS_HIP(hipGetLastError());
        d2h(&maxlen, mx.get(), 1, s);
    }
    const bool longrows = maxlen > ILU_WIDE_LG;
    if (longrows) longq.resize((size_t)std::max(n, 1));
    for (int l = 0; l < lo.nlev; ++l) {
        const int a = lo.hptr[(size_t)l], b = lo.hptr[(size_t)l + 1];
        if (b <= a) continue;
        if (longrows) SS_HIP(hipMemsetAsync(nlong.get(), 0, sizeof(int), s));
        k_ilu0_level<ILU_WIDE_LG><<<div_up((int64_t)(b - a) * ILU_WIDE_LG, ILU_LEVEL_BS), ILU_LEVEL_BS, 0, s>>>(
            j, a, b, detect, boost, longrows ? longq.get() : nullptr, nlong.get());
        if (longrows) k_ilu0_long<<<8, ILU_LONG_BS, 0, s>>>(j, longq.get(), nlong.get(), detect, boost);
    }
    SS_HIP(hipGetLastError());
    IluResult r;
    d2h(&r.guarded, nguard.get(), 1, s);  // (synchronises before the work array is released)
    return r;
}

// ------------------------------------------------ fixed-point ILU(0)
// The zero-fill factors as the fixed point of (LU)_ij = a_ij on the pattern
// (Chow and Patel 2015), by synchronous sweeps: every entry is recomputed
// from the previous sweep's values,
//   u_ij = a_ij - sum_{k < i} l_ik u_kj,  l_ij = (a_ij - sum_{k < j} l_ik u_kj) / u_jj,
// the products subtracted in increasing k as the elimination does, and the
// pivot guard applied to each new u_ii.  Start: u_ii = a_ii through the
// same guard, then l_ij = a_ij / u_jj and u_ij = a_ij (a tiny a_jj, as in
// the shifted zero diagonal of inverse power, would otherwise put huge
// multipliers into the first sweeps).  A sweep has no order between rows:
// one launch, FP_G lanes
// per row.  A row of at most FP_G entries keeps them one per lane; the U
// part of each row k it eliminates with comes FP_G entries at a time, each
// entry finds its column among the row's (in LDS) by binary search, and a
// match reaches the lane holding that column through LDS.  Longer rows
// (a trace row) take one lane per entry, each merging on its own.
constexpr int FP_G = 32;

// the largest |a_ij| of the row over the lane group (every lane)
__device__ __forceinline__ double fp_row_norm(const double2 *a, int rs, int re, int lane) {
    double rn = 0.0;
    for (int e = rs + lane; e < re; e += FP_G) {
        const double2 v = a[e];
        rn = fmax(rn, sqrt(v.x * v.x + v.y * v.y));
    }
    for (int off = FP_G / 2; off > 0; off >>= 1) rn = fmax(rn, __shfl_xor(rn, off, FP_G));
    return rn;
}

// the pivot guard of the elimination: below detect * rn, the pivot becomes
// boost * rn with its phase kept (boost itself if rn is zero)
__device__ __forceinline__ double2 fp_guard(double2 v, double rn, double detect, double boost, bool *hit) {
    const double mag = sqrt(v.x * v.x + v.y * v.y);
    *hit = !(mag >= detect * rn);
    if (!*hit) return v;
    const double b = (rn > 0.0) ? boost * rn : 1.0;
    return (mag > 0.0) ? cscale(v, b / mag) : mk(b, 0.0);
}

// start, first the pivots: x = a, with u_ii = a_ii through the guard
__global__ void __launch_bounds__(ILU_LEVEL_BS) k_ilu_fp_pivots(int n, const int *rowptr, const int *diag,
                                                                const double2 *a, double2 *x, double detect,
                                                                double boost) {
    const int t = blockIdx.x * ILU_LEVEL_BS + threadIdx.x;
    const int row = t / FP_G, lane = t % FP_G;
    if (row >= n) return;
    const int rs = rowptr[row], re = rowptr[row + 1];
    const double rn = fp_row_norm(a, rs, re, lane);
    for (int e = rs + lane; e < re; e += FP_G) x[e] = a[e];
    if (lane == 0) {
        bool hit;
        x[diag[row]] = fp_guard(a[diag[row]], rn, detect, boost, &hit);
    }
}

// then the multipliers: l_ij = a_ij / u_jj
__global__ void __launch_bounds__(ILU_LEVEL_BS) k_ilu_fp_start(int n, const int *rowptr, const int *col,
                                                               const int *diag, const double2 *a, double2 *x) {
    const int t = blockIdx.x * ILU_LEVEL_BS + threadIdx.x;
    const int row = t / FP_G, lane = t % FP_G;
    if (row >= n) return;
    for (int e = rowptr[row] + lane; e < diag[row]; e += FP_G) x[e] = cdiv(a[e], x[diag[col[e]]]);
}

// the new value of entry e = (row, j) from v = a_ij minus its products
__device__ __forceinline__ double2 fp_finish(double2 v, int row, int j, const int *diag, const double2 *old,
                                             double rn, double detect, double boost, int *nguard) {
    if (j < row) return cdiv(v, old[diag[j]]);
    if (j == row) {
        bool hit;
        v = fp_guard(v, rn, detect, boost, &hit);
        if (hit) atomicAdd(nguard, 1);
    }
    return v;
}

__global__ void __launch_bounds__(ILU_LEVEL_BS) k_ilu_fp_sweep(int n, const int *rowptr, const int *col,
                                                               const int *diag, const double2 *a,
                                                               const double2 *old, double2 *out, double detect,
                                                               double boost, int *nguard) {
    __shared__ int scol[ILU_LEVEL_BS], stag[ILU_LEVEL_BS];
    __shared__ double2 su[ILU_LEVEL_BS];
    const int t = blockIdx.x * ILU_LEVEL_BS + threadIdx.x;
    const int row = t / FP_G, lane = t % FP_G;
    if (row >= n) return;  // (whole groups)
    const int gb = (int)threadIdx.x - lane;
    const int rs = rowptr[row], re = rowptr[row + 1], dg = diag[row];
    const int len = re - rs, nl = dg - rs;
    const double rn = fp_row_norm(a, rs, re, lane);
    if (len > FP_G) {
        // one lane per entry, merging with each row k on its own
        for (int e = rs + lane; e < re; e += FP_G) {
            const int j = col[e];
            double2 v = a[e];
            for (int e2 = rs; e2 < dg; ++e2) {
                const int k = col[e2];
                if (k >= j) break;
                int lo = diag[k] + 1, hi = rowptr[k + 1] - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int c = col[mid];
                    if (c == j) {
                        v = csub(v, cmul(old[e2], old[mid]));
                        break;
                    }
                    if (c < j) lo = mid + 1; else hi = mid - 1;
                }
            }
            out[e] = fp_finish(v, row, j, diag, old, rn, detect, boost, nguard);
        }
        return;
    }
    const bool in = lane < len;
    const int cj = in ? col[rs + lane] : INT_MAX;
    double2 v = in ? a[rs + lane] : mk(0.0, 0.0);
    const double2 lo_v = in ? old[rs + lane] : mk(0.0, 0.0);
    scol[gb + lane] = cj;
    stag[gb + lane] = -1;
    ilu_wave_sync();
    int tag = 0;
    for (int p = 0; p < nl; ++p) {
        const int k = __shfl(cj, p, FP_G);
        double2 l;
        l.x = __shfl(lo_v.x, p, FP_G);
        l.y = __shfl(lo_v.y, p, FP_G);
        const int ks = diag[k] + 1, ke = rowptr[k + 1];
        for (int c0 = ks; c0 < ke; c0 += FP_G, ++tag) {
            const int f = c0 + lane;
            if (f < ke) {
                const int uc = col[f];
                int pos = 0;
                for (int st = FP_G / 2; st > 0; st >>= 1)
                    if (scol[gb + pos + st - 1] < uc) pos += st;
                if (scol[gb + pos] < uc) ++pos;
                if (pos < FP_G && scol[gb + pos] == uc) {
                    su[gb + pos] = old[f];
                    stag[gb + pos] = tag;
                }
            }
            ilu_wave_sync();
            if (stag[gb + lane] == tag) v = csub(v, cmul(l, su[gb + lane]));
            ilu_wave_sync();
        }
    }
    if (in) out[rs + lane] = fp_finish(v, row, cj, diag, old, rn, detect, boost, nguard);
}

IluResult ilu0_fixed_point(const CsrBuf<double2> &A, const int *diag, int sweeps, double detect, double boost,
                           CsrBuf<double2> &LU, hipStream_t s) {
    SS_REQUIRE(sweeps >= 1, SS_E_INVALID_ARG, "fixed-point ILU: at least one sweep");
    const int n = A.n, nnz = A.nnz;
    LU.alloc(n, nnz);
    SS_HIP(hipMemcpyAsync(LU.rowptr.get(), A.rowptr.get(), sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) SS_HIP(hipMemcpyAsync(LU.col.get(), A.col.get(), sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
    DevBuf<double2> other((size_t)std::max(nnz, 1));
    DevBuf<int> nguard(1);
    IluResult r;
    if (n == 0) return r;
    // the sweeps alternate between the two buffers and end in LU.val
    double2 *buf[2] = {LU.val.get(), other.get()};
    int cur = (sweeps % 2 == 0) ? 0 : 1;
    const int grid = div_up((int64_t)n * FP_G, ILU_LEVEL_BS);
    k_ilu_fp_pivots<<<grid, ILU_LEVEL_BS, 0, s>>>(n, A.rowptr.get(), diag, A.val.get(), buf[cur], detect, boost);
    k_ilu_fp_start<<<grid, ILU_LEVEL_BS, 0, s>>>(n, A.rowptr.get(), A.col.get(), diag, A.val.get(), buf[cur]);
    SS_HIP(hipGetLastError());
    for (int k = 0; k < sweeps; ++k) {
        SS_HIP(hipMemsetAsync(nguard.get(), 0, sizeof(int), s));  // (the last sweep's count)
        k_ilu_fp_sweep<<<grid, ILU_LEVEL_BS, 0, s>>>(n, A.rowptr.get(), A.col.get(), diag, A.val.get(), buf[cur],
                                                     buf[1 - cur], detect, boost, nguard.get());
        SS_HIP(hipGetLastError());
        cur = 1 - cur;
    }
    d2h(&r.guarded, nguard.get(), 1, s);  // (synchronises before the other buffer is released)
    return r;
}

IluResult ilu0_factor(const CsrBuf<double2> &A, const int *diag, double detect, double boost, CsrBuf<double2> &LU,
                      hipStream_t s) {
    const int n = A.n, nnz = A.nnz;
    LU.alloc(n, nnz);
    SS_HIP(hipMemcpyAsync(LU.rowptr.get(), A.rowptr.get(), sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) SS_HIP(hipMemcpyAsync(LU.col.get(), A.col.get(), sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
    DevBuf<double2> work((size_t)nnz);
    fill_sentinel<double2>(nnz, LU.val.get(), s);
    DevBuf<unsigned> status(1);
    DevBuf<int> nguard(1);
    SS_HIP(hipMemsetAsync(status.get(), 0, sizeof(unsigned), s));
    SS_HIP(hipMemsetAsync(nguard.get(), 0, sizeof(int), s));
    BlockCounter bc;
    bc.init(s);
    const unsigned grid = (unsigned)div_up(n, ILU_WPB);
    if (n) {
        k_ilu0<<<grid, ILU_WPB * 64, 0, s>>>(n, A.rowptr.get(), A.col.get(), diag, A.val.get(), work.get(),
                                              LU.val.get(), bc.ctr.get(), bc.take(grid), detect, boost,
                                              status.get(), nguard.get());
        SS_HIP(hipGetLastError());
    }
    IluResult r;
    unsigned st = 0;
    d2h(&st, status.get(), 1, s);
    d2h(&r.guarded, nguard.get(), 1, s);
    SS_REQUIRE(!(st & STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "ILU(0): dependency wait timed out");
    return r;
}

// ------------------------------------------------ triangular solves
// One thread per row.  Each pass a lane loads the next batch of dependency
// values (independent loads, issued together) and consumes them in column
// order while they are published, so the accumulation order is fixed.
constexpr int TRSV_BS = 256;
constexpr int TRSV_BATCH = 8;

// y = L^-1 b with L unit lower (strict lower part of LU); resets `reset`
// (the output of the following upper solve) to the sentinel.
template <typename T>
__global__ void __launch_bounds__(TRSV_BS) k_trsv_lower(int n, const int *rowptr, const int *col, const T *val,
                                                        const int *diag, const T *b, T *y, T *reset,
                                                        unsigned *ctr, unsigned base, unsigned *status,
                                                        const int *skip) {
    const unsigned bid = ordered_block(ctr, base);
    if (skip && *skip) return;
    const int row = (int)bid * TRSV_BS + threadIdx.x;
    const bool active = row < n;
    int e = 0, ee = 0;
    T acc = czero<T>();
    if (active) {
        e = rowptr[row];
        ee = diag[row];
        acc = b[row];
        if (reset) set_sentinel(reset + row);
    }
    bool done = !active;
    unsigned spins = 0;
    while (true) {
        if (!done) {
            T v[TRSV_BATCH];
            bool ok[TRSV_BATCH];
#pragma unroll
            for (int q = 0; q < TRSV_BATCH; ++q) {
                ok[q] = false;
                if (e + q < ee) ok[q] = try_load(y + col[e + q], v[q]);
            }
            bool run = true;
            int used = 0;
#pragma unroll
            for (int q = 0; q < TRSV_BATCH; ++q) {
                if (run && e + q < ee && ok[q]) {
                    acc = csub(acc, cmul(val[e + q], v[q]));
                    ++used;
                } else {
                    run = false;
                }
            }
            e += used;
            if (used) {
                spins = 0;
            } else if (e < ee) {
                ++spins;
                if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
                    atomicOr(status, STATUS_SPIN_TIMEOUT);
                    e = ee;
                }
            }
            if (e >= ee) {
                publish(y + row, acc);
                done = true;
            }
        }
        if (__all(done)) break;
    }
}

// z = U^-1 y (U = diagonal and upper part of LU), rows from the last one
// up; resets y to the sentinel for the next lower solve.
template <typename T>
__global__ void __launch_bounds__(TRSV_BS) k_trsv_upper(int n, const int *rowptr, const int *col, const T *val,
                                                        const int *diag, T *y, T *z, unsigned *ctr, unsigned base,
                                                        unsigned *status, const int *skip) {
    const unsigned bid = ordered_block(ctr, base);
    if (skip && *skip) return;
    const int lin = (int)bid * TRSV_BS + threadIdx.x;
    const bool active = lin < n;
    const int row = n - 1 - lin;
    int e = 0, ee = 0, dg = 0;
    T acc = czero<T>();
    if (active) {
        dg = diag[row];
        e = dg + 1;
        ee = rowptr[row + 1];
        acc = y[row];
        set_sentinel(y + row);
    }
    bool done = !active;
    unsigned spins = 0;
    while (true) {
        if (!done) {
            T v[TRSV_BATCH];
            bool ok[TRSV_BATCH];
#pragma unroll
            for (int q = 0; q < TRSV_BATCH; ++q) {
                ok[q] = false;
                if (e + q < ee) ok[q] = try_load(z + col[e + q], v[q]);
            }
            bool run = true;
            int used = 0;
#pragma unroll
            for (int q = 0; q < TRSV_BATCH; ++q) {
                if (run && e + q < ee && ok[q]) {
                    acc = csub(acc, cmul(val[e + q], v[q]));
                    ++used;
                } else {
                    run = false;
                }
            }
            e += used;
            if (used) {
                spins = 0;
            } else if (e < ee) {
                ++spins;
                if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
                    atomicOr(status, STATUS_SPIN_TIMEOUT);
                    e = ee;
                }
            }
            if (e >= ee) {
                publish(z + row, cdiv(acc, val[dg]));
                done = true;
            }
        }
        if (__all(done)) break;
    }
}

template <typename T>
void Precond<T>::setup(const CsrBuf<T> *lu, const int *dg, int n_, hipStream_t s) {
    LU = lu;
    diag = dg;
    n = n_;
    y.resize((size_t)n);
    fill_sentinel<T>(n, y.get(), s);
    status.resize(1);
    SS_HIP(hipMemsetAsync(status.get(), 0, sizeof(unsigned), s));
    counter.init(s);
}

// Sync-free triangular solve in level order over the packed level layout
// (rows sorted by level): a persistent set of wavefronts takes chunks of 64
// consecutive slots in increasing order from an atomic counter, so the rows
// of a chunk belong to one or two adjacent levels and every row a chunk
// waits on lies in an earlier chunk already taken by a running wavefront.
// Keeping only ~1k wavefronts in flight (instead of one thread per row)
// keeps the polling traffic from crowding out the loads that make progress.
// The first WgK<T> entries of a row come coalesced from the packed copy, the
// rest from the CSR factor; entries are consumed in CSR order
// (deterministic rounding), each pass issuing the loads of every pending
// packed entry at once.
constexpr int LEV_WAVES_PER_BLOCK = 4;
constexpr int LEV_MAX_WAVES = 1024;

template <typename T, bool UPPER>
__global__ void __launch_bounds__(LEV_WAVES_PER_BLOCK * 64)
    k_trsv_slots(int n, const int4 *slot, const int *pcol, const T *pval, const T *aux, const int *col,
                 const T *val, T *in, T *out, T *reset, unsigned *ctr, unsigned nwaves, unsigned *status,
                 const int *skip) {
    constexpr int K = WgK<T>::value;
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned chunk = 0;
        if (lane == 0) chunk = atomicAdd(ctr, 1u);
        chunk = __shfl(chunk, 0, 64);
        if ((long long)chunk * 64 >= n) {
            // the last wavefront out resets both counters for the next launch
            if (lane == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (atomicAdd(ctr + 1, 1u) == nwaves - 1) {
                    __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            break;
        }
        const int idx = (int)chunk * 64 + lane;
        const bool active = idx < n;
        int row = 0, start = 0, len = 0;
        int c[K];
        T v[K];
        T acc = czero<T>(), piv = czero<T>();
        if (active) {
            const int4 sl = slot[idx];
            row = sl.x;
            start = sl.y;
            len = sl.z;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                c[k] = pcol[(size_t)k * n + idx];
                v[k] = pval[(size_t)k * n + idx];
            }
            acc = in[row];
            if (UPPER) {
                piv = aux[idx];
                set_sentinel(in + row);  // the lower result goes back to the sentinel
            }
            if (reset) set_sentinel(reset + row);
        }
        int q = 0;  // entries consumed
        bool done = !active;
        unsigned spins = 0;
        while (true) {
            if (!done) {
                int used = 0;
                if (q < K) {
                    T y[K];
                    bool ok[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        ok[k] = false;
                        if (k >= q && k < len) ok[k] = try_load(out + c[k], y[k]);
                    }
                    bool run = true;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        if (k >= q && k < len) {
                            if (run && ok[k]) {
                                acc = csub(acc, cmul(v[k], y[k]));
                                ++used;
                            } else {
                                run = false;
                            }
                        }
                    }
                } else {
                    T y[TRSV_BATCH];
                    bool ok[TRSV_BATCH];
#pragma unroll
                    for (int b = 0; b < TRSV_BATCH; ++b) {
                        ok[b] = false;
                        if (q + b < len) ok[b] = try_load(out + col[start + q + b], y[b]);
                    }
                    bool run = true;
#pragma unroll
                    for (int b = 0; b < TRSV_BATCH; ++b) {
                        if (run && q + b < len && ok[b]) {
                            acc = csub(acc, cmul(val[start + q + b], y[b]));
                            ++used;
                        } else {
                            run = false;
                        }
                    }
                }
                q += used;
                if (used) {
                    spins = 0;
                } else if (q < len) {
                    ++spins;
                    if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
                        atomicOr(status, STATUS_SPIN_TIMEOUT);
                        q = len;
                    }
                }
                if (q >= len) {
                    publish(out + row, UPPER ? cdiv(acc, piv) : acc);
                    done = true;
                }
            }
            if (__all(done)) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

// workgroups of one level-order solve
inline unsigned slots_blocks(int n) {
    const long long chunks = (n + 63) / 64;
    const long long waves = std::min<long long>(chunks, LEV_MAX_WAVES);
    return (unsigned)((waves + LEV_WAVES_PER_BLOCK - 1) / LEV_WAVES_PER_BLOCK);
}

template <typename T>
void Precond<T>::use_levels(const Csr<double2> &lu64, hipStream_t s, int m, const int *order) {
    build_levels(lu64, diag, lo, up, s, order);
    if (m == PRE_AUTO) {
        const bool shallow = std::max(lo.nlev, up.nlev) <= PRE_CLASSES_MAX_LEVELS;
        m = (n <= PRE_BLOCK_MAX_N) ? PRE_BLOCK : shallow ? PRE_CLASSES : PRE_GROUPS;
    }
    if (m == PRE_CLASSES) {
        mode = m;
        return;
    }
    if (m == PRE_GROUPS) {
        // the 16-byte coherent accesses address the vector through a buffer
        // resource limited to 2^31 bytes
        SS_REQUIRE((int64_t)n * (int64_t)sizeof(T) < ((int64_t)1 << 31), SS_E_INVALID_ARG,
                   "row-group triangular solves: system too large");
        group_gates(lo, n, gate_lo, s);
        group_gates(up, n, gate_up, s);
    } else {
        pack_side<T>(lo, LU->view(), false, pl, s);
        pack_side<T>(up, LU->view(), true, pu, s);
    }
    if (m == PRE_BLOCK) bl.resize((size_t)std::max(n, 1));
    if (m == PRE_LEVELS || m == PRE_GROUPS) {
        lev_ctr.resize(4);
        SS_HIP(hipMemsetAsync(lev_ctr.get(), 0, 4 * sizeof(unsigned), s));
    }
    mode = m;
}

template <typename T>
void Precond<T>::borrow_groups(const LevelSched *lo_, const LevelSched *up_, const int *glo, const int *gup,
                               hipStream_t s) {
    blo = lo_;
    bup = up_;
    bglo = glo;
    bgup = gup;
    lev_ctr.resize(4);
    SS_HIP(hipMemsetAsync(lev_ctr.get(), 0, 4 * sizeof(unsigned), s));
    mode = PRE_GROUPS;
}

template <typename T>
void Precond<T>::borrow_classes(const LevelSched *lo_, const LevelSched *up_) {
    blo = lo_;
    bup = up_;
    mode = PRE_CLASSES;
}

// y[q] = x[idx[q]] (gather) or y[idx[q]] = x[q] (scatter); nothing when *skip
template <typename T, bool SCATTER>
__global__ void k_permute_vec(int n, const int *idx, const T *x, T *y, const int *skip) {
    if (skip && *skip) return;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    if (SCATTER) y[idx[q]] = x[q];
    else y[q] = x[idx[q]];
}

template <typename T>
void Precond<T>::apply(const T *b, T *out, hipStream_t s, const int *skip) {
    if (n == 0) return;
    if (pin) {
        pz.resize((size_t)n);
        if (mode == PRE_CLASSES) {
            // the permutation folded into the first and the last substitution
            const LevelSched &L0 = blo ? *blo : lo, &U0 = bup ? *bup : up;
            trsv_classes<T>(L0, false, LU->view(), b, y.get(), skip, s, pin, nullptr);
            trsv_classes<T>(U0, true, LU->view(), y.get(), pz.get(), skip, s, pin, out);
            return;
        }
        pb.resize((size_t)n);
        k_permute_vec<T, false><<<div_up(n, 256), 256, 0, s>>>(n, pin, b, pb.get(), skip);
        const int *keep = pin;
        pin = nullptr;
        apply(pb.get(), pz.get(), s, skip);
        pin = keep;
        k_permute_vec<T, true><<<div_up(n, 256), 256, 0, s>>>(n, pin, pz.get(), out, skip);
        SS_HIP(hipGetLastError());
        return;
    }
    if (mode == PRE_CLASSES) {
        // y takes the lower result (the sentinel is not kept in this mode)
        const LevelSched &L0 = blo ? *blo : lo, &U0 = bup ? *bup : up;
        trsv_classes<T>(L0, false, LU->view(), b, y.get(), skip, s);
        trsv_classes<T>(U0, true, LU->view(), y.get(), out, skip, s);
        return;
    }
    if (mode == PRE_BLOCK) {
        BlockPrecond<T> B;
        B.lo = &lo;
        B.up = &up;
        B.pl = &pl;
        B.pu = &pu;
        precond_block<T>(B, LU->view(), b, out, bl.get(), s, skip);
        return;
    }
    if (mode == PRE_GROUPS) {
        // y holds the sentinel between applies (the upper solve puts it
        // back); the lower solve resets `out` for the upper one
        const LevelSched &L0 = blo ? *blo : lo, &U0 = bup ? *bup : up;
        const int *g0 = blo ? bglo : gate_lo.get(), *g1 = bup ? bgup : gate_up.get();
        trsv_groups<T>(L0, g0, false, LU->view(), b, y.get(), out, lev_ctr.get(), status.get(), skip, s);
        trsv_groups<T>(U0, g1, true, LU->view(), y.get(), out, nullptr, lev_ctr.get(), status.get(), skip, s);
        return;
    }
    if (mode == PRE_LEVELS) {
        const unsigned blocks = slots_blocks(n);
        const unsigned bs = LEV_WAVES_PER_BLOCK * 64, nwaves = blocks * LEV_WAVES_PER_BLOCK;
        // y holds the sentinel between applies; the lower solve reads b
        // through `in` without modifying it (reset = out prepares the upper).
        // The chunk counters return to zero at the end of each launch.
        k_trsv_slots<T, false><<<blocks, bs, 0, s>>>(n, pl.slot.get(), pl.col.get(), pl.val.get(), nullptr,
                                                     LU->col.get(), LU->val.get(), const_cast<T *>(b), y.get(),
                                                     out, lev_ctr.get(), nwaves, status.get(), skip);
        k_trsv_slots<T, true><<<blocks, bs, 0, s>>>(n, pu.slot.get(), pu.col.get(), pu.val.get(), pu.aux.get(),
                                                    LU->col.get(), LU->val.get(), y.get(), out, nullptr,
                                                    lev_ctr.get(), nwaves, status.get(), skip);
        SS_HIP(hipGetLastError());
        return;
    }
    const unsigned grid = (unsigned)div_up(n, TRSV_BS);
    k_trsv_lower<T><<<grid, TRSV_BS, 0, s>>>(n, LU->rowptr.get(), LU->col.get(), LU->val.get(), diag, b, y.get(),
                                              out, counter.ctr.get(), counter.take(grid), status.get(), skip);
    k_trsv_upper<T><<<grid, TRSV_BS, 0, s>>>(n, LU->rowptr.get(), LU->col.get(), LU->val.get(), diag, y.get(), out,
                                              counter.ctr.get(), counter.take(grid), status.get(), skip);
    SS_HIP(hipGetLastError());
}

template <typename T>
void Precond<T>::lower(const T *b, T *out, hipStream_t s) {
    // out = L^-1 b: run the lower solve into y, then copy (out must not alias y)
    if (n == 0) return;
    if (pin) {
        pb.resize((size_t)n);
        pz.resize((size_t)n);
        k_permute_vec<T, false><<<div_up(n, 256), 256, 0, s>>>(n, pin, b, pb.get(), nullptr);
        const int *keep = pin;
        pin = nullptr;
        lower(pb.get(), pz.get(), s);
        pin = keep;
        k_permute_vec<T, true><<<div_up(n, 256), 256, 0, s>>>(n, pin, pz.get(), out, nullptr);
        SS_HIP(hipGetLastError());
        return;
    }
    const unsigned grid = (unsigned)div_up(n, TRSV_BS);
    k_trsv_lower<T><<<grid, TRSV_BS, 0, s>>>(n, LU->rowptr.get(), LU->col.get(), LU->val.get(), diag, b, y.get(),
                                              nullptr, counter.ctr.get(), counter.take(grid), status.get(),
                                              nullptr);
    SS_HIP(hipGetLastError());
    SS_HIP(hipMemcpyAsync(out, y.get(), sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    fill_sentinel<T>(n, y.get(), s);
}

template <typename T>
void Precond<T>::upper(const T *b, T *out, hipStream_t s) {
    if (n == 0) return;
    if (pin) {
        pb.resize((size_t)n);
        pz.resize((size_t)n);
        k_permute_vec<T, false><<<div_up(n, 256), 256, 0, s>>>(n, pin, b, pb.get(), nullptr);
        const int *keep = pin;
        pin = nullptr;
        upper(pb.get(), pz.get(), s);
        pin = keep;
        k_permute_vec<T, true><<<div_up(n, 256), 256, 0, s>>>(n, pin, pz.get(), out, nullptr);
        SS_HIP(hipGetLastError());
        return;
    }
    SS_HIP(hipMemcpyAsync(y.get(), b, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    fill_sentinel<T>(n, out, s);
    const unsigned grid = (unsigned)div_up(n, TRSV_BS);
    k_trsv_upper<T><<<grid, TRSV_BS, 0, s>>>(n, LU->rowptr.get(), LU->col.get(), LU->val.get(), diag, y.get(), out,
                                              counter.ctr.get(), counter.take(grid), status.get(), nullptr);
    SS_HIP(hipGetLastError());
}

template <typename T>
unsigned Precond<T>::read_status(hipStream_t s) {
    unsigned st = 0;
    d2h(&st, status.get(), 1, s);
    return st;
}

template struct Precond<double2>;
template struct Precond<float2>;

}  // namespace ss
