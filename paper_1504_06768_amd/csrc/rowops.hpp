// Row-level device functions shared by the one-system set-up kernels and
// their batched forms, so that both give the same matrices entry for entry.
#pragma once
#include "ss_internal.hpp"

namespace ss {

// Row rt of L~ is the merge of row rt of L with w at the trace columns; all
// other rows are copied.  Entries that cancel to exactly zero are dropped.
template <bool FILL>
__device__ inline int trace_row0(int d, int rt, const int *rowptr, const int *col, const double2 *val, double2 w,
                                 int *ocol, double2 *oval) {
    int e = rowptr[rt];
    const int ee = rowptr[rt + 1];
    int k = 0;
    int cnt = 0;
    while (e < ee || k < d) {
        const int ce = (e < ee) ? col[e] : 0x7fffffff;
        const int ct = (k < d) ? k * (d + 1) : 0x7fffffff;
        const int c = min(ce, ct);
        double2 v = mk(0.0, 0.0);
        if (ce == c) { v = val[e]; ++e; }
        if (ct == c) { v = cadd(v, w); ++k; }
        if (v.x != 0.0 || v.y != 0.0) {
            if (FILL) { ocol[cnt] = c; oval[cnt] = v; }
            ++cnt;
        }
    }
    return cnt;
}

// Row r of L - sigma I (the diagonal inserted when absent).
template <bool FILL>
__device__ inline int shift_row(int r, const int *rowptr, const int *col, const double2 *val, double sigma,
                                int *ocol, double2 *oval) {
    int cnt = 0;
    bool placed = false;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int c = col[e];
        if (!placed && c > r) {
            if (FILL) { ocol[cnt] = r; oval[cnt] = mk(-sigma, 0.0); }
            ++cnt;
            placed = true;
        }
        double2 v = val[e];
        if (c == r) {
            v.x -= sigma;
            placed = true;
        }
        if (v.x != 0.0 || v.y != 0.0) {
            if (FILL) { ocol[cnt] = c; oval[cnt] = v; }
            ++cnt;
        }
    }
    if (!placed) {
        if (FILL) { ocol[cnt] = r; oval[cnt] = mk(-sigma, 0.0); }
        ++cnt;
    }
    return cnt;
}

// One block of 256 threads: the trace row k (d + 1), k = forced if >= 0,
// else the population row with the smallest |L_rr| (lowest k among ties).
// Every thread of the block must call it; the result is valid in thread 0.
__device__ inline int pick_trace_row_block(int d, const int *rowptr, const int *col, const double2 *val,
                                           int forced) {
    __shared__ double sm[256];
    __shared__ int sk[256];
    double best = INFINITY;
    int bk = 0x7fffffff;
    for (int k = threadIdx.x; k < d; k += 256) {
        const int r = k * (d + 1);
        double mag = 0.0;
        int lo = rowptr[r], hi = rowptr[r + 1] - 1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int c = col[mid];
            if (c == r) { mag = sqrt(val[mid].x * val[mid].x + val[mid].y * val[mid].y); break; }
            if (c < r) lo = mid + 1; else hi = mid - 1;
        }
        if (mag < best || (mag == best && k < bk)) { best = mag; bk = k; }
    }
    sm[threadIdx.x] = best;
    sk[threadIdx.x] = bk;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double m2 = sm[threadIdx.x + off];
            const int k2 = sk[threadIdx.x + off];
            if (m2 < sm[threadIdx.x] || (m2 == sm[threadIdx.x] && k2 < sk[threadIdx.x])) {
                sm[threadIdx.x] = m2;
                sk[threadIdx.x] = k2;
            }
        }
        __syncthreads();
    }
    return (forced >= 0 ? forced : sk[0]) * (d + 1);
}

// Row r of the union of two sorted patterns (a and b); FILL writes the
// columns (and value 1 when oval != null).  Returns the row length.
template <bool FILL>
__device__ inline int union_row(int r, const int *ar, const int *ac, const int *br, const int *bc, int *ocol,
                                double2 *oval) {
    int a = ar[r], ae = ar[r + 1], b = br[r], be = br[r + 1], o = 0;
    while (a < ae || b < be) {
        const int x = (a < ae) ? ac[a] : 0x7fffffff;
        const int y = (b < be) ? bc[b] : 0x7fffffff;
        const int m = min(x, y);
        if (x <= y) ++a;
        if (y <= x) ++b;
        if (FILL) {
            ocol[o] = m;
            if (oval) oval[o] = mk(1.0, 0.0);
        }
        ++o;
    }
    return o;
}

// The same union by a group of G lanes when each row has at most G entries
// (rows [as, as + na) of ac and [bs, bs + nb) of bc, columns sorted and
// unique within each): lane t holds entry t of both rows, and each output
// position is counted from the other lanes' columns by shuffle.  An entry of
// the first row lands at its index plus the entries of the second row below
// it that the first row lacks; such an entry of the second row lands at the
// entries of the first row below it plus those of its own row before it.
// Returns the union's length on every lane; with FILL it is written to ocol
// (and 1 to oval).  All G lanes call this with the same rows.
template <bool FILL, int G>
__device__ inline int union_row_group(int as, int na, int bs, int nb, const int *ac, const int *bc, int *ocol,
                                      double2 *oval) {
    const int t = threadIdx.x & (G - 1);
    const int x = (t < na) ? ac[as + t] : 0x7fffffff;
    const int y = (t < nb) ? bc[bs + t] : 0x7fffffff;
    int dup = 0;  // y is also in the first row
    for (int v = 0; v < na; ++v) dup |= (__shfl(x, v, G) == y);
    dup &= (t < nb);
    int ndup = 0, bx = 0, before = 0, ay = 0;
    for (int u = 0; u < nb; ++u) {
        const int yu = __shfl(y, u, G);
        const int du = __shfl(dup, u, G);
        ndup += du;
        bx += (!du && yu < x);
        before += (du && u < t);
    }
    for (int v = 0; v < na; ++v) ay += (__shfl(x, v, G) < y);
    if (FILL) {
        if (t < na) {
            ocol[t + bx] = x;
            if (oval) oval[t + bx] = mk(1.0, 0.0);
        }
        if (t < nb && !dup) {
            const int p = ay + (t - before);
            ocol[p] = y;
            if (oval) oval[p] = mk(1.0, 0.0);
        }
    }
    return na + nb - ndup;
}

// A group of G lanes (a whole wavefront by default) sorts the entries
// [rs, re) by column (unique within a row): rank sort, so the result does
// not depend on the order of the input.
template <typename T, int G = 64>
__device__ inline void sort_row_wave(int rs, int re, const int *col_in, const T *val_in, int *col_out, T *val_out) {
    const int lane = threadIdx.x & (G - 1);
    if (re - rs <= G) {
        // one pass: ranks from the other lanes' columns by shuffle (all G
        // lanes call this with the same row)
        const int e = rs + lane;
        const int c = (e < re) ? col_in[e] : 0x7fffffff;
        int rank = 0;
        for (int f = 0; f < re - rs; ++f) rank += (__shfl(c, f, G) < c);
        if (e < re) {
            col_out[rs + rank] = c;
            if (val_in) val_out[rs + rank] = val_in[e];
        }
        return;
    }
    for (int e = rs + lane; e < re; e += G) {
        const int c = col_in[e];
        int rank = 0;
        for (int f = rs; f < re; ++f) rank += (col_in[f] < c);
        col_out[rs + rank] = c;
        if (val_in) val_out[rs + rank] = val_in[e];
    }
}

}  // namespace ss
