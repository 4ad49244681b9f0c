/* Dual-threshold incomplete LU with column pivoting (ILUTP), in plain C --
 * test infrastructure (oracle), never linked into the solver library.
 *
 * Paper, section "Iterative Solvers": the preconditioner is "iLUT with
 * dual-threshold and pivoting".  The dropping rules are those of the
 * oracle's ILUT (oracle/c/ilut.c): row i is eliminated in the row-wise IKJ
 * form, multipliers below tau = drop_tol * ||a_i||_inf are dropped, and each
 * strict part keeps the entries with |w_j| >= tau, at most
 * ceil(fill * nnz(a_i)) of them, largest first (ties: lower position first).
 *
 * Pivoting (Saad, "Iterative Methods for Sparse Linear Systems", 2nd ed.,
 * sec. 10.4.4): the factorisation is A Q = L U with a column permutation Q
 * built as the rows are processed.  Columns are referred to by their
 * original index c and by their current position iperm[c]; position p holds
 * column perm[p].  While row i is processed, an entry of column c belongs
 * to the lower part when iperm[c] < i, is the diagonal candidate when
 * iperm[c] == i and to the upper part otherwise; lower entries are
 * eliminated in increasing position.  After dropping, let c* be the kept
 * upper entry of largest magnitude (first in position on ties); when
 * permtol * |w_c*| > |w_diag| (the diagonal candidate, 0 if absent) the
 * columns at positions i and iperm[c*] are exchanged, so that c* becomes the
 * pivot of row i and the former diagonal candidate an upper entry.  Only
 * positions >= i move, so a lower entry's position is final when it is
 * stored.  permtol = 0 never pivots and gives the ILUT of oracle/c/ilut.c bit
 * for bit; permtol = 1 with drop_tol = 0 and no fill limit is Gaussian
 * elimination with partial pivoting by columns.  The pivot guard of the ILUT
 * applies to the chosen pivot.
 *
 * Complex arithmetic as in ilut.c (product (ac - bd) + (ad + bc)i, Smith's
 * quotient, hypot for the modulus).
 *
 * Input: CSR with sorted column indices (indptr int64[n+1], indices int32,
 * data interleaved re/im doubles).  Output: perm[n] (position -> original
 * column) and the factors in position space -- strict lower part of L (unit
 * diagonal implied) and U with its diagonal -- rows sorted, into caller
 * arrays of capacity cap entries.  Returns the number of guarded pivots
 * (>= 0), -1 on allocation failure, -2 when cap is exceeded, -3 for a zero
 * pivot with guard == 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;

static cplx p_mul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static cplx p_sub(cplx a, cplx b) {
    cplx r = {a.re - b.re, a.im - b.im};
    return r;
}

static cplx p_div(cplx a, cplx b) {
    cplx r;
    if (fabs(b.re) >= fabs(b.im)) {
        double ratio = b.im / b.re, den = b.re + b.im * ratio;
        r.re = (a.re + a.im * ratio) / den;
        r.im = (a.im - a.re * ratio) / den;
    } else {
        double ratio = b.re / b.im, den = b.re * ratio + b.im;
        r.re = (a.re * ratio + a.im) / den;
        r.im = (a.im * ratio - a.re) / den;
    }
    return r;
}

static double p_abs(cplx a) { return hypot(a.re, a.im); }

/* candidates keyed by position: magnitude descending, then position ascending */
typedef struct { int32_t pos, col; double mag; } pcand;

static int cmp_pcand(const void *x, const void *y) {
    const pcand *a = (const pcand *)x, *b = (const pcand *)y;
    if (a->mag != b->mag) return a->mag > b->mag ? -1 : 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

typedef struct { int32_t pos; cplx v; } pent;

static int cmp_pent(const void *x, const void *y) {
    const pent *a = (const pent *)x, *b = (const pent *)y;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

/* binary min-heap of positions */
static void ph_push(int32_t *h, int64_t *len, int32_t v) {
    int64_t i = (*len)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p] <= v) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = v;
}

static int32_t ph_pop(int32_t *h, int64_t *len) {
    int32_t top = h[0], v = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= *len) break;
        if (c + 1 < *len && h[c + 1] < h[c]) ++c;
        if (h[c] >= v) break;
        h[i] = h[c];
        i = c;
    }
    if (*len > 0) h[i] = v;
    return top;
}

int oracle_ilutp(int64_t n, const int64_t *indptr, const int32_t *indices, const double *data, double drop_tol,
                 double fill, double permtol, double guard, double boost, int64_t cap, int32_t *perm,
                 int64_t *lu_indptr, int32_t *lu_indices, double *lu_data) {
    const cplx *A = (const cplx *)data;
    cplx *LU = (cplx *)lu_data;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    cplx *w = malloc(sizeof(cplx) * nn);
    int64_t *stamp = malloc(sizeof(int64_t) * nn);
    int32_t *cols = malloc(sizeof(int32_t) * nn);
    int32_t *heap = malloc(sizeof(int32_t) * nn);
    int32_t *iperm = malloc(sizeof(int32_t) * nn);
    /* U rows stored by original column while the factorisation runs */
    int64_t *uptr = malloc(sizeof(int64_t) * (nn + 1));
    int32_t *ucol = malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    cplx *uval = malloc(sizeof(cplx) * (size_t)(cap > 0 ? cap : 1));
    /* L rows (positions final when stored) */
    int64_t *lptr = malloc(sizeof(int64_t) * (nn + 1));
    int32_t *lpos = malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    cplx *lval = malloc(sizeof(cplx) * (size_t)(cap > 0 ? cap : 1));
    pcand *lo = malloc(sizeof(pcand) * nn);
    pcand *up = malloc(sizeof(pcand) * nn);
    pent *row = malloc(sizeof(pent) * (nn + 1));
    int rc = 0, guarded = 0;
    if (!w || !stamp || !cols || !heap || !iperm || !uptr || !ucol || !uval || !lptr || !lpos || !lval || !lo ||
        !up || !row) {
        rc = -1;
        goto out;
    }
    for (int64_t j = 0; j < n; ++j) {
        stamp[j] = -1;
        perm[j] = (int32_t)j;
        iperm[j] = (int32_t)j;
    }
    uptr[0] = 0;
    lptr[0] = 0;
    int64_t nu = 0, nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a0 = indptr[i], a1 = indptr[i + 1];
        const int64_t nz = a1 - a0;
        double rownorm = 0.0;
        for (int64_t e = a0; e < a1; ++e) {
            double m = p_abs(A[e]);
            if (m > rownorm) rownorm = m;
        }
        const double tau = drop_tol * rownorm;
        const int64_t keep = (int64_t)ceil(fill * (double)nz);
        int64_t ncols = 0, hlen = 0;
        for (int64_t e = a0; e < a1; ++e) {
            int32_t c = indices[e];
            w[c] = A[e];
            stamp[c] = i;
            cols[ncols++] = c;
            if (iperm[c] < i) ph_push(heap, &hlen, iperm[c]);
        }
        /* elimination in increasing position; a dropped multiplier is
           marked with stamp = -2 - i */
        while (hlen > 0) {
            int32_t k = ph_pop(heap, &hlen);   /* a position < i */
            int32_t c = perm[k];
            /* the pivot of row k is the first stored entry of its U row */
            cplx l = p_div(w[c], uval[uptr[k]]);
            if (p_abs(l) < tau) {
                stamp[c] = -2 - i;
                continue;
            }
            w[c] = l;
            for (int64_t f = uptr[k] + 1; f < uptr[k + 1]; ++f) {
                int32_t cj = ucol[f];
                cplx t = p_mul(l, uval[f]);
                if (stamp[cj] == i) {
                    w[cj] = p_sub(w[cj], t);
                } else {
                    cplx z = {0.0, 0.0};
                    w[cj] = p_sub(z, t);
                    stamp[cj] = i;
                    cols[ncols++] = cj;
                    if (iperm[cj] < i) ph_push(heap, &hlen, iperm[cj]);
                }
            }
        }
        /* dropping: second rule and the fill cap */
        int64_t nlo = 0, nup = 0;
        int have_diag = 0;
        cplx piv = {0.0, 0.0};
        int32_t dcol = perm[i];
        for (int64_t q = 0; q < ncols; ++q) {
            int32_t c = cols[q];
            if (stamp[c] != i) continue;
            int32_t p = iperm[c];
            if (p == i) {
                piv = w[c];
                have_diag = 1;
                continue;
            }
            double m = p_abs(w[c]);
            if (m < tau) continue;
            pcand cd = {p, c, m};
            if (p < i) lo[nlo++] = cd;
            else up[nup++] = cd;
        }
        qsort(lo, (size_t)nlo, sizeof(pcand), cmp_pcand);
        qsort(up, (size_t)nup, sizeof(pcand), cmp_pcand);
        if (nlo > keep) nlo = keep;
        if (nup > keep) nup = keep;
        /* pivoting: up[0] is the kept upper entry of largest magnitude */
        if (permtol > 0.0 && nup > 0 && permtol * up[0].mag > p_abs(piv)) {
            int32_t cs = up[0].col, ps = up[0].pos;
            /* exchange positions i and ps */
            perm[i] = cs;
            perm[ps] = dcol;
            iperm[cs] = (int32_t)i;
            iperm[dcol] = ps;
            cplx newpiv = w[cs];
            /* the former diagonal candidate takes the pivot's place among the
               upper entries (kept when it is non-zero) */
            if (have_diag && (piv.re != 0.0 || piv.im != 0.0)) {
                up[0].col = dcol;
                up[0].pos = ps;
                up[0].mag = p_abs(piv);
            } else {
                up[0] = up[--nup];
            }
            piv = newpiv;
            dcol = cs;
        }
        if (guard > 0.0) {
            double bound = guard * rownorm, value = boost * rownorm;
            double m = p_abs(piv);
            if (!(m >= bound)) {
                if (value <= 0.0) value = 1.0;
                if (piv.re == 0.0 && piv.im == 0.0) {
                    piv.re = value;
                    piv.im = 0.0;
                } else {
                    piv.re = piv.re / m * value;
                    piv.im = piv.im / m * value;
                }
                ++guarded;
            }
        } else if (piv.re == 0.0 && piv.im == 0.0) {
            rc = -3;
            goto out;
        }
        if (nu + nup + 1 > cap || nl + nlo > cap) {
            rc = -2;
            goto out;
        }
        /* store: L by final position (ascending), U pivot first then the
           other upper entries by original column */
        for (int64_t q = 0; q < nlo; ++q) {
            row[q].pos = lo[q].pos;
            row[q].v = w[lo[q].col];
        }
        qsort(row, (size_t)nlo, sizeof(pent), cmp_pent);
        for (int64_t q = 0; q < nlo; ++q) {
            lpos[nl] = row[q].pos;
            lval[nl] = row[q].v;
            ++nl;
        }
        lptr[i + 1] = nl;
        ucol[nu] = dcol;
        uval[nu] = piv;
        ++nu;
        for (int64_t q = 0; q < nup; ++q) {
            int32_t c = up[q].col;
            ucol[nu] = c;
            /* the former diagonal candidate keeps its value from before the swap */
            uval[nu] = w[c];
            ++nu;
        }
        uptr[i + 1] = nu;
        for (int64_t q = 0; q < ncols; ++q) stamp[cols[q]] = -1;
    }
    /* output in final position space, rows sorted */
    {
        int64_t pos = 0;
        lu_indptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t m = 0;
            for (int64_t f = lptr[i]; f < lptr[i + 1]; ++f) {
                row[m].pos = lpos[f];
                row[m].v = lval[f];
                ++m;
            }
            for (int64_t f = uptr[i]; f < uptr[i + 1]; ++f) {
                row[m].pos = iperm[ucol[f]];
                row[m].v = uval[f];
                ++m;
            }
            qsort(row, (size_t)m, sizeof(pent), cmp_pent);
            if (pos + m > cap) {
                rc = -2;
                goto out;
            }
            for (int64_t q = 0; q < m; ++q) {
                lu_indices[pos] = row[q].pos;
                LU[pos] = row[q].v;
                ++pos;
            }
            lu_indptr[i + 1] = pos;
        }
    }
    rc = guarded;
out:
    free(w);
    free(stamp);
    free(cols);
    free(heap);
    free(iperm);
    free(uptr);
    free(ucol);
    free(uval);
    free(lptr);
    free(lpos);
    free(lval);
    free(lo);
    free(up);
    free(row);
    return rc;
}
