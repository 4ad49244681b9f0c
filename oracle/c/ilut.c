/* Dual-threshold incomplete LU (ILUT) without pivoting, in plain C -- test
 * infrastructure (oracle), never linked into the solver library.
 *
 * Paper, section "Iterative Solvers": the preconditioner is an incomplete LU
 * factorisation of the (permuted) modified Liouvillian with a drop tolerance
 * and a fill limit.  Row i is eliminated in increasing column order (the
 * row-wise IKJ form of Gaussian elimination):
 *   w = a_i (the working row), tau = drop_tol * ||a_i||_inf,
 *   keep = ceil(fill * nnz(a_i));
 *   for each k < i present in w, smallest first:
 *       l = w_k / u_kk; if |l| < tau drop w_k, else w_k = l and
 *       w_j -= l * u_kj for every stored u_kj, j > k (new entries are fill);
 *   the strict lower (multipliers) and strict upper parts of w are cut to
 *   the entries with |w_j| >= tau, then to the `keep` largest in magnitude
 *   (ties: lower column first); the diagonal is always kept.
 * A pivot with |u_ii| < guard * ||a_i||_inf becomes boost * ||a_i||_inf
 * times its phase (that value when it is exactly zero) and is counted.
 *
 * The same steps as the Python ILUT of the oracle, with the same complex
 * arithmetic (product (ac - bd) + (ad + bc)i; quotient by Smith's method,
 * R. L. Smith, CACM 5 (1962) 435), so the two agree bit for bit when built
 * without floating-point contraction; this one runs the full-size systems.
 *
 * Input: CSR with sorted column indices (indptr int64[n+1], indices int32,
 * data interleaved re/im doubles).  Output: the strict lower part of L and U
 * (diagonal included), rows sorted, into caller arrays of capacity cap
 * entries (cap >= n + 2 * sum_i ceil(fill * nnz(a_i)) always suffices).
 * Returns the number of guarded pivots (>= 0), -1 on allocation failure,
 * -2 when cap is exceeded, -3 for a zero pivot with guard == 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;

static cplx c_mul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static cplx c_sub(cplx a, cplx b) {
    cplx r = {a.re - b.re, a.im - b.im};
    return r;
}

/* Smith's method */
static cplx c_div(cplx a, cplx b) {
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

static double c_abs(cplx a) { return hypot(a.re, a.im); }

typedef struct { int32_t col; double mag; } cand;

/* magnitude descending, then column ascending */
static int cmp_cand(const void *x, const void *y) {
    const cand *a = (const cand *)x, *b = (const cand *)y;
    if (a->mag != b->mag) return a->mag > b->mag ? -1 : 1;
    return (a->col > b->col) - (a->col < b->col);
}

static int cmp_int(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* binary min-heap of column indices */
static void heap_push(int32_t *h, int64_t *len, int32_t v) {
    int64_t i = (*len)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p] <= v) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = v;
}

static int32_t heap_pop(int32_t *h, int64_t *len) {
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

int oracle_ilut(int64_t n, const int64_t *indptr, const int32_t *indices, const double *data, double drop_tol,
                double fill, double guard, double boost, int64_t cap, int64_t *lu_indptr, int32_t *lu_indices,
                double *lu_data) {
    const cplx *A = (const cplx *)data;
    cplx *LU = (cplx *)lu_data;
    cplx *w = malloc(sizeof(cplx) * (size_t)(n > 0 ? n : 1));
    int64_t *stamp = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cols = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *heap = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *udiag = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    cand *lo = malloc(sizeof(cand) * (size_t)(n > 0 ? n : 1));
    cand *up = malloc(sizeof(cand) * (size_t)(n > 0 ? n : 1));
    int32_t *sel = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int rc = 0, guarded = 0;
    if (!w || !stamp || !cols || !heap || !udiag || !lo || !up || !sel) {
        rc = -1;
        goto out;
    }
    for (int64_t j = 0; j < n; ++j) stamp[j] = -1;
    lu_indptr[0] = 0;
    int64_t pos = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a0 = indptr[i], a1 = indptr[i + 1];
        const int64_t nz = a1 - a0;
        double rownorm = 0.0;
        for (int64_t e = a0; e < a1; ++e) {
            double m = c_abs(A[e]);
            if (m > rownorm) rownorm = m;
        }
        const double tau = drop_tol * rownorm;
        const int64_t keep = (int64_t)ceil(fill * (double)nz);
        /* scatter the row; `dead` marks dropped multipliers via stamp = -2 - i */
        int64_t ncols = 0, hlen = 0;
        for (int64_t e = a0; e < a1; ++e) {
            int32_t j = indices[e];
            w[j] = A[e];
            stamp[j] = i;
            cols[ncols++] = j;
            if (j < i) heap_push(heap, &hlen, j);
        }
        while (hlen > 0) {
            int32_t k = heap_pop(heap, &hlen);
            cplx l = c_div(w[k], LU[udiag[k]]);
            if (c_abs(l) < tau) {
                stamp[k] = -2 - i;
                continue;
            }
            w[k] = l;
            for (int64_t f = udiag[k] + 1; f < lu_indptr[k + 1]; ++f) {
                int32_t j = lu_indices[f];
                cplx t = c_mul(l, LU[f]);
                if (stamp[j] == i) {
                    w[j] = c_sub(w[j], t);
                } else {
                    cplx z = {0.0, 0.0};
                    w[j] = c_sub(z, t);
                    stamp[j] = i;
                    cols[ncols++] = j;
                    if (j < i) heap_push(heap, &hlen, j);
                }
            }
        }
        /* second dropping rule and the fill cap */
        int64_t nlo = 0, nup = 0;
        cplx piv = {0.0, 0.0};
        for (int64_t c = 0; c < ncols; ++c) {
            int32_t j = cols[c];
            if (stamp[j] != i) continue; /* dropped multiplier */
            if (j == i) {
                piv = w[j];
                continue;
            }
            double m = c_abs(w[j]);
            if (m < tau) continue;
            cand cd = {j, m};
            if (j < i) lo[nlo++] = cd;
            else up[nup++] = cd;
        }
        qsort(lo, (size_t)nlo, sizeof(cand), cmp_cand);
        qsort(up, (size_t)nup, sizeof(cand), cmp_cand);
        if (nlo > keep) nlo = keep;
        if (nup > keep) nup = keep;
        if (guard > 0.0) {
            double bound = guard * rownorm, value = boost * rownorm;
            double m = c_abs(piv);
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
        if (pos + nlo + nup + 1 > cap) {
            rc = -2;
            goto out;
        }
        int64_t ns = 0;
        for (int64_t c = 0; c < nlo; ++c) sel[ns++] = lo[c].col;
        sel[ns++] = (int32_t)i;
        for (int64_t c = 0; c < nup; ++c) sel[ns++] = up[c].col;
        qsort(sel, (size_t)ns, sizeof(int32_t), cmp_int);
        for (int64_t c = 0; c < ns; ++c) {
            int32_t j = sel[c];
            lu_indices[pos] = j;
            if (j == i) {
                LU[pos] = piv;
                udiag[i] = pos;
            } else {
                LU[pos] = w[j];
            }
            ++pos;
        }
        lu_indptr[i + 1] = pos;
        for (int64_t c = 0; c < ncols; ++c) stamp[cols[c]] = -1;
    }
    rc = guarded;
out:
    free(w);
    free(stamp);
    free(cols);
    free(heap);
    free(udiag);
    free(lo);
    free(up);
    free(sel);
    return rc;
}
