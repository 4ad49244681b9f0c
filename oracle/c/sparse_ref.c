/* Zero-fill incomplete LU and the triangular solves with its factors, in
 * plain C -- test infrastructure (oracle), never linked into the solver
 * library.  They serve the CPU fp64 sparse reference solve of the oracle
 * (oracle/sparse_ref.py) at sizes where the Python loops would take hours.
 *
 * Paper, section "Iterative Solvers": the preconditioner is an incomplete LU
 * factorisation M = L U of the (permuted) modified Liouvillian, and each
 * Krylov iteration applies M^-1 by forward and backward substitution.
 *
 * oracle_ilu0: ILU(0) in the row-wise (IKJ) elimination order.  L is unit
 *   lower and U upper, both on the pattern of A: for each row i and each
 *   stored k < i in ascending order, l_ik = a_ik / u_kk, then
 *   a_ij -= l_ik u_kj for every stored u_kj (j > k) whose position (i, j) is
 *   in the pattern; entries outside the pattern are dropped.  A pivot below
 *   guard * ||a_i||_inf (the input row) becomes boost * ||a_i||_inf times its
 *   phase (that value when it is exactly zero) and is counted.  The same steps
 *   and complex arithmetic as the Python ilu0 of the oracle (product
 *   (ac - bd) + (ad + bc)i, quotient by Smith's method, R. L. Smith, CACM 5
 *   (1962) 435).
 *
 * oracle_lu_solve: x = U^-1 L^-1 b from the combined factor (strict lower
 *   part of L, U with its diagonal), rows in order for L, reverse for U.
 *
 * Input CSR: indptr int64[n+1], indices int32 (sorted per row), values as
 * interleaved re/im doubles.  oracle_ilu0 works in place on vals and needs a
 * stored diagonal in every row; it returns the number of guarded pivots, -1
 * on allocation failure, -2 for a row without a diagonal entry, -3 for a
 * zero pivot with guard == 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { double re, im; } cplx;

static cplx c_mul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static cplx c_sub(cplx a, cplx b) {
    cplx r = {a.re - b.re, a.im - b.im};
    return r;
}

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

int oracle_ilu0(int64_t n, const int64_t *indptr, const int32_t *indices, double *vals_ri, double guard,
                double boost) {
    cplx *v = (cplx *)vals_ri;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!pos || !diag) {
        free(pos);
        free(diag);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j) pos[j] = -1;
    for (int64_t i = 0; i < n; ++i) {
        diag[i] = -1;
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e)
            if (indices[e] == i) diag[i] = e;
        if (diag[i] < 0) {
            free(pos);
            free(diag);
            return -2;
        }
    }
    int guarded = 0;
    for (int64_t i = 0; i < n; ++i) {
        double rownorm = 0.0;
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
            double m = c_abs(v[e]);
            if (m > rownorm) rownorm = m;
            pos[indices[e]] = e;
        }
        for (int64_t e = indptr[i]; e < diag[i]; ++e) {
            const int64_t k = indices[e];
            v[e] = c_div(v[e], v[diag[k]]);
            const cplx lik = v[e];
            for (int64_t f = diag[k] + 1; f < indptr[k + 1]; ++f) {
                const int64_t p = pos[indices[f]];
                if (p >= 0) v[p] = c_sub(v[p], c_mul(lik, v[f]));
            }
        }
        cplx piv = v[diag[i]];
        if (guard > 0) {
            const double bound = guard * rownorm;
            if (c_abs(piv) < bound) {
                double value = boost * rownorm;
                if (value <= 0) value = 1.0;
                if (piv.re == 0.0 && piv.im == 0.0) {
                    piv.re = value;
                    piv.im = 0.0;
                } else {
                    const double m = c_abs(piv);
                    piv.re = piv.re / m * value;
                    piv.im = piv.im / m * value;
                }
                v[diag[i]] = piv;
                ++guarded;
            }
        } else if (piv.re == 0.0 && piv.im == 0.0) {
            free(pos);
            free(diag);
            return -3;
        }
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) pos[indices[e]] = -1;
    }
    free(pos);
    free(diag);
    return guarded;
}

void oracle_lu_solve(int64_t n, const int64_t *indptr, const int32_t *indices, const double *vals_ri,
                     const int64_t *diag, const double *b_ri, double *x_ri) {
    const cplx *v = (const cplx *)vals_ri;
    const cplx *b = (const cplx *)b_ri;
    cplx *x = (cplx *)x_ri;
    for (int64_t i = 0; i < n; ++i) {  /* L y = b, unit diagonal */
        cplx s = b[i];
        for (int64_t e = indptr[i]; e < diag[i]; ++e) s = c_sub(s, c_mul(v[e], x[indices[e]]));
        x[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {  /* U x = y */
        cplx s = x[i];
        for (int64_t e = diag[i] + 1; e < indptr[i + 1]; ++e) s = c_sub(s, c_mul(v[e], x[indices[e]]));
        x[i] = c_div(s, v[diag[i]]);
    }
}
