/* A plain C99 client of the solver library: builds the Liouvillian of a
 * driven damped cavity (H = Delta a+a + E (a + a+), C = sqrt(kappa) a) in a
 * Fock space of N states, solves for the steady state on the GPU and checks
 * it against the coherent state |alpha><alpha|, alpha = -iE / (kappa/2 +
 * i Delta), which is the exact steady state of this model (up to the
 * truncation, negligible at N = 40 for |alpha|^2 = 2).  Exit status 0 on
 * success.  Only include/ss.h and libss.so are used. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ss.h"

#define NMAX 64

static int fail(const char *what, int rc) {
    fprintf(stderr, "%s failed: %d (%s)\n", what, rc, ss_last_error());
    return 1;
}

int main(int argc, char **argv) {
    const int N = argc > 1 ? atoi(argv[1]) : 40;
    if (N < 2 || N > NMAX) return 2;
    const double delta = 0.5, E = 1.0, kappa = 1.0;
    /* H: tridiagonal; a: one superdiagonal */
    int64_t hp[NMAX + 1], ap[NMAX + 1];
    int32_t hi[3 * NMAX], ai[NMAX];
    double hv[6 * NMAX], av[2 * NMAX];
    int64_t nh = 0, na = 0;
    for (int i = 0; i < N; ++i) {
        hp[i] = nh;
        if (i > 0) { hi[nh] = i - 1; hv[2 * nh] = E * sqrt((double)i); hv[2 * nh + 1] = 0; ++nh; }
        hi[nh] = i; hv[2 * nh] = delta * i; hv[2 * nh + 1] = 0; ++nh;
        if (i + 1 < N) { hi[nh] = i + 1; hv[2 * nh] = E * sqrt((double)(i + 1)); hv[2 * nh + 1] = 0; ++nh; }
        ap[i] = na;
        if (i + 1 < N) { ai[na] = i + 1; av[2 * na] = sqrt(kappa * (i + 1)); av[2 * na + 1] = 0; ++na; }
    }
    hp[N] = nh;
    ap[N] = na;
    ss_csr_z H = {N, nh, hp, hi, hv};
    ss_csr_z C = {N, na, ap, ai, av};
    ss_liouv L = NULL;
    int rc = ss_build_liouvillian(&H, &C, 1, N, &L);
    if (rc != SS_OK) return fail("ss_build_liouvillian", rc);
    ss_options opt;
    ss_options_default(&opt);
    opt.prec = SS_MIXED;
    double *rho = malloc(sizeof(double) * 2 * N * N);
    ss_info info;
    rc = ss_solve(L, SS_TRACE_BICGSTAB, 1e-10, &opt, rho, &info);
    if (rc != SS_OK) return fail("ss_solve", rc);
    /* coherent state amplitudes c_k = e^{-|alpha|^2/2} alpha^k / sqrt(k!) */
    const double complex alpha = -I * E / (kappa / 2 + I * delta);
    double complex c[NMAX];
    c[0] = cexp(-0.5 * creal(alpha * conj(alpha)));
    for (int k = 1; k < N; ++k) c[k] = c[k - 1] * alpha / sqrt((double)k);
    double err = 0;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            const double complex r = rho[2 * (i + N * j)] + I * rho[2 * (i + N * j) + 1];
            const double e = cabs(r - c[i] * conj(c[j]));
            if (e > err) err = e;
        }
    printf("N=%d ||L rho||=%.3e inner=%d max|rho - |alpha><alpha||=%.3e %s\n", N, info.resid_l2, info.inner_its, err,
           ss_version());
    free(rho);
    ss_liouv_free(L);
    return (err <= 1e-6 && info.resid_l2 <= 1e-10) ? 0 : 3;
}
