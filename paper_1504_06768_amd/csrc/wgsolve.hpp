// Workgroup-resident solver for small systems (wgsolve.hip): the whole
// refinement loop, BiCGSTAB and level-scheduled ILU triangular solves of one
// system run inside one workgroup, with the triangular-solve vector in LDS.
#pragma once
#include "blas.hpp"
#include "levels.hpp"

namespace ss {

// Outcome of a workgroup solve (device struct, one per system).
struct WgResult {
    int status;     // SS_OK, SS_E_NOT_CONVERGED or SS_E_BREAKDOWN
    int outer;
    int inner;
    int breakdowns;
    double resid;   // last outer certificate ||L x|| / |Tr x|
    long long ticks_precond;  // device wall-clock ticks (100 MHz) spent in
    long long ticks_spmv;     // the triangular solves, the SpMVs and the
    long long ticks_total;    // whole kernel, measured by thread 0
};

template <typename T>
struct WgProblem {
    int n, d, q0, trace;      // trace: 1 = trace-row system, 0 = inverse power
    int nlev_l, nlev_u;
    int maxiter, max_outer;
    int force_breakdown;      // SS_FLAG_FORCE_BREAKDOWN: every breakdown test fires
    double tol, rtol_in, sigma;
    double2 w;
    Csr<T> A;                 // inner-precision P A P^T
    Csr<double2> A64;         // fp64 P A P^T (outer residual)
    Csr<T> LU;                // ILU factors (inner precision)
    const int *diag;
    const int *lptr;
    const int4 *lslot;        // packed level layout of L (see PackedSide)
    const int *lcol;
    const T *lval;
    const int *uptr;
    const int4 *uslot;        // packed level layout of U
    const int *ucol;
    const T *uval;
    const T *uaux;
    const int *tpos;          // permuted positions of the diagonal of rho
    const double2 *b64;       // trace-row right-hand side (permuted), or null
    double2 *x64;             // solution (fp64, permuted); inverse power: start vector
    double2 *r64;             // fp64 residual scratch
    T *work;                  // 11 n inner-precision scratch
    T *ysc;                   // n scratch for the triangular solves when LDS is too small
    WgResult *res;
};

constexpr int WG_BS = 512;

// Largest n whose triangular-solve vector of type T fits the LDS budget.
template <typename T>
int wg_lds_capacity();

// Launch one workgroup per problem (probs: device array of count entries);
// max_n and max_levels (largest nlev_l + nlev_u) size the LDS.
template <typename T>
void wg_solve(const WgProblem<T> *probs, int count, int max_n, int max_levels, hipStream_t s);

// whether a system of n entries of elem bytes and `levels` levels keeps its
// triangular-solve vector in LDS
bool wg_fits_lds(size_t n, size_t elem, int levels);

}  // namespace ss
