// Workgroup-resident solver for small systems (wgsolve.hip): the whole
// refinement loop, BiCGSTAB and level-scheduled ILU triangular solves of one
// system run inside one workgroup, with the triangular-solve vector in LDS.
#pragma once
#include "blas.hpp"
#include "ilu.hpp"

namespace ss {

// Level schedule of one triangular factor: slots in level order, each slot
// {row, first entry, end entry, 0}; levels delimited by ptr.
struct LevelSched {
    int nlev = 0;
    DevBuf<int> ptr;    // nlev + 1
    DevBuf<int4> slot;  // n
};

// Level sets of the strict lower part (forward) and of the strict upper part
// (backward) of the ILU factors; a row's level is one more than the largest
// level among the rows it depends on.
void build_levels(const Csr<double2> &LU, const int *diag, LevelSched &lo, LevelSched &up, hipStream_t s);

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

// factor entries per row kept in the packed level layout (fewer for
// complex128 so that three levels of them fit in registers)
template <typename T> struct WgK;
template <> struct WgK<float2> { static constexpr int value = 8; };
template <> struct WgK<double2> { static constexpr int value = 4; };

// Level-ordered packed copy of one triangular factor in precision T: for
// slot idx (level order), slot[idx] = {row, first CSR entry, length, 0}, and
// the first WgK<T> column indices and values of the row at
// col[k * n + idx], val[k * n + idx] (zero padded); aux[idx] is the pivot
// u_ii for the upper factor.  Every load of a slot is addressed by idx alone.
template <typename T>
struct PackedSide {
    DevBuf<int4> slot;
    DevBuf<int> col;
    DevBuf<T> val;
    DevBuf<T> aux;
};

template <typename T>
void pack_side(const LevelSched &ls, const Csr<T> &LU, bool upper, PackedSide<T> &out, hipStream_t s);

template <typename T>
struct WgProblem {
    int n, d, q0, trace;      // trace: 1 = trace-row system, 0 = inverse power
    int nlev_l, nlev_u;
    int maxiter, max_outer;
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
