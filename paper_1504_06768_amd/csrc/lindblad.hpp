// The Lindblad generator applied without the assembled n x n matrix
// (lindblad.hip).
//
// Eq. (lindblad) in column stacking, vec(A rho B) = (B^T (x) A) vec(rho):
//   L vec(rho) = vec(Gpre rho + rho Gpost^T + sum_k C_k rho C_k^+),
// with Gpre = -i H - 1/2 D, Gpost = (i H - 1/2 D)^T, D = sum_k C_k^+ C_k.
// Only the d x d operators Gpre, Gpost and C_k are kept (a few non-zeros per
// row for the paper's models), so a residual in fp64 streams rho and the
// result instead of the complex128 n x n matrix.
#pragma once
#include "ss_internal.hpp"

namespace ss {

constexpr int MAX_COPS = 16;

// Device views of the d x d operators, passed by value to kernels.
struct LindbladOp {
    int d = 0;
    int nops = 0;
    Csr<double2> Gp;              // Gpre, rows i
    Csr<double2> Gq;              // Gpost, rows j
    Csr<double2> C[MAX_COPS];     // collapse operators
};

// Owning storage of the operators (kept on the handle after assembly).
struct LindbladBuf {
    int d = 0;
    CsrBuf<double2> Gp, Gq;
    std::vector<CsrBuf<double2>> C;
    LindbladOp view() const;
    size_t bytes() const;
};

// For every r < n = d^2:
//   v      = (L vec rho)_r  (+ w * (*trace) when trace != null and r == trow)
//   o      = iperm ? iperm[r] : r
//   y[o]   = b ? b[o] - v : v
// rho is the natural-order (column-stacked) density matrix; with iperm the
// output is in the ordering's numbering.  When partials is non-null, block
// partial sums of |y|^2 go to partials[0 .. nb), nb = lindblad_blocks(d)
// (sum them with sum_partials).
void lindblad_apply(const LindbladOp &A, const double2 *rho, const int *iperm, int trow, double2 w,
                    const double2 *trace, const double2 *b, double2 *y, double2 *partials, hipStream_t s);
int lindblad_blocks(int d);

// rho[r] = x[iperm[r]]: a vector in the ordering's numbering back to the
// natural one.
void unpermute(int n, const int *iperm, const double2 *x, double2 *rho, hipStream_t s);

}  // namespace ss
