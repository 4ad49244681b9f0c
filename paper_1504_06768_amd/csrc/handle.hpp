// The Liouvillian handle and the set-up / solve drivers (solve.hip).
#pragma once
#include "blas.hpp"
#include "ilu.hpp"
#include "krylov.hpp"

struct ss_liouv_s {
    int64_t N = 0;
    int d = 0;
    int n = 0;
    hipStream_t own_stream = nullptr;
    ss::CsrBuf<double2> L;  // assembled Liouvillian, natural order

    // results of the set-up stage (ss_prepare)
    bool prepared = false;
    int p_method = -1;
    ss_options p_opt{};
    ss::CsrBuf<double2> A;     // L~ or L - sigma I, natural order
    ss::CsrBuf<double2> S;     // symmetrised pattern of A
    ss::DevBuf<int> perm, iperm;
    ss::CsrBuf<double2> Ap;    // P A P^T (fp64)
    ss::CsrBuf<float2> Ap32;   // P A P^T (complex64, mixed precision)
    ss::DevBuf<int> diag;      // diagonal positions in Ap
    ss::CsrBuf<double2> LU;    // ILU factors (fp64)
    ss::CsrBuf<float2> LU32;   // ILU factors rounded to complex64
    ss::DevBuf<int> lu_diag;   // diagonal positions in LU
    ss::DevBuf<int> tpos;      // permuted positions of the diagonal of rho
    ss::DevBuf<double2> d_w;   // trace-row weight (device)
    double2 w = {0, 0};
    int trow = 0;              // row of L~ carrying the trace row T
    int q0 = 0;                // its position after the ordering
    int guarded = 0;
    int diag_added = 0;        // explicit zero diagonals added to Ap
    double t_setup_ms = 0;
};

namespace ss {

hipStream_t stream_of(ss_liouv h);
void prepare(ss_liouv h, int method, const ss_options &o);
int solve(ss_liouv h, int method, double tol, const ss_options &o, double *rho_out, ss_info *info);

}  // namespace ss
