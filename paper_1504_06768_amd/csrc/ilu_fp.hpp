// Fixed-point ILU(0) (ilu.hip).
#pragma once
#include "ilu.hpp"

namespace ss {

// The zero-fill factors as the fixed point of (LU)_ij = a_ij on A's pattern,
// after `sweeps` synchronous sweeps from l_ij = a_ij / a_jj, u_ij = a_ij
// (Chow and Patel 2015); exact once the sweeps cover the longest chain of
// dependencies.  guarded: pivots guarded in the last sweep.
IluResult ilu0_fixed_point(const CsrBuf<double2> &A, const int *diag, int sweeps, double detect, double boost,
                           CsrBuf<double2> &LU, hipStream_t s);

}  // namespace ss
