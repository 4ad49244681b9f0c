// Problem transforms (transform.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

// *d_out = mean of the diagonal of L (device scalar).
void mean_diagonal(const CsrBuf<double2> &L, double2 *d_out, hipStream_t s);

// A = L + w T, T = ones in row 0 at columns k (d + 1); w read from device.
void make_modified(const CsrBuf<double2> &L, int d, const double2 *d_w, CsrBuf<double2> &A, hipStream_t s);

// A = L - sigma I.
void make_shifted(const CsrBuf<double2> &L, double sigma, CsrBuf<double2> &A, hipStream_t s);

}  // namespace ss
