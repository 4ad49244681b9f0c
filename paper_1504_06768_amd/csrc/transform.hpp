// Problem transforms (transform.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

// *d_out = mean of the diagonal of L (device scalar).
void mean_diagonal(const CsrBuf<double2> &L, double2 *d_out, hipStream_t s);

// Row index k (d + 1) that carries T: population `forced` if >= 0, else the
// population row with the smallest |L_rr| (lowest k among ties).
int pick_trace_row(const CsrBuf<double2> &L, int d, int forced, hipStream_t s);

// A = L + w T, T = ones in row rt at columns k (d + 1); w read from device.
void make_modified(const CsrBuf<double2> &L, int d, int rt, const double2 *d_w, CsrBuf<double2> &A, hipStream_t s);

// A = L - sigma I.
void make_shifted(const CsrBuf<double2> &L, double sigma, CsrBuf<double2> &A, hipStream_t s);

}  // namespace ss
