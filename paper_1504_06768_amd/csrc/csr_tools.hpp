// Declarations of the generic CSR kernels (csr_tools.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

// Validate a caller CSR (host or device arrays) and copy it to the device.
void upload_csr(const ss_csr_z *in, int64_t N, CsrBuf<double2> &out, hipStream_t s, const char *what);

// Sort the entries of every row by column (columns unique within a row).
template <typename T>
void sort_rows(int n, const int *rowptr, const int *col_in, const T *val_in, int *col_out, T *val_out,
               hipStream_t s);

// A^T as CSR with sorted rows; pattern only when with_values is false.
template <typename T>
void transpose(const CsrBuf<T> &A, CsrBuf<T> &At, hipStream_t s, bool with_values);

// diag[r] = position of (r, r) or -1; returns the number of rows without one.
int find_diagonal(int n, const int *rowptr, const int *col, int *diag, hipStream_t s);

// Bandwidth B = ub + lb + 1 and profile P = up + lp of a CSR pattern.
void bandwidth_profile(int n, const int *rowptr, const int *col, int64_t *B, int64_t *P, hipStream_t s);

}  // namespace ss
