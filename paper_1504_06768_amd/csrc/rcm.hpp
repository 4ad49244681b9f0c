// Ordering (rcm.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

// pattern of A + A^T (values set to 1)
void symmetrize_pattern(const CsrBuf<double2> &A, CsrBuf<double2> &S, hipStream_t s);

// reverse Cuthill-McKee of a symmetric pattern: perm[new] = old, iperm[old] = new
void rcm_order(const CsrBuf<double2> &S, DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s);

// Many graphs at once, one workgroup each (graphs of up to RCM_BLOCK_MAX_N
// nodes): the same ordering as rcm_order.
constexpr int RCM_BLOCK_MAX_N = 65536;
struct RcmJob {
    int n;
    const int *rowptr, *col;  // symmetric pattern, sorted rows
    int *deg, *pos_of, *owner, *order, *offs;  // scratch: n, n, n, n, n + 1
    int *perm, *iperm;                          // results
};
struct RcmScratch {
    DevBuf<int> deg, pos_of, owner, order, offs;
    void alloc(int n);
    RcmJob job(const CsrBuf<double2> &S, int *perm, int *iperm) const;
};
bool rcm_batchable(int n);
void rcm_batch(const RcmJob *jobs, int count, hipStream_t s);

void identity_order(int n, DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s);

// Colour classes over a base order (colour.hip): the greedy colouring of the
// symmetric pattern S visited in a seeded random order, classes in
// increasing colour, each in base order.  Returns the number of colours;
// class_ptr (optional) receives where each class starts in the new order,
// then n.
int colour_order(const CsrBuf<double2> &S, const DevBuf<int> &base_perm, const DevBuf<int> &base_iperm,
                 DevBuf<int> &perm, DevBuf<int> &iperm, hipStream_t s, std::vector<int> *class_ptr = nullptr);

// B = P A P^T (rows and columns permuted, rows sorted)
void permute_matrix(const CsrBuf<double2> &A, const int *perm, const int *iperm, CsrBuf<double2> &B, hipStream_t s);

// y[q] = x[idx[q]]
void gather(int n, const int *idx, const double2 *x, double2 *y, hipStream_t s);

}  // namespace ss
