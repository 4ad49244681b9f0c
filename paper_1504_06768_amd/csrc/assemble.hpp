// Liouvillian assembly (assemble.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

constexpr int MAX_COPS = 16;

struct OpPair {
    Csr<double2> C;   // collapse operator
    Csr<double2> Ct;  // its transpose (C^T, not conjugated)
};

// L of eq. (lindblad) as an n x n CSR (n = N^2), exact zeros dropped.
void assemble_liouvillian(const ss_csr_z *H, const ss_csr_z *c_ops, int n_cops, int64_t N, hipStream_t s,
                          CsrBuf<double2> &L);

}  // namespace ss
