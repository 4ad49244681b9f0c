// Liouvillian assembly (assemble.hip).
#pragma once
#include "lindblad.hpp"

namespace ss {

struct OpPair {
    Csr<double2> C;   // collapse operator
    Csr<double2> Ct;  // its transpose (C^T, not conjugated)
};

// L of eq. (lindblad) as an n x n CSR (n = N^2), exact zeros dropped.  The
// d x d operators it is built from (Gpre, Gpost, C_k) go to `ops` for the
// matrix-free application of L.
void assemble_liouvillian(const ss_csr_z *H, const ss_csr_z *c_ops, int n_cops, int64_t N, hipStream_t s,
                          CsrBuf<double2> &L, LindbladBuf &ops);

}  // namespace ss
