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

// Batched assembly: systems k < count with H[k] (N_k = H[k].n) and the
// n_cops[k] matrices c_ops[k][0..), every array device-resident and
// N_k <= ASM_BATCH_MAX_N; out[k] receives L and the d x d operators, its
// blocks tagged with out[k].tag (the stream the handle works on).  The
// kernels run on s; on return the work is complete.  Throws on the first
// invalid system (nothing is usable then).
constexpr int64_t ASM_BATCH_MAX_N = 1024;
constexpr size_t ASM_BATCH_STAGE_BYTES = size_t(512) << 20;

struct AsmTarget {
    CsrBuf<double2> *L;
    LindbladBuf *lin;
    hipStream_t tag;
};

bool batch_assembly_fits(int64_t N);
// (on_device: the caller guarantees every array is device memory)
void assemble_batch(int count, const ss_csr_z *H, const ss_csr_z *const *c_ops, const int *n_cops,
                    const AsmTarget *out, hipStream_t s, bool on_device = false);

}  // namespace ss
