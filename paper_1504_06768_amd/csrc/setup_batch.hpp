// Batched set-up stages (setup_batch.hip).
#pragma once
#include "handle.hpp"

namespace ss {

// For every handle: the trace-row transform (trace) or the shift by
// o.sigma, the weight and trace row, and the symmetrised pattern S -- what
// the transform stage of ss_prepare computes, with the same results -- for
// the whole batch at once, kernels on s.  Options must have been validated.
void transform_batch(ss_liouv *hs, int count, bool trace, const ss_options &o, hipStream_t s);

// For every handle with its ordering: P A P^T, the diagonal positions, the
// trace positions and q0 (as prepare_permute and prepare_finish give them),
// and with ilu0 the factor's pattern (that of P A P^T, values at the
// sentinel) and its diagonal positions.  res[k].missing counts the rows of
// P A P^T without a diagonal entry: such a handle needs the explicit zero
// diagonal of prepare_permute before its factorisation (and its factor
// pattern again).
struct PermResult {
    int missing = 0;
};
void permute_batch(ss_liouv *hs, int count, bool ilu0, hipStream_t s, std::vector<PermResult> &res);

}  // namespace ss
