// Batched set-up stages (setup_batch.hip).
#pragma once
#include "handle.hpp"

namespace ss {

// For every handle: the trace-row transform (trace) or the shift by
// o.sigma, the weight and trace row, and the symmetrised pattern S -- what
// the transform stage of ss_prepare computes, with the same results -- for
// the whole batch at once, kernels on s.  Options must have been validated.
void transform_batch(ss_liouv *hs, int count, bool trace, const ss_options &o, hipStream_t s);

}  // namespace ss
