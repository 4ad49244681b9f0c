// Stable bucket sort of positions by small integer keys (bucket.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

// Positions 0..n-1 in (key[p], p) order, keys in [0, nkeys):
//   out[q]          = items ? items[p] : p   for the q-th position p,
//   inv[out[q]]     = q                      (if inv is not null),
//   starts[k]       = first q of key k, starts[nkeys] = n (if not null).
// Deterministic; one wavefront per chunk of positions, no contended atomics.
void bucket_sort(int n, const int *key, int nkeys, const int *items, int *out, int *inv, int *starts,
                 hipStream_t s);

}  // namespace ss
