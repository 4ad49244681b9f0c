// Start vectors of the inverse-power driver (solve.hip, setup_batch.hip).
#pragma once
#include "ss_internal.hpp"

namespace ss {

// ------------------------------------------------------- random start
// Element r = i + d j (column stacking) of the random trace-1 Hermitian start
// matrix of inverse power: 1/d on the diagonal; above it c (u + i v) with u,
// v uniform in [-1, 1) from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
// of the pair's index and the seed, c = 0.5 / d; below it the conjugate.
__host__ __device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline double2 random_start_value(int d, int r, uint64_t seed) {
    const int i = r % d, j = r / d;
    if (i == j) return make_double2(1.0 / d, 0.0);
    const int a = i < j ? i : j, b = i < j ? j : i;
    const uint64_t key = splitmix64(seed ^ splitmix64((uint64_t)a * (uint64_t)d + (uint64_t)b));
    const double u = (double)(key >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    const double v = (double)(splitmix64(key) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    const double c = 0.5 / d;
    return make_double2(c * u, i < j ? c * v : -c * v);
}

}  // namespace ss
