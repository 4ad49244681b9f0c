// Device helpers for the sync-free (dependency-polling) kernels: ILU
// factorisation and sparse triangular solves.
//
// A row's result is published with relaxed agent-scope atomic stores into an
// array pre-filled with a sentinel bit pattern; a dependent row polls the
// values it needs with relaxed agent-scope atomic loads until they differ
// from the sentinel.  No flag/data ordering is needed because the data itself
// is the flag.  Workgroups take an ordered index from an atomic counter, so
// every row a workgroup waits on belongs to a workgroup that has already
// started; waits are additionally bounded (SPIN_LIMIT) and report a status
// bit instead of hanging.
#pragma once
#include "ss_internal.hpp"

namespace ss {

__device__ inline unsigned long long ld_relaxed(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_relaxed(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long canon_bits(double v) {
    return isnan(v) ? 0x7FF8000000000000ull : (unsigned long long)__double_as_longlong(v);
}
__device__ inline unsigned canon_bits(float v) {
    return isnan(v) ? 0x7FC00000u : (unsigned)__float_as_uint(v);
}

// ---- complex128: two 64-bit words, each polled separately
__device__ inline bool try_load(const double2 *p, double2 &out) {
    const unsigned long long *q = reinterpret_cast<const unsigned long long *>(p);
    const unsigned long long x = ld_relaxed(q);
    const unsigned long long y = ld_relaxed(q + 1);
    if (x == SENT_F64 || y == SENT_F64) return false;
    out.x = __longlong_as_double((long long)x);
    out.y = __longlong_as_double((long long)y);
    return true;
}
__device__ inline void publish(double2 *p, double2 v) {
    unsigned long long *q = reinterpret_cast<unsigned long long *>(p);
    st_relaxed(q, canon_bits(v.x));
    st_relaxed(q + 1, canon_bits(v.y));
}
__device__ inline void set_sentinel(double2 *p) {
    unsigned long long *q = reinterpret_cast<unsigned long long *>(p);
    q[0] = SENT_F64;
    q[1] = SENT_F64;
}

// ---- complex64: one 64-bit word
__device__ inline bool try_load(const float2 *p, float2 &out) {
    const unsigned long long w = ld_relaxed(reinterpret_cast<const unsigned long long *>(p));
    if ((unsigned)(w & 0xffffffffull) == SENT_F32 || (unsigned)(w >> 32) == SENT_F32) return false;
    out.x = __uint_as_float((unsigned)(w & 0xffffffffull));
    out.y = __uint_as_float((unsigned)(w >> 32));
    return true;
}
__device__ inline void publish(float2 *p, float2 v) {
    const unsigned long long w = ((unsigned long long)canon_bits(v.y) << 32) | canon_bits(v.x);
    st_relaxed(reinterpret_cast<unsigned long long *>(p), w);
}
__device__ inline void set_sentinel(float2 *p) {
    *reinterpret_cast<unsigned long long *>(p) = SENT_F32x2;
}

__device__ inline bool aborted(const unsigned *status) {
    return (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & STATUS_SPIN_TIMEOUT) != 0;
}

// Poll until published (bounded).  On timeout, flag the status word and
// return 0; once any wait has timed out every other wait gives up at once,
// so a broken dependency chain ends the kernel quickly instead of hanging.
template <typename T>
__device__ inline T wait_load(const T *p, unsigned *status) {
    T v;
    unsigned spins = 0;
    while (!try_load(p, v)) {
        ++spins;
        if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(status))) {
            atomicOr(status, STATUS_SPIN_TIMEOUT);
            return czero<T>();
        }
        if (spins > 32) __builtin_amdgcn_s_sleep(1);
    }
    return v;
}

// Ordered workgroup index: the k-th workgroup to start gets k - base.
__device__ inline unsigned ordered_block(unsigned *ctr, unsigned base) {
    __shared__ unsigned sbid;
    if (threadIdx.x == 0) sbid = atomicAdd(ctr, 1u) - base;
    __syncthreads();
    return sbid;
}

// Host side of an ordered-block counter: tracks how many workgroups have
// taken an index so each launch knows its base.
struct BlockCounter {
    DevBuf<unsigned> ctr;
    unsigned next = 0;
    void init(hipStream_t s) {
        ctr.resize(1);
        SS_HIP(hipMemsetAsync(ctr.get(), 0, sizeof(unsigned), s));
        next = 0;
    }
    unsigned take(unsigned blocks) {
        const unsigned b = next;
        next += blocks;
        return b;
    }
};

}  // namespace ss
