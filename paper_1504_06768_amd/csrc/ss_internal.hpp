// Internal declarations shared by the solver's HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ss.h"

namespace ss {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// A failed HIP call also leaves its code behind as the calling thread's
// "last error", which the hipGetLastError() that follows a kernel launch
// would report as that launch's failure.  Every failure is therefore read
// back (cleared) where it is handled: SS_HIP clears before it throws, and a
// call whose failure is tolerated goes through hip_quiet.
inline hipError_t hip_quiet(hipError_t e) {
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

#define SS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (void)hipGetLastError();                                                   \
            throw ::ss::Error(e_ == hipErrorOutOfMemory ? SS_E_OOM : SS_E_HIP,         \
                              std::string(#call) + ": " + hipGetErrorString(e_));      \
        }                                                                              \
    } while (0)

#define SS_REQUIRE(cond, code, msg)                                                    \
    do {                                                                               \
        if (!(cond)) throw ::ss::Error((code), (msg));                                 \
    } while (0)

// ------------------------------------------------------------ device memory
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// stream on which the calling thread issues its work: blocks allocated
// meanwhile are tagged with it, and their release waits (through an event on
// it) for the work queued there, never for the host
void set_current_stream(hipStream_t s);
hipStream_t current_stream();
// Releases by this thread, during the scope, of blocks tagged with stream s
// share one event recorded on s when the scope opens (instead of one event
// per block): for tearing down an object whose work on s is all queued.
struct FreeScope {
    explicit FreeScope(hipStream_t s);
    ~FreeScope();
    FreeScope(const FreeScope &) = delete;
    FreeScope &operator=(const FreeScope &) = delete;

  private:
    hipEvent_t ev_ = nullptr, prev_ev = nullptr;
    hipStream_t prev_s = nullptr;
};
// the calling thread's current stream is s for the lifetime of the scope
struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s) : prev(current_stream()) { set_current_stream(s); }
    ~StreamScope() { set_current_stream(prev); }
    StreamScope(const StreamScope &) = delete;
    StreamScope &operator=(const StreamScope &) = delete;
};
// release every cached block (waits for their last uses)
void trim_device_cache();
// caller allocator for the underlying blocks (NULL: hipMalloc / hipFree)
void set_allocator(ss_alloc_fn a, ss_free_fn f, void *ctx);
// a stream from the library's fixed pool
hipStream_t pooled_stream();

template <typename T>
class DevBuf {
  public:
    DevBuf() = default;
    explicit DevBuf(size_t n) { resize(n); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
        return *this;
    }
    void resize(size_t n) {
        if (n == n_ && p_) return;
        release();
        n_ = n;
        p_ = static_cast<T *>(dev_alloc(sizeof(T) * (n ? n : 1)));
    }
    void release() {
        if (p_) dev_free(p_);
        p_ = nullptr;
        n_ = 0;
    }
    T *get() const { return p_; }
    size_t size() const { return n_; }
    size_t bytes() const { return n_ * sizeof(T); }

  private:
    T *p_ = nullptr;
    size_t n_ = 0;
};

// ----------------------------------------------------------- complex types
// complex128 = double2, complex64 = float2, (x, y) = (re, im)
template <typename T> struct RealOf;
template <> struct RealOf<double2> { using type = double; };
template <> struct RealOf<float2> { using type = float; };

__host__ __device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline float2 mkf(float a, float b) { return make_float2(a, b); }

template <typename T> __host__ __device__ inline T cadd(T a, T b) { T r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename T> __host__ __device__ inline T csub(T a, T b) { T r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename T> __host__ __device__ inline T cmul(T a, T b) {
    T r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename T> __host__ __device__ inline T cmulc(T a, T b) {
    T r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename T> __host__ __device__ inline T cconj(T a) { T r; r.x = a.x; r.y = -a.y; return r; }
template <typename T, typename R> __host__ __device__ inline T cscale(T a, R s) { T r; r.x = a.x * s; r.y = a.y * s; return r; }
// a / b, scaled to avoid overflow in |b|^2 for the magnitudes used here
template <typename T> __host__ __device__ inline T cdiv(T a, T b) {
    using R = typename RealOf<T>::type;
    R s = fabs(b.x) + fabs(b.y);
    R bx = b.x / s, by = b.y / s;
    R den = bx * bx + by * by;
    T r;
    r.x = ((a.x / s) * bx + (a.y / s) * by) / den;
    r.y = ((a.y / s) * bx - (a.x / s) * by) / den;
    return r;
}
template <typename T> __host__ __device__ inline typename RealOf<T>::type cabs2(T a) { return a.x * a.x + a.y * a.y; }
template <typename T> __host__ __device__ inline typename RealOf<T>::type cabs1(T a) { return fabs(a.x) + fabs(a.y); }
// Loads and stores through address-space-1 (global) pointers.  A pointer
// read from memory is generic to the compiler, and a plain access through it
// becomes a flat instruction, which also counts against the LDS wait counter:
// every wait for an LDS access would then wait for every global load in
// flight.  Vector types go through clang vector types so that the copy does
// not fall back to a generic reference.
template <typename U> struct GlobalRaw { using type = U; };
template <> struct GlobalRaw<float2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct GlobalRaw<double2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct GlobalRaw<int4> { typedef int __attribute__((ext_vector_type(4))) type; };
template <typename U>
__device__ __forceinline__ U gld(const U *p) {
    using R = typename GlobalRaw<U>::type;
    const R r = *(const __attribute__((address_space(1))) R *)p;
    return __builtin_bit_cast(U, r);
}
template <typename U>
__device__ __forceinline__ void gst(U *p, const U &v) {
    using R = typename GlobalRaw<U>::type;
    *(__attribute__((address_space(1))) R *)p = __builtin_bit_cast(R, v);
}

template <typename T> __host__ __device__ inline T czero() { T r; r.x = 0; r.y = 0; return r; }

__host__ __device__ inline float2 to_c64(double2 a) { return make_float2((float)a.x, (float)a.y); }
__host__ __device__ inline double2 to_c128(float2 a) { return make_double2((double)a.x, (double)a.y); }
template <typename T> __device__ inline T from_c128(double2 a);
template <> __device__ inline double2 from_c128<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_c128<float2>(double2 a) { return to_c64(a); }
__device__ inline double2 widen(double2 a) { return a; }
__device__ inline double2 widen(float2 a) { return to_c128(a); }

// ------------------------------------------------------ sparse matrix views
template <typename T>
struct Csr {  // non-owning device view
    int n = 0;
    int nnz = 0;
    const int *rowptr = nullptr;
    const int *col = nullptr;
    const T *val = nullptr;
};

template <typename T>
struct CsrBuf {  // owning device storage
    int n = 0;
    int nnz = 0;
    DevBuf<int> rowptr, col;
    DevBuf<T> val;
    void alloc(int n_, int nnz_) {
        n = n_;
        nnz = nnz_;
        rowptr.resize((size_t)n + 1);
        col.resize((size_t)nnz);
        val.resize((size_t)nnz);
    }
    Csr<T> view() const {
        Csr<T> v;
        v.n = n; v.nnz = nnz; v.rowptr = rowptr.get(); v.col = col.get(); v.val = val.get();
        return v;
    }
    size_t bytes() const { return rowptr.bytes() + col.bytes() + val.bytes(); }
};

// -------------------------------------------------------------- utilities
inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// exclusive scan of n ints: out[0..n], out[n] = total (in == out allowed);
// returns the total (synchronises the stream) when want_total is true
int64_t scan_exclusive(const int *in, int *out, int64_t n, hipStream_t s, bool want_total);

// copy helpers
template <typename T>
inline void d2h(T *h, const T *d, size_t n, hipStream_t s) {
    SS_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
}
template <typename T>
inline void h2d(T *d, const T *h, size_t n, hipStream_t s) {
    SS_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
}

bool is_device_ptr(const void *p);

// ----------------------------------------------- device-wide bounded waits
// Device status word bits, set by kernels, read by the host after a solve.
enum : unsigned { STATUS_SPIN_TIMEOUT = 1u, STATUS_ZERO_PIVOT = 2u, STATUS_OVERFLOW = 4u };

// Large enough that a healthy dependency wait never reaches it, small enough
// that a broken one ends in seconds.
constexpr unsigned SPIN_LIMIT = 1u << 20;

// Sentinel bit patterns marking "not yet written" in the sync-free kernels;
// computed NaNs are canonicalised so they never equal a sentinel.
constexpr uint64_t SENT_F64 = 0x7FF4DEADBEEF1234ull;
constexpr uint32_t SENT_F32 = 0x7FA5EEDDu;
constexpr uint64_t SENT_F32x2 = ((uint64_t)SENT_F32 << 32) | SENT_F32;

}  // namespace ss
