// ss_apply_noalloc: the operators of ss_apply for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The scratch the operators need -- the intermediate vector of the two
// triangular solves, complex64 copies of the operands in mixed precision,
// the status word and the control words of the row-group solves -- lives in
// one file-scope device array of NOALLOC_SCRATCH_BYTES.  Its device address
// is taken once per device with hipGetSymbolAddress, on the first call made
// with that device current, and kept; host code never passes the array's
// name to a kernel.  Every call on a device shares that device's array and
// leaves its last contents behind: what must start at zero or at the
// sentinel is set by a kernel at the start of each call, and calls that
// overlap on one device race.
#include <mutex>

#include "handle.hpp"

namespace ss {
void set_last_error(const std::string &msg);
}

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr size_t CONTROL_BYTES = 256;  // status word at 0, control words at 64
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
unsigned char *g_scratch[MAX_DEVICES] = {};

// the scratch array's device address on the current device
unsigned char *scratch_ptr() {
    int dev = 0;
    SS_HIP(hipGetDevice(&dev));
    SS_REQUIRE(dev >= 0 && dev < MAX_DEVICES, SS_E_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        SS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SS_REQUIRE(p != nullptr, SS_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch[dev] = static_cast<unsigned char *>(p);
    }
    return g_scratch[dev];
}

__global__ void k_zero_words(unsigned *p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0u;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// y[q] = x[idx[q]] (gather) or y[idx[q]] = x[q] (scatter)
template <typename T, bool SCATTER>
__global__ void k_permute_vec(int n, const int *idx, const T *x, T *y) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    if (SCATTER) y[idx[q]] = x[q];
    else y[q] = x[idx[q]];
}

// y = (L U)^-1 x with the row-group solves over the handle's schedules;
// x, y in precision T, ysol: n of scratch; for factors in the colour-class
// order under an RCM-ordered solve (h->split), xs and ys (n each) hold x and
// the result in the factors' order
template <typename T>
void precond(ss_liouv h, const ss::CsrBuf<T> &LU, const T *x, T *y, T *ysol, T *xs, T *ys, unsigned *status,
             unsigned *ctl, hipStream_t s) {
    const int n = h->n;
    const T *in = x;
    T *out = y;
    if (h->split) {
        k_permute_vec<T, false><<<ss::div_up(n, 256), 256, 0, s>>>(n, h->cp.get(), x, xs);
        SS_HIP(hipGetLastError());
        in = xs;
        out = ys;
    }
    ss::fill_sentinel<T>(n, ysol, s);
    ss::trsv_groups<T>(h->sched_lo, h->gate_lo.get(), false, LU.view(), in, ysol, out, ctl, status, nullptr, s);
    ss::trsv_groups<T>(h->sched_up, h->gate_up.get(), true, LU.view(), ysol, out, nullptr, ctl, status, nullptr, s);
    if (h->split) {
        k_permute_vec<T, true><<<ss::div_up(n, 256), 256, 0, s>>>(n, h->cp.get(), ys, y);
        SS_HIP(hipGetLastError());
    }
}

int run(ss_liouv L, int op, int prec, const double *x, double *y) {
    SS_REQUIRE(L != nullptr && x != nullptr && y != nullptr, SS_E_INVALID_ARG, "null argument");
    SS_REQUIRE(prec == SS_FP64 || prec == SS_MIXED, SS_E_INVALID_ARG, "unknown precision");
    SS_REQUIRE(op == SS_OP_SPMV_L || op == SS_OP_SPMV_APERM || op == SS_OP_APPLY_L || op == SS_OP_PRECOND,
               SS_E_INVALID_ARG, "ss_apply_noalloc: operator must be SPMV_L, SPMV_APERM, APPLY_L or PRECOND");
    SS_REQUIRE(ss::is_device_ptr(x) && ss::is_device_ptr(y), SS_E_INVALID_ARG,
               "ss_apply_noalloc: x and y must be device pointers");
    const bool natural = (op == SS_OP_SPMV_L || op == SS_OP_APPLY_L);
    SS_REQUIRE(!natural || prec == SS_FP64, SS_E_INVALID_ARG, "SPMV_L and APPLY_L run in fp64 only");
    SS_REQUIRE(natural || L->prepared, SS_E_STATE, "ss_prepare not called");
    SS_REQUIRE(natural || prec == SS_FP64 || L->p_opt.prec == SS_MIXED, SS_E_STATE,
               "complex64 operators exist only after a mixed-precision ss_prepare");
    SS_REQUIRE(op != SS_OP_PRECOND || L->sched_ready, SS_E_STATE,
               "ss_apply_noalloc: the handle has no device-wide triangular-solve schedules (prepare it for the "
               "device-wide path: n > 4096, a GMRES method or SS_FLAG_DEVICE_WIDE)");
    const int n = L->n;
    const size_t nn = (size_t)n;
    // scratch needed: control block, then the operator's vectors
    size_t need = CONTROL_BYTES;
    const size_t es = prec == SS_MIXED ? sizeof(float2) : sizeof(double2);
    if (op == SS_OP_PRECOND) need += (L->split ? 3 : 1) * align256(nn * es);
    if (prec == SS_MIXED) need += 2 * align256(nn * sizeof(float2));
    SS_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, SS_E_INVALID_ARG,
               "ss_apply_noalloc: system too large for the " + std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                   " MiB scratch array (needs " + std::to_string(need) + " bytes)");
    hipStream_t s = ss::stream_of(L);
    unsigned char *base = scratch_ptr();
    unsigned *status = reinterpret_cast<unsigned *>(base);
    unsigned *ctl = reinterpret_cast<unsigned *>(base + 64);
    unsigned char *vec = base + CONTROL_BYTES;
    k_zero_words<<<1, 64, 0, s>>>(status, 64);  // status word and control words
    SS_HIP(hipGetLastError());
    const double2 *xd = reinterpret_cast<const double2 *>(x);
    double2 *yd = reinterpret_cast<double2 *>(y);
    if (op == SS_OP_SPMV_L) {
        const ss::Csr<double2> A = L->L.view();
        ss::spmv<double2>(A, xd, yd, ss::spmv_group(A.n, A.nnz), s);
    } else if (op == SS_OP_APPLY_L) {
        ss::lindblad_apply(L->lin.view(), xd, nullptr, 0, ss::mk(0.0, 0.0), nullptr, nullptr, yd, nullptr, s);
    } else if (prec == SS_FP64) {
        if (op == SS_OP_SPMV_APERM) {
            const ss::Csr<double2> A = L->Ap.view();
            ss::spmv<double2>(A, xd, yd, ss::spmv_group(A.n, A.nnz), s);
        } else {
            double2 *v0 = reinterpret_cast<double2 *>(vec);
            double2 *v1 = reinterpret_cast<double2 *>(vec + align256(nn * sizeof(double2)));
            double2 *v2 = reinterpret_cast<double2 *>(vec + 2 * align256(nn * sizeof(double2)));
            precond<double2>(L, L->LU, xd, yd, v0, v1, v2, status, ctl, s);
        }
    } else {
        float2 *ysol = reinterpret_cast<float2 *>(vec);
        float2 *xs = reinterpret_cast<float2 *>(vec + align256(nn * sizeof(float2)));
        float2 *ys = reinterpret_cast<float2 *>(vec + 2 * align256(nn * sizeof(float2)));
        if (op == SS_OP_PRECOND) vec += (L->split ? 3 : 1) * align256(nn * sizeof(float2));
        float2 *xf = reinterpret_cast<float2 *>(vec);
        float2 *yf = reinterpret_cast<float2 *>(vec + align256(nn * sizeof(float2)));
        ss::convert<float2, double2>(n, xd, xf, nullptr, s);
        if (op == SS_OP_SPMV_APERM) {
            const ss::Csr<float2> A = L->Ap32.view();
            ss::spmv<float2>(A, xf, yf, ss::spmv_group(A.n, A.nnz), s);
        } else {
            precond<float2>(L, L->LU32, xf, yf, ysol, xs, ys, status, ctl, s);
        }
        ss::convert<double2, float2>(n, yf, yd, nullptr, s);
    }
    unsigned st = 0;
    SS_HIP(hipMemcpyAsync(&st, status, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    SS_REQUIRE(!(st & ss::STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "triangular solve: dependency wait timed out");
    return SS_OK;
}

}  // namespace

extern "C" int ss_apply_noalloc(ss_liouv L, int32_t op, int32_t prec, const double *x, double *y) {
    (void)hipGetLastError();
    try {
        return run(L, op, prec, x, y);
    } catch (const ss::Error &e) {
        ss::set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        ss::set_last_error(e.what());
        return SS_E_HIP;
    }
}
