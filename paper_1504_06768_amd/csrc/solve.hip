// Set-up and solve drivers.
//
// Set-up (ss_prepare): problem transform (trace row or shift), symmetrised
// pattern, reverse Cuthill-McKee, P A P^T, ILU factors -- all on the device.
//
// Trace-row driver (section "Direct factorization", eq. linear, solved
// iteratively as in section "Iterative Solvers", eq. modified): fp64
// iterative refinement around the inner Krylov solve,
//     r = b - L~ x   (fp64),  solve L~ d = r / ||r||  (inner precision),
//     x += ||r|| d   (fp64),
// until ||L vec(rho)||_2 <= tol with rho = unvec(x) / Tr x.  With fp64 inner
// solves this is plain preconditioned Krylov plus a residual check.
//
// Inverse-power driver (the doubly-iterative inverse-power method, section
// "Iterative Solvers", eqs. inverse and inverseiter): the normalised step
// x <- (L - sigma I)^-1 x / || . || is taken in the equivalent correction
// form  (L - sigma I)^-1 x = -(x - d) / sigma  with  (L - sigma I) d = L x,
// i.e. x <- x - d, then x <- x / Tr x.  The direction is the same; the inner
// right-hand side is the (trace-free) residual, which stays meaningful when
// the inner solve runs in complex64, where sigma = 1e-15 cannot be
// represented next to O(1) diagonal entries.  Inner tolerance one decade
// below the outer one (relative to the current residual).
#include <chrono>
#include <thread>
#include <cstdio>
#include <cstdlib>

#include "start.hpp"
#include "assemble.hpp"
#include "csr_tools.hpp"
#include "handle.hpp"
#include "ilu_fp.hpp"
#include "rcm.hpp"
#include "setup_batch.hpp"
#include "transform.hpp"
#include "wgsolve.hpp"

namespace ss {

static thread_local hipStream_t tls_stream = nullptr;

void set_thread_stream(hipStream_t s) { tls_stream = s; }
hipStream_t stream_peek(ss_liouv h) { return tls_stream ? tls_stream : h->own_stream; }

hipStream_t stream_of(ss_liouv h) {
    hipStream_t s = tls_stream ? tls_stream : h->own_stream;
    set_current_stream(s);
    return s;
}

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

__global__ void k_trace_positions(int d, const int *iperm, int *tpos) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < d) tpos[k] = iperm[(int64_t)k * (d + 1)];
}

__global__ void k_copy_d2(const double2 *src, double2 *dst) { *dst = *src; }

template <typename TD>
__global__ void k_round_vals(int64_t n, const double2 *a, TD *b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = from_c128<TD>(a[i]);
}

static void copy_pattern_c64(const CsrBuf<double2> &a, CsrBuf<float2> &b, hipStream_t s) {
    b.alloc(a.n, a.nnz);
    SS_HIP(hipMemcpyAsync(b.rowptr.get(), a.rowptr.get(), sizeof(int) * (a.n + 1), hipMemcpyDeviceToDevice, s));
    if (a.nnz) {
        SS_HIP(hipMemcpyAsync(b.col.get(), a.col.get(), sizeof(int) * a.nnz, hipMemcpyDeviceToDevice, s));
        round_to_c64(a.nnz, a.val.get(), b.val.get(), s);
    }
}

static bool is_trace(int method) { return method == SS_TRACE_BICGSTAB || method == SS_TRACE_GMRES; }
static bool is_gmres(int method) { return method == SS_TRACE_GMRES || method == SS_INVPOW_GMRES; }

// The set-up in stages, so that a batch can run the ordering and the ILU(0)
// of all its systems in one launch each (one workgroup per system).
static void check_options(int method, const ss_options &o) {
    SS_REQUIRE(method >= 0 && method <= 3, SS_E_INVALID_ARG, "unknown method");
    SS_REQUIRE(o.prec == SS_FP64 || o.prec == SS_MIXED, SS_E_INVALID_ARG, "unknown precision");
    SS_REQUIRE(o.ilu == SS_ILU0 || o.ilu == SS_ILUT, SS_E_INVALID_ARG, "unknown ILU kind");
    SS_REQUIRE(o.ordering == SS_ORDER_RCM || o.ordering == SS_ORDER_NATURAL || o.ordering == SS_ORDER_COLOUR,
               SS_E_INVALID_ARG, "unknown ordering");
    SS_REQUIRE(o.ilu_sweeps >= 0, SS_E_INVALID_ARG, "ilu_sweeps must be >= 0");
    SS_REQUIRE(o.ilu_sweeps == 0 || o.ilu == SS_ILU0, SS_E_INVALID_ARG, "ilu_sweeps applies to SS_ILU0 only");
}

static void prepare_transform(ss_liouv h, int method, const ss_options &o, hipStream_t s) {
    check_options(method, o);
    h->prepared = false;
    const int d = h->d;
    h->d_w.resize(1);
    if (is_trace(method)) {
        if (o.weight != 0.0) {
            const double2 w = mk(o.weight, 0.0);
            h2d(h->d_w.get(), &w, 1, s);
        } else {
            mean_diagonal(h->L, h->d_w.get(), s);
        }
        d2h(&h->w, h->d_w.get(), 1, s);
        if (h->w.x == 0.0 && h->w.y == 0.0) {
            // zero mean diagonal (e.g. N = 1, where L = 0, or no dissipation):
            // any nonzero weight gives the same rho
            SS_REQUIRE(o.weight == 0.0, SS_E_INVALID_ARG, "trace-row weight is zero");
            h->w = mk(1.0, 0.0);
            h2d(h->d_w.get(), &h->w, 1, s);
        }
        SS_REQUIRE(o.trace_row < d, SS_E_INVALID_ARG, "trace_row must be < N");
        h->trow = pick_trace_row(h->L, d, o.trace_row, s);
        make_modified(h->L, d, h->trow, h->d_w.get(), h->A, s);
    } else {
        h->w = mk(0.0, 0.0);
        h->trow = 0;
        make_shifted(h->L, o.sigma, h->A, s);
    }
    symmetrize_pattern(h->A, h->S, s);
    h->perm.resize((size_t)h->n);
    h->iperm.resize((size_t)h->n);
}

// Rows whose diagonal is structurally zero (e.g. the ground-state population
// of a Jaynes-Cummings system when the trace row sits elsewhere) get an
// explicit zero diagonal entry, so the zero-fill ILU has a pivot position;
// the matrix itself is unchanged.
static void add_zero_diagonal(ss_liouv h, hipStream_t s) {
    CsrBuf<double2> aug;
    make_shifted(h->Ap, 0.0, aug, s);
    h->Ap = std::move(aug);
    const int still = find_diagonal(h->n, h->Ap.rowptr.get(), h->Ap.col.get(), h->diag.get(), s);
    SS_REQUIRE(still == 0, SS_E_ZERO_PIVOT, "could not give every row a diagonal entry");
}

__global__ void k_rows_by_rcm(int n, const int *rcm_perm, const int *iperm, int *lorder) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) lorder[p] = iperm[rcm_perm[p]];
}

// cp[lorder[p]] = p
__global__ void k_invert(int n, const int *lorder, int *cp) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) cp[lorder[p]] = p;
}

// RCM order -> colour-class order (SS_ORDER_COLOUR).  lorder keeps, for
// each RCM position, the row it became: rows inside a level of the factors'
// schedules are taken in RCM order, so that the rows running together
// gather from nearby parts of every class.  With keep_rcm (the device-wide
// path) perm and iperm stay the RCM order, which the Krylov iteration and
// its SpMV keep, and cp maps the factors' rows to it; otherwise the whole
// solve runs in the colour-class order.
static void recolour(ss_liouv h, bool keep_rcm, hipStream_t s) {
    DevBuf<int> perm, iperm;
    h->colours = colour_order(h->S, h->perm, h->iperm, perm, iperm, s, &h->class_ptr);
    const int n = h->n;
    h->lorder.resize((size_t)std::max(n, 1));
    if (n) {
        k_rows_by_rcm<<<div_up(n, 256), 256, 0, s>>>(n, h->perm.get(), iperm.get(), h->lorder.get());
        SS_HIP(hipGetLastError());
    }
    h->split = keep_rcm;
    if (keep_rcm) {
        h->cp.resize((size_t)std::max(n, 1));
        if (n) {
            k_invert<<<div_up(n, 256), 256, 0, s>>>(n, h->lorder.get(), h->cp.get());
            SS_HIP(hipGetLastError());
        }
    } else {
        h->perm = std::move(perm);
        h->iperm = std::move(iperm);
    }
}

static void prepare_permute(ss_liouv h, hipStream_t s) {
    const int n = h->n;
    permute_matrix(h->A, h->perm.get(), h->iperm.get(), h->Ap, s);
    h->diag.resize((size_t)n);
    h->diag_added = find_diagonal(n, h->Ap.rowptr.get(), h->Ap.col.get(), h->diag.get(), s);
    if (h->diag_added > 0) add_zero_diagonal(h, s);
}

static void prepare_finish(ss_liouv h, int method, const ss_options &o, hipStream_t s, double t0,
                           bool batched = false) {
    const int n = h->n, d = h->d;
    if (o.ilu == SS_ILU0 && !batched && !h->split) {
        h->lu_diag.resize((size_t)n);
        if (n) SS_HIP(hipMemcpyAsync(h->lu_diag.get(), h->diag.get(), sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    }
    if (o.prec == SS_MIXED) {
        if (!batched) {  // (a batch makes these copies together)
            copy_pattern_c64(h->Ap, h->Ap32, s);
            copy_pattern_c64(h->LU, h->LU32, s);
        }
    } else {
        h->Ap32 = CsrBuf<float2>();
        h->LU32 = CsrBuf<float2>();
    }
    if (!batched) {
        h->tpos.resize((size_t)d);
        k_trace_positions<<<div_up(d, 256), 256, 0, s>>>(d, h->iperm.get(), h->tpos.get());
        SS_HIP(hipGetLastError());
        d2h(&h->q0, h->iperm.get() + h->trow, 1, s);
    }
    h->p_method = method;
    h->p_opt = o;
    h->prepared = true;
    h->t_setup_ms = now_ms() - t0;
}

void prepare(ss_liouv h, int method, const ss_options &o) {
    hipStream_t s = stream_of(h);
    const double t0 = now_ms();
    const bool dbg = std::getenv("SS_DEBUG") != nullptr;
    double tp = t0;
    auto phase = [&](const char *name) {
        if (!dbg) return;
        SS_HIP(hipStreamSynchronize(s));
        const double t = now_ms();
        std::fprintf(stderr, "[ss] prepare %-10s %.3f ms\n", name, t - tp);
        tp = t;
    };
    prepare_transform(h, method, o, s);
    phase("transform");
    // device-wide solves use level schedules of the factors
    const bool want_sched = !use_workgroup(h, method, o) && (int64_t)h->n * (int64_t)sizeof(double2) < ((int64_t)1 << 31);
    SS_REQUIRE(o.ilu_sweeps == 0 || want_sched, SS_E_INVALID_ARG,
               "ilu_sweeps: fixed-point ILU(0) on the device-wide path only");
    if (o.ordering == SS_ORDER_NATURAL) identity_order(h->n, h->perm, h->iperm, s);
    else rcm_order(h->S, h->perm, h->iperm, s);
    h->colours = 0;
    h->split = false;
    if (o.ordering == SS_ORDER_COLOUR) recolour(h, want_sched, s);
    phase("ordering");
    prepare_permute(h, s);
    phase("permute");
    // the matrix to factorise: Ap, or its colour-class reordering (split)
    CsrBuf<double2> Ac;
    DevBuf<int> cdiag;
    if (h->split) {
        permute_matrix(h->Ap, h->cp.get(), h->lorder.get(), Ac, s);
        cdiag.resize((size_t)std::max(h->n, 1));
        const int missing = find_diagonal(h->n, Ac.rowptr.get(), Ac.col.get(), cdiag.get(), s);
        SS_REQUIRE(missing == 0, SS_E_ZERO_PIVOT, "colour-class reordering lost a diagonal entry");
    }
    const CsrBuf<double2> &F = h->split ? Ac : h->Ap;
    const int *fdiag = h->split ? cdiag.get() : h->diag.get();
    // zero fill keeps the pattern, so for ILU(0) the schedules are built
    // first and drive the factorisation too when they are shallow
    bool sched_built = false;
    if (o.ilu == SS_ILU0 && want_sched) {
        // (zero fill: the factors keep A's pattern, so no entry joins two
        // rows of one colour class)
        build_levels(F.view(), fdiag, h->sched_lo, h->sched_up, s, h->colours ? h->lorder.get() : nullptr,
                     h->colours ? &h->class_ptr : nullptr);
        sched_built = true;
        phase("levels");
    }
    if (o.ilu == SS_ILU0 && o.ilu_sweeps > 0) {
        h->guarded = ilu0_fixed_point(F, fdiag, o.ilu_sweeps, PIVOT_DETECT, PIVOT_BOOST, h->LU, s).guarded;
    } else if (o.ilu == SS_ILU0 && sched_built && h->sched_lo.nlev <= PRE_CLASSES_MAX_LEVELS) {
        h->guarded = ilu0_factor_levels(F, fdiag, h->sched_lo, PIVOT_DETECT, PIVOT_BOOST, h->LU, s).guarded;
    } else if (o.ilu == SS_ILU0) {
        h->guarded = ilu0_factor(F, fdiag, PIVOT_DETECT, PIVOT_BOOST, h->LU, s).guarded;
    } else {
        h->guarded =
            ilut_factor(F, fdiag, o.drop_tol, o.fill, PIVOT_DETECT, PIVOT_BOOST, h->LU, h->lu_diag, s).guarded;
    }
    if (o.ilu == SS_ILU0 && h->split) {
        h->lu_diag = std::move(cdiag);  // (prepare_finish leaves it)
    }
    phase("ilu");
    prepare_finish(h, method, o, s, t0);
    phase("finish");
    h->sched_ready = false;
    if (want_sched) {
        if (!sched_built)
            build_levels(h->LU.view(), h->lu_diag.get(), h->sched_lo, h->sched_up, s,
                         h->colours ? h->lorder.get() : nullptr);
        group_gates(h->sched_lo, h->n, h->gate_lo, s);
        group_gates(h->sched_up, h->n, h->gate_up, s);
        h->sched_ready = true;
        h->t_setup_ms = now_ms() - t0;
        phase("levels");
    }
}

// ------------------------------------------------------------ helpers
__global__ void k_set_scalar(double2 *dst, double2 v) { *dst = v; }

// x[idx[k]] = v for k < m
__global__ void k_set_at(int m, const int *idx, double2 *x, double2 v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) x[idx[k]] = v;
}

// x *= 1 / t (complex)
__global__ void k_scale_inv(int n, double2 *x, const double2 *t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 inv = cdiv(mk(1.0, 0.0), *t);
    x[i] = cmul(x[i], inv);
}

// y[perm[q]] = x[q] / t   (undo the ordering, normalise the trace)
__global__ void k_unpermute_scale(int n, const int *perm, const double2 *x, const double2 *t, double2 *y) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double2 inv = cdiv(mk(1.0, 0.0), *t);
    y[perm[q]] = cmul(x[q], inv);
}

// max |rho_ij - conj(rho_ji)| over the d x d matrix stored column-major
__global__ void k_herm_err(int d, const double2 *rho, double2 *partials) {
    __shared__ double sh[256];
    double m = 0;
    const int64_t nn = (int64_t)d * d;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nn; q += (int64_t)gridDim.x * 256) {
        const int i = (int)(q % d), j = (int)(q / d);
        const double2 a = rho[q], b = rho[(int64_t)i * d + j];
        const double dx = a.x - b.x, dy = a.y + b.y;
        m = fmax(m, sqrt(dx * dx + dy * dy));
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = mk(sh[0], 0.0);
}

__global__ void k_hermitize(int d, const double2 *rho, double2 *out) {
    const int64_t nn = (int64_t)d * d;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nn) return;
    const int i = (int)(q % d), j = (int)(q / d);
    const double2 a = rho[q], b = rho[(int64_t)i * d + j];
    out[q] = mk(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
}

__global__ void k_max_part(const double2 *p, int nb, double2 *out) {
    if (threadIdx.x) return;
    double m = 0;
    for (int b = 0; b < nb; ++b) m = fmax(m, p[b].x);
    *out = mk(m, 0.0);
}

// host threads preparing the systems of a batch (environment variable
// SS_SETUP_THREADS overrides it, 1..64)
constexpr int BATCH_SETUP_THREADS = 8;

static int setup_threads() {
    const char *e = std::getenv("SS_SETUP_THREADS");
    if (!e) return BATCH_SETUP_THREADS;
    const int v = std::atoi(e);
    return (v >= 1 && v <= 64) ? v : BATCH_SETUP_THREADS;
}

static thread_local std::string tl_batch_error;
static void set_batch_error(const std::string &e) { tl_batch_error = e; }
const std::string &batch_error() { return tl_batch_error; }

// ------------------------------------------------------------- driver
// Largest system solved by the workgroup-resident kernel unless forced.
constexpr int WG_AUTO_MAX_N = 4096;

bool use_workgroup_n(int64_t n, int method, const ss_options &o) {
    if (is_gmres(method)) return false;
    if (o.flags & (SS_FLAG_DEVICE_WIDE | SS_FLAG_MATRIX_FREE)) return false;
    if (o.flags & SS_FLAG_WORKGROUP) return true;
    return n <= WG_AUTO_MAX_N;
}

bool use_workgroup(ss_liouv h, int method, const ss_options &o) { return use_workgroup_n(h->n, method, o); }

__global__ void k_random_start(int n, int d, const int *perm, uint64_t seed, double2 *x) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = random_start_value(d, perm[q], seed);
}

// Start vector and right-hand side in the permuted order: trace row
// b = w e_rt, x = 0; inverse power x = vec(I / d), or the random trace-1
// Hermitian start of SS_FLAG_RANDOM_START.
static void init_vectors(ss_liouv h, bool trace, double2 *x, double2 *b, const ss_options &o, hipStream_t s) {
    const int n = h->n, d = h->d;
    zero<double2>(n, x, s);
    if (trace) {
        zero<double2>(n, b, s);
        k_set_at<<<1, 1, 0, s>>>(1, h->iperm.get() + h->trow, b, h->w);
    } else if (o.flags & SS_FLAG_RANDOM_START) {
        k_random_start<<<div_up(n, 256), 256, 0, s>>>(n, d, h->perm.get(), (uint64_t)o.seed, x);
    } else {
        k_set_at<<<div_up(d, 256), 256, 0, s>>>(d, h->tpos.get(), x, mk(1.0 / d, 0.0));
    }
    SS_HIP(hipGetLastError());
}

template <typename T>
void make_wg(ss_liouv h, int method, double tol, const ss_options &o, const CsrBuf<T> &Ain, const CsrBuf<T> &LUin,
             WgBundle<T> &B, hipStream_t s, bool levels_built) {
    const int n = h->n;
    const bool trace = is_trace(method);
    B.x.resize((size_t)n);
    B.r.resize((size_t)n);
    B.b.resize((size_t)n);
    init_vectors(h, trace, B.x.get(), B.b.get(), o, s);
    if (!levels_built) build_levels(h->LU.view(), h->lu_diag.get(), B.lo, B.up, s);
    pack_side<T>(B.lo, LUin.view(), false, B.pl, s);
    pack_side<T>(B.up, LUin.view(), true, B.pu, s);
    B.work.resize((size_t)11 * n);
    B.ysc.resize((size_t)n);
    B.res.resize(1);
    B.levels = B.lo.nlev + B.up.nlev;
    WgProblem<T> &P = B.P;
    std::memset(&P, 0, sizeof(P));
    P.n = n;
    P.d = h->d;
    P.q0 = h->q0;
    P.trace = trace ? 1 : 0;
    P.nlev_l = B.lo.nlev;
    P.nlev_u = B.up.nlev;
    P.maxiter = o.maxiter;
    P.max_outer = o.max_outer > 0 ? o.max_outer : 20;
    P.tol = tol;
    P.rtol_in = (o.inner_tol > 0) ? o.inner_tol : (o.prec == SS_MIXED ? 1e-4 : 0.0);
    P.force_breakdown = (o.flags & SS_FLAG_FORCE_BREAKDOWN) ? 1 : 0;
    P.sigma = o.sigma;
    P.w = h->w;
    P.A = Ain.view();
    P.A64 = h->Ap.view();
    P.LU = LUin.view();
    P.diag = h->lu_diag.get();
    P.lptr = B.lo.ptr.get();
    P.lslot = B.pl.slot.get();
    P.lcol = B.pl.col.get();
    P.lval = B.pl.val.get();
    P.uptr = B.up.ptr.get();
    P.uslot = B.pu.slot.get();
    P.ucol = B.pu.col.get();
    P.uval = B.pu.val.get();
    P.uaux = B.pu.aux.get();
    P.tpos = h->tpos.get();
    P.b64 = trace ? B.b.get() : nullptr;
    P.x64 = B.x.get();
    P.r64 = B.r.get();
    P.work = B.work.get();
    P.ysc = B.ysc.get();
    P.res = B.res.get();
}
template void make_wg<double2>(ss_liouv, int, double, const ss_options &, const CsrBuf<double2> &,
                               const CsrBuf<double2> &, WgBundle<double2> &, hipStream_t, bool);
template void make_wg<float2>(ss_liouv, int, double, const ss_options &, const CsrBuf<float2> &,
                              const CsrBuf<float2> &, WgBundle<float2> &, hipStream_t, bool);

// ||(L U)^-1 e||_inf with e = (1, ..., 1): the paper's stability measure of
// the preconditioner (section "Iterative Solvers"), with the fp64 factors
// and the level-scheduled solve.
__global__ void k_fill_ones(int n, double2 *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = mk(1.0, 0.0);
}

static double condition_estimate(ss_liouv h, hipStream_t s) {
    const int n = h->n;
    if (n == 0 || h->LU.nnz == 0) return 0.0;
    DevBuf<double2> e((size_t)n), y((size_t)n), part((size_t)VEC_MAX_BLOCKS), sc(1);
    k_fill_ones<<<div_up(n, 256), 256, 0, s>>>(n, e.get());
    SS_HIP(hipGetLastError());
    Precond<double2> M;
    M.setup(&h->LU, h->lu_diag.get(), n, s);
    if (h->split) M.pin = h->cp.get();
    M.use_levels(h->LU.view(), s);
    M.apply(e.get(), y.get(), s);
    norm_inf<double2>(n, y.get(), part.get(), sc.get(), s);
    double2 v;
    d2h(&v, sc.get(), 1, s);
    return v.x;
}

// The outcome and the info record of a finished solve.
int fill_info(ss_liouv h, const ss_options &o, double tol, const SolveStats &st, double final_res, double herm_err,
              double2 trx, int64_t bandwidth, int64_t profile, ss_info *info, hipStream_t s) {
    const int n = h->n;
    int status = st.status;
    if (status == SS_E_NOT_CONVERGED && final_res <= tol) status = SS_OK;
    if (info) {
        info->status = status;
        info->outer_its = st.outer;
        info->inner_its = st.inner;
        info->breakdowns = st.breakdowns;
        info->pivots_guarded = h->guarded;
        info->fell_back = st.fell_back;
        info->nnz_matrix = h->Ap.nnz;
        info->nnz_factors = h->LU.nnz;
        info->fill_factor = h->Ap.nnz ? (double)h->LU.nnz / h->Ap.nnz : 0.0;
        info->resid_l2 = final_res;
        info->herm_err = herm_err;
        info->trace_err = sqrt((trx.x - 1.0) * (trx.x - 1.0) + trx.y * trx.y);
        info->weight = h->w.x;
        info->method = h->p_method;
        info->colours = h->colours;
        info->bandwidth = (int32_t)bandwidth;
        info->profile = profile;
        info->cond_est = (o.flags & SS_FLAG_COND_EST) ? condition_estimate(h, s) : 0.0;
        info->t_setup_ms = h->t_setup_ms;
        info->t_solve_ms = st.t_solve_ms;
        info->t_kernel_ms = st.t_kernel_ms;
        info->path = st.path;
        // algorithmic bytes: per BiCGSTAB iteration two SpMV and two triangular
        // solve pairs plus about 24 vector passes; per outer step one fp64
        // SpMV and about 6 vector passes (values, indices, row pointers and
        // vectors each counted once per use)
        const double sT = st.elem_bytes;
        const double spmvT = (double)h->Ap.nnz * (sT + 4) + 4.0 * (n + 1) + 2.0 * n * sT;
        const double trsvT = (double)h->LU.nnz * (sT + 4) + 8.0 * (n + 1) + 8.0 * n + 4.0 * n * sT;
        const double spmv64 = (double)h->Ap.nnz * 20.0 + 4.0 * (n + 1) + 32.0 * n;
        info->bytes_alg = st.inner * (2 * spmvT + 2 * trsvT + 24.0 * n * sT) + (st.outer + 1) * (spmv64 + 96.0 * n);
    }
    return status;
}

// Finish a solve: unpermute, normalise the trace, certify with L itself,
// Hermiticity error, copy rho out (host or device), fill info.
int finish(ss_liouv h, const double2 *x, const ss_options &o, double tol, const SolveStats &st, double *rho_out,
           ss_info *info, hipStream_t s) {
    const int n = h->n, d = h->d;
    DevBuf<double2> scal(4), part((size_t)VEC_MAX_BLOCKS), rho((size_t)n), Lr((size_t)n);
    double2 *sc = scal.get();
    gather_sum(d, h->tpos.get(), x, sc, s);
    double2 trx;
    d2h(&trx, sc, 1, s);
    k_unpermute_scale<<<div_up(n, 256), 256, 0, s>>>(n, h->perm.get(), x, sc, rho.get());
    SS_HIP(hipGetLastError());
    if (o.flags & SS_FLAG_HERMITIZE) {
        k_hermitize<<<div_up(n, 256), 256, 0, s>>>(d, rho.get(), Lr.get());
        SS_HIP(hipMemcpyAsync(rho.get(), Lr.get(), sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
    }
    if (o.flags & SS_FLAG_MATRIX_FREE) {
        lindblad_apply(h->lin.view(), rho.get(), nullptr, 0, mk(0.0, 0.0), nullptr, nullptr, Lr.get(), part.get(), s);
        sum_partials(part.get(), lindblad_blocks(d), 1, sc + 1, s);
    } else {
        const Csr<double2> Lv = h->L.view();
        spmv<double2>(Lv, rho.get(), Lr.get(), spmv_group(Lv.n, Lv.nnz), s);
        norm2<double2>(n, Lr.get(), part.get(), sc + 1, s);
    }
    const int nbh = vec_blocks(n);
    k_herm_err<<<nbh, 256, 0, s>>>(d, rho.get(), part.get());
    k_max_part<<<1, 64, 0, s>>>(part.get(), nbh, sc + 2);
    SS_HIP(hipGetLastError());
    double2 fin[2];
    d2h(fin, sc + 1, 2, s);
    if (rho_out) {
        const hipMemcpyKind k = is_device_ptr(rho_out) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        SS_HIP(hipMemcpyAsync(rho_out, rho.get(), sizeof(double2) * n, k, s));
        SS_HIP(hipStreamSynchronize(s));
    }
    int64_t bw = 0, pf = 0;
    if (info) bandwidth_profile(h->Ap.n, h->Ap.rowptr.get(), h->Ap.col.get(), &bw, &pf, s);
    const int status = fill_info(h, o, tol, st, sqrt(fin[0].x), fin[1].x, trx, bw, pf, info, s);
    return status;
}

// Outer steps in a row without halving the best fp64 residual after which
// a device-wide solve stops (SS_E_NOT_CONVERGED with the last iterate).
constexpr int STALL_STEPS = 4;

template <typename T>
static int run(ss_liouv h, int method, double tol, const ss_options &o, const CsrBuf<T> &Ain, const CsrBuf<T> &LUin,
               double *rho_out, ss_info *info) {
    hipStream_t s = stream_of(h);
    const int n = h->n, d = h->d;
    const double t0 = now_ms();
    const bool trace = is_trace(method);
    const bool mixed = (o.prec == SS_MIXED);
    const int maxouter = o.max_outer > 0 ? o.max_outer : 20;
    SolveStats st;
    st.elem_bytes = (double)sizeof(T);
    bool use_gmres = is_gmres(method);
    int gm_m = o.gmres_m;
    DevBuf<double2> xbuf, bbuf;
    double2 *x = nullptr, *bvec = nullptr;
    WgBundle<T> B;
    bool done_wg = false;
    if (use_workgroup(h, method, o)) {
        // whole solve in one workgroup: level schedules, then one launch
        make_wg<T>(h, method, tol, o, Ain, LUin, B, s);
        x = B.x.get();
        bvec = B.b.get();
        DevBuf<WgProblem<T>> dP(1);
        h2d(dP.get(), &B.P, 1, s);
        hipEvent_t e0, e1;
        SS_HIP(hipEventCreate(&e0));
        SS_HIP(hipEventCreate(&e1));
        SS_HIP(hipEventRecord(e0, s));
        st.path = wg_fits_lds((size_t)n, sizeof(T), B.levels) ? 2 : 1;
        wg_solve<T>(dP.get(), 1, n, B.levels, s);
        SS_HIP(hipEventRecord(e1, s));
        WgResult hr;
        d2h(&hr, B.res.get(), 1, s);
        float kms = 0.f;
        SS_HIP(hipEventElapsedTime(&kms, e0, e1));
        hip_quiet(hipEventDestroy(e0));
        hip_quiet(hipEventDestroy(e1));
        st.t_kernel_ms = kms;
        if (std::getenv("SS_DEBUG")) {
            std::fprintf(stderr,
                         "[ss] workgroup solve: n=%d levels L/U=%d/%d inner=%d outer=%d kernel=%.3f ms "
                         "precond=%.3f ms spmv=%.3f ms total=%.3f ms (device clock)\n",
                         n, B.lo.nlev, B.up.nlev, hr.inner, hr.outer, kms, hr.ticks_precond * 1e-5,
                         hr.ticks_spmv * 1e-5, hr.ticks_total * 1e-5);
        }
        st.status = hr.status;
        st.outer = hr.outer;
        st.inner = hr.inner;
        st.breakdowns = hr.breakdowns;
        done_wg = true;
        if (st.status == SS_E_BREAKDOWN && !(o.flags & SS_FLAG_NO_FALLBACK)) {
            // continue from the current iterate with the device-wide GMRES
            done_wg = false;
            use_gmres = true;
            st.fell_back = 1;
            st.status = SS_E_NOT_CONVERGED;
        }
    } else {
        xbuf.resize((size_t)n);
        bbuf.resize((size_t)n);
        x = xbuf.get();
        bvec = bbuf.get();
        init_vectors(h, trace, x, bvec, o, s);
    }
    if (!done_wg) {
        Precond<T> M;
        M.setup(&LUin, h->lu_diag.get(), n, s);
        if (h->split) M.pin = h->cp.get();
        if (!(o.flags & SS_FLAG_SYNCFREE)) {
            const int mode = (o.flags & SS_FLAG_TRSV_BLOCK)     ? PRE_BLOCK
                             : (o.flags & SS_FLAG_TRSV_LEVELS)  ? PRE_LEVELS
                             : (o.flags & SS_FLAG_TRSV_GROUPS)  ? PRE_GROUPS
                             : (o.flags & SS_FLAG_TRSV_CLASSES) ? PRE_CLASSES
                                                                : PRE_AUTO;
            // shallow schedules (the colour-class order) above the
            // one-workgroup size take one launch per level
            const bool shallow = h->sched_ready && std::max(h->sched_lo.nlev, h->sched_up.nlev) <= PRE_CLASSES_MAX_LEVELS;
            const bool classes = mode == PRE_CLASSES || (mode == PRE_AUTO && shallow && n > PRE_BLOCK_MAX_N);
            // the one-workgroup solve takes long factor rows one entry at a
            // time: iLUT factors (rows of ~100 entries) go to the row groups
            const bool groups =
                mode == PRE_GROUPS || (mode == PRE_AUTO && (n > PRE_BLOCK_MAX_N || o.ilu == SS_ILUT));
            if (classes && h->sched_ready)
                M.borrow_classes(&h->sched_lo, &h->sched_up);
            else if (classes)
                M.use_levels(h->LU.view(), s, PRE_CLASSES, h->colours ? h->lorder.get() : nullptr);
            else if (groups && h->sched_ready)
                M.borrow_groups(&h->sched_lo, &h->sched_up, h->gate_lo.get(), h->gate_up.get(), s);
            else
                M.use_levels(h->LU.view(), s, mode, h->colours ? h->lorder.get() : nullptr);
        }
        Krylov<T> K;
        K.init(Ain.view(), &M, s);
        const Csr<double2> A64 = h->Ap.view();
        const int gA = spmv_group(A64.n, A64.nnz);
        // matrix-free residual: x back to the natural order, then L applied
        // from the d x d operators with the transform and the ordering folded
        // into the same kernel
        const bool mfree = (o.flags & SS_FLAG_MATRIX_FREE) != 0;
        const LindbladOp lin = h->lin.view();
        DevBuf<double2> rho_nat(mfree ? (size_t)n : 0);
        DevBuf<double2> r((size_t)n), part(4 * (size_t)VEC_MAX_BLOCKS), scal(16);
        DevBuf<T> bT((size_t)n), dT((size_t)n);
        double2 *sc = scal.get();
        int outer, stalled = 0;
        double best_resid = INFINITY;
        for (outer = 0; outer <= maxouter; ++outer) {
            // fp64 residual and trace
            double2 hs[3];
            double resid;
            if (trace) {
                gather_sum(d, h->tpos.get(), x, sc + 1, s);
                if (mfree) {
                    unpermute(n, h->iperm.get(), x, rho_nat.get(), s);
                    lindblad_apply(lin, rho_nat.get(), h->iperm.get(), h->trow, h->w, sc + 1, bvec, r.get(),
                                   part.get(), s);
                    sum_partials(part.get(), lindblad_blocks(d), 1, sc, s);
                } else {
                    spmv_residual(A64, bvec, x, r.get(), part.get(), gA, s);
                    sum_partials(part.get(), vec_blocks(n), 1, sc, s);
                }
                k_copy_d2<<<1, 1, 0, s>>>(r.get() + h->q0, sc + 2);
                SS_HIP(hipGetLastError());
                d2h(hs, sc, 3, s);
                const double r2 = hs[0].x;
                const double2 tr = hs[1], rq = hs[2];
                // L x = -r + w (1 - Tr x) e_q0  (permuted row q0 carries T)
                const double2 one_m_tr = mk(1.0 - tr.x, -tr.y);
                const double2 e0 = csub(cmul(h->w, one_m_tr), rq);
                const double lx2 = fmax(r2 - (rq.x * rq.x + rq.y * rq.y), 0.0) + e0.x * e0.x + e0.y * e0.y;
                const double trm = sqrt(tr.x * tr.x + tr.y * tr.y);
                resid = (trm > 0) ? sqrt(lx2) / trm : INFINITY;
                if (outer > 0 && resid <= tol) { st.status = SS_OK; break; }
                if (outer == maxouter) break;
                const double rn = sqrt(r2);
                if (rn == 0.0) { st.status = SS_OK; break; }
                double2 den = mk(rn, 0.0);
                h2d(sc + 4, &den, 1, s);
            } else {
                // r = L x = (L - sigma I) x + sigma x
                if (mfree) {
                    unpermute(n, h->iperm.get(), x, rho_nat.get(), s);
                    lindblad_apply(lin, rho_nat.get(), h->iperm.get(), 0, mk(0.0, 0.0), nullptr, nullptr, r.get(),
                                   part.get(), s);
                    sum_partials(part.get(), lindblad_blocks(d), 1, sc, s);
                } else {
                    spmv_residual(A64, nullptr, x, r.get(), part.get(), gA, s);
                    double2 sg = mk(o.sigma, 0.0);
                    h2d(sc + 5, &sg, 1, s);
                    axpy_widen<double2>(n, sc + 5, x, r.get(), s);
                    norm2<double2>(n, r.get(), part.get(), sc, s);
                }
                gather_sum(d, h->tpos.get(), x, sc + 1, s);
                d2h(hs, sc, 2, s);
                const double trm = sqrt(hs[1].x * hs[1].x + hs[1].y * hs[1].y);
                resid = (trm > 0) ? sqrt(hs[0].x) / trm : INFINITY;
                if (resid <= tol) { st.status = SS_OK; break; }
                if (outer == maxouter) break;
                double2 den = mk(sqrt(hs[0].x), 0.0);
                h2d(sc + 4, &den, 1, s);
            }
            // give up when the outer steps stop making progress: no halving of
            // the best residual in STALL_STEPS consecutive steps
            if (resid < 0.5 * best_resid) {
                best_resid = resid;
                stalled = 0;
            } else if (++stalled >= STALL_STEPS) {
                break;
            }
            // inner solve of A d = r / ||r||
            double2 hden;
            d2h(&hden, sc + 4, 1, s);
            double rtol_in = o.inner_tol;
            if (rtol_in <= 0) rtol_in = mixed ? 1e-4 : std::max(0.1 * tol / hden.x, 1e-13);
            rtol_in = std::min(rtol_in, 0.5);
            convert<T, double2>(n, r.get(), bT.get(), sc + 4, s);
            KrylovResult kr;
            if (!use_gmres) {
                kr = K.bicgstab(bT.get(), dT.get(), rtol_in, o.maxiter, (o.flags & SS_FLAG_FORCE_BREAKDOWN) != 0);
                st.breakdowns += kr.breakdown;
                if (!kr.converged && kr.breakdown) {
                    st.inner += kr.iters;
                    if (o.flags & SS_FLAG_NO_FALLBACK) {
                        st.status = SS_E_BREAKDOWN;
                        break;
                    }
                    // fall back to GMRES for this and the remaining steps
                    use_gmres = true;
                    st.fell_back = 1;
                    kr = K.gmres(bT.get(), dT.get(), rtol_in, o.maxiter, gm_m);
                }
            } else {
                kr = K.gmres(bT.get(), dT.get(), rtol_in, o.maxiter, gm_m);
            }
            // restarted GMRES that stagnates gets a longer Krylov basis next time
            if (use_gmres && !kr.converged) gm_m = std::min(2 * gm_m, 128);
            st.inner += kr.iters;
            const unsigned pst = M.read_status(s);
            SS_REQUIRE(!(pst & STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT, "triangular solve: dependency wait timed out");
            if (trace) {
                axpy_widen<T>(n, sc + 4, dT.get(), x, s);  // x += ||r|| d
            } else {
                double2 neg = mk(-hden.x, 0.0);
                h2d(sc + 6, &neg, 1, s);
                axpy_widen<T>(n, sc + 6, dT.get(), x, s);  // x -= ||r|| d
                gather_sum(d, h->tpos.get(), x, sc + 7, s);
                k_scale_inv<<<div_up(n, 256), 256, 0, s>>>(n, x, sc + 7);  // x /= Tr x
                SS_HIP(hipGetLastError());
            }
        }
        st.outer += outer;
    }
    st.t_solve_ms = now_ms() - t0;
    return finish(h, x, o, tol, st, rho_out, info, s);
}

// ------------------------------------------------------------- batches
// Independent systems solved together: set-up of every handle on its own
// stream from a few host threads, then one launch of the workgroup-resident
// solver with one workgroup per system (the systems run side by side on the
// CUs), then the finish of every handle.  A system whose BiCGSTAB broke
// down is solved again on its own with the device-wide kernels (unless
// SS_FLAG_NO_FALLBACK).  Each system's arithmetic stays in its own
// workgroup, so its result is the same as in a batch of one.
template <typename T>
static int run_batch(ss_liouv *hs, int count, int method, const double *tols, const ss_options &o,
                     double **rho_out, ss_info *infos, int *status) {
    const int nthreads = std::max(1, std::min(count, setup_threads()));
    std::vector<std::string> err((size_t)count);
    std::vector<int> code((size_t)count, SS_OK);
    auto parallel = [&](auto &&fn) {
        std::vector<std::thread> th;
        for (int t = 0; t < nthreads; ++t)
            th.emplace_back([&, t]() {
                for (int i = t; i < count; i += nthreads) {
                    if (code[(size_t)i] != SS_OK) continue;
                    try {
                        fn(i);
                    } catch (const Error &e) {
                        code[(size_t)i] = e.code;
                        err[(size_t)i] = e.what();
                    } catch (const std::exception &e) {
                        code[(size_t)i] = SS_E_HIP;
                        err[(size_t)i] = e.what();
                    }
                }
            });
        for (auto &x : th) x.join();
    };
    const double t0 = now_ms();
    hipStream_t s0 = stream_of(hs[0]);
    const bool dbg = std::getenv("SS_DEBUG") != nullptr;
    double tmark = t0;
    auto mark = [&](const char *name) {
        if (!dbg) return;
        SS_HIP(hipStreamSynchronize(s0));
        const double t = now_ms();
        std::fprintf(stderr, "[ss] batch of %d: %-22s %8.3f ms\n", count, name, t - tmark);
        tmark = t;
    };
    // stage 1: transform and symmetrised pattern of every system together
    check_options(method, o);
    SS_REQUIRE(o.ilu_sweeps == 0, SS_E_INVALID_ARG, "ilu_sweeps: fixed-point ILU(0) on the device-wide path only");
    {
        std::vector<ss_liouv> ok;
        std::vector<int> idx;
        for (int i = 0; i < count; ++i) {
            if (is_trace(method) && o.trace_row >= hs[i]->d) {
                code[(size_t)i] = SS_E_INVALID_ARG;
                err[(size_t)i] = "trace_row must be < N";
                continue;
            }
            ok.push_back(hs[i]);
            idx.push_back(i);
        }
        try {
            transform_batch(ok.data(), (int)ok.size(), is_trace(method), o, s0);
        } catch (const Error &e) {
            for (int i : idx) {
                code[(size_t)i] = e.code;
                err[(size_t)i] = e.what();
            }
        }
    }
    mark("transform+pattern");
    // stage 2: RCM of every graph in one launch (small graphs), else per system
    const bool rcm = o.ordering != SS_ORDER_NATURAL;  // the colour order starts from RCM
    std::vector<RcmScratch> rs((size_t)count);
    {
        std::vector<RcmJob> jobs;
        for (int i = 0; i < count; ++i) {
            if (code[(size_t)i] != SS_OK || !rcm || !rcm_batchable(hs[i]->n) || hs[i]->n == 0) continue;
            rs[(size_t)i].alloc(hs[i]->n);
            jobs.push_back(rs[(size_t)i].job(hs[i]->S, hs[i]->perm.get(), hs[i]->iperm.get()));
        }
        rcm_batch(jobs.data(), (int)jobs.size(), s0);
    }
    mark("rcm (batched)");
    // stage 3: orderings the batched RCM does not cover, per system (rare),
    // and the colour classes over RCM
    parallel([&](int i) {
        ss_liouv h = hs[i];
        hipStream_t s = stream_of(h);
        h->colours = 0;
        if (!(rcm && rcm_batchable(h->n) && h->n > 0)) {
            if (!rcm) identity_order(h->n, h->perm, h->iperm, s);
            else rcm_order(h->S, h->perm, h->iperm, s);
        }
        h->split = false;
        if (o.ordering == SS_ORDER_COLOUR) recolour(h, false, s);
        SS_HIP(hipStreamSynchronize(s));
    });
    {
        FreeScope fs(s0);  // the batched RCM is complete: one event for all its scratch
        rs.clear();
    }
    // P A P^T, diagonal and trace positions and the ILU(0) pattern of every
    // system together; rows without a diagonal entry (rare) are fixed per system
    const bool ilu0 = (o.ilu == SS_ILU0);
    std::vector<Ilu0Batch> ib((size_t)count);
    std::vector<Ilu0Job> ijobs((size_t)count);
    std::vector<char> own_ilu((size_t)count, 0);
    DevBuf<double2> ilu_work;
    DevBuf<unsigned> ilu_flags;
    {
        std::vector<ss_liouv> ok;
        std::vector<int> idx;
        for (int i = 0; i < count; ++i)
            if (code[(size_t)i] == SS_OK) {
                ok.push_back(hs[i]);
                idx.push_back(i);
            }
        std::vector<PermResult> pres;
        try {
            permute_batch(ok.data(), (int)ok.size(), ilu0, s0, pres);
        } catch (const Error &e) {
            for (int i : idx) {
                code[(size_t)i] = e.code;
                err[(size_t)i] = e.what();
            }
            pres.assign(ok.size(), PermResult{});
        }
        // rows without a diagonal: explicit zeros, then the factor's own scratch
        parallel([&](int i) {
            ss_liouv h = hs[i];
            if (h->diag_added == 0) return;
            hipStream_t s = stream_of(h);
            add_zero_diagonal(h, s);
            if (ilu0) {
                ijobs[(size_t)i] = ib[(size_t)i].prepare(h->Ap, h->diag.get(), h->LU, s);
                SS_HIP(hipMemcpyAsync(h->lu_diag.get(), h->diag.get(), sizeof(int) * h->n, hipMemcpyDeviceToDevice,
                                      s));
                own_ilu[(size_t)i] = 1;
            }
            SS_HIP(hipStreamSynchronize(s));
        });
        if (ilu0) {
            // ILU(0) scratch of the other systems in two arenas
            size_t wtot = 0;
            for (int i : idx)
                if (code[(size_t)i] == SS_OK && !own_ilu[(size_t)i]) wtot += (size_t)std::max(hs[i]->Ap.nnz, 1);
            StreamScope scope(s0);
            ilu_work.resize(std::max<size_t>(wtot, 1));
            ilu_flags.resize(2 * (size_t)count);
            SS_HIP(hipMemsetAsync(ilu_flags.get(), 0, ilu_flags.bytes(), s0));
            size_t w = 0;
            for (int i : idx) {
                if (code[(size_t)i] != SS_OK || own_ilu[(size_t)i]) continue;
                ss_liouv h = hs[i];
                Ilu0Job &j = ijobs[(size_t)i];
                j.n = h->n;
                j.rowptr = h->Ap.rowptr.get();
                j.col = h->Ap.col.get();
                j.diag = h->diag.get();
                j.a = h->Ap.val.get();
                j.w = ilu_work.get() + w;
                j.out = h->LU.val.get();
                j.status = ilu_flags.get() + 2 * i;
                j.nguard = reinterpret_cast<int *>(ilu_flags.get() + 2 * i + 1);
                w += (size_t)std::max(h->Ap.nnz, 1);
            }
        }
    }
    mark("permute+ilu prep");
    // level schedules of both factor sides; with ILU(0) the factor has the
    // pattern of P A P^T, so they exist before the factorisation and its lower
    // side schedules the factorisation itself
    LevelBatch lb;
    auto schedule = [&]() {
        std::vector<ss_liouv> ok;
        std::vector<int> idx;
        for (int i = 0; i < count; ++i)
            if (code[(size_t)i] == SS_OK) {
                ok.push_back(hs[i]);
                idx.push_back(i);
            }
        try {
            levels_setup_batch(ok.data(), (int)ok.size(), s0, lb);
        } catch (const Error &e) {
            for (int i : idx) {
                code[(size_t)i] = e.code;
                err[(size_t)i] = e.what();
            }
        }
    };
    if (ilu0) schedule();
    mark("levels (batched)");
    // stage 4: ILU(0) of every system in one launch, level by level
    std::vector<unsigned> hflags;
    if (ilu0) {
        std::vector<Ilu0Job> jobs;
        for (int i = 0; i < count; ++i) {
            if (code[(size_t)i] != SS_OK) continue;
            Ilu0Job j = ijobs[(size_t)i];
            const int q = lb.pos.at(hs[i]);
            j.nlev = lb.nl[(size_t)q];
            j.lptr = lb.lptr[(size_t)q];
            j.lslot = lb.lslot[(size_t)q];
            jobs.push_back(j);
        }
        ilu0_levels_batch(jobs.data(), (int)jobs.size(), PIVOT_DETECT, PIVOT_BOOST, s0);
        hflags.resize(2 * (size_t)count);
        d2h(hflags.data(), ilu_flags.get(), hflags.size(), s0);
    }
    mark("ilu0 (batched)");
    // stage 5: ILUT or the outcome of the ILU(0), the rest of the set-up, per system
    parallel([&](int i) {
        ss_liouv h = hs[i];
        hipStream_t s = stream_of(h);
        if (ilu0 && own_ilu[(size_t)i]) {
            h->guarded = ib[(size_t)i].result(s).guarded;
        } else if (ilu0) {
            SS_REQUIRE(!(hflags[2 * (size_t)i] & STATUS_SPIN_TIMEOUT), SS_E_TIMEOUT,
                       "ILU(0): dependency wait timed out");
            h->guarded = (int)hflags[2 * (size_t)i + 1];
        } else {
            h->guarded = ilut_factor(h->Ap, h->diag.get(), o.drop_tol, o.fill, PIVOT_DETECT, PIVOT_BOOST, h->LU,
                                     h->lu_diag, s)
                             .guarded;
        }
        prepare_finish(h, method, o, s, t0, true);
        SS_HIP(hipStreamSynchronize(s));
    });
    ib.clear();
    if (o.prec == SS_MIXED) {
        std::vector<ss_liouv> ok;
        std::vector<int> idx;
        for (int i = 0; i < count; ++i)
            if (code[(size_t)i] == SS_OK) {
                ok.push_back(hs[i]);
                idx.push_back(i);
            }
        try {
            c64_copies_batch(ok.data(), (int)ok.size(), s0);
        } catch (const Error &e) {
            for (int i : idx) {
                code[(size_t)i] = e.code;
                err[(size_t)i] = e.what();
            }
        }
    }
    mark("ilu result+finish prep");
    // stage 6: (ILUT: level schedules now) packed factors and the
    // workgroup problems of every system together
    if (!ilu0) schedule();
    WgBatch<T> wb;
    std::vector<int> slot((size_t)count, -1);
    {
        std::vector<ss_liouv> ok;
        std::vector<int> idx;
        for (int i = 0; i < count; ++i)
            if (code[(size_t)i] == SS_OK) {
                slot[(size_t)i] = (int)ok.size();
                ok.push_back(hs[i]);
                idx.push_back(i);
            }
        std::vector<double> tl;
        for (int i : idx) tl.push_back(tols[i]);
        try {
            wg_setup_batch<T>(ok.data(), (int)ok.size(), method, tl.data(), o, lb, s0, wb);
        } catch (const Error &e) {
            for (int i : idx) {
                code[(size_t)i] = e.code;
                err[(size_t)i] = e.what();
            }
        }
    }
    mark("schedules+wg problem");
    const double t_setup = now_ms() - t0;
    std::vector<WgProblem<T>> probs;
    int max_n = 0, max_lev = 0;
    for (int i = 0; i < count; ++i) {
        if (code[(size_t)i] != SS_OK) continue;
        const int k = slot[(size_t)i];
        probs.push_back(wb.probs[(size_t)k]);
        max_n = std::max(max_n, wb.probs[(size_t)k].n);
        max_lev = std::max(max_lev, wb.levels[(size_t)k]);
    }
    float kms = 0.f;
    const double t1 = now_ms();
    if (!probs.empty()) {
        hipStream_t s = stream_of(hs[0]);
        DevBuf<WgProblem<T>> dP(probs.size());
        h2d(dP.get(), probs.data(), probs.size(), s);
        hipEvent_t e0, e1;
        SS_HIP(hipEventCreate(&e0));
        SS_HIP(hipEventCreate(&e1));
        SS_HIP(hipEventRecord(e0, s));
        wg_solve<T>(dP.get(), (int)probs.size(), max_n, max_lev, s);
        SS_HIP(hipEventRecord(e1, s));
        SS_HIP(hipEventSynchronize(e1));
        SS_HIP(hipEventElapsedTime(&kms, e0, e1));
        hip_quiet(hipEventDestroy(e0));
        hip_quiet(hipEventDestroy(e1));
    }
    const double t_solve = now_ms() - t1;
    mark("workgroup solve");
    const int path = wg_fits_lds((size_t)max_n, sizeof(T), max_lev) ? 2 : 1;
    // outcomes of every system, read back together
    std::vector<int> solved;
    std::vector<const WgResult *> rptr;
    for (int i = 0; i < count; ++i)
        if (code[(size_t)i] == SS_OK) {
            solved.push_back(i);
            rptr.push_back(wb.probs[(size_t)slot[(size_t)i]].res);
        }
    std::vector<WgResult> hres;
    read_results(rptr, hres, s0);
    if (dbg && !hres.empty()) {
        // device wall-clock ticks (100 MHz) inside the solver, mean over the batch
        double tp = 0, ts = 0, tt = 0, its = 0;
        for (const WgResult &r : hres) {
            tp += (double)r.ticks_precond;
            ts += (double)r.ticks_spmv;
            tt += (double)r.ticks_total;
            its += r.inner;
        }
        const double m = (double)hres.size() * 100.0;  // ticks -> us
        std::fprintf(stderr, "[ss] batch of %d: solver per system: %.0f us total, %.0f us preconditioner, %.0f us SpMV, "
                     "%.1f inner iterations\n", count, tt / m, tp / m, ts / m, its / (double)hres.size());
    }
    // systems whose BiCGSTAB broke down or stagnated: again on their own
    // with iLUT and the device-wide GMRES; the others finish together
    std::vector<char> again((size_t)count, 0);
    std::vector<ss_liouv> fh;
    std::vector<const double2 *> fx;
    std::vector<SolveStats> fst;
    std::vector<double *> fout;
    std::vector<ss_info *> finfo;
    std::vector<int> fidx;
    std::vector<double> ftol;
    for (size_t k = 0; k < solved.size(); ++k) {
        const int i = solved[k];
        const WgResult &hr = hres[k];
        if (hr.status == SS_E_BREAKDOWN && !(o.flags & SS_FLAG_NO_FALLBACK)) {
            again[(size_t)i] = 1;
            continue;
        }
        SolveStats st;
        st.status = hr.status;
        st.outer = hr.outer;
        st.inner = hr.inner;
        st.breakdowns = hr.breakdowns;
        st.path = path;
        st.t_kernel_ms = kms;
        st.t_solve_ms = t_solve;
        st.elem_bytes = (double)sizeof(T);
        fh.push_back(hs[i]);
        fx.push_back(wb.probs[(size_t)slot[(size_t)i]].x64);
        fst.push_back(st);
        fout.push_back(rho_out ? rho_out[i] : nullptr);
        finfo.push_back(infos ? infos + i : nullptr);
        fidx.push_back(i);
        ftol.push_back(tols[i]);
    }
    {
        std::vector<int> fstat(fh.size(), SS_OK);
        try {
            finish_batch(fh.data(), (int)fh.size(), fx.data(), o, ftol.data(), fst.data(), fout.data(), finfo.data(),
                         fstat.data(), s0);
        } catch (const Error &e) {
            for (size_t k = 0; k < fh.size(); ++k) {
                fstat[k] = e.code;
                err[(size_t)fidx[k]] = e.what();
            }
        }
        for (size_t k = 0; k < fh.size(); ++k) {
            code[(size_t)fidx[k]] = fstat[k];
            if (infos) infos[fidx[k]].t_setup_ms = t_setup;
        }
    }
    parallel([&](int i) {
        if (!again[(size_t)i]) return;
        ss_liouv h = hs[i];
        code[(size_t)i] = solve_ilut_gmres(h, method, tols[i], o, rho_out ? rho_out[i] : nullptr,
                                           infos ? infos + i : nullptr);
    });
    mark("finish (+ fallbacks)");
    int first = SS_OK;
    for (int i = 0; i < count; ++i) {
        if (status) status[i] = code[(size_t)i];
        if (infos) infos[i].status = code[(size_t)i];
        if (code[(size_t)i] != SS_OK && first == SS_OK) {
            first = code[(size_t)i];
            if (!err[(size_t)i].empty()) set_batch_error(err[(size_t)i]);
        }
    }
    return first;
}

int solve_batch(ss_liouv *hs, int count, int method, double tol, const ss_options &o, double **rho_out,
                ss_info *infos, int *status, const double *tols) {
    SS_REQUIRE(tols || (tol > 0 && std::isfinite(tol)), SS_E_INVALID_ARG, "tol must be positive");
    SS_REQUIRE(method == SS_TRACE_BICGSTAB || method == SS_INVPOW_BICGSTAB, SS_E_INVALID_ARG,
               "batched solves use BiCGSTAB (the workgroup-resident solver)");
    SS_REQUIRE(!(o.flags & SS_FLAG_MATRIX_FREE), SS_E_INVALID_ARG,
               "SS_FLAG_MATRIX_FREE implies the device-wide path; batched solves run the workgroup-resident solver");
    std::vector<double> uniform;
    if (!tols) {
        uniform.assign((size_t)std::max(count, 0), tol);
        tols = uniform.data();
    }
    if (o.prec == SS_MIXED) return run_batch<float2>(hs, count, method, tols, o, rho_out, infos, status);
    return run_batch<double2>(hs, count, method, tols, o, rho_out, infos, status);
}

// SS_AUTO: RCM bandwidths of L~ and of L - sigma I decide the driver.
constexpr double AUTO_BANDWIDTH_RATIO = 1.5;
// a diagonal entry below this fraction of its row's largest counts as zero
constexpr double AUTO_ZERO_DIAG = 1e-12;

__global__ void k_count_small_diag(int n, const int *rowptr, const double2 *val, const int *diag, double eps,
                                   int *cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) m = fmax(m, sqrt(val[e].x * val[e].x + val[e].y * val[e].y));
    const double2 a = val[diag[i]];
    if (sqrt(a.x * a.x + a.y * a.y) <= eps * m) atomicAdd(cnt, 1);
}

static int choose_method(ss_liouv h, const ss_options &o) {
    hipStream_t s = stream_of(h);
    int64_t bt = 0, bs = 0, p = 0;
    ss_options oo = o;
    oo.ilu = SS_ILU0;
    prepare_transform(h, SS_TRACE_BICGSTAB, oo, s);
    rcm_order(h->S, h->perm, h->iperm, s);
    prepare_permute(h, s);
    bandwidth_profile(h->Ap.n, h->Ap.rowptr.get(), h->Ap.col.get(), &bt, &p, s);
    // zero diagonal entries that the trace row does not cover (e.g. the
    // populations under pure dephasing) leave zero-fill ILU of L~ with
    // boosted pivots: inverse power then
    int zero_diag = h->diag_added;
    if (zero_diag == 0) {
        DevBuf<int> cnt(1);
        SS_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int), s));
        k_count_small_diag<<<div_up(h->n, 256), 256, 0, s>>>(h->n, h->Ap.rowptr.get(), h->Ap.val.get(), h->diag.get(),
                                                            AUTO_ZERO_DIAG, cnt.get());
        SS_HIP(hipGetLastError());
        d2h(&zero_diag, cnt.get(), 1, s);
    }
    prepare_transform(h, SS_INVPOW_BICGSTAB, oo, s);
    rcm_order(h->S, h->perm, h->iperm, s);
    prepare_permute(h, s);
    bandwidth_profile(h->Ap.n, h->Ap.rowptr.get(), h->Ap.col.get(), &bs, &p, s);
    if (std::getenv("SS_DEBUG"))
        std::fprintf(stderr, "[ss] auto: B(L~) = %lld, B(L - sigma I) = %lld, zero diagonals of L~ = %d\n",
                     (long long)bt, (long long)bs, zero_diag);
    if (zero_diag > 0 || (double)bt > AUTO_BANDWIDTH_RATIO * (double)bs) return SS_INVPOW_BICGSTAB;
    // the trace row: GMRES (the paper's first choice) where the device-wide
    // kernels solve; BiCGSTAB where the workgroup-resident launch does
    return use_workgroup_n(h->n, SS_TRACE_BICGSTAB, o) ? SS_TRACE_BICGSTAB : SS_TRACE_GMRES;
}

// When zero-fill ILU cannot precondition a system (no diagonal dominance:
// element growth in the factors, the failure the paper attributes to iLU),
// the paper's own combination takes over: the dual-threshold iLUT with
// restarted GMRES (section "Iterative Solvers"; GMRES on the trace-row
// system is its recommended first choice, section "Conclusion").  Used
// after BiCGSTAB and the GMRES fallback on the ILU(0) factors have both
// failed; the solve is flagged info.fell_back.
int solve_ilut_gmres(ss_liouv h, int method, double tol, const ss_options &o, double *rho_out, ss_info *info) {
    ss_options od = o;
    od.ilu = SS_ILUT;
    od.ilu_sweeps = 0;
    od.flags |= SS_FLAG_DEVICE_WIDE;
    od.flags &= ~SS_FLAG_WORKGROUP;
    const int gm = is_trace(method) ? SS_TRACE_GMRES : SS_INVPOW_GMRES;
    prepare(h, gm, od);
    int st;
    if (od.prec == SS_MIXED) st = run<float2>(h, gm, tol, od, h->Ap32, h->LU32, rho_out, info);
    else st = run<double2>(h, gm, tol, od, h->Ap, h->LU, rho_out, info);
    if (info) info->fell_back = 1;
    return st;
}

int solve(ss_liouv h, int method, double tol, const ss_options &o, double *rho_out, ss_info *info) {
    SS_REQUIRE(tol > 0 && std::isfinite(tol), SS_E_INVALID_ARG, "tol must be positive");
    if (method == SS_AUTO) method = choose_method(h, o);
    prepare(h, method, o);
    int st;
    if (o.prec == SS_MIXED) st = run<float2>(h, method, tol, o, h->Ap32, h->LU32, rho_out, info);
    else st = run<double2>(h, method, tol, o, h->Ap, h->LU, rho_out, info);
    if ((st == SS_E_NOT_CONVERGED || st == SS_E_BREAKDOWN) && o.ilu == SS_ILU0 && !(o.flags & SS_FLAG_NO_FALLBACK))
        st = solve_ilut_gmres(h, method, tol, o, rho_out, info);
    return st;
}

}  // namespace ss
