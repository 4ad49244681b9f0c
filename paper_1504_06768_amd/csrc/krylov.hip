// Preconditioned Krylov solvers (section "Iterative Solvers"): BiCGSTAB
// (van der Vorst) and restarted GMRES(m), both right-preconditioned with the
// ILU factors, A M^-1 y = b, x = M^-1 y, so the monitored residual is the
// residual of the original system.  The paper writes the preconditioned
// system with M^-1 on the left; the solution is the same.
//
// All scalars (rho, alpha, omega, the Hessenberg matrix and Givens rotations)
// stay on the device: one-thread "finalise" kernels turn reduction results
// into the next step's coefficients, and a skip flag makes every kernel of
// an already-finished solve return at once, so the host only reads the state
// every few iterations.
#include <limits>

#include "krylov.hpp"

namespace ss {

constexpr int BATCH_ITERS = 4;  // BiCGSTAB iterations enqueued between host checks
constexpr int GM_BATCH = 4;     // GMRES steps enqueued between host checks

// ------------------------------------------------------------ BiCGSTAB
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_init(int n, const T *b, T *r, T *rhat, T *p, T *v, T *x,
                                                   double2 *partials) {
    double2 d[1] = {mk(0.0, 0.0)};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const T bi = b[i];
        r[i] = bi;
        rhat[i] = bi;
        p[i] = czero<T>();
        v[i] = czero<T>();
        x[i] = czero<T>();
        const double2 w = widen(bi);
        d[0].x += w.x * w.x + w.y * w.y;
    }
    __shared__ double2 sh[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double a = d[0].x;
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0) sh[wave] = mk(a, 0.0);
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = mk(sh[0].x + sh[1].x + sh[2].x + sh[3].x, 0.0);
}

__global__ void k_bicg_init_fin(BicgState *st, const double2 *scal, double rtol, int maxiter, double bd_eps) {
    const double b2 = scal[0].x;
    st->bnorm2 = b2;
    st->rhat2 = b2;
    st->rnorm2 = b2;
    st->rho = mk(b2, 0.0);
    st->rho_old = mk(1.0, 0.0);
    st->alpha = mk(1.0, 0.0);
    st->omega = mk(1.0, 0.0);
    st->tol2 = rtol * rtol * b2;
    st->bd_eps = bd_eps;
    st->iters = 0;
    st->maxiter = maxiter;
    st->state = (b2 == 0.0) ? 2 : 0;
    st->skip = (st->state != 0) || (maxiter <= 0);
}

// restart after a breakdown: r^ = r, p = v = 0
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_restart(int n, const T *r, T *rhat, T *p, T *v, double2 *partials) {
    double a = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const T ri = r[i];
        rhat[i] = ri;
        p[i] = czero<T>();
        v[i] = czero<T>();
        const double2 w = widen(ri);
        a += w.x * w.x + w.y * w.y;
    }
    __shared__ double sh[4];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = mk(sh[0] + sh[1] + sh[2] + sh[3], 0.0);
}

__global__ void k_bicg_restart_fin(BicgState *st, const double2 *scal) {
    const double r2 = scal[0].x;
    st->rhat2 = r2;
    st->rho = mk(r2, 0.0);
    st->rho_old = mk(1.0, 0.0);
    st->alpha = mk(1.0, 0.0);
    st->omega = mk(1.0, 0.0);
    st->state = 0;
    st->skip = (st->iters >= st->maxiter);
}

// p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega)
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_p(int n, const BicgState *st, const T *r, T *p, const T *v) {
    if (st->skip) return;
    const double2 beta = cmul(cdiv(st->rho, st->rho_old), cdiv(st->alpha, st->omega));
    const double2 om = st->omega;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double2 pi = widen(p[i]), vi = widen(v[i]), ri = widen(r[i]);
        const double2 q = csub(pi, cmul(om, vi));
        p[i] = from_c128<T>(cadd(ri, cmul(beta, q)));
    }
}

// alpha = rho / (r^, v); breakdown when (r^, v) vanishes relative to |r^||v|
__device__ void fin_alpha(BicgState *st, const double2 *scal) {
    if (st->skip) return;
    const double2 rv = scal[0];
    const double vv = scal[1].x;
    st->dot_rv = rv;
    const double m2 = rv.x * rv.x + rv.y * rv.y;
    if (!(m2 > st->bd_eps * st->bd_eps * st->rhat2 * vv)) {
        st->state = 3;
        st->skip = 1;
        return;
    }
    st->alpha = cdiv(st->rho, rv);
}

// s = r - alpha v, partial ||s||^2
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_s(int n, const BicgState *st, const T *r, const T *v, T *s,
                                                double2 *partials) {
    if (st->skip) return;
    const double2 al = st->alpha;
    double a = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double2 si = csub(widen(r[i]), cmul(al, widen(v[i])));
        const T sv = from_c128<T>(si);
        s[i] = sv;
        const double2 w = widen(sv);
        a += w.x * w.x + w.y * w.y;
    }
    __shared__ double sh[4];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = mk(sh[0] + sh[1] + sh[2] + sh[3], 0.0);
}

__device__ void fin_s(BicgState *st, const double2 *scal) {
    if (st->skip) return;
    if (scal[0].x <= st->tol2) {
        st->state = 1;
        st->skip = 1;
    }
}

// omega = (t, s) / (t, t) = conj(s^H t) / |t|^2  (scal[0] holds s^H t)
__device__ void fin_omega(BicgState *st, const double2 *scal) {
    if (st->skip) return;
    st->dot_ts = cconj(scal[0]);
    st->dot_tt = scal[1].x;
    st->omega = (scal[1].x > 0.0) ? cscale(cconj(scal[0]), 1.0 / scal[1].x) : mk(0.0, 0.0);
}

// x += alpha p^ + omega s^, r = s - omega t, partials (r^, r) and ||r||^2
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_x(int n, const BicgState *st, T *x, const T *phat, const T *shat,
                                                T *r, const T *s, const T *t, const T *rhat, double2 *partials) {
    const int state = st->state;
    if (state != 0 && state != 1) return;
    if (state == 0 && st->skip) return;
    const double2 al = st->alpha, om = st->omega;
    double2 d0 = mk(0.0, 0.0);
    double d1 = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double2 xi = cadd(widen(x[i]), cmul(al, widen(phat[i])));
        if (state == 0) {
            xi = cadd(xi, cmul(om, widen(shat[i])));
            const T ri = from_c128<T>(csub(widen(s[i]), cmul(om, widen(t[i]))));
            r[i] = ri;
            const double2 rw = widen(ri);
            d0 = cadd(d0, cmulc(widen(rhat[i]), rw));
            d1 += rw.x * rw.x + rw.y * rw.y;
        } else {
            r[i] = s[i];
        }
        x[i] = from_c128<T>(xi);
    }
    __shared__ double sh[3][4];
    double a = d0.x, b = d0.y, c = d1;
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[0][wave] = a; sh[1][wave] = b; sh[2][wave] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = mk(sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3], sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
        partials[gridDim.x + blockIdx.x] = mk(sh[2][0] + sh[2][1] + sh[2][2] + sh[2][3], 0.0);
    }
}

__device__ void fin_x(BicgState *st, const double2 *scal) {
    const int state = st->state;
    if (state == 1) {
        st->state = 2;
        st->iters += 1;
        st->skip = 1;
        return;
    }
    if (state != 0 || st->skip) return;
    st->rho_old = st->rho;
    st->rho = scal[0];
    st->rnorm2 = scal[1].x;
    st->iters += 1;
    const double2 rho = scal[0];
    const double m2 = rho.x * rho.x + rho.y * rho.y;
    if (st->rnorm2 <= st->tol2) {
        st->state = 2;
        st->skip = 1;
    } else if (!(st->omega.x != 0.0 || st->omega.y != 0.0) ||
               !(m2 > st->bd_eps * st->bd_eps * st->rhat2 * st->rnorm2)) {
        st->state = 3;
        st->skip = 1;
    } else if (st->iters >= st->maxiter) {
        st->skip = 1;
    }
}

// The k sums of one reduction (one workgroup, fixed order) and the scalar
// step that uses them, in one launch.
enum FinStep { FIN_ALPHA, FIN_S, FIN_OMEGA, FIN_X };

template <int STEP>
__global__ void __launch_bounds__(SUM_BS) k_sum_fin(const double2 *partials, int nb, int k, double2 *scal,
                                                    BicgState *st) {
    for (int j = 0; j < k; ++j) {
        const double2 v = sum_partials_block(partials + (int64_t)j * nb, nb);
        if (threadIdx.x == 0) scal[j] = v;
    }
    if (threadIdx.x != 0) return;
    if (STEP == FIN_ALPHA) fin_alpha(st, scal);
    else if (STEP == FIN_S) fin_s(st, scal);
    else if (STEP == FIN_OMEGA) fin_omega(st, scal);
    else fin_x(st, scal);
}

template <typename T>
void Krylov<T>::init(const Csr<T> &A_, Precond<T> *M_, hipStream_t s_) {
    A = A_;
    M = M_;
    s = s_;
    n = A.n;
    group = spmv_group(A.n, A.nnz);
    const size_t nn = (size_t)std::max(n, 1);
    r.resize(nn); rhat.resize(nn); p.resize(nn); v.resize(nn); sv.resize(nn); t.resize(nn);
    phat.resize(nn); shat.resize(nn);
    partials.resize(std::max<size_t>(4 * (size_t)VEC_MAX_BLOCKS * 24, 2 * (size_t)SPMV_DOTS_MAX_BLOCKS));
    scal.resize(128);
    bst.resize(1);
    gst.resize(1);
}

template <typename T>
KrylovResult Krylov<T>::bicgstab(const T *b, T *x, double rtol, int maxiter, bool force_breakdown) {
    const int nb = vec_blocks(n);
    // (a threshold whose square overflows makes every breakdown test fire)
    const double bd_eps = force_breakdown ? 1e300 : (sizeof(typename RealOf<T>::type) == 8 ? 1e-30 : 1e-14);
    BicgState *st = bst.get();
    const int *skip = &st->skip;
    double2 *sc = scal.get();
    double2 *pp = partials.get();
    KrylovResult res;

    k_bicg_init<T><<<nb, 256, 0, s>>>(n, b, r.get(), rhat.get(), p.get(), v.get(), x, pp);
    sum_partials(pp, nb, 1, sc, s);
    k_bicg_init_fin<<<1, 1, 0, s>>>(st, sc, rtol, maxiter, bd_eps);
    SS_HIP(hipGetLastError());

    int restarts = 0;
    BicgState h;
    while (true) {
        for (int it = 0; it < BATCH_ITERS; ++it) {
            k_bicg_p<T><<<nb, 256, 0, s>>>(n, st, r.get(), p.get(), v.get());
            M->apply(p.get(), phat.get(), s, skip);
            const int nbv = spmv_dots<T>(A, phat.get(), v.get(), rhat.get(), v.get(), pp, group, s, skip);
            k_sum_fin<FIN_ALPHA><<<1, SUM_BS, 0, s>>>(pp, nbv, 2, sc, st);
            k_bicg_s<T><<<nb, 256, 0, s>>>(n, st, r.get(), v.get(), sv.get(), pp);
            k_sum_fin<FIN_S><<<1, SUM_BS, 0, s>>>(pp, nb, 1, sc + 2, st);
            M->apply(sv.get(), shat.get(), s, skip);
            const int nbt = spmv_dots<T>(A, shat.get(), t.get(), sv.get(), t.get(), pp, group, s, skip);
            k_sum_fin<FIN_OMEGA><<<1, SUM_BS, 0, s>>>(pp, nbt, 2, sc + 4, st);
            k_bicg_x<T><<<nb, 256, 0, s>>>(n, st, x, phat.get(), shat.get(), r.get(), sv.get(), t.get(),
                                           rhat.get(), pp);
            k_sum_fin<FIN_X><<<1, SUM_BS, 0, s>>>(pp, nb, 2, sc + 6, st);
            SS_HIP(hipGetLastError());
        }
        d2h(&h, st, 1, s);
        if (h.state == 3 && restarts < 3 && h.iters < maxiter) {
            // breakdown: restart with r^ = current residual
            ++restarts;
            ++res.breakdown;
            k_bicg_restart<T><<<nb, 256, 0, s>>>(n, r.get(), rhat.get(), p.get(), v.get(), pp);
            sum_partials(pp, nb, 1, sc, s);
            k_bicg_restart_fin<<<1, 1, 0, s>>>(st, sc);
            SS_HIP(hipGetLastError());
            continue;
        }
        if (h.skip) break;
    }
    res.iters = h.iters;
    res.converged = (h.state == 2);
    if (h.state == 3) res.breakdown += 1;
    res.rel_res = h.bnorm2 > 0 ? sqrt(h.rnorm2 / h.bnorm2) : 0.0;
    return res;
}

// --------------------------------------------------------------- GMRES
// partials of V_k^H w for k = blockIdx.y, w^H w at k = self_at; skip set,
// or gate given and clear: nothing.  (One workgroup per row slice and k:
// one workgroup per slice for every k, w read once, measured slower.)
template <typename T>
__global__ void __launch_bounds__(256) k_multidot(int n, const T *V, int64_t ldv, const T *w, int self_at,
                                                  double2 *partials, const int *skip, const int *gate) {
    if ((skip && *skip) || (gate && !*gate)) return;
    const int k = blockIdx.y;
    const T *vk = (k == self_at) ? w : V + (int64_t)k * ldv;
    double2 acc[1] = {mk(0.0, 0.0)};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        acc[0] = cadd(acc[0], cmulc(widen(vk[i]), widen(w[i])));
    block_partials<1>(acc, partials + (int64_t)k * gridDim.x);
}

// w = sign * sum_k h[k] V_k + (accumulate ? w : 0)
template <typename T>
// (with npart: block partials of the result's ||w||^2 there as well)
__global__ void __launch_bounds__(256) k_multi_axpy(int n, int nk, const T *V, int64_t ldv, const double2 *h,
                                                    double sign, bool accumulate, T *w, const int *skip = nullptr,
                                                    const int *gate = nullptr, double2 *npart = nullptr) {
    if ((skip && *skip) || (gate && !*gate)) return;
    double2 nrm[1] = {mk(0.0, 0.0)};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double2 acc = accumulate ? widen(w[i]) : mk(0.0, 0.0);
        for (int k = 0; k < nk; ++k) acc = cadd(acc, cscale(cmul(h[k], widen(V[(int64_t)k * ldv + i])), sign));
        const T wi = from_c128<T>(acc);
        w[i] = wi;
        const double2 ww = widen(wi);
        nrm[0].x += ww.x * ww.x + ww.y * ww.y;
    }
    if (npart) block_partials<1>(nrm, npart);
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale_into(int n, const T *w, const double2 *den, T *out,
                                                    const int *skip = nullptr) {
    if (skip && *skip) return;
    const double inv = 1.0 / den->x;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) out[i] = from_c128<T>(cscale(widen(w[i]), inv));
}

template <typename T>
__global__ void __launch_bounds__(256) k_sub_into(int n, const T *b, const T *a, T *out) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) out[i] = from_c128<T>(csub(widen(b[i]), widen(a[i])));
}

template <typename T>
__global__ void __launch_bounds__(256) k_add_into(int n, const T *a, T *x) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) x[i] = from_c128<T>(cadd(widen(x[i]), widen(a[i])));
}

// hcol[k] = the sum of partial group k (k < nk), and H[k, j] (+)= hcol[k]
// for k <= j; one workgroup per group
__global__ void __launch_bounds__(SUM_BS) k_gm_sum_hcol(const double2 *partials, int nb, double2 *hcol, double2 *H,
                                                        int ldh, int j, bool accumulate, const int *skip,
                                                        const int *gate) {
    if (*skip || (gate && !*gate)) return;
    const int k = blockIdx.x;
    const double2 v = sum_partials_block(partials + (int64_t)k * nb, nb);
    if (threadIdx.x != 0) return;
    hcol[k] = v;
    if (k <= j) H[(int64_t)j * ldh + k] = accumulate ? cadd(H[(int64_t)j * ldh + k], v) : v;
}

// the stopping test's bounds (absolute tolerance, iterations)
__global__ void k_gm_init(GmresState *st, double tol_abs, int maxiter) {
    st->tol = tol_abs;
    st->maxiter = maxiter;
    st->iters = 0;
}
// cycle start: beta = ||r||, g = beta e_1
__global__ void k_gm_start(GmresState *st, const double2 *norm2, double2 *g, int ldh) {
    const double beta = sqrt(norm2->x);
    st->beta = beta;
    st->res = beta;
    st->j = 0;
    st->skip = 0;
    for (int k = 0; k < ldh; ++k) g[k] = mk(0.0, 0.0);
    g[0] = mk(beta, 0.0);
}

// second orthogonalisation pass only when the first cancelled w to below
// sqrt(eps) of its norm (||w'||^2 < eps ||w||^2, eps the unit roundoff of
// the Krylov vectors): the first pass leaves w' with an error of order
// eps ||w||, so only then does w' lose more than sqrt(eps) of its
// orthogonality to the basis.  (The criterion of Daniel, Gragg, Kaufman and
// Stewart, ||w'||^2 < ||w||^2 / 2, ran the second pass at almost every step
// on the Liouvillians here with the same iteration counts as never.)
// The first pass's ||w'||^2 goes from its partials into wnorm2_after.
__global__ void __launch_bounds__(SUM_BS) k_gm_need2(GmresState *st, const double2 *npart, int nb,
                                                     double2 *wnorm2_after, const double2 *wnorm2_before,
                                                     double eps) {
    if (st->skip) return;
    const double2 v = sum_partials_block(npart, nb);
    if (threadIdx.x != 0) return;
    *wnorm2_after = v;
    st->pass2 = (v.x < eps * wnorm2_before->x) ? 1 : 0;
}
// new column j: h_{j+1,j} = ||w||, previous rotations, new rotation, g
// update, and the stopping test (which sets skip for the steps queued after)
__device__ void gm_givens(GmresState *st, double2 *H, int ldh, int j, const double2 *wnorm2, double *cs,
                          double2 *sn, double2 *g, double2 *den) {
    if (st->skip) return;
    double2 *h = H + (int64_t)j * ldh;
    const double hn = sqrt(wnorm2->x);
    st->hnext = hn;
    den->x = hn;
    den->y = 0.0;
    for (int k = 0; k < j; ++k) {
        // [c s; -conj(s) c] applied to (h_k, h_{k+1})
        const double2 a = h[k], b = h[k + 1];
        h[k] = cadd(cscale(a, cs[k]), cmul(sn[k], b));
        h[k + 1] = csub(cscale(b, cs[k]), cmulc(sn[k], a));
    }
    const double2 a = h[j];
    const double amag = sqrt(a.x * a.x + a.y * a.y);
    const double nrm = sqrt(amag * amag + hn * hn);
    double c;
    double2 sv;
    if (nrm == 0.0) {
        c = 1.0;
        sv = mk(0.0, 0.0);
    } else if (amag == 0.0) {
        c = 0.0;
        sv = mk(1.0, 0.0);
    } else {
        c = amag / nrm;
        // s = (a / |a|) * conj(hn) / nrm, hn real
        sv = cscale(a, hn / (amag * nrm));
    }
    cs[j] = c;
    sn[j] = sv;
    h[j] = (amag == 0.0) ? mk(hn, 0.0) : cscale(a, nrm / amag);
    h[j + 1] = mk(0.0, 0.0);
    const double2 gj = g[j];
    g[j] = cscale(gj, c);
    g[j + 1] = cscale(cmulc(sv, gj), -1.0);
    st->res = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
    st->j = j + 1;
    st->iters += 1;
    if (st->res <= st->tol || hn == 0.0 || st->iters >= st->maxiter) st->skip = 1;
}

// ||w||^2 after the second pass (from its partials when it ran, else the
// first pass's), then the Givens step
__global__ void __launch_bounds__(SUM_BS) k_gm_givens(GmresState *st, const double2 *npart, int nb,
                                                      double2 *wnorm2, double2 *H, int ldh, int j, double *cs,
                                                      double2 *sn, double2 *g, double2 *den) {
    if (st->skip) return;
    if (st->pass2) {
        const double2 v = sum_partials_block(npart, nb);
        if (threadIdx.x == 0) *wnorm2 = v;
    }
    if (threadIdx.x == 0) gm_givens(st, H, ldh, j, wnorm2, cs, sn, g, den);
}

// y = R^-1 g over the first jj columns (back substitution)
__global__ void k_gm_solve(const double2 *H, int ldh, int jj, const double2 *g, double2 *y) {
    for (int k = jj - 1; k >= 0; --k) {
        double2 acc = g[k];
        for (int c = k + 1; c < jj; ++c) acc = csub(acc, cmul(H[(int64_t)c * ldh + k], y[c]));
        y[k] = cdiv(acc, H[(int64_t)k * ldh + k]);
    }
}

template <typename T>
KrylovResult Krylov<T>::gmres(const T *b, T *x, double rtol, int maxiter, int m) {
    KrylovResult res;
    if (m < 1) m = 1;
    if (m > 128) m = 128;
    const int ldh = m + 1;
    if (m_alloc != m) {
        V.resize((size_t)(m + 1) * std::max(n, 1));
        w.resize((size_t)std::max(n, 1));
        z.resize((size_t)std::max(n, 1));
        u.resize((size_t)std::max(n, 1));
        H.resize((size_t)ldh * m);
        g.resize((size_t)ldh);
        sn.resize((size_t)m);
        cs.resize((size_t)m);
        yv.resize((size_t)m);
        hcol.resize((size_t)ldh);
        // (m + 1) groups of products, then the norm's partials
        if (partials.size() < (size_t)(m + 2) * VEC_MAX_BLOCKS) partials.resize((size_t)(m + 2) * VEC_MAX_BLOCKS);
        m_alloc = m;
    }
    const int nb = vec_blocks(n);
    double2 *pp = partials.get();
    double2 *sc = scal.get();
    GmresState *st = gst.get();
    T *Vp = V.get();
    const int64_t ldv = n;

    zero<T>(n, x, s);
    norm2<T>(n, b, pp, sc, s);
    double2 hb;
    d2h(&hb, sc, 1, s);
    const double bnorm = sqrt(hb.x);
    if (bnorm == 0.0) {
        res.converged = 1;
        return res;
    }
    const double tol_abs = rtol * bnorm;
    k_gm_init<<<1, 1, 0, s>>>(st, tol_abs, maxiter);
    SS_HIP(hipGetLastError());
    const int *skip = &st->skip, *pass2 = &st->pass2;
    int total = 0;
    bool first = true;
    double last_res = bnorm;
    GmresState hs;
    while (true) {
        // r = b - A x into V_0 (x = 0 on the first cycle)
        if (first) {
            SS_HIP(hipMemcpyAsync(w.get(), b, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
        } else {
            spmv<T>(A, x, z.get(), group, s);
            k_sub_into<T><<<nb, 256, 0, s>>>(n, b, z.get(), w.get());
        }
        first = false;
        norm2<T>(n, w.get(), pp, sc, s);
        k_gm_start<<<1, 1, 0, s>>>(st, sc, g.get(), ldh);
        SS_HIP(hipGetLastError());
        d2h(&hs, st, 1, s);
        last_res = hs.beta;
        if (hs.beta <= tol_abs || total >= maxiter) {
            res.converged = hs.beta <= tol_abs;
            break;
        }
        {
            double2 den = mk(hs.beta, 0.0);
            h2d(sc + 8, &den, 1, s);
            k_scale_into<T><<<nb, 256, 0, s>>>(n, w.get(), sc + 8, Vp);
            SS_HIP(hipGetLastError());
        }
        // Arnoldi steps, queued GM_BATCH at a time: the step that meets the
        // stopping test sets skip, and the kernels of the steps queued after
        // it do nothing; the host reads the state once per batch
        bool stop = false;
        for (int j0 = 0; j0 < m && !stop; j0 += GM_BATCH) {
            const int j1 = std::min(m, j0 + GM_BATCH);
            for (int j = j0; j < j1; ++j) {
                T *vj = Vp + (int64_t)j * ldv;
                M->apply(vj, z.get(), s, skip);
                spmv<T>(A, z.get(), w.get(), group, s, skip);
                // classical Gram-Schmidt; the first pass also forms w^H w,
                // each update also the partials of the new ||w||^2
                double2 *np = pp + (int64_t)(m + 1) * nb;
                k_multidot<T><<<dim3(nb, j + 2), 256, 0, s>>>(n, Vp, ldv, w.get(), j + 1, pp, skip, nullptr);
                k_gm_sum_hcol<<<j + 2, SUM_BS, 0, s>>>(pp, nb, hcol.get(), H.get(), ldh, j, false, skip, nullptr);
                k_multi_axpy<T><<<nb, 256, 0, s>>>(n, j + 1, Vp, ldv, hcol.get(), -1.0, true, w.get(), skip, nullptr,
                                                   np);
                k_gm_need2<<<1, SUM_BS, 0, s>>>(st, np, nb, sc, hcol.get() + j + 1,
                                                std::numeric_limits<typename RealOf<T>::type>::epsilon() / 2);
                k_multidot<T><<<dim3(nb, j + 1), 256, 0, s>>>(n, Vp, ldv, w.get(), -1, pp, skip, pass2);
                k_gm_sum_hcol<<<j + 1, SUM_BS, 0, s>>>(pp, nb, hcol.get(), H.get(), ldh, j, true, skip, pass2);
                k_multi_axpy<T><<<nb, 256, 0, s>>>(n, j + 1, Vp, ldv, hcol.get(), -1.0, true, w.get(), skip, pass2,
                                                   np);
                k_gm_givens<<<1, SUM_BS, 0, s>>>(st, np, nb, sc, H.get(), ldh, j, cs.get(), sn.get(), g.get(),
                                                 sc + 9);
                k_scale_into<T><<<nb, 256, 0, s>>>(n, w.get(), sc + 9, Vp + (int64_t)(j + 1) * ldv, skip);
                SS_HIP(hipGetLastError());
            }
            d2h(&hs, st, 1, s);
            stop = hs.skip != 0;
        }
        const int jj = hs.j;
        total = hs.iters;
        last_res = hs.res;
        // x += M^-1 (V y)
        k_gm_solve<<<1, 1, 0, s>>>(H.get(), ldh, jj, g.get(), yv.get());
        k_multi_axpy<T><<<nb, 256, 0, s>>>(n, jj, Vp, ldv, yv.get(), 1.0, false, u.get());
        M->apply(u.get(), z.get(), s);
        k_add_into<T><<<nb, 256, 0, s>>>(n, z.get(), x);
        SS_HIP(hipGetLastError());
        if (stop) {
            res.converged = last_res <= tol_abs || hs.hnext == 0.0;
            if (hs.hnext == 0.0) last_res = 0.0;
            break;
        }
    }
    res.iters = total;
    res.rel_res = last_res / bnorm;
    return res;
}

template struct Krylov<double2>;
template struct Krylov<float2>;

}  // namespace ss
