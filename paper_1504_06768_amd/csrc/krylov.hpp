// Right-preconditioned Krylov solvers (krylov.hip).
#pragma once
#include "blas.hpp"
#include "ilu.hpp"

namespace ss {

struct KrylovResult {
    int iters = 0;
    int converged = 0;
    int breakdown = 0;     // BiCGSTAB: r^ orthogonal to r, or omega = 0
    double rel_res = 0.0;  // final (recursive) residual / ||b||
};

// Device-side state of one BiCGSTAB solve.
struct BicgState {
    double2 rho, rho_old, alpha, omega;
    double2 dot_rv, dot_ts;
    double dot_tt, rnorm2, bnorm2, tol2, rhat2, bd_eps;
    int state;  // 0 running, 1 converged after the half step, 2 converged, 3 breakdown
    int iters;
    int maxiter;
    int skip;   // != 0 once the solve has stopped: later kernels return at once
};

struct GmresState {
    double beta, bnorm, tol, res, hnext;
    int j, state, iters, maxiter, skip;
    int pass2;  // the step's second orthogonalisation pass runs
};

template <typename T>
struct Krylov {
    int n = 0;
    Csr<T> A;
    int group = 8;
    Precond<T> *M = nullptr;
    hipStream_t s = nullptr;
    // BiCGSTAB workspace
    DevBuf<T> r, rhat, p, v, sv, t, phat, shat;
    DevBuf<double2> partials, scal;
    DevBuf<BicgState> bst;
    // GMRES workspace
    int m_alloc = 0;
    DevBuf<T> V, w, z, u;
    DevBuf<double2> H, g, sn, yv, hcol;
    DevBuf<double> cs;
    DevBuf<GmresState> gst;

    void init(const Csr<T> &A_, Precond<T> *M_, hipStream_t s_);
    // x = solution of A x = b from x = 0, relative tolerance rtol on the
    // recursive residual; returns iterations and flags
    // force_breakdown: every breakdown test fires (SS_FLAG_FORCE_BREAKDOWN)
    KrylovResult bicgstab(const T *b, T *x, double rtol, int maxiter, bool force_breakdown = false);
    KrylovResult gmres(const T *b, T *x, double rtol, int maxiter, int m);
};

}  // namespace ss
