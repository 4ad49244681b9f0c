// The Liouvillian handle and the set-up / solve drivers (solve.hip).
#pragma once
#include "blas.hpp"
#include "ilu.hpp"
#include "krylov.hpp"
#include "lindblad.hpp"

struct ss_liouv_s {
    int64_t N = 0;
    int d = 0;
    int n = 0;
    hipStream_t own_stream = nullptr;
    ss::CsrBuf<double2> L;  // assembled Liouvillian, natural order
    ss::LindbladBuf lin;    // its d x d operators (matrix-free application)

    // results of the set-up stage (ss_prepare)
    bool prepared = false;
    int p_method = -1;
    ss_options p_opt{};
    ss::CsrBuf<double2> A;     // L~ or L - sigma I, natural order
    ss::CsrBuf<double2> S;     // symmetrised pattern of A
    ss::DevBuf<int> perm, iperm;
    ss::CsrBuf<double2> Ap;    // P A P^T (fp64)
    ss::CsrBuf<float2> Ap32;   // P A P^T (complex64, mixed precision)
    ss::DevBuf<int> diag;      // diagonal positions in Ap
    ss::CsrBuf<double2> LU;    // ILU factors (fp64)
    ss::CsrBuf<float2> LU32;   // ILU factors rounded to complex64
    ss::DevBuf<int> lu_diag;   // diagonal positions in LU
    ss::DevBuf<int> tpos;      // permuted positions of the diagonal of rho
    ss::DevBuf<double2> d_w;   // trace-row weight (device)
    double2 w = {0, 0};
    int trow = 0;              // row of L~ carrying the trace row T
    int q0 = 0;                // its position after the ordering
    int guarded = 0;
    int diag_added = 0;        // explicit zero diagonals added to Ap
    int colours = 0;           // colour classes of SS_ORDER_COLOUR (else 0)
    ss::DevBuf<int> lorder;    // SS_ORDER_COLOUR: row of each RCM position (rows' order inside a level)
    std::vector<int> class_ptr;  // SS_ORDER_COLOUR: first row of each class in the factors' order, then n
    // SS_ORDER_COLOUR on the device-wide path: the Krylov iteration runs in
    // RCM order (perm, Ap) and the factors in the colour-class order; cp[q]
    // is the RCM position of factor row q (lorder is its inverse)
    bool split = false;
    ss::DevBuf<int> cp;
    double t_setup_ms = 0;
    // level schedules of the factors and the gates of the row-group
    // triangular solves, built by ss_prepare for the device-wide path and
    // used by its solves and by ss_apply_noalloc
    bool sched_ready = false;
    ss::LevelSched sched_lo, sched_up;
    ss::DevBuf<int> gate_lo, gate_up;
};

#include "wgsolve.hpp"

namespace ss {

hipStream_t stream_of(ss_liouv h);    // the handle's stream, made the thread's current one
hipStream_t stream_peek(ss_liouv h);  // the handle's stream (current stream unchanged)
void prepare(ss_liouv h, int method, const ss_options &o);
int solve(ss_liouv h, int method, double tol, const ss_options &o, double *rho_out, ss_info *info);
// The same system again with iLUT and GMRES on the device-wide path (the
// fallback when ILU(0)-preconditioned solves fail); sets info->fell_back.
int solve_ilut_gmres(ss_liouv h, int method, double tol, const ss_options &o, double *rho_out, ss_info *info);
// tols (optional, count entries) gives each system its own tolerance.
int solve_batch(ss_liouv *hs, int count, int method, double tol, const ss_options &o, double **rho_out,
                ss_info *infos, int *status, const double *tols = nullptr);
const std::string &batch_error();  // message of the first failed system of the last batch (this thread)
bool use_workgroup(ss_liouv h, int method, const ss_options &o);
bool use_workgroup_n(int64_t n, int method, const ss_options &o);  // the same rule for a size n = N^2

// Counters of one solve, handed to finish().
struct SolveStats {
    int status = SS_E_NOT_CONVERGED;
    int outer = 0, inner = 0, breakdowns = 0, fell_back = 0, path = 0;
    double t_solve_ms = 0.0, t_kernel_ms = 0.0, elem_bytes = 16.0;
};

// Device state of one workgroup-resident solve.
template <typename T>
struct WgBundle {
    LevelSched lo, up;
    PackedSide<T> pl, pu;
    DevBuf<T> work, ysc;
    DevBuf<double2> x, r, b;
    DevBuf<WgResult> res;
    WgProblem<T> P;
    int levels = 0;
};

// Build the workgroup problem of a prepared handle (level schedules, packed
// factors, start vector, scratch).
template <typename T>
void make_wg(ss_liouv h, int method, double tol, const ss_options &o, const CsrBuf<T> &Ain, const CsrBuf<T> &LUin,
             WgBundle<T> &B, hipStream_t s, bool levels_built = false);

// The outcome (status) of a solve and its info record (when info != null)
// from the certificate ||L rho||, the Hermiticity and trace errors and the
// bandwidth and profile of P A P^T.
int fill_info(ss_liouv h, const ss_options &o, double tol, const SolveStats &st, double final_res, double herm_err,
              double2 trx, int64_t bandwidth, int64_t profile, ss_info *info, hipStream_t s);

// Unpermute, normalise, certify and copy out the solution x (permuted, fp64).
int finish(ss_liouv h, const double2 *x, const ss_options &o, double tol, const SolveStats &st, double *rho_out,
           ss_info *info, hipStream_t s);

}  // namespace ss
