/*
 * ss.h -- C ABI of the MI355X steady-state solver for Lindblad master equations.
 *
 * Method: P. D. Nation, "Steady-state solution methods for open quantum
 * optical systems".  Given a Hamiltonian H and collapse operators C_k (d x d
 * sparse matrices), find the density matrix rho with L vec(rho) = 0 and
 * Tr rho = 1, where L is the Lindblad Liouvillian (section "Steady-state
 * density matrix", eqs. lindblad and eigval) in column-stacking order,
 * vec(rho)[i + d*j] = rho[i, j].
 *
 * Every step of the solve runs in HIP kernels on the current GPU: Liouvillian
 * assembly, the trace-row or shift transform, reverse Cuthill-McKee ordering,
 * incomplete LU factorisation, sparse triangular solves, sparse
 * matrix-vector products and the preconditioned Krylov iterations.
 *
 * Conventions for every entry point:
 *   - return value: SS_OK (0) on success, a negative SS_E_* code on error,
 *     SS_PENDING (1) from ss_poll while a request is still running;
 *   - on error, ss_last_error() returns a message for the calling thread;
 *   - complex numbers are stored as interleaved (re, im) doubles;
 *   - pointers marked "host or device" may point to host memory or to memory
 *     allocated on the current HIP device; the library inspects the pointer;
 *   - input buffers are borrowed for the duration of the call only.
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define SS_OK               0
#define SS_PENDING          1
#define SS_E_INVALID_ARG   -1  /* bad shape, index, NaN/Inf, unknown enum   */
#define SS_E_OOM           -2  /* device or host allocation failed          */
#define SS_E_NOT_CONVERGED -3  /* iteration limit reached (section "Iterative
                                  Solvers": maximum number of iterations);
                                  the best iterate and its residual are still
                                  returned                                  */
#define SS_E_BREAKDOWN     -4  /* BiCGSTAB breakdown (residual orthogonal to
                                  the shadow residual, section "Numerical
                                  Simulations") and no fallback allowed     */
#define SS_E_ZERO_PIVOT    -5  /* structurally zero diagonal in the ILU      */
#define SS_E_HIP           -6  /* HIP runtime error                          */
#define SS_E_STATE         -7  /* call not valid for the handle's state      */
#define SS_E_TIMEOUT       -8  /* a bounded device-side wait gave up         */

/* --------------------------------------------------------------- inputs */
/* d x d complex sparse matrix in CSR form.  indptr has n+1 entries, column
 * indices are strictly increasing within a row and lie in [0, n); data holds
 * 2*nnz doubles (re, im).  All three arrays may be host or device memory
 * (all three on the same side). */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t *indptr;
    const int32_t *indices;
    const double *data;
} ss_csr_z;

/* opaque handles; each owns device memory until freed */
typedef struct ss_liouv_s *ss_liouv;
typedef struct ss_server_s *ss_server;

/* ------------------------------------------------------------ methods */
/* SS_TRACE_*  : the unit-trace linear system L~ x = w e_0 with
 *               L~ = L + w T (section "Direct factorization", eq. linear),
 *               w = mean of the diagonal of L (Fig. 4 caption), solved by
 *               ILU-preconditioned BiCGSTAB or restarted GMRES(m) (section
 *               "Iterative Solvers", eq. modified).
 * SS_INVPOW_* : the doubly-iterative inverse-power method (section
 *               "Iterative Solvers", last paragraph): shifted inverse power
 *               on L - sigma I (eqs. inverse, inverseiter) whose linear
 *               solves are ILU-preconditioned Krylov iterations with a
 *               tolerance one decade below the outer one. */
#define SS_TRACE_BICGSTAB   0
#define SS_TRACE_GMRES      1
#define SS_INVPOW_BICGSTAB  2
#define SS_INVPOW_GMRES     3
/* SS_AUTO: choose between the two drivers from the structure (section
 * "Numerical Simulations": the trace row can inflate the bandwidth of the
 * RCM-ordered matrix, and then inverse power is faster).  Both L~ and
 * L - sigma I are RCM-ordered; if the bandwidth of L~ exceeds 1.5 times that
 * of L - sigma I, or L~ has a diagonal entry below 1e-12 of its row's
 * largest (a zero diagonal the trace row does not cover, e.g. populations
 * under pure dephasing), SS_INVPOW_BICGSTAB is used.  Otherwise the trace
 * row: with GMRES, the paper's recommended first choice (section
 * "Conclusion"), for systems the device-wide kernels solve (n > 4096), and
 * with BiCGSTAB below that, where the whole solve runs in one
 * workgroup-resident launch (which has no GMRES) and is faster.
 * ss_solve only; info.method reports the choice. */
#define SS_AUTO             4

/* precision: SS_FP64 runs everything in complex128.  SS_MIXED runs the
 * inner Krylov iterations, ILU factors and SpMV in complex64 and keeps the
 * outer residual, correction accumulation and trace normalisation in fp64
 * (iterative refinement). */
#define SS_FP64   0
#define SS_MIXED  1

#define SS_ILU0   0  /* zero-fill ILU on the pattern of the permuted matrix */
#define SS_ILUT   1  /* dual-threshold ILU (drop_tol, fill), section
                        "Iterative Solvers" (iLUTP without pivoting)        */

#define SS_ORDER_RCM      0  /* reverse Cuthill-McKee on L~ + L~^T      */
#define SS_ORDER_NATURAL  1
#define SS_ORDER_COLOUR   2  /* colour classes: the greedy colouring of the
                                structure of L~ + L~^T visited in a seeded
                                random order (vertex v has priority
                                SplitMix64(v)), classes in increasing colour,
                                each in RCM order.  Not in the paper: no
                                off-diagonal entry joins two rows of one
                                class, so the ILU(0) substitutions have at
                                most as many dependent levels as colours
                                (about 14 on the Liouvillians here, against
                                ~10^3 in RCM order), at the price of more
                                Krylov iterations.  On the device-wide path
                                only the factors take this order: the
                                Krylov iteration and its SpMV stay in RCM
                                order, the permutation folded into the
                                first and last substitution.
                                ss_info.colours reports the count.        */

typedef struct {
    int32_t prec;       /* SS_FP64 | SS_MIXED                       (SS_FP64)  */
    int32_t ilu;        /* SS_ILU0 | SS_ILUT                        (SS_ILU0)  */
    int32_t ordering;   /* SS_ORDER_RCM | _NATURAL | _COLOUR        (RCM)      */
    int32_t gmres_m;    /* GMRES restart length m                   (20);
                           after an outer step whose GMRES did not converge
                           the next uses 2 m, up to 128                        */
    int32_t maxiter;    /* inner Krylov iteration limit per solve   (1000)     */
    int32_t max_outer;  /* outer refinement / inverse-power steps   (20)       */
    int32_t flags;      /* SS_FLAG_* bits                           (0)        */
    int32_t trace_row;  /* population k whose row k (N + 1) carries the trace
                           row T; -1 = the population row with the smallest
                           |L_rr| (ties: lowest k).  The paper notes the row
                           is arbitrary and uses row 0.                (-1)    */
    double drop_tol;    /* ILUT drop tolerance relative to ||row||_inf (1e-4)  */
    double fill;        /* ILUT entries kept per part, x nnz(row)     (10)     */
    double sigma;       /* inverse-power shift                        (1e-15)  */
    double inner_tol;   /* relative inner Krylov tolerance; 0 = default:
                           tol/10 relative to the outer residual in FP64,
                           1e-4 in SS_MIXED                                     */
    double weight;      /* trace-row weight w; 0 = mean diagonal of L          */
    int64_t seed;       /* seed of the random start (SS_FLAG_RANDOM_START) (0) */
    int32_t ilu_sweeps; /* SS_ILU0 on the device-wide path: 0 = the factors by
                           elimination; s > 0 = the same zero-fill factors as
                           the fixed point of (LU)_ij = a_ij on the pattern,
                           after s synchronous sweeps from l_ij = a_ij / a_jj,
                           u_ij = a_ij (Chow and Patel 2015; exact once s
                           covers the longest dependency chain, an
                           approximation of them before).  Not with the
                           workgroup-resident solve or ss_solve_batch
                           (SS_E_INVALID_ARG).                        (0)     */
    int32_t reserved;   /* 0                                                   */
} ss_options;

#define SS_FLAG_HERMITIZE   1  /* return (rho + rho^+)/2                      */
#define SS_FLAG_NO_FALLBACK 2  /* no fallback: neither GMRES after a BiCGSTAB
                                  breakdown nor iLUT + GMRES after an ILU(0)
                                  solve that fails                            */
#define SS_FLAG_DEVICE_WIDE 4  /* force the device-wide kernels (one kernel
                                  per step, all CUs) even for small systems   */
#define SS_FLAG_WORKGROUP   8  /* force the workgroup-resident solve (whole
                                  BiCGSTAB solve in one workgroup; chosen by
                                  default for BiCGSTAB up to n = 4096)        */
#define SS_FLAG_SYNCFREE   16  /* device-wide path: triangular solves
                                  sync-free over all CUs in row order         */
#define SS_FLAG_TRSV_BLOCK 32  /* device-wide path: triangular solves in one
                                  workgroup, level by level                   */
#define SS_FLAG_COND_EST  128  /* fill info.cond_est (one extra application
                                  of the preconditioner)                      */
#define SS_FLAG_TRSV_LEVELS 64 /* device-wide path: triangular solves
                                  sync-free over all CUs in level order     */
#define SS_FLAG_TRSV_GROUPS 1024 /* device-wide path: triangular solves
                                  sync-free over all CUs in level order, 16
                                  lanes per row, polling gated near the
                                  frontier (default: BLOCK up to n = 65536,
                                  else GROUPS)                               */
#define SS_FLAG_FORCE_BREAKDOWN 512 /* testing hook: every BiCGSTAB breakdown
                                  test fires (as if the shadow residual were
                                  orthogonal to the residual), so the restart
                                  and GMRES fallback paths run; not for
                                  production solves                          */
#define SS_FLAG_RANDOM_START 2048 /* inverse power starts from a random
                                  trace-1 Hermitian matrix (unit diagonal / N,
                                  off-diagonal entries drawn from opt.seed by
                                  a counter-based generator) instead of I / N;
                                  section "Eigenvalue Methods" starts the
                                  power iteration from a random vector        */
#define SS_FLAG_TRSV_CLASSES 4096 /* device-wide path: triangular solves with
                                  one launch per level (the default above
                                  n = 65536 when neither factor has more than
                                  64 levels, as in the colour-class order)  */
#define SS_FLAG_MATRIX_FREE 256 /* the fp64 residual of every outer step
                                  and the final certificate apply L from the
                                  d x d operators of eq. (lindblad) instead of
                                  streaming the assembled complex128 matrices
                                  (same values up to rounding order); implies
                                  the device-wide path                        */

typedef struct {
    int32_t status;          /* the call's return code                        */
    int32_t outer_its;       /* refinement or inverse-power steps             */
    int32_t inner_its;       /* total Krylov iterations                       */
    int32_t breakdowns;      /* BiCGSTAB restarts after breakdown             */
    int32_t pivots_guarded;  /* ILU pivots replaced by the guard value        */
    int32_t fell_back;       /* 1 if the solve left its first method: BiCGSTAB
                                breakdown -> GMRES, or, when ILU(0) cannot
                                precondition the system, the whole solve
                                again with iLUT and GMRES (device-wide)      */
    int32_t bandwidth;       /* B of the ordered matrix that was factorised   */
    int32_t path;            /* 0 device-wide kernels, 1 workgroup-resident
                                with the solve vector in global memory, 2
                                workgroup-resident with it in LDS             */
    int64_t profile;         /* P of the matrix that was factorised           */
    int64_t nnz_matrix;      /* nnz of L~ or L - sigma I                      */
    int64_t nnz_factors;     /* nnz(L) + nnz(U) of the ILU                    */
    double resid_l2;         /* ||L vec(rho)||_2 in fp64 with Tr rho = 1      */
    double herm_err;         /* max |rho - rho^+|                             */
    double trace_err;        /* |Tr rho - 1| before normalisation's rounding  */
    double cond_est;         /* ||(LU)^-1 e||_inf, e = ones (SS_FLAG_COND_EST) */
    double fill_factor;      /* nnz_factors / nnz_matrix                      */
    double weight;           /* w used by the trace row                       */
    double t_setup_ms;       /* transform + ordering + factorisation          */
    double t_solve_ms;       /* Krylov iterations + finish                    */
    double t_kernel_ms;      /* device time of the iteration kernels (HIP
                                events), workgroup-resident path only         */
    double bytes_alg;        /* algorithmic HBM bytes of the iterations:
                                matrix, factors and vectors once per use      */
    int32_t method;          /* the method that ran (resolves SS_AUTO)        */
    int32_t colours;         /* colour classes of SS_ORDER_COLOUR (else 0)    */
} ss_info;

/* fills *opt with the defaults listed above */
int ss_options_default(ss_options *opt);

/* ----------------------------------------------------- core entry points */
/* Assemble the Liouvillian of eq. (lindblad) on the device:
 *   L = -i (I (x) H - H^T (x) I)
 *       + sum_k [ conj(C_k) (x) C_k - 1/2 I (x) C_k^+ C_k - 1/2 (C_k^+ C_k)^T (x) I ]
 * as an n x n CSR matrix, n = N^2, with entries that sum to exactly zero
 * dropped.  H and c_ops[k] are N x N (host or device).  n_cops may be 0.
 * Limits: N <= 46340 and nnz(L) < 2^31.  *out receives a new handle. */
int ss_build_liouvillian(const ss_csr_z *H, const ss_csr_z *c_ops, int32_t n_cops,
                         int64_t N, ss_liouv *out);

/* Assemble count Liouvillians together: system k has H[k] (N_k = H[k].n)
 * and the n_cops[k] collapse operators c_ops[k][0 .. n_cops[k]) (c_ops[k]
 * may be NULL when n_cops[k] == 0).  Systems whose arrays are all device
 * memory and N_k <= 1024 are assembled by one set of launches for the whole
 * batch (the host waits twice per batch instead of several times per
 * system); any other system is built as by ss_build_liouvillian.  The
 * result is the same L as ss_build_liouvillian gives.  out[k] receives a new
 * handle.  On error every out[k] is NULL, no handle is left allocated, and
 * ss_last_error names the first invalid system. */
int ss_build_liouvillian_batch(int32_t count, const ss_csr_z *H, const ss_csr_z *const *c_ops,
                               const int32_t *n_cops, ss_liouv *out);

/* Solve for the steady state.  method: SS_TRACE_* or SS_INVPOW_*; tol: the
 * target for ||L vec(rho)||_2 with Tr rho = 1; opt: NULL for defaults.
 * rho_out: N*N complex (2*N*N doubles), column-major (= vec order), host or
 * device, caller-owned.  info may be NULL.  rho is always trace-normalised;
 * on SS_E_NOT_CONVERGED it holds the best iterate. */
int ss_solve(ss_liouv L, int32_t method, double tol, const ss_options *opt,
             double *rho_out, ss_info *info);

/* Solve `count` independent systems together (a parameter sweep, say): each
 * handle is set up on its own stream, then one launch of the workgroup-
 * resident solver runs one workgroup per system, side by side on the CUs.
 * method: SS_TRACE_BICGSTAB or SS_INVPOW_BICGSTAB; tol and opt as in
 * ss_solve, shared by all systems.  Ls: count distinct handles (borrowed).
 * rho_out: NULL or count pointers, each NULL or an N_i*N_i complex buffer
 * (host or device, caller-owned); infos: NULL or count entries; status:
 * NULL or count entries receiving each system's status.  Each system's
 * result equals that of a batch of one.  Returns SS_OK when every system
 * converged, else the status of the first one that did not. */
/* (The set-up runs on 8 host threads; the environment variable
 * SS_SETUP_THREADS = 1..64 changes that.) */
int ss_solve_batch(ss_liouv *Ls, int32_t count, int32_t method, double tol,
                   const ss_options *opt, double **rho_out, ss_info *infos,
                   int32_t *status);

void ss_liouv_free(ss_liouv L);

/* N, n = N^2 and nnz of the assembled Liouvillian */
int ss_liouv_shape(ss_liouv L, int64_t *N, int64_t *n, int64_t *nnz);

/* ------------------------------------------------ stage-wise inspection */
/* Run the problem transform, ordering and factorisation of a method (the
 * set-up half of ss_solve) and keep the results on the handle. */
int ss_prepare(ss_liouv L, int32_t method, const ss_options *opt);

#define SS_MAT_L         0  /* assembled Liouvillian, natural order            */
#define SS_MAT_A         1  /* transformed matrix (L~ or L - sigma I), natural  */
#define SS_MAT_A_PERM    2  /* transformed matrix after the ordering: P A P^T,
                               the matrix the Krylov iteration multiplies (in
                               RCM order when SS_ORDER_COLOUR factors run on
                               the device-wide path)                          */
#define SS_MAT_LU        3  /* ILU factors in one CSR: strict lower part of the
                               unit-lower L, then U with its diagonal          */
#define SS_MAT_SYM       4  /* symmetrised pattern of A used by RCM (data = 1)  */

/* Copy a matrix to host arrays.  Call first with indptr = indices = data =
 * NULL to get *nnz; then with arrays of n+1, nnz and 2*nnz entries. */
int ss_export_csr(ss_liouv L, int32_t which, int64_t *nnz, int64_t *indptr,
                  int32_t *indices, double *data);

/* Copy the ordering of the ILU factors, perm[new] = old (n entries), to a
 * host array.  With SS_ORDER_COLOUR on the device-wide path this is the
 * colour-class order while SS_MAT_A_PERM, the Krylov vectors and the vectors
 * of the SS_OP_* operators stay in RCM order: the preconditioner operators
 * apply (LU)^-1 through that permutation. */
int ss_export_perm(ss_liouv L, int32_t *perm);

#define SS_OP_SPMV_L      0  /* y = L x          (natural order, fp64)         */
#define SS_OP_SPMV_APERM  1  /* y = (P A P^T) x  (prec selects c128 / c64)     */
#define SS_OP_PRECOND     2  /* y = (LU)^-1 x    (prec selects c128 / c64),
                                the solver's own choice of the ways below:
                                BLOCK up to n = 65536; above, CLASSES when
                                no factor has more than 64 levels, else
                                GROUPS                                     */
#define SS_OP_LSOLVE      3  /* y = L_f^-1 x     unit lower factor             */
#define SS_OP_USOLVE      4  /* y = U_f^-1 x     upper factor                  */
#define SS_OP_PRECOND_SYNCFREE 5 /* y = (LU)^-1 x, sync-free solves over all
                                    CUs in row order                       */
#define SS_OP_PRECOND_BLOCK    6 /* y = (LU)^-1 x, one workgroup stepping
                                    through the level schedule             */
#define SS_OP_PRECOND_LEVELS   7 /* y = (LU)^-1 x, sync-free solves over all
                                    CUs in level order                     */
#define SS_OP_APPLY_L          8 /* y = L x (natural order, fp64) evaluated
                                    without the assembled matrix: vec of
                                    Gpre X + X Gpost^T + sum_k C_k X C_k^+,
                                    X the d x d matrix whose columns are the
                                    consecutive d-blocks of x (eq. lindblad,
                                    column stacking); needs no ss_prepare  */
#define SS_OP_PRECOND_GROUPS   9 /* y = (LU)^-1 x, sync-free solves over all
                                    CUs in level order, 16 lanes per row
                                    (one factor entry each), polling gated
                                    two levels behind the frontier         */
#define SS_OP_PRECOND_CLASSES 10 /* y = (LU)^-1 x with one launch per level
                                    of each factor: fast when the levels are
                                    few (the colour-class order); each row
                                    sums its products in a tree, so the
                                    result equals the others' to rounding */

/* Apply one operator of the prepared handle to x (n complex, host or
 * device) giving y (n complex, host or device).  prec = SS_FP64 or SS_MIXED:
 * in SS_MIXED x is rounded to complex64, the operator runs in complex64 and
 * y is widened back to complex128. */
int ss_apply(ss_liouv L, int32_t op, int32_t prec, const double *x, double *y);

/* ss_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same operators with the same kernels, no hipMalloc, hipFree or allocating
 * library call.  op = SS_OP_SPMV_L or SS_OP_APPLY_L (fp64), SS_OP_SPMV_APERM
 * or SS_OP_PRECOND (fp64 or SS_MIXED); SS_OP_PRECOND always takes the
 * row-group triangular solves (SS_OP_PRECOND_GROUPS) and needs the
 * schedules ss_prepare builds for the device-wide path (n > 4096, a GMRES
 * method or SS_FLAG_DEVICE_WIDE), else SS_E_STATE.  x and y: n complex128
 * (interleaved re, im), DEVICE pointers (else SS_E_INVALID_ARG), not
 * aliased.  Scratch: one library-owned device array of 64 MiB per device,
 * held until the process ends; a call needs 256 B plus 16 n B (fp64
 * PRECOND) or 24 n B (mixed PRECOND) or 16 n B (mixed SPMV_APERM), the
 * PRECOND vectors three times over (48 n B fp64, 40 n B mixed) when the
 * factors take the colour-class order on the device-wide path, and returns
 * SS_E_INVALID_ARG beyond that (n above ~4.19e6 fp64 and ~2.79e6 mixed, or
 * ~1.39e6 and ~1.67e6 in the colour-class order).
 * Every call on a device shares that array: calls that overlap on one
 * device (other threads, other handles) race.  Synchronous: returns after
 * the result is in y. */
int ss_apply_noalloc(ss_liouv L, int32_t op, int32_t prec, const double *x, double *y);

/* Time `reps` back-to-back applications of an operator of the prepared
 * handle (SS_OP_SPMV_L, SS_OP_APPLY_L, SS_OP_SPMV_APERM or one of the
 * SS_OP_PRECOND* operators; prec as in
 * ss_apply) on the handle's stream, bracketed by HIP events; *avg_ms
 * receives the mean time per application.  Input and output vectors are
 * library-owned device scratch.  Used to measure achieved bandwidth. */
int ss_time_operator(ss_liouv L, int32_t op, int32_t prec, int32_t reps, double *avg_ms);

/* Bandwidth B and profile P of a stage matrix (definitions of the section
 * "Direct factorization"), computed on the device. */
int ss_bandwidth_profile(ss_liouv L, int32_t which, int64_t *B, int64_t *P);

/* ------------------------------------------------------------- serving */
/* A server keeps many small solves resident on the device and advances them
 * side by side (continuous batching; not in the paper: a deployment of its
 * method for parameter sweeps).  Requests are admitted in arrival order while
 * fewer than max_slots are resident and their predicted device footprint
 * (an upper bound of the bytes a request holds while it runs) fits in
 * hbm_budget_bytes; a request larger than the whole budget is admitted
 * alone.  Several workers (host threads, environment SS_SERVER_WORKERS =
 * 1..16, default 4) each take a group -- the admitted head of the queue plus
 * later queued requests with the same method and options, at most one per
 * compute unit -- and run it on their own stream: batched assembly and set-up
 * stages, one launch of the workgroup-resident solver with one workgroup per
 * request, the finish.  A request that arrives while groups are on the
 * device is admitted as soon as a worker, a slot and memory are free, and
 * its work overlaps theirs on the device; a group's slots and memory return
 * to the budget when it finishes.  A worker that finds the queue still
 * growing waits until no request has arrived for SS_SERVER_WINDOW_US
 * microseconds (0..100000, default 200) or a full group is queued.
 * Each request's arithmetic stays in its own workgroup, so its result is
 * the same alone and in any group.  Returns SS_E_INVALID_ARG for a zero
 * budget or max_slots <= 0. */
int ss_server_create(size_t hbm_budget_bytes, int32_t max_slots, ss_server *out);

/* Queue a steady-state request (inputs, host or device, are copied to the
 * host and validated before return: a malformed matrix gives
 * SS_E_INVALID_ARG here, never a failed group).  method, tol and opt as in
 * ss_solve (SS_AUTO included).  Requests with SS_TRACE_BICGSTAB or
 * SS_INVPOW_BICGSTAB that the workgroup-resident solver takes (N^2 <= 4096,
 * or SS_FLAG_WORKGROUP; N <= 1024, at most 16 collapse operators) are
 * batched; any other request (GMRES, SS_AUTO, larger systems) is solved on
 * its own by a worker with the kernels of ss_solve.  *ticket identifies the
 * request. */
int ss_submit(ss_server S, const ss_csr_z *H, const ss_csr_z *c_ops, int32_t n_cops,
              int64_t N, int32_t method, double tol, const ss_options *opt,
              uint64_t *ticket);

/* Non-blocking.  Returns SS_PENDING while the request runs; otherwise the
 * request's status, with rho_out (N*N complex, host or device; NULL to
 * discard) and info filled, and the ticket retired.  An unknown or retired
 * ticket gives SS_E_INVALID_ARG. */
int ss_poll(ss_server S, uint64_t ticket, double *rho_out, ss_info *info);

/* Block until every queued request has finished. */
int ss_server_drain(ss_server S);

/* Occupancy of a server: the budget, the predicted footprint of the
 * requests resident now and the largest it has been, resident and queued
 * requests, groups run so far and the largest of them, workers, and the
 * largest group a worker forms. */
typedef struct {
    uint64_t budget_bytes;
    uint64_t resident_bytes;
    uint64_t peak_resident_bytes;
    int32_t resident;
    int32_t queued;
    uint64_t groups;
    uint64_t largest_group;
    int32_t workers;
    int32_t max_group;
} ss_server_stats_t;
int ss_server_stats(ss_server S, ss_server_stats_t *st);

/* Stops the workers after their current groups (queued requests are
 * dropped) and releases the server. */
void ss_server_destroy(ss_server S);

/* ---------------------------------------------------------------- misc */
/* thread-local message describing the last error */
const char *ss_last_error(void);

/* Make subsequent calls of this thread enqueue their work on a HIP stream
 * (a hipStream_t cast to void*; NULL = the library's own stream per handle).
 * The stream must outlive every handle used with it: device blocks released
 * by those handles are returned to the library's cache behind events
 * recorded on it. */
int ss_set_stream(void *hip_stream);

/* Route the library's device allocations through caller callbacks (e.g. a
 * framework's caching allocator): alloc(bytes, ctx) returns device memory or
 * NULL, free(ptr, ctx) releases it.  Pass NULL callbacks to return to
 * hipMalloc / hipFree.  Set it before any handle exists and do not change it
 * while device memory of the library is alive (blocks are returned to the
 * allocator that made them only by ss_trim_cache or at their release). */
typedef void *(*ss_alloc_fn)(size_t bytes, void *ctx);
typedef void (*ss_free_fn)(void *ptr, void *ctx);
int ss_set_allocator(ss_alloc_fn alloc, ss_free_fn free_fn, void *ctx);

/* Release every device block the library keeps cached for reuse (waits for
 * the last work that used them). */
int ss_trim_cache(void);

/* library version string */
const char *ss_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SS_H */
