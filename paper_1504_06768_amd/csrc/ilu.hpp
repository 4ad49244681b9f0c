// ILU factorisation and its application (ilu.hip).
#pragma once
#include "ss_internal.hpp"
#include "syncfree.hpp"
#include "levels.hpp"

namespace ss {

struct IluResult {
    int guarded = 0;
};

// ILU(0) of A (rows sorted, diagonal positions in diag) in fp64; pivots below
// detect * ||a_i||_inf become boost * ||a_i||_inf (phase kept).
IluResult ilu0_factor(const CsrBuf<double2> &A, const int *diag, double detect, double boost, CsrBuf<double2> &LU,
                      hipStream_t s);

// ILU(0) of many systems in one launch, one workgroup each.  prepare() sets
// up one system (factor storage, scratch, flags) on its stream; after
// ilu0_batch has run every job, result() reads that system's outcome.
struct Ilu0Job {
    int n;
    const int *rowptr, *col, *diag;
    const double2 *a;
    double2 *w, *out;
    unsigned *status;
    int *nguard;
    // level schedule of the strict lower part (ilu0_levels_batch only)
    int nlev;
    const int *lptr;
    const int4 *lslot;
};
struct Ilu0Batch {
    DevBuf<double2> work;
    DevBuf<unsigned> flags;  // status word, guarded-pivot count
    Ilu0Job prepare(const CsrBuf<double2> &A, const int *diag, CsrBuf<double2> &LU, hipStream_t s);
    IluResult result(hipStream_t s);
};
void ilu0_batch(const Ilu0Job *jobs, int count, double detect, double boost, hipStream_t s);
// The same factorisation level by level (jobs carry their lower-part level
// schedules; no dependency waits); the factor values need no sentinel.
void ilu0_levels_batch(const Ilu0Job *jobs, int count, double detect, double boost, hipStream_t s);

// The same factors with one launch per level of the lower schedule `lo`
// (built from A's pattern, which zero fill keeps): no dependency waits, so
// fast when the levels are few and wide (the colour-class order).
IluResult ilu0_factor_levels(const CsrBuf<double2> &A, const int *diag, const LevelSched &lo, double detect,
                             double boost, CsrBuf<double2> &LU, hipStream_t s);

// Dual-threshold ILUT (drop_tol relative to ||row||_inf, at most
// ceil(fill * nnz(row)) entries kept in each of L and U per row).
IluResult ilut_factor(const CsrBuf<double2> &A, const int *diag, double drop_tol, double fill, double detect,
                      double boost, CsrBuf<double2> &LU, DevBuf<int> &lu_diag, hipStream_t s);

constexpr double PIVOT_DETECT = 1e-8;  // relative to ||a_i||_inf
constexpr double PIVOT_BOOST = 1e-1;

template <typename T>
void fill_sentinel(int64_t n, T *p, hipStream_t s);

void round_to_c64(int64_t n, const double2 *a, float2 *b, hipStream_t s);

// Ways of applying (L U)^-1: sync-free in row order over all CUs, one
// workgroup stepping through the levels, sync-free in level order over all
// CUs, the choice by size, row groups in level order, or one launch per
// level (shallow schedules).
enum : int { PRE_ROWS = 0, PRE_BLOCK = 1, PRE_LEVELS = 2, PRE_AUTO = 3, PRE_GROUPS = 4, PRE_CLASSES = 5 };
constexpr int PRE_BLOCK_MAX_N = 65536;
// deepest schedule (levels per factor) the automatic choice solves with one
// launch per level
constexpr int PRE_CLASSES_MAX_LEVELS = 64;

// One triangular solve over the level schedule `ls` with one launch per level
// (trsv_classes.hip): lower out = L^-1 in, upper out = U^-1 in.  No sentinels
// are used or restored; nothing runs when *skip != 0 on the device.  With
// pin (a permutation: factor row q is position pin[q] of the caller's
// vectors) the lower solve reads in[pin[q]] and the upper one also writes
// outp[pin[q]].
template <typename T>
void trsv_classes(const LevelSched &ls, bool upper, const Csr<T> &LU, const T *in, T *out, const int *skip,
                  hipStream_t s, const int *pin = nullptr, T *outp = nullptr);

// Sync-free triangular solves over all CUs with 16 lanes per row, in level
// order, polling gated two levels behind the frontier (trsv_groups.hip).
// group_gates: for every task of 4 consecutive slots, the last row of the
// level two below the level of its first slot (-1 if none).
constexpr int GROUP_WAVES = 2048;  // persistent wavefronts per launch
void group_gates(const LevelSched &ls, int n, DevBuf<int> &gate, hipStream_t s);
// One triangular solve over the level schedule `ls` (lower: out = L^-1 in,
// and `reset` -- the output of the following upper solve -- back to the
// sentinel; upper: out = U^-1 in, and `in` back to the sentinel).  `out`
// must hold the sentinel on entry; ctl: four control words at zero (zero
// again on return).
template <typename T>
void trsv_groups(const LevelSched &ls, const int *gate, bool upper, const Csr<T> &LU, const T *in, T *out, T *reset,
                 unsigned *ctl, unsigned *status, const int *skip, hipStream_t s);

// M^-1 = (L U)^-1 applied with the sync-free triangular solves.
template <typename T>
struct Precond {
    const CsrBuf<T> *LU = nullptr;
    const int *diag = nullptr;
    int n = 0;
    DevBuf<T> y;           // lower-solve result, kept at the sentinel between applies
    // pin (optional): factor row q is position pin[q] of the vectors apply()
    // takes and returns (the colour-class factors of a solve run in RCM
    // order); pb/pz hold the permuted vectors
    const int *pin = nullptr;
    DevBuf<T> pb, pz;
    DevBuf<unsigned> status;
    BlockCounter counter;
    // level-scheduled modes (apply() uses them once built)
    int mode = PRE_ROWS;
    LevelSched lo, up;
    PackedSide<T> pl, pu;
    DevBuf<int> gate_lo, gate_up;  // PRE_GROUPS
    DevBuf<T> bl;
    DevBuf<unsigned> lev_ctr;  // control words of the level-order launches (PRE_LEVELS, PRE_GROUPS)
    void setup(const CsrBuf<T> *lu, const int *dg, int n_, hipStream_t s);
    // Build the level schedules (from the fp64 factors' pattern, which the
    // rounded copy shares) and packed factors, and switch apply() to a
    // level-scheduled solve: PRE_BLOCK (one workgroup, barrier per level),
    // PRE_LEVELS (sync-free over all CUs in level order), PRE_GROUPS (the
    // same with 16 lanes per row and gated polling), PRE_CLASSES (one launch
    // per level) or PRE_AUTO (PRE_BLOCK for n <= PRE_BLOCK_MAX_N, else
    // PRE_CLASSES when no factor has more than PRE_CLASSES_MAX_LEVELS
    // levels, else PRE_GROUPS).
    void use_levels(const Csr<double2> &lu64, hipStream_t s, int m = PRE_AUTO, const int *order = nullptr);
    // PRE_GROUPS over level schedules and gates owned by the caller (they
    // must outlive this object)
    void borrow_groups(const LevelSched *lo_, const LevelSched *up_, const int *glo, const int *gup, hipStream_t s);
    // PRE_CLASSES over level schedules owned by the caller (they must
    // outlive this object)
    void borrow_classes(const LevelSched *lo_, const LevelSched *up_);
    const LevelSched *blo = nullptr, *bup = nullptr;
    const int *bglo = nullptr, *bgup = nullptr;
    // out = (LU)^-1 b; out must not alias b or y.  When *skip != 0 on the
    // device, both solves return at once (used after convergence).
    void apply(const T *b, T *out, hipStream_t s, const int *skip = nullptr);
    void lower(const T *b, T *out, hipStream_t s);
    void upper(const T *b, T *out, hipStream_t s);
    unsigned read_status(hipStream_t s);
};

}  // namespace ss
