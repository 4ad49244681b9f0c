// Level schedules of the ILU triangular factors and their packed level-order
// copies (wgsolve.hip), shared by the workgroup-resident solver and the
// single-workgroup triangular solves of the device-wide path.
#pragma once
#include "ss_internal.hpp"

namespace ss {

// Level schedule of one triangular factor: slots in level order, each slot
// {row, first entry, end entry, w} with w the row's end in the factor for
// the lower side (the ILU(0) of a batch reads it) and 0 for the upper side;
// levels delimited by ptr.
struct LevelSched {
    int nlev = 0;
    DevBuf<int> ptr;    // nlev + 1
    DevBuf<int4> slot;  // n; rows in increasing order within a level
    std::vector<int> hptr;  // host copy of ptr
};

// Level sets of the strict lower part (forward) and of the strict upper part
// (backward) of the ILU factors; a row's level is one more than the largest
// level among the rows it depends on.
// order (optional, n entries): the rows in the order they take inside a
// level (default: increasing row index).
// classes (optional, host, ascending, first 0 and last n): runs of rows with
// no entry between two rows of one run (the colour-class order of a
// zero-fill factor); each run's levels then take one launch with no waits,
// and an entry inside a run is an error.
void build_levels(const Csr<double2> &LU, const int *diag, LevelSched &lo, LevelSched &up, hipStream_t s,
                  const int *order = nullptr, const std::vector<int> *classes = nullptr);

// The level analysis of many systems in one launch (one workgroup each):
// job() sets up one system's scratch on its stream, levels_batch runs every
// job of one side, finish() turns one system's levels into its schedule.
struct LevelJob {
    int n;
    const int *rowptr, *col, *diag;
    int *lvl;
    unsigned *status;
    int *maxlvl;
};
struct LevelBuild {
    DevBuf<int> lvl, misc;
    DevBuf<unsigned> status;
    LevelJob job(const Csr<double2> &LU, const int *diag, hipStream_t s);
    template <bool UPPER>
    void finish(const Csr<double2> &LU, const int *diag, LevelSched &ls, hipStream_t s, const int *order = nullptr);
};
template <bool UPPER>
void levels_batch(const LevelJob *jobs, int count, hipStream_t s);

// factor entries per row kept in the packed level layout (fewer for
// complex128 so that three levels of them fit in registers).  Longer rows
// take their remaining entries from the factor's CSR arrays, one dependent
// load at a time.  For complex64, 7 covers all but two rows per triangle of
// the Jaynes-Cummings Liouvillian (cavity 40 x qubit) and measured fastest of
// 6, 7 and 8 there (preconditioner time per system 11.7, 9.9, 10.4 ms).  For
// complex128, 5 is the widest without register spills (6 and 7 spill); on
// the same batch the fp64 solver launch takes 56.9 ms against 62.0 ms at 4.
template <typename T> struct WgK;
template <> struct WgK<float2> { static constexpr int value = 7; };
template <> struct WgK<double2> { static constexpr int value = 5; };

// Level-ordered packed copy of one triangular factor in precision T: for
// slot idx (level order), slot[idx] = {row, first CSR entry, length, 0}, and
// the first WgK<T> column indices and values of the row at
// col[k * n + idx], val[k * n + idx] (zero padded); aux[idx] is the pivot
// u_ii for the upper factor.  Every load of a slot is addressed by idx alone.
template <typename T>
struct PackedSide {
    DevBuf<int4> slot;
    DevBuf<int> col;
    DevBuf<T> val;
    DevBuf<T> aux;
};

template <typename T>
void pack_side(const LevelSched &ls, const Csr<T> &LU, bool upper, PackedSide<T> &out, hipStream_t s);

// Level schedules and packed factors for the single-workgroup triangular
// solve pair of the device-wide path.
template <typename T>
struct BlockPrecond {
    const LevelSched *lo = nullptr, *up = nullptr;
    const PackedSide<T> *pl = nullptr, *pu = nullptr;
};

// out = (L U)^-1 b in one workgroup (bl: n scratch); returns at once when
// *skip != 0 on the device.
template <typename T>
void precond_block(const BlockPrecond<T> &B, const Csr<T> &LU, const T *b, T *out, T *bl, hipStream_t s,
                   const int *skip);

}  // namespace ss
