// Batched set-up stages (setup_batch.hip).
#pragma once
#include <unordered_map>

#include "handle.hpp"

namespace ss {

// For every handle: the trace-row transform (trace) or the shift by
// o.sigma, the weight and trace row, and the symmetrised pattern S -- what
// the transform stage of ss_prepare computes, with the same results -- for
// the whole batch at once, kernels on s.  Options must have been validated.
void transform_batch(ss_liouv *hs, int count, bool trace, const ss_options &o, hipStream_t s);

// For every handle with its ordering: P A P^T, the diagonal positions, the
// trace positions and q0 (as prepare_permute and prepare_finish give them),
// and with ilu0 the factor's pattern (that of P A P^T, values at the
// sentinel) and its diagonal positions.  res[k].missing counts the rows of
// P A P^T without a diagonal entry: such a handle needs the explicit zero
// diagonal of prepare_permute before its factorisation (and its factor
// pattern again).
struct PermResult {
    int missing = 0;
};
void permute_batch(ss_liouv *hs, int count, bool ilu0, hipStream_t s, std::vector<PermResult> &res);

// Level analysis of both factor sides of many handles (their LU pattern
// and diagonal positions in place -- for ILU(0) the pattern of P A P^T, so
// the lower side also schedules the factorisation itself) and the level
// schedules: ptr (nlev + 1) and slots {row, first, end, 0} in level order.
struct LevelBatch {
    DevBuf<unsigned char> arena;
    std::vector<ss_liouv> hs;
    std::unordered_map<ss_liouv, int> pos;
    std::vector<int> nl, nu;
    std::vector<const int *> lptr, uptr;
    std::vector<const int4 *> lslot, uslot;
};
void levels_setup_batch(ss_liouv *hs, int count, hipStream_t s, LevelBatch &out);

// Workgroup-resident problems of many prepared handles with their level
// schedules (lb): packed factors, start vectors and scratch -- what make_wg
// builds for one handle -- in one arena for the whole batch; tols[k] is the
// tolerance of hs[k].  probs[k] and levels[k] (nlev_l + nlev_u) belong to
// hs[k]; the arenas must outlive the solve.
template <typename T>
struct WgBatch {
    DevBuf<unsigned char> arena;
    std::vector<WgProblem<T>> probs;
    std::vector<int> levels;
};
template <typename T>
void wg_setup_batch(ss_liouv *hs, int count, int method, const double *tols, const ss_options &o,
                    const LevelBatch &lb, hipStream_t s, WgBatch<T> &out);

// finish() for many systems in one launch (one block each): xs[k] is the
// permuted fp64 solution of hs[k], rho_out[k] (host, device or null) and
// infos[k] (or null) receive its results, status[k] its outcome.
void finish_batch(ss_liouv *hs, int count, const double2 *const *xs, const ss_options &o, const double *tols,
                  const SolveStats *st, double *const *rho_out, ss_info *const *infos, int *status, hipStream_t s);

// The complex64 copies of P A P^T and of the ILU factor of every handle
// (mixed precision), one launch.
void c64_copies_batch(ss_liouv *hs, int count, hipStream_t s);

// out[k] = *src[k] (device result records), one host wait.
void read_results(const std::vector<const WgResult *> &src, std::vector<WgResult> &out, hipStream_t s);

// the handle's P A P^T and ILU factor in precision T
template <typename T> const CsrBuf<T> &ap_of(ss_liouv h);
template <typename T> const CsrBuf<T> &lu_of(ss_liouv h);
template <> inline const CsrBuf<float2> &ap_of<float2>(ss_liouv h) { return h->Ap32; }
template <> inline const CsrBuf<double2> &ap_of<double2>(ss_liouv h) { return h->Ap; }
template <> inline const CsrBuf<float2> &lu_of<float2>(ss_liouv h) { return h->LU32; }
template <> inline const CsrBuf<double2> &lu_of<double2>(ss_liouv h) { return h->LU; }

}  // namespace ss
