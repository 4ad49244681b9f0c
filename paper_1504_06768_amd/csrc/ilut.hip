// Dual-threshold incomplete LU (ILUT) -- see ilu.hpp.
#include "ilu.hpp"

namespace ss {

IluResult ilut_factor(const CsrBuf<double2> &, const int *, double, double, double, double, CsrBuf<double2> &,
                      DevBuf<int> &, hipStream_t) {
    throw Error(SS_E_INVALID_ARG, "ILUT is not available in this build");
}

}  // namespace ss
