// Sketch-width instantiations above 32 (40, 50 and 60) of the per-slice
// completion (slice_impl.h) and of the second-stage small kernels
// (stage2_impl.h).
#include "stage2_impl.h"

namespace dpar2 {

hipError_t slice_dispatch_3(int L, int64_t K, int J, int R, const int32_t* slice_ptr,
                            const int32_t* slice_list, const double* partG, const double* partP,
                            const double* partS, double* xnorm2, double* Mt, double* Phi, double* sig1,
                            float* omega_next, float* msgn, Ctl* ctl, const int32_t* slice_t, hipStream_t s) {
  switch (L) {
#define DPAR2_SF(L_)                                                                                        \
  case L_:                                                                                                  \
    return slice_fin_launch<L_>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, \
                                omega_next, msgn, ctl, slice_t, s);
    DPAR2_SF(40) DPAR2_SF(50) DPAR2_SF(60)
#undef DPAR2_SF
    default: return hipErrorInvalidValue;
  }
}

hipError_t s2_small_dispatch_3(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                               double* D, double* E, double* U2s, double* small, Ctl* ctl, double* scratch,
                               hipStream_t s) {
  switch (L2) {
    case 40: return s2_small_launch<40>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 50: return s2_small_launch<50>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 60: return s2_small_launch<60>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
