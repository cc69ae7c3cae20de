// Sketch-width instantiations 1..16 of the per-slice completion
// (slice_impl.h) and of the second-stage small kernels (stage2_impl.h).
#include "stage2_impl.h"

namespace dpar2 {

hipError_t slice_dispatch_1(int L, int64_t K, int J, int R, const int32_t* slice_ptr,
                              const int32_t* slice_list, const double* partG, const double* partP,
                              const double* partS, double* xnorm2, double* Mt, double* Phi, double* sig1,
                              float* omega_next, float* msgn, Ctl* ctl, const int32_t* slice_t, hipStream_t s) {
  switch (L) {
    case 1: return slice_fin_launch<1>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 2: return slice_fin_launch<2>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 3: return slice_fin_launch<3>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 4: return slice_fin_launch<4>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 5: return slice_fin_launch<5>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 6: return slice_fin_launch<6>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 7: return slice_fin_launch<7>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 8: return slice_fin_launch<8>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 9: return slice_fin_launch<9>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 10: return slice_fin_launch<10>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 11: return slice_fin_launch<11>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 12: return slice_fin_launch<12>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 13: return slice_fin_launch<13>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 14: return slice_fin_launch<14>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 15: return slice_fin_launch<15>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 16: return slice_fin_launch<16>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t s2_small_dispatch_1(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                                 double* D, double* E, double* U2s, double* small, Ctl* ctl, double* scratch,
                                 hipStream_t s) {
  switch (L2) {
    case 1: return s2_small_launch<1>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 2: return s2_small_launch<2>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 3: return s2_small_launch<3>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 4: return s2_small_launch<4>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 5: return s2_small_launch<5>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 6: return s2_small_launch<6>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 7: return s2_small_launch<7>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 8: return s2_small_launch<8>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 9: return s2_small_launch<9>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 10: return s2_small_launch<10>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 11: return s2_small_launch<11>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 12: return s2_small_launch<12>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 13: return s2_small_launch<13>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 14: return s2_small_launch<14>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 15: return s2_small_launch<15>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 16: return s2_small_launch<16>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
