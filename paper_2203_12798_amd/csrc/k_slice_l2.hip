// Sketch-width instantiations 17..32 of the per-slice completion
// (slice_impl.h) and of the second-stage small kernels (stage2_impl.h).
#include "stage2_impl.h"

namespace dpar2 {

hipError_t slice_dispatch_2(int L, int64_t K, int J, int R, const int32_t* slice_ptr,
                              const int32_t* slice_list, const double* partG, const double* partP,
                              const double* partS, double* xnorm2, double* Mt, double* Phi, double* sig1,
                              float* omega_next, float* msgn, Ctl* ctl, const int32_t* slice_t, hipStream_t s) {
  switch (L) {
    case 17: return slice_fin_launch<17>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 18: return slice_fin_launch<18>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 19: return slice_fin_launch<19>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 20: return slice_fin_launch<20>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 21: return slice_fin_launch<21>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 22: return slice_fin_launch<22>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 23: return slice_fin_launch<23>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 24: return slice_fin_launch<24>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 25: return slice_fin_launch<25>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 26: return slice_fin_launch<26>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 27: return slice_fin_launch<27>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 28: return slice_fin_launch<28>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 29: return slice_fin_launch<29>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 30: return slice_fin_launch<30>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 31: return slice_fin_launch<31>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    case 32: return slice_fin_launch<32>(K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t s2_small_dispatch_2(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                                 double* D, double* E, double* U2s, double* small, Ctl* ctl, double* scratch,
                                 hipStream_t s) {
  switch (L2) {
    case 17: return s2_small_launch<17>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 18: return s2_small_launch<18>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 19: return s2_small_launch<19>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 20: return s2_small_launch<20>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 21: return s2_small_launch<21>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 22: return s2_small_launch<22>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 23: return s2_small_launch<23>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 24: return s2_small_launch<24>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 25: return s2_small_launch<25>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 26: return s2_small_launch<26>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 27: return s2_small_launch<27>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 28: return s2_small_launch<28>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 29: return s2_small_launch<29>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 30: return s2_small_launch<30>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 31: return s2_small_launch<31>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    case 32: return s2_small_launch<32>(nt, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
