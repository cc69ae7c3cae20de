// Launch sequence of PARAFAC2-ALS on the uncompressed slices (Alg. 2), the
// rank-templated kernels of plain_impl.h for R = 1..32.
#include "plain_impl.h"

namespace dpar2 {

template <int R>
static hipError_t plain_launch(int phase, const PlainArgs& a, const PlainLaunch& pl, hipStream_t s) {
  constexpr int RR = R * R;
  const int64_t K = a.K;
  const int J = a.J;
  hipError_t e;
  if (phase == 0) {   // begin
    hipLaunchKernelGGL(k_pl_begin<R>, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (phase == 2) {   // U output: Theta_k H
    hipLaunchKernelGGL(k_pl_theta<R>, dim3((unsigned)K), dim3(64), 0, s, a);
    return hipGetLastError();
  }
  const int n = J * R;
  hipLaunchKernelGGL(k_pl_commit, dim3((unsigned)std::min(64, (n + 255) / 256)), dim3(256), 0, s, a, n);
  if ((e = launch_slab(pl.slab, pl.dtype, pl.n_items, pl.vec, false, pl.wide, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl_slice<R>, dim3((unsigned)K), dim3(64), 0, s, a);
  if ((e = launch_segsum(1, nullptr, K, RR, RR, a.g1p, a.red, RR, s)) != hipSuccess) return e;
  if ((e = launch_segsum(1, nullptr, K, 1, 1, a.xnorm2, a.red + RED_WIDTH * RR + 1, 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl_h<R>, dim3(1), dim3(EPI_THREADS), 0, s, a);
  const unsigned nvb = (unsigned)((K + PL_VSLICES - 1) / PL_VSLICES);
  hipLaunchKernelGGL(k_pl_v<R>, dim3(nvb, (unsigned)((J + 255) / 256)), dim3(256), 0, s, a);
  if ((e = launch_segsum(1, nullptr, nvb, (int64_t)J * R, (int64_t)J * R, a.g2p, a.g2, (int64_t)J * R, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_pl_vupd<R>, dim3(1), dim3(EPI_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_pl_w<R>, dim3((unsigned)K), dim3(64), 0, s, a);
  if ((e = launch_segsum(1, nullptr, K, RR + 2, RR + 2, a.wp, a.red + 2 * RR, RR + 2, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl_err<R>, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_plain(int phase, int R, const PlainArgs& a, const PlainLaunch& pl, hipStream_t s) {
  switch (R) {
#define DPAR2_PL(R_) \
  case R_:           \
    return plain_launch<R_>(phase, a, pl, s);
    DPAR2_PL(1) DPAR2_PL(2) DPAR2_PL(3) DPAR2_PL(4) DPAR2_PL(5) DPAR2_PL(6) DPAR2_PL(7) DPAR2_PL(8)
    DPAR2_PL(9) DPAR2_PL(10) DPAR2_PL(11) DPAR2_PL(12) DPAR2_PL(13) DPAR2_PL(14) DPAR2_PL(15) DPAR2_PL(16)
    DPAR2_PL(17) DPAR2_PL(18) DPAR2_PL(19) DPAR2_PL(20) DPAR2_PL(21) DPAR2_PL(22) DPAR2_PL(23) DPAR2_PL(24)
    DPAR2_PL(25) DPAR2_PL(26) DPAR2_PL(27) DPAR2_PL(28) DPAR2_PL(29) DPAR2_PL(30) DPAR2_PL(31) DPAR2_PL(32)
#undef DPAR2_PL
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
