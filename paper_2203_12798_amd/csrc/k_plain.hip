// Launch sequence of PARAFAC2-ALS on the uncompressed slices (Alg. 2), the
// rank-templated kernels of plain_impl.h for R = 1..32 (40 and 50: k_plain_big.hip).
#include "plain_impl.h"

namespace dpar2 {

hipError_t launch_plain_big(int phase, int R, const PlainArgs& a, const PlainLaunch& pl, hipStream_t s);

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
      return launch_plain_big(phase, R, a, pl, s);
  }
}

}  // namespace dpar2
