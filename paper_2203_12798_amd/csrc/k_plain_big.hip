// Rank instantiations above 32 (40 and 50) of PARAFAC2-ALS on the
// uncompressed slices (plain_impl.h).
#include "plain_impl.h"

namespace dpar2 {

hipError_t launch_plain_big(int phase, int R, const PlainArgs& a, const PlainLaunch& pl, hipStream_t s) {
  switch (R) {
    case 40: return plain_launch<40>(phase, a, pl, s);
    case 50: return plain_launch<50>(phase, a, pl, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
