// Rank instantiations above 32 (40 and 50) of the compressed ALS kernels
// (als_impl.h).
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_5(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s) {
  switch (R) {
    case 40: return als_launch<40>(phase, a, nb, nb0, seg, seg0, s);
    case 50: return als_launch<50>(phase, a, nb, nb0, seg, seg0, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
