// Rank instantiations 17..24 of the compressed ALS kernels (als_impl.h).
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_3(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s) {
  switch (R) {
    case 17: return als_launch<17>(phase, a, nb, nb0, seg, seg0, s);
    case 18: return als_launch<18>(phase, a, nb, nb0, seg, seg0, s);
    case 19: return als_launch<19>(phase, a, nb, nb0, seg, seg0, s);
    case 20: return als_launch<20>(phase, a, nb, nb0, seg, seg0, s);
    case 21: return als_launch<21>(phase, a, nb, nb0, seg, seg0, s);
    case 22: return als_launch<22>(phase, a, nb, nb0, seg, seg0, s);
    case 23: return als_launch<23>(phase, a, nb, nb0, seg, seg0, s);
    case 24: return als_launch<24>(phase, a, nb, nb0, seg, seg0, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
