// Rank instantiations 1..8 of the compressed ALS kernels (als_impl.h).
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_1(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s) {
  switch (R) {
    case 1: return als_launch<1>(phase, a, nb, nb0, seg, seg0, s);
    case 2: return als_launch<2>(phase, a, nb, nb0, seg, seg0, s);
    case 3: return als_launch<3>(phase, a, nb, nb0, seg, seg0, s);
    case 4: return als_launch<4>(phase, a, nb, nb0, seg, seg0, s);
    case 5: return als_launch<5>(phase, a, nb, nb0, seg, seg0, s);
    case 6: return als_launch<6>(phase, a, nb, nb0, seg, seg0, s);
    case 7: return als_launch<7>(phase, a, nb, nb0, seg, seg0, s);
    case 8: return als_launch<8>(phase, a, nb, nb0, seg, seg0, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
