// Rank instantiations 9..16 of the compressed ALS kernels (als_impl.h).
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_2(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s) {
  switch (R) {
    case 9: return als_launch<9>(phase, a, nb, nb0, seg, seg0, s);
    case 10: return als_launch<10>(phase, a, nb, nb0, seg, seg0, s);
    case 11: return als_launch<11>(phase, a, nb, nb0, seg, seg0, s);
    case 12: return als_launch<12>(phase, a, nb, nb0, seg, seg0, s);
    case 13: return als_launch<13>(phase, a, nb, nb0, seg, seg0, s);
    case 14: return als_launch<14>(phase, a, nb, nb0, seg, seg0, s);
    case 15: return als_launch<15>(phase, a, nb, nb0, seg, seg0, s);
    case 16: return als_launch<16>(phase, a, nb, nb0, seg, seg0, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
