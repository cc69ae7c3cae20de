// Rank instantiations 25..32 of the compressed ALS kernels (als_impl.h).
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_4(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s) {
  switch (R) {
    case 25: return als_launch<25>(phase, a, nb, nb0, seg, seg0, s);
    case 26: return als_launch<26>(phase, a, nb, nb0, seg, seg0, s);
    case 27: return als_launch<27>(phase, a, nb, nb0, seg, seg0, s);
    case 28: return als_launch<28>(phase, a, nb, nb0, seg, seg0, s);
    case 29: return als_launch<29>(phase, a, nb, nb0, seg, seg0, s);
    case 30: return als_launch<30>(phase, a, nb, nb0, seg, seg0, s);
    case 31: return als_launch<31>(phase, a, nb, nb0, seg, seg0, s);
    case 32: return als_launch<32>(phase, a, nb, nb0, seg, seg0, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dpar2
