// Slab-pass instantiations for f32 slabs (sketch_impl.h).
#include "sketch_impl.h"

namespace dpar2 {

hipError_t slab_launch_f32(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s) {
  return uout ? slab_launch<DPAR2_F32, true, true>(a, n_items, vec, s)
              : slab_launch<DPAR2_F32, false, true>(a, n_items, vec, s);
}

}  // namespace dpar2
