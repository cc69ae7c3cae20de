// Slab-pass instantiations for fp8 slabs (sketch_impl.h).
#include "sketch_impl.h"

namespace dpar2 {

hipError_t slab_launch_fp8(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s) {
  return uout ? slab_launch<DPAR2_FP8_E4M3, true>(a, n_items, vec, s) : slab_launch<DPAR2_FP8_E4M3, false>(a, n_items, vec, s);
}

}  // namespace dpar2
