// Slab-pass instantiations for bf16 slabs (sketch_impl.h).
#include "sketch_impl.h"

namespace dpar2 {

hipError_t slab_launch_bf16(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s) {
  return uout ? slab_launch<DPAR2_BF16, true>(a, n_items, vec, s) : slab_launch<DPAR2_BF16, false>(a, n_items, vec, s);
}

}  // namespace dpar2
