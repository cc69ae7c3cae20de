// Slab-pass instantiations for bf16 slabs (sketch_impl.h): Omega rounded to bf16
// for the first pass, split into three bf16 pieces for a power step's
// per-slice sketch matrices.
#include "sketch_impl.h"

namespace dpar2 {

hipError_t slab_launch_bf16(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s) {
  if (a.omega)
    return uout ? slab_launch<DPAR2_BF16, true, true>(a, n_items, vec, s) : slab_launch<DPAR2_BF16, false, true>(a, n_items, vec, s);
  return uout ? slab_launch<DPAR2_BF16, true, false>(a, n_items, vec, s) : slab_launch<DPAR2_BF16, false, false>(a, n_items, vec, s);
}

}  // namespace dpar2
