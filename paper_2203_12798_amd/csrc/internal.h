// Host-side interfaces between the C ABI (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace dpar2 {

// One unit of first-stage work: rows [row0, row1) of slice `slice`.  Items are
// listed longest first (the GPU form of Alg. 4: the dispatcher hands the next
// item to the first free compute unit, which is the least-loaded one).
struct Item {
  int64_t row0;
  int64_t row1;
  int32_t slice;
  int32_t pad;
};

constexpr int SKETCH_TM = 64;          // rows per tile of the slab pass
constexpr int MAX_CHUNK_ROWS = 16384;  // longest item (rows)
constexpr int STAGE2_CHUNK = 256;      // rows of M^T per second-stage block
constexpr int ALS_THREADS = 256;

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
  int64_t K, J, N, n_items;
  int R, L, L2, max_iter;
  int64_t n2;             // second-stage row chunks of M^T
  int nblkA, nblkB, nblkC, nblkF;
  size_t ctl, items, slice_ptr, slice_list;
  size_t partG, partP, partS;
  size_t xnorm2, Mt, Phi, sig1;
  size_t Y2p, Y2, B2t, S2p, U2;
  size_t D, E, F, FtFp;
  size_t Psi, Pw, Mk, small, partA, partB, partC, partBegin, red, fitp, trace, om1, omq;
  size_t total;
};

// indices of R x R blocks inside Layout::small
enum SmallSlot {
  SM_BM = 0,     // E D^T V (current V)
  SM_GAM,        // Hadamard Gram (scratch)
  SM_HTH,        // H^T H
  SM_VTV,        // V^T V
  SM_WTW,        // W^T W
  SM_G3INV,      // (V^T V * H^T H)^dagger
  SM_HV,         // H^T H * V^T V
  SM_DTD,        // D^T D
  SM_FTF,        // F^T F
  SM_VC,         // V = D VC after a V update (R x R coordinates of V)
  SM_COUNT
};

constexpr int RED_MAXBLK = 1024;         // grid size cap of the per-slice kernels

// --- launchers (each returns the hipGetLastError() of its launches) ---------
// Arguments of the slab pass (sketch_impl.h, k_sketch.hip).
struct SlabArgs {
  const void* slab;        // N x J elements of the input type
  const float* scale;      // per-slice dequantisation scale (fp8), else unused
  int J, L, R;
  const float* omega;      // J x L (om_stride 0) or K x J x L (om_stride J L)
  int64_t om_stride;
  const Item* items;
  double *partG, *partP, *partS;
  const double* theta;     // U variant: K x L x R
  double* U;               // U variant: N x R
};
// Slab pass over all work items: per-item partials of Y^T Y, Y^T X and
// ||X||^2, or (uout) U = Y Theta_k.  dtype: dpar2_dtype.
hipError_t launch_slab(const SlabArgs& a, int dtype, int64_t n_items, bool uout, hipStream_t s);
// Per-slice completion of the first stage; omega_next (K x J x L float32, or
// NULL) receives the sketch matrix of a power step, the orthonormal right
// singular vectors of B_k (Alg. 1's power iteration in stabilised form).
hipError_t launch_slice_finish(int64_t K, int J, int L, int R, const int32_t* slice_ptr,
                               const int32_t* slice_list, const double* partG,
                               const double* partP, const double* partS, double* xnorm2,
                               double* Mt, double* Phi, double* sig1, float* omega_next, Ctl* ctl,
                               hipStream_t s);
hipError_t launch_stage2(const Layout& lay, char* ws, const float* omega2, hipStream_t s);
// out[e] = sum_{b < nb} part[b * stride + e] for e < width, in a fixed order
hipError_t launch_colsum(int64_t nb, int64_t stride, int64_t width, const double* part, double* out,
                         hipStream_t s);
hipError_t launch_als_begin(const Layout& lay, char* ws, double* H, double* V, double* W, hipStream_t s);
hipError_t launch_als_iteration(const Layout& lay, char* ws, double* H, double* V, double* W,
                                double* err_trace, double tol, hipStream_t s);
hipError_t launch_fitness(const Layout& lay, char* ws, const double* H, const double* V,
                          const double* W, double* fit, hipStream_t s);
hipError_t launch_theta(const Layout& lay, char* ws, const double* H, double* theta,
                        hipStream_t s);

hipError_t launch_pw_identity(const Layout& lay, char* ws, hipStream_t s);
hipError_t launch_als_end(const Layout& lay, char* ws, double* V, hipStream_t s);
int als_blocks(int64_t K, int R);

bool sketch_supported(int J, int L, int dtype);

}  // namespace dpar2
