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
  int64_t tslot;   // first slot of the item's tiles in the wide pass's Y-digit buffer
};

constexpr int SKETCH_TM = 64;          // rows per tile of the slab pass
// Ranks and sketch widths: every value up to 32, and above 32 the ranks 40 and
// 50 and the sketch widths 40, 50 and 60 (the per-slice R x R and L x L
// factorisations give each column one lane of a 64-lane wave)
constexpr int MAX_RANK = 64;
inline bool rank_supported(int R) { return (R >= 1 && R <= 32) || R == 40 || R == 50; }
inline bool width_supported(int L) { return (L >= 1 && L <= 32) || L == 40 || L == 50 || L == 60; }
constexpr int MAX_CHUNK_ROWS = 16384;  // longest item (rows)
constexpr int STAGE2_CHUNK = 256;      // rows of M^T per second-stage block (one per thread)
// J from which the second stage's J-long steps (Gram and whitening of Y2,
// D = Q2 U2_R, D^T D) run on one wave per 64 rows instead of one per tensor
constexpr int S2_WIDE_J = 512;
// doubles of second-stage scratch for that form (nt tensors, sketch width
// L2, rank R): the 64-row partials, the summed Gram and Wh / U2_R
inline int64_t s2_scratch_doubles(int64_t nt, int64_t J, int64_t L2, int64_t R) {
  if (J < S2_WIDE_J) return 0;
  const int64_t M = L2 > R ? L2 : R;
  return nt * (((J + 63) / 64) * M * M + 2 * L2 * L2);
}
// rows of M^T per block of the second-stage sketch Y2 = M Omega_2 (one wave
// per 64 columns): about 8192 waves over a tensor's K R rows, 64 to 2048
// rows each, a multiple of 64 (per tensor, so that a tensor in a batch is
// blocked as when decomposed alone)
inline int64_t stage2_ychunk(int64_t KR, int64_t J) {
  int64_t r = (KR * ((J + 63) / 64) + 8191) / 8192;
  r = (r + 63) / 64 * 64;
  return r < 64 ? 64 : (r > 2048 ? 2048 : r);
}
constexpr int ALS_THREADS = 256;

// A group: tensors decomposed together, sharing J, R, L, L2, the dtype and the
// iteration options (a single-tensor call is a group of one).  Per-slice work
// runs over the concatenated slices of the group (global slice index); each
// tensor keeps its own small state, addressed by its index t.
struct TDesc {
  int64_t K;            // slices of the tensor
  int64_t k0;           // its first global slice
  const void* slab;     // N_t x J elements
  const float* scale;   // fp8 per-slice scales (K), else NULL
  const float* om1;     // J x L
  const float* om2;     // (K R) x L2
  double *H, *V, *W;    // factors (caller memory)
  double* trace;        // per-iteration error (caller memory) or NULL
  double tol;
  int64_t rbase;        // first row of the tensor in the group's row space (wide-J sketch buffer)
};

// One block of a per-slice kernel: rows [s0, s1) of tensor t (global slice
// indices for the iteration kernels, local rows for the begin kernel).
struct Blk {
  int32_t t, s0, s1, pad;
};

// One second-stage chunk: rows [r0, r1) of M^T (global), all of tensor t.
struct Chunk {
  int64_t r0, r1;
  int32_t t, pad;
};

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
  int nt;                 // tensors in the group
  int64_t K, J, N, n_items;
  int R, L, L2, max_iter, q;
  int64_t n2;             // second-stage row chunks of M^T
  int64_t n2y;            // row chunks of the second-stage sketch (STAGE2_YCHUNK rows)
  int nblk, nblk0;        // blocks of the iteration / begin per-slice kernels
  // tables (device)
  size_t tdesc, blk, blk0, chunks, ychunks, seg_blk, seg_blk0, seg_chunk, seg_ychunk, seg_slice, slice_t;
  // first stage (global slice index)
  size_t ctl, items, slice_ptr, slice_list;
  size_t partG, partP, partS;
  size_t xnorm2, Mt, Phi, sig1, msgn;
  // second stage (per chunk / per tensor)
  size_t Y2p, Y2, B2t, S2p, S2, U2, s2s;   // s2s: scratch of the long-J second stage
  size_t D, E, F, FtFp;
  // iteration
  size_t Psi, Pw, Mk, small, partA, partB, partC, partBegin, red, fitp, trace, om1, omq;
  size_t ybuf;            // wide-J slab pass: Y of every row (N x 16 LT floats), else empty
  bool wide;              // slab pass in 128-column chunks (J above the narrow limit, or asked for)
  bool det;               // resumable mode (DPAR2_FLAG_DETERMINISTIC)
  size_t tables_end;     // end of the host-built tables [tdesc, tables_end)
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

constexpr int RED_WIDTH = 6;             // (6 R R + 2) doubles of column sums per tensor

// --- launchers (each returns the hipGetLastError() of its launches) ---------
// Arguments of the slab pass (sketch_impl.h, k_sketch.hip).
struct SlabArgs {
  const TDesc* td;         // tensors of the group (slab, scales, Omega_1)
  int J, L, R;
  const float* omega;      // NULL: each tensor's Omega_1; else K x J x L per slice
  const Item* items;       // Item::pad = tensor index
  double *partG, *partP, *partS;
  const double* theta;     // U variant: K x L x R
  double* U;               // U variant: N x R (single tensor)
  float* ybuf;             // wide-J pass: Y digits and exponents per tile (wide_tile_bytes(L) each,
                           // tile t of an item at slot Item::tslot + t)
  const int32_t* skip;     // NULL, or a flag: every block returns at once while it is nonzero
};
// J above which the slab pass takes the two-kernel wide form (sketch, then
// projection per 128-column chunk): 256 for float32 slabs, 128 otherwise
inline int narrow_j_limit(int dtype) { return dtype == 0 ? 256 : 128; }
// bytes per 64-row tile of the wide pass's Y-digit buffer: three digit planes
// of 16 LT columns x 64 row bytes, then the 16 LT column exponents
// (16 LT columns: LT = 1, 2 or 4 for L up to 16, 32 or 64)
__host__ __device__ inline int wide_lt(int L) { return L <= 16 ? 1 : L <= 32 ? 2 : 4; }
__host__ __device__ inline size_t wide_tile_bytes(int L) { return (size_t)wide_lt(L) * (3 * 16 * 64 + 16 * 4); }
constexpr int MAX_J = 16384;
// Slab pass over all work items: per-item partials of Y^T Y, Y^T X and
// ||X||^2, or (uout) U = Y Theta_k.  dtype: dpar2_dtype; vec: every slab is
// aligned for 4-element loads and J % 4 == 0.
hipError_t launch_slab(const SlabArgs& a, int dtype, int64_t n_items, bool vec, bool uout, bool wide,
                       hipStream_t s);
// the wide form (J above narrow_j_limit), k_slab_wide.hip
hipError_t launch_slab_wide(const SlabArgs& a, int dtype, int64_t n_items, bool vec, bool uout, hipStream_t s);
// Per-slice completion of the first stage; omega_next (K x J x L float32, or
// NULL) receives the sketch matrix of a power step, the orthonormal right
// singular vectors of B_k (Alg. 1's power iteration in stabilised form);
// msgn (K x R) is scratch for the sign gauge of C_k B_k.
hipError_t launch_slice_finish(int64_t K, int J, int L, int R, const int32_t* slice_ptr,
                               const int32_t* slice_list, const double* partG,
                               const double* partP, const double* partS, double* xnorm2,
                               double* Mt, double* Phi, double* sig1, float* omega_next, float* msgn, Ctl* ctl,
                               const int32_t* slice_t, hipStream_t s);
hipError_t launch_stage2(const Layout& lay, char* ws, hipStream_t s);
// out[t * ostride + e] = sum_{b in [seg[t], seg[t+1])} part[b * stride + e],
// e < width, t < nt, in a fixed order (one block per (e, t)).  n1 >= 0 gives
// the row count of a single tensor (nt == 1, seg = {0, n1}) so that the
// kernel need not read seg first; -1 otherwise.
hipError_t launch_segsum(int nt, const int64_t* seg, int64_t n1, int64_t stride, int64_t width,
                         const double* part, double* out, int64_t ostride, hipStream_t s);
hipError_t launch_als_begin(const Layout& lay, char* ws, hipStream_t s);
hipError_t launch_als_iteration(const Layout& lay, char* ws, hipStream_t s);
hipError_t launch_als_end(const Layout& lay, char* ws, hipStream_t s);
hipError_t launch_fitness(const Layout& lay, char* ws, double* fit, hipStream_t s);
hipError_t launch_theta(const Layout& lay, char* ws, const double* H, double* theta, hipStream_t s);
hipError_t launch_pw_identity(const Layout& lay, char* ws, hipStream_t s);
int als_slices_per_block(int R);

bool sketch_supported(int J, int L, int dtype);

// --- PARAFAC2-ALS on the uncompressed slices (Alg. 2), k_plain.hip -----------
constexpr int PL_VSLICES = 32;   // slices per block of the V pass
struct PlainArgs {
  int64_t K;
  int J;
  const int32_t* slice_ptr;       // K + 1: items of each slice
  const int32_t* slice_list;
  const double *partG, *partP, *partS;
  double* xnorm2;                 // K
  double *H, *V, *W;              // factors (caller memory)
  double* trace;                  // per-iteration error or NULL
  double tol;
  double* Y;                      // K x R x J: Y_k = Q_k^T X_k
  double* theta;                  // K x R x R: T_k G_k^{-1/2} (Q_k = X_k V Theta_k)
  double* g1p;                    // K x R R
  double* g2p;                    // ceil(K / PL_VSLICES) x J x R
  double* wp;                     // K x (R R + 2)
  double* small;                  // SM_COUNT x R R
  double* red;                    // RED_WIDTH R R + 2 (summed partials)
  double* g2;                     // J x R (summed)
  float *om_next, *om_cur;        // J x R float32 copies of V (next pass / last pass run)
  Ctl* ctl;
};
// The slab pass of an iteration: arguments and launch shape.
struct PlainLaunch {
  SlabArgs slab;
  int dtype;
  int64_t n_items;
  bool vec, wide;
};
// phase 0: begin of a call; 1: one iteration; 2: Theta_k <- Theta_k H (U output)
hipError_t launch_plain(int phase, int R, const PlainArgs& a, const PlainLaunch& pl, hipStream_t s);

// --- post-processing of the factors (Sec. IV-E), k_down.hip -----------------
hipError_t launch_pcc(int64_t J, int R, const double* V, double* C, hipStream_t s);
hipError_t launch_similarity(int n, int64_t M, int R, const int64_t* off, const int32_t* idx, const double* U,
                             double gamma, double* S, hipStream_t s);
hipError_t launch_topk(const double* v, int n, int exclude, int k, int32_t* out, hipStream_t s);
hipError_t launch_rwr(const double* S, int n, int target, double c, int iters, double* r, double* work,
                      hipStream_t s);

// --- learned warm start (k_warm.hip) ------------------------------------------
constexpr int WARM_WIDTH = 128;   // hidden width of the set encoder
// float offsets of the parameter blocks (row-major), P = total
struct WarmLayout {
  int F;                                            // tokens: R (R + 1) / 2 features
  int W1, b1, W2, b2, WH, bH, WV, bV, Ww, bw, P;
};
__host__ __device__ WarmLayout warm_layout(int R);
hipError_t launch_warm_feat(int64_t K, int J, int R, const double* F, const double* E, const double* D, float* tok,
                            hipStream_t s);
hipError_t launch_warm_targets(int64_t K, int J, int R, const double* D, const double* E, const double* H,
                               const double* V, const double* W, float* tH, float* tV, float* tW, hipStream_t s);
hipError_t launch_warm_apply(int64_t K, int J, int R, const double* D, const double* E, const float* pH,
                             const float* pV, const float* pW, double* H, double* V, double* W, hipStream_t s);
hipError_t launch_warm_forward(int R, int n, const int32_t* tok_off, const float* tok, const float* theta,
                               float* act, float* pH, float* pV, float* pW, hipStream_t s);
hipError_t launch_warm_backward(int R, int n, const int32_t* tok_off, const float* tok, const float* theta,
                                float* act, const float* pH, const float* pV, const float* pW, const float* tH,
                                const float* tV, const float* tW, float* gpart, float* grad, float* loss,
                                hipStream_t s);
hipError_t launch_warm_adam(int R, float* theta, const float* grad, float* m, float* v, int step, float lr,
                            float b1, float b2, float eps, float scale, hipStream_t s);

}  // namespace dpar2
