// Device-side building blocks shared by the libdpar2 kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpar2 {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Matrix-core (MFMA) tiles.  Lane layouts (checked on gfx950):
//   16x16x4 f32 and f64: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k.
//   f32 result: lane l, element v holds D[4 (l / 16) + v][l % 16].
//   f64 result: lane l, element v holds D[(l / 16) + 4 v][l % 16].
// ---------------------------------------------------------------------------
__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int f32_row(int lane, int v) { return 4 * (lane >> 4) + v; }
__device__ __forceinline__ int f64_row(int lane, int v) { return (lane >> 4) + 4 * v; }

// ---------------------------------------------------------------------------
// Shared control block of one decomposition (lives in the workspace).
// ---------------------------------------------------------------------------
struct Ctl {
  int32_t iters;        // iterations whose error is recorded
  int32_t done;         // stop rule fired: later iterations are no-ops
  int32_t base;         // value of `iters` when the current als_step call began
  uint32_t warn;        // DPAR2_WARN_* bits
  int32_t vc_valid;     // V is held as D VC (V not yet written back)
  int32_t bad;          // the slab held NaN or Inf: the iteration is skipped
  double e_prev;        // last recorded error
  double e0;            // sum_k ||F^(k) E D^T||_F^2 (constant part of e)
  double xnorm2;        // sum_k ||X_k||_F^2
  double fit_true;
};

// ---------------------------------------------------------------------------
// Round-robin (circle) pairing of n = 2m' players over n-1 rounds: in round r
// the pairs are (r, n-1) and (r - i mod (n-1), r + i mod (n-1)), i = 1..n/2-1.
// Every unordered pair meets exactly once per sweep.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rr_partner(int x, int r, int n) {
  const int m = n - 1;
  if (x == m) return r;
  int p = (2 * r - x) % m;
  if (p < 0) p += m;
  return (p == x) ? m : p;
}

// 1/x and 1/sqrt(x) for normal finite x > 0: the hardware estimate (relative
// error below 2^-24 on gfx950, measured over 4M values spread across 200
// binades) refined by one Newton-Raphson step, which squares that error to
// below 2^-48: a few ulp, enough for Jacobi rotations and Cholesky pivots,
// with a far shorter dependency chain than IEEE division or square root.
__device__ __forceinline__ double nr_rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double nr_rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  const double e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

// Jacobi rotation (Golub & Van Loan, symmetric Schur decomposition): for the
// 2x2 symmetric [app apq; apq aqq] (apq != 0) returns c, s with
// J = [c s; -s c] such that J^T A J is diagonal:
//   zeta = (aqq - app) / (2 apq), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1 / sqrt(1 + t^2), s = c t.
// Also used for one-sided Jacobi with app = ||a||^2, aqq = ||b||^2, apq = a.b.
__device__ __forceinline__ void jacobi_cs(double app, double aqq, double apq, double* c, double* s) {
  const double zeta = (aqq - app) * nr_rcp(2.0 * apq);
  const double az = fabs(zeta);
  double t;
  if (az < 1e150) {
    const double q = fma(zeta, zeta, 1.0);
    t = nr_rcp(az + q * nr_rsq(q));
  } else {
    t = 0.5 / az;   // 1 + zeta^2 would overflow; t = 1 / (2 |zeta|) to rounding
  }
  t = (zeta >= 0.0) ? t : -t;
  const double cc = nr_rsq(fma(t, t, 1.0));
  *c = cc;
  *s = cc * t;
}

// Sum over the block (blockDim.x a multiple of 64, <= 1024); every thread
// gets the total.  red: LDS scratch of >= 16 doubles.
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

}  // namespace dpar2
