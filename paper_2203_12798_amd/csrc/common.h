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
  int32_t pad0;
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
__device__ __forceinline__ void rr_pair(int i, int r, int n, int* p, int* q) {
  const int m = n - 1;
  if (i == 0) { *p = r; *q = m; return; }
  int a = (r - i) % m; if (a < 0) a += m;
  int b = (r + i) % m;
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// Jacobi rotation (Golub & Van Loan, symmetric Schur decomposition): for the
// 2x2 symmetric [app apq; apq aqq] returns c, s with J = [c s; -s c] such that
// J^T A J is diagonal.  Also used for one-sided Jacobi with app = ||a||^2,
// aqq = ||b||^2, apq = a.b.
__device__ __forceinline__ void jacobi_cs(double app, double aqq, double apq, double* c, double* s) {
  const double zeta = (aqq - app) / (2.0 * apq);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cc = 1.0 / sqrt(1.0 + t * t);
  *c = cc;
  *s = cc * t;
}

// ---------------------------------------------------------------------------
// Block-cooperative dense routines on small (n <= 32) float64 matrices held in
// LDS.  Every thread of the block must call them (they contain barriers).
// Matrices are row-major with leading dimension ld.
// ---------------------------------------------------------------------------

// Symmetric eigen-decomposition by cyclic Jacobi with parallel (round-robin)
// ordering.  A pair is rotated while |a_pq| > 1e-14 sqrt(|a_pp a_qq|) (a
// relative threshold above the rounding floor, which keeps the small
// eigenvalues of a Gram matrix relatively accurate); the sweeps stop after
// one without rotations.  On return A's diagonal holds the eigenvalues, V
// (n x n) the eigenvectors as columns.  cs: LDS scratch of >= 2*16+2 doubles.
// Returns 1 if the sweep cap was reached.
__device__ inline int block_sym_evd(double* A, int ld, double* V, int n, double* cs) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) V[(e / n) * ld + (e % n)] = ((e / n) == (e % n)) ? 1.0 : 0.0;
  __syncthreads();
  if (n <= 1) return 0;
  const int ne = n + (n & 1);        // players (one dummy when n is odd)
  const int npair = ne / 2;
  const int max_sweeps = 40;
  int capped = 1;
  double* flag = cs + 2 * 16;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) flag[0] = 0.0;
    __syncthreads();
    for (int r = 0; r < ne - 1; ++r) {
      if (tid < npair) {
        int p, q;
        rr_pair(tid, r, ne, &p, &q);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * ld + q];
          const double app = A[p * ld + p], aqq = A[q * ld + q];
          if (apq != 0.0 && fabs(apq) > 1e-14 * sqrt(fabs(app * aqq))) {
            jacobi_cs(app, aqq, apq, &c, &s);
            flag[0] = 1.0;
          }
        }
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < npair * n; e += nt) {
        const int i = e / n, m = e % n;
        int p, q;
        rr_pair(i, r, ne, &p, &q);
        if (q < n && cs[2 * i + 1] != 0.0) {
          const double c = cs[2 * i], s = cs[2 * i + 1];
          const double ap = A[p * ld + m], aq = A[q * ld + m];
          A[p * ld + m] = c * ap - s * aq;
          A[q * ld + m] = s * ap + c * aq;
        }
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < npair * n; e += nt) {
        const int i = e / n, m = e % n;
        int p, q;
        rr_pair(i, r, ne, &p, &q);
        if (q < n && cs[2 * i + 1] != 0.0) {
          const double c = cs[2 * i], s = cs[2 * i + 1];
          const double ap = A[m * ld + p], aq = A[m * ld + q];
          A[m * ld + p] = c * ap - s * aq;
          A[m * ld + q] = s * ap + c * aq;
          const double vp = V[m * ld + p], vq = V[m * ld + q];
          V[m * ld + p] = c * vp - s * vq;
          V[m * ld + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    if (flag[0] == 0.0) {
      capped = 0;
      break;
    }
    __syncthreads();
  }
  __syncthreads();
  return capped;
}

// Order eigenpairs by decreasing eigenvalue: writes perm[0..n) (LDS ints) with
// perm[rank] = index.  Ties keep the lower index first.
__device__ inline void block_sort_desc(const double* A, int ld, int n, int* perm) {
  const int tid = threadIdx.x;
  if (tid < n) {
    const double li = A[tid * ld + tid];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * ld + j];
      if (lj > li || (lj == li && j < tid)) ++rank;
    }
    perm[rank] = tid;
  }
  __syncthreads();
}

// Whitening of a symmetric positive semidefinite n x n Gram matrix G = Y^T Y
// (LDS; destroyed): G = V diag(lambda) V^T and Wh = V diag(lambda^{-1/2}) over
// eigenvalues above 64 eps lambda_max (zero columns for the others), so that
// Y Wh is an orthonormal basis of the numerical range of Y (an eigen-based
// CholeskyQR that stays defined when Y is rank deficient).  V: LDS scratch.
// Returns 1 if the Jacobi sweep cap was reached.
__device__ inline int block_whiten(double* G, int ld, int n, double* Wh, double* V, double* cs) {
  const int capped = block_sym_evd(G, ld, V, n, cs);
  double lmax = 0.0;
  for (int i = 0; i < n; ++i) lmax = fmax(lmax, G[i * ld + i]);
  const double cut = 64.0 * 2.220446049250313e-16 * lmax;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int a = e / n, b = e % n;
    const double lam = G[b * ld + b];
    Wh[a * ld + b] = (lam > cut && lam > 0.0) ? V[a * ld + b] / sqrt(lam) : 0.0;
  }
  __syncthreads();
  return capped;
}

// Moore-Penrose pseudoinverse of a symmetric positive semidefinite n x n
// matrix G (LDS): Ginv = U diag(1/lambda) U^T over eigenvalues above
// n * eps * lambda_max.  G is destroyed.  U: LDS n x n scratch.
__device__ inline int block_spd_pinv(double* G, int ld, double* Ginv, double* U, int n, double* cs) {
  int capped = block_sym_evd(G, ld, U, n, cs);
  double lmax = 0.0;
  for (int i = 0; i < n; ++i) lmax = fmax(lmax, fabs(G[i * ld + i]));
  const double cut = (double)n * 2.220446049250313e-16 * lmax;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int a = e / n, b = e % n;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double li = G[i * ld + i];
      if (li > cut) s += U[a * ld + i] * U[b * ld + i] / li;
    }
    Ginv[a * ld + b] = s;
  }
  __syncthreads();
  return capped;
}

// Block-wide sum of one double per thread (blockDim.x multiple of 64, <= 1024).
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
