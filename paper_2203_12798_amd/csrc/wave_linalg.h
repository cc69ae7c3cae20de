// Small dense FP64 linear algebra done by one 64-lane wave on an n x n
// matrix (n <= 64), in a "split" layout: column c is held by H = 64 / RM
// lanes (lane = h RM + c, RM = the power of two >= n rounded up to even),
// lane h holding rows h LH .. h LH + LH - 1.  A Jacobi round then exchanges
// LH rows per lane instead of n, and every lane of the wave has work (above
// n = 32 one lane per column: H = 1).
#pragma once

#include "internal.h"

namespace dpar2 {

constexpr double EPS64 = 2.220446049250313e-16;
// Jacobi pairs are rotated while |a.b| > JACOBI_TOL |a| |b|: above the
// rounding floor of an n-term dot product, so converged columns stop.
constexpr double JACOBI_TOL = 1e-13;
constexpr int JACOBI_SWEEPS = 30;

__host__ __device__ constexpr int pow2ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}

template <int L>
struct SC {
  static constexpr int N = L + (L & 1);                          // Jacobi players
  static constexpr int RM = pow2ceil(N) < 2 ? 2 : pow2ceil(N);   // column groups
  static constexpr int H = 64 / RM;                              // lanes per column
  static constexpr int LH = (L + H - 1) / H;                     // rows per lane
  // LDS leading dimension: padded up to L = 32; above, unpadded, so that the
  // per-slice completion's four L x L matrices at L = 50 leave room for two
  // blocks per compute unit
  static constexpr int LD = (L > 32) ? L : L + 1;
  static constexpr int CW = 32;                                  // P columns per chunk
};

// One-sided Jacobi (Hestenes) on L columns split over H lanes each: lane
// (h, c) holds rows h LH .. of column c of T in t[] and, if WITHV, of the
// accumulated rotation in v[].  Round-robin pairing; both lanes of a pair, and
// all H lanes of a column, compute the same rotation from the same sums (the
// butterfly sums are symmetric, hence identical on every lane).  A pair is
// rotated while |a.b| > JACOBI_TOL |a| |b|; the sweeps stop after one without
// rotations, or after one whose largest |a.b| / (|a| |b|) was below 1e-7
// (convergence is quadratic, so the next sweep would not rotate).  All 64
// lanes must call it.  Returns the number of sweeps.
template <int L, bool WITHV>
__device__ inline int split_jacobi(double (&t)[SC<L>::LH], double (&v)[SC<L>::LH], int c, int h) {
  constexpr int N = SC<L>::N, RM = SC<L>::RM, LH = SC<L>::LH;
  int sweep;
  for (sweep = 0; sweep < JACOBI_SWEEPS; ++sweep) {
    int rotated = 0;
    int big = 0;   // some rotation had |a.b| / (|a| |b|) above 1e-7
    for (int r = 0; r < N - 1; ++r) {
      const int pc = (c < N) ? rr_partner(c, r, N) : c;
      const int src = h * RM + pc;
      double tp[LH], vp[LH];
#pragma unroll
      for (int i = 0; i < LH; ++i) tp[i] = __shfl(t[i], src, 64);
      if constexpr (WITHV) {
#pragma unroll
        for (int i = 0; i < LH; ++i) vp[i] = __shfl(v[i], src, 64);
      }
      double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
      for (int i = 0; i < LH; ++i) {
        aa = fma(t[i], t[i], aa);
        bb = fma(tp[i], tp[i], bb);
        ab = fma(t[i], tp[i], ab);
      }
#pragma unroll
      for (int o = RM; o < 64; o <<= 1) {
        aa += __shfl_xor(aa, o, 64);
        bb += __shfl_xor(bb, o, 64);
        ab += __shfl_xor(ab, o, 64);
      }
      const bool low = c < pc;
      const double alpha = low ? aa : bb, beta = low ? bb : aa;
      const double ab2 = ab * ab, ref = alpha * beta;
      if (c < N && pc != c && ab != 0.0 && ab2 > (JACOBI_TOL * JACOBI_TOL) * ref) {
        big |= (ab2 > 1e-14 * ref) ? 1 : 0;
        double cs, sn;
        jacobi_cs(alpha, beta, ab, &cs, &sn);
        rotated = 1;
        const double sa = low ? -sn : sn;
#pragma unroll
        for (int i = 0; i < LH; ++i) t[i] = fma(cs, t[i], sa * tp[i]);
        if constexpr (WITHV) {
#pragma unroll
          for (int i = 0; i < LH; ++i) v[i] = fma(cs, v[i], sa * vp[i]);
        }
      }
    }
    if (!__any(rotated)) break;
    if (!__any(big)) {   // largest |a.b| / (|a| |b|) below 1e-7
      ++sweep;
      break;
    }
  }
  return sweep;
}

// sum over the H lanes of a column (identical result on each of them)
template <int L>
__device__ __forceinline__ double col_sum(double x) {
#pragma unroll
  for (int o = SC<L>::RM; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Upper Cholesky factor of a symmetric positive semidefinite L x L matrix
// held by columns (lane c < L: a[i] = A[i][c]), right-looking; lane p
// publishes its column through LDS `row` at step p.  A pivot <= tau gives a
// zero row of the factor.  On return lane c < L holds C[i][c] in a[i]
// (a[i] = 0 below the diagonal) and rinv[p] = 1 / C[p][p] (0 for a zero
// pivot).  Returns the number of zero pivots (the same on every lane).  All
// 64 lanes must call it.
template <int L>
__device__ inline int lane_cholesky(double (&a)[L], double* row, double* rinv, double tau) {
  const int c = threadIdx.x;
  int zeros = 0;
#pragma unroll
  for (int p = 0; p < L; ++p) {
    if (c == p) {
#pragma unroll
      for (int i = p; i < L; ++i) row[i] = a[i];
    }
    __syncthreads();
    const double d = row[p];
    const double ri = (d > tau) ? nr_rsq(d) : 0.0;
    zeros += (d > tau) ? 0 : 1;
    if (c >= p && c < L) {
      const double rpc = a[p] * ri;   // C[p][c]
      if (c > p) {
#pragma unroll
        for (int i = p + 1; i < L; ++i) a[i] = fma(-(row[i] * ri), rpc, a[i]);
      }
      a[p] = rpc;
    }
    if (c == 0) rinv[p] = ri;
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (i > c) a[i] = 0.0;
  return zeros;
}

}  // namespace dpar2
