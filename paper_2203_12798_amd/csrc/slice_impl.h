// Per-slice completion of the first-stage randomized SVD (the QR, projection
// and small-SVD steps of Alg. 1 for every X_k, Eq. 4), templated on the sketch
// width L.  One 64-lane wave per slice, from the slab pass's exact partial sums
// G = Y^T Y (L x L), P = Y^T X (L x J):
//   whitening Wh with Q = Y Wh orthonormal (QR step): Wh = R^{-1} from the
//     Cholesky factor G = R^T R; when a pivot falls below 1e-9 max_i G_ii the
//     eigen form Wh = V Lambda^{-1/2} over the eigenvalues above
//     64 eps lambda_max is used instead (defined also for a rank-deficient Y)
//   B B^T = Wh^T (P P^T) Wh with B = Q^T X = Wh^T P (projection)
//   B B^T = U~ Lambda~ U~^T (one-sided Jacobi; small SVD), sigma = sqrt(lambda~)
//   Phi = Wh U~_R (A_k = Y Phi = Q U~_R), C_k B_k = B^T U~_R = P^T Phi
// Each column of C_k B_k is signed so that its largest-magnitude entry is
// positive (first one on ties); Phi's column follows.
//
// Lane layout for the L x L matrices: column c is split over H = 64 / RM lanes
// (lane = h RM + c), lane h holding rows h LH .. h LH + LH - 1.  The Jacobi
// rounds then exchange LH rows per lane instead of L.
#pragma once

#include "als_impl.h"

namespace dpar2 {

template <int L>
struct SC {
  static constexpr int N = L + (L & 1);                          // Jacobi players
  static constexpr int RM = pow2ceil(N) < 2 ? 2 : pow2ceil(N);   // column groups
  static constexpr int H = 64 / RM;                              // lanes per column
  static constexpr int LH = (L + H - 1) / H;                     // rows per lane
  static constexpr int LD = L + 1;                               // LDS leading dimension
  static constexpr int CW = 32;                                  // P columns per chunk
};

// One-sided Jacobi (Hestenes) on L columns split over H lanes each: lane
// (h, c) holds rows h LH .. of column c of T in t[] and of the accumulated
// rotation in v[].  Round-robin pairing; both lanes of a pair, and all H lanes
// of a column, compute the same rotation from the same sums (the butterfly
// sums are symmetric, hence identical on every lane).  All 64 lanes must call
// it.  Returns the number of sweeps.
template <int L>
__device__ inline int split_jacobi(double (&t)[SC<L>::LH], double (&v)[SC<L>::LH], int c, int h) {
  constexpr int N = SC<L>::N, RM = SC<L>::RM, LH = SC<L>::LH;
  int sweep;
  for (sweep = 0; sweep < JACOBI_SWEEPS; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < N - 1; ++r) {
      const int pc = (c < N) ? rr_partner(c, r, N) : c;
      const int src = h * RM + pc;
      double tp[LH], vp[LH];
#pragma unroll
      for (int i = 0; i < LH; ++i) tp[i] = __shfl(t[i], src, 64);
#pragma unroll
      for (int i = 0; i < LH; ++i) vp[i] = __shfl(v[i], src, 64);
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
      if (c < N && pc != c && ab != 0.0 && fabs(ab) > JACOBI_TOL * sqrt(alpha * beta)) {
        double cs, sn;
        jacobi_cs(alpha, beta, ab, &cs, &sn);
        rotated = 1;
        const double sa = low ? -sn : sn;
#pragma unroll
        for (int i = 0; i < LH; ++i) {
          t[i] = fma(cs, t[i], sa * tp[i]);
          v[i] = fma(cs, v[i], sa * vp[i]);
        }
      }
    }
    if (!__any(rotated)) break;
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

template <int L>
__global__ __launch_bounds__(64) void k_slice_fin(int K, int J, int R, const int32_t* __restrict__ slice_ptr,
                                                  const int32_t* __restrict__ slice_list,
                                                  const double* __restrict__ partG,
                                                  const double* __restrict__ partP,
                                                  const double* __restrict__ partS, double* __restrict__ xnorm2,
                                                  double* __restrict__ Mt, double* __restrict__ Phi,
                                                  double* __restrict__ sig1, Ctl* ctl) {
  constexpr int RM = SC<L>::RM, LH = SC<L>::LH, LD = SC<L>::LD, CW = SC<L>::CW, LL = L * L;
  __shared__ double Gs[L * LD];    // G, then its Cholesky factor (upper triangle)
  __shared__ double Ss[L * LD];    // S' = P P^T; then Phi
  __shared__ double Ws[L * LD];    // whitening Wh
  __shared__ double Xs[L * LD];    // S' Wh; then sorted eigenvectors U~
  __shared__ double Pc[L * CW];    // chunk of P
  __shared__ double Mc[L * CW];    // chunk of C_k B_k (rows r < R)
  __shared__ double sgn[L];

  const int lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const int k = blockIdx.x;
  const int i0 = slice_ptr[k], i1 = slice_ptr[k + 1];
  const bool cv = c < L;
  unsigned warn = 0;

  // G column c (own rows) and ||X_k||^2
  double t[LH], v[LH];
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int a = h * LH + ii;
    double s = 0.0;
    if (cv && a < L)
      for (int q = i0; q < i1; ++q) s += partG[(size_t)slice_list[q] * LL + a * L + c];
    t[ii] = s;
    v[ii] = (a == c) ? 1.0 : 0.0;
    if (cv && a < L) Gs[a * LD + c] = s;
  }
  if (lane == 0) {
    double s = 0.0;
    for (int q = i0; q < i1; ++q) s += partS[slice_list[q]];
    xnorm2[k] = s;
  }

  // S' = P P^T, P streamed through LDS in chunks of CW columns
  double sp[LH];
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) sp[ii] = 0.0;
  for (int jc = 0; jc < J; jc += CW) {
    for (int e = lane; e < L * CW; e += 64) {
      const int a = e / CW, jj = e % CW;
      double p = 0.0;
      if (jc + jj < J)
        for (int q = i0; q < i1; ++q) p += partP[(size_t)slice_list[q] * L * J + (size_t)a * J + jc + jj];
      Pc[e] = p;
    }
    __syncthreads();
    if (cv) {
      for (int jj = 0; jj < CW; ++jj) {
        const double pc = Pc[c * CW + jj];
#pragma unroll
        for (int ii = 0; ii < LH; ++ii) {
          const int a = h * LH + ii;
          if (a < L) sp[ii] = fma(Pc[a * CW + jj], pc, sp[ii]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int a = h * LH + ii;
    if (cv && a < L) Ss[a * LD + c] = sp[ii];
  }
  __syncthreads();

  // Whitening.  Cholesky G = R^T R in Gs (upper triangle, row p = row p of R)
  double dmax = 0.0;
  for (int a = 0; a < L; ++a) dmax = fmax(dmax, Gs[a * LD + a]);
  const double tau = 1e-9 * dmax;
  bool chol = dmax > 0.0;
  for (int p = 0; p < L && chol; ++p) {
    const double d = Gs[p * LD + p];
    __syncthreads();
    if (!(d > tau)) {
      chol = false;   // every lane read the same d
      break;
    }
    const double rp = sqrt(d);
    if (lane >= p && lane < L) Gs[p * LD + lane] = (lane == p) ? rp : Gs[p * LD + lane] / rp;
    __syncthreads();
    const int m = L - p - 1;
    for (int e = lane; e < m * m; e += 64) {
      const int i = p + 1 + e / m, j = p + 1 + e % m;
      if (j >= i) Gs[i * LD + j] -= Gs[p * LD + i] * Gs[p * LD + j];
    }
    __syncthreads();
  }
  if (chol) {
    // Wh = R^{-1}: lane c < L solves R x = e_c by back substitution
    if (lane < L) {
      double x[L];
#pragma unroll
      for (int i = L - 1; i >= 0; --i) {
        double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int j = i + 1; j < L; ++j) s = fma(-Gs[i * LD + j], x[j], s);
        x[i] = (i > lane) ? 0.0 : s / Gs[i * LD + i];
      }
#pragma unroll
      for (int i = 0; i < L; ++i) Ws[i * LD + lane] = x[i];
    }
  } else {
    // eigen form: G = V Lambda V^T, Wh column c = v_c / sqrt(lambda_c) or 0
    if (split_jacobi<L>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
    double lam = 0.0;
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) lam = fma(t[ii], t[ii], lam);
    lam = sqrt(col_sum<L>(lam));
    double lmax = cv ? lam : 0.0;
    for (int o = 1; o < 64; o <<= 1) lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
    const double ws = (lam > 64.0 * EPS64 * lmax && lam > 0.0) ? 1.0 / sqrt(lam) : 0.0;
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      if (cv && a < L) Ws[a * LD + c] = v[ii] * ws;
    }
  }
  __syncthreads();

  // S = Wh^T S' Wh, column c (own rows)
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int a = h * LH + ii;
    if (cv && a < L) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < L; ++b) s = fma(Ss[a * LD + b], Ws[b * LD + c], s);
      Xs[a * LD + c] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int a = h * LH + ii;
    double s = 0.0;
    if (cv && a < L)
#pragma unroll
      for (int b = 0; b < L; ++b) s = fma(Ws[b * LD + a], Xs[b * LD + c], s);
    t[ii] = s;
    v[ii] = (a == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  // B B^T = U~ Lambda~ U~^T
  if (split_jacobi<L>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
  double mu = 0.0;
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) mu = fma(t[ii], t[ii], mu);
  mu = sqrt(col_sum<L>(mu));   // eigenvalue of the PSD matrix B B^T
  // rank by decreasing eigenvalue (ties: lower index first)
  int rank = 0;
  for (int c2 = 0; c2 < L; ++c2) {
    const double m2 = __shfl(mu, c2, 64);
    if (m2 > mu || (m2 == mu && c2 < c)) ++rank;
  }
  if (cv) {
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      if (a < L) Xs[a * LD + rank] = v[ii];
    }
    if (h == 0 && rank < R) sig1[(size_t)k * R + rank] = sqrt(mu > 0.0 ? mu : 0.0);
  }
  __syncthreads();
  // Phi = Wh U~_R (into Ss)
  for (int e = lane; e < L * R; e += 64) {
    const int a = e / R, r = e % R;
    double s = 0.0;
    for (int b = 0; b < L; ++b) s = fma(Ws[a * LD + b], Xs[b * LD + r], s);
    Ss[a * LD + r] = s;
  }
  __syncthreads();

  // C_k B_k = P^T Phi.  Pass 0 finds the signed leading entry of each column
  // (lane r < R scans the chunk), pass 1 writes the signed rows of M^T.
  double bv = -1.0, bs = 0.0;
  double* Mk = Mt + (size_t)k * R * J;
  for (int pass = 0; pass < 2; ++pass) {
    for (int jc = 0; jc < J; jc += CW) {
      for (int e = lane; e < L * CW; e += 64) {
        const int a = e / CW, jj = e % CW;
        double p = 0.0;
        if (jc + jj < J)
          for (int q = i0; q < i1; ++q) p += partP[(size_t)slice_list[q] * L * J + (size_t)a * J + jc + jj];
        Pc[e] = p;
      }
      __syncthreads();
      for (int e = lane; e < R * CW; e += 64) {
        const int r = e / CW, jj = e % CW;
        double m = 0.0;
#pragma unroll
        for (int a = 0; a < L; ++a) m = fma(Ss[a * LD + r], Pc[a * CW + jj], m);
        if (pass == 0) Mc[e] = m;
        else if (jc + jj < J) Mk[(size_t)r * J + jc + jj] = sgn[r] * m;
      }
      __syncthreads();
      if (pass == 0 && lane < R) {
        const int nj = (J - jc < CW) ? J - jc : CW;
        for (int jj = 0; jj < nj; ++jj) {
          const double m = Mc[lane * CW + jj];
          if (fabs(m) > bv) {
            bv = fabs(m);
            bs = m;
          }
        }
      }
      __syncthreads();
    }
    if (pass == 0) {
      if (lane < R) sgn[lane] = (bs < 0.0) ? -1.0 : 1.0;
      __syncthreads();
    }
  }
  for (int e = lane; e < L * R; e += 64) {
    const int a = e / R, r = e % R;
    Phi[(size_t)k * L * R + e] = sgn[r] * Ss[a * LD + r];
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl->warn, warn);
}

template <int L>
hipError_t slice_fin_launch(int64_t K, int J, int R, const int32_t* slice_ptr, const int32_t* slice_list,
                            const double* partG, const double* partP, const double* partS, double* xnorm2,
                            double* Mt, double* Phi, double* sig1, Ctl* ctl, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_fin<L>, dim3((unsigned)K), dim3(64), 0, s, (int)K, J, R, slice_ptr, slice_list,
                     partG, partP, partS, xnorm2, Mt, Phi, sig1, ctl);
  return hipGetLastError();
}

}  // namespace dpar2
