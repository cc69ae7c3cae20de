// Per-slice completion of the first-stage randomized SVD (the QR, projection
// and small-SVD steps of Alg. 1 for every X_k, Eq. 4), templated on the sketch
// width L.  One 64-lane wave per slice, from the slab pass's exact partial sums
// G = Y^T Y (L x L), P = Y^T X (L x J):
//   whitening Wh with Q = Y Wh orthonormal (QR step): Wh = R^{-1} from the
//     Cholesky factor G = R^T R; when a pivot falls below 1e-9 max_i G_ii the
//     eigen form Wh = V Lambda^{-1/2} over the eigenvalues above
//     64 eps lambda_max is used instead (defined also for a rank-deficient Y)
//   B = Q^T X = Wh^T P (projection), streamed by chunks of P, and S = B B^T
//   S = C^T C (Cholesky), one-sided Jacobi on C^T: C^T V = U~ Sigma gives the
//     eigenvectors U~ of S and the singular values Sigma of B (small SVD)
//   Phi = Wh U~_R (A_k = Y Phi = Q U~_R), C_k B_k = B^T U~_R = P^T Phi
// Each column of C_k B_k is signed so that its largest-magnitude entry is
// positive (first one on ties); Phi's column follows.  P is streamed twice (for
// S, and for C_k B_k written unsigned with the sign found on the way; a second
// kernel flips the rows of M^T whose sign is negative), three times with a
// power step.
//
// Lane layout for the L x L matrices: the split layout of wave_linalg.h.
#pragma once

#include "wave_linalg.h"

namespace dpar2 {

// D(nrow x 32) += A^T(nrow x L) B(L x 32) on the FP64 matrix cores for one
// chunk of 32 columns, A from the L x LD matrix `a` (column r of a = row r of
// the product), B from the chunk `b` (row stride CP); acc[tr][tj] is the
// 16 x 16 tile (rows 16 tr, columns 16 tj), lane l holding rows
// f64_row(l, v) and column l % 16; nrow <= 16 TRN.  All 64 lanes take part.
template <int L>
constexpr int row_tiles() { return L > 32 ? 4 : 2; }

template <int L, int LD, int CP, int TRN>
__device__ __forceinline__ void chunk_atb(const double* a, const double* b, int nrow, v4d (&acc)[TRN][2],
                                          int lane) {
  const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < (L + 3) / 4; ++kk) {
    const int k = 4 * kk + k4;
    double av[TRN], bv[2];
#pragma unroll
    for (int t = 0; t < TRN; ++t) {
      const int r = 16 * t + i16;
      av[t] = (k < L && r < nrow) ? a[k * LD + r] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) bv[t] = (k < L) ? b[k * CP + 16 * t + i16] : 0.0;
#pragma unroll
    for (int tr = 0; tr < TRN; ++tr) {
      if (16 * tr >= nrow) continue;   // wave-uniform
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) acc[tr][tj] = mfma_f64(av[tr], bv[tj], acc[tr][tj]);
    }
  }
}

template <int L>
__global__ __launch_bounds__(64) void k_slice_fin(int K, int J, int R, const int32_t* __restrict__ slice_ptr,
                                                  const int32_t* __restrict__ slice_list,
                                                  const double* __restrict__ partG,
                                                  const double* __restrict__ partP,
                                                  const double* __restrict__ partS, double* __restrict__ xnorm2,
                                                  double* __restrict__ Mt, double* __restrict__ Phi,
                                                  double* __restrict__ sig1, float* __restrict__ omega_next,
                                                  float* __restrict__ msgn, Ctl* ctl,
                                                  const int32_t* __restrict__ slice_t) {
  constexpr int RM = SC<L>::RM, LH = SC<L>::LH, LD = SC<L>::LD, CW = SC<L>::CW, LL = L * L;
  constexpr int TRN = row_tiles<L>();   // 16-row tiles of the L- and R-row products
  constexpr int CP = CW + 1;        // padded chunk row (conflict-free column reads)
  constexpr int NPX = (L * CP > L * LD) ? L * CP : L * LD;
  // G and its Cholesky factors are not needed while P is streamed: the chunks
  // of B = Wh^T P and of C_k B_k (rows r < R) share their space
  __shared__ double GM[NPX];
  double* const Gs = GM;            // G, its Cholesky factor (upper), later that of S
  double* const Mc = GM;            // chunk of B; chunk of C_k B_k
  __shared__ double Ss[L * LD];    // S = B B^T; then Phi
  __shared__ double Ws[L * LD];    // whitening Wh
  // the sorted eigenvectors U~ live only between the Jacobi and Phi, when no
  // chunk of P is streamed: they share the chunk's space
  __shared__ double PX[NPX];
  double* const Pc = PX;            // chunk of P
  double* const Xs = PX;            // sorted eigenvectors U~
  __shared__ double sgn[L], row[L], rinv[L], sv[L];

  const int lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const int k = blockIdx.x;
  const int i0 = slice_ptr[k], i1 = slice_ptr[k + 1];
  const bool cv = c < L;
  unsigned warn = 0;

  // G column c (own rows) and ||X_k||^2
  double t[LH], v[LH];
  {
    double gs[LH];
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) gs[ii] = 0.0;
    // loads are unconditional (clamped index, value masked) so that they are
    // issued back to back instead of one branch and wait each
    for (int q = i0; q < i1; ++q) {
      const double* g = partG + (size_t)slice_list[q] * LL;
#pragma unroll
      for (int ii = 0; ii < LH; ++ii) {
        const int a = h * LH + ii;
        const bool ok = cv && a < L;
        const double x = g[ok ? a * L + c : 0];
        gs[ii] += ok ? x : 0.0;
      }
    }
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      if (cv && a < L) Gs[a * LD + c] = gs[ii];
    }
  }
  if (lane == 0) {
    double s = 0.0;
    for (int q = i0; q < i1; ++q) s += partS[slice_list[q]];
    xnorm2[k] = s;
  }

  // P is streamed through LDS in chunks of CW columns: fetch(jc) loads chunk
  // jc (summed over the slice's items) into registers, stash() puts it into
  // Pc; the next chunk's loads are in flight while the current one is used
  constexpr int NE = (L * CW + 63) / 64;
  double pv[NE];
  auto fetch = [&](int jc) {
#pragma unroll
    for (int u = 0; u < NE; ++u) pv[u] = 0.0;
    for (int q = i0; q < i1; ++q) {
      const double* base = partP + (size_t)slice_list[q] * L * J + jc;
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = lane + 64 * u, a = e / CW, jj = e % CW;
        const bool ok = e < L * CW && jc + jj < J;
        const double x = base[ok ? (size_t)a * J + jj : 0];
        pv[u] += ok ? x : 0.0;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = lane + 64 * u;
      if (e < L * CW) Pc[(e / CW) * CP + e % CW] = pv[u];
    }
  };
  __syncthreads();   // G complete in Gs
  // Whitening: G = R^T R (lane_cholesky), Wh = R^{-1}
  double dmax = 0.0;
  for (int a = 0; a < L; ++a) dmax = fmax(dmax, Gs[a * LD + a]);
  double col[L];
#pragma unroll
  for (int i = 0; i < L; ++i) col[i] = (lane < L) ? Gs[i * LD + lane] : 0.0;
  __syncthreads();
  const bool chol = dmax > 0.0 && lane_cholesky<L>(col, row, rinv, 1e-9 * dmax) == 0;
  if (chol) {
    if (lane < L) {
#pragma unroll
      for (int i = 0; i < L; ++i) Gs[i * LD + lane] = col[i];
    }
    __syncthreads();
    // lane c < L solves R x = e_c by back substitution
    if (lane < L) {
      double x[L];
#pragma unroll
      for (int i = L - 1; i >= 0; --i) {
        double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int j = i + 1; j < L; ++j) s = fma(-Gs[i * LD + j], x[j], s);
        x[i] = (i > lane) ? 0.0 : s * rinv[i];
      }
#pragma unroll
      for (int i = 0; i < L; ++i) Ws[i * LD + lane] = x[i];
    }
  } else {
    // eigen form: G = V Lambda V^T, Wh column c = v_c / sqrt(lambda_c) or 0
    // (Gs still holds G: the factor is written back only on success)
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      t[ii] = (cv && a < L) ? Gs[a * LD + c] : 0.0;
      v[ii] = (a == c) ? 1.0 : 0.0;
    }
    if (split_jacobi<L, true>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
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

  // S = B B^T with B = Wh^T P = Q^T X (the projection), streamed in chunks of
  // CW columns on the FP64 matrix cores: each chunk of P is whitened first,
  // B_c = Wh^T P_c, and then S += B_c B_c^T.  (Forming P P^T before the
  // whitening would square the condition of Y as well as that of B: a slice
  // with one dominant row then loses its small singular values.)
  v4d sacc[TRN][TRN];
#pragma unroll
  for (int x = 0; x < TRN; ++x)
#pragma unroll
    for (int y2 = 0; y2 < TRN; ++y2) sacc[x][y2] = v4d{0.0, 0.0, 0.0, 0.0};
  {
    const int i16 = lane & 15, k4 = lane >> 4;
    fetch(0);
    for (int jc = 0; jc < J; jc += CW) {
      stash();
      if (jc + CW < J) fetch(jc + CW);
      __syncthreads();
      v4d bacc[TRN][2];
#pragma unroll
      for (int x = 0; x < TRN; ++x)
#pragma unroll
        for (int y2 = 0; y2 < 2; ++y2) bacc[x][y2] = v4d{0.0, 0.0, 0.0, 0.0};
      chunk_atb<L, LD, CP, TRN>(Ws, Pc, L, bacc, lane);
#pragma unroll
      for (int tr = 0; tr < TRN; ++tr)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = 16 * tr + f64_row(lane, v), jj = 16 * tj + i16;
            if (a < L) Mc[a * CP + jj] = bacc[tr][tj][v];
          }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < CW / 4; ++kk) {
        const int j = 4 * kk + k4;
        double bv2[TRN];
#pragma unroll
        for (int t = 0; t < TRN; ++t) bv2[t] = (16 * t + i16 < L) ? Mc[(16 * t + i16) * CP + j] : 0.0;
        // the upper triangle of tiles that L covers
#pragma unroll
        for (int tr = 0; tr < TRN; ++tr)
#pragma unroll
          for (int tj = tr; tj < TRN; ++tj)
            if (16 * tj < L) sacc[tr][tj] = mfma_f64(bv2[tr], bv2[tj], sacc[tr][tj]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int tr = 0; tr < TRN; ++tr)
#pragma unroll
      for (int tj = tr; tj < TRN; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * tr + f64_row(lane, v), b = 16 * tj + i16;
          if (a < L && b < L) {
            Ss[a * LD + b] = sacc[tr][tj][v];
            if (tr != tj) Ss[b * LD + a] = sacc[tr][tj][v];
          }
        }
  }
  __syncthreads();
  // column c of S, Cholesky S = C^T C (semidefinite)
#pragma unroll
  for (int i = 0; i < L; ++i) col[i] = (lane < L) ? Ss[i * LD + lane] : 0.0;
  double smax = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (i == lane) smax = col[i];
  for (int o = 1; o < 64; o <<= 1) smax = fmax(smax, __shfl_xor(smax, o, 64));
  lane_cholesky<L>(col, row, rinv, 1e-13 * smax);
  // rows of C become the Jacobi columns (A = C^T, A A^T = S): lane (h, c)
  // takes entries h LH .. of row c
  if (lane < L) {
#pragma unroll
    for (int i = 0; i < L; ++i) Gs[i * LD + lane] = col[i];
  }
  __syncthreads();
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int b = h * LH + ii;
    t[ii] = (cv && b < L) ? Gs[c * LD + b] : 0.0;
  }
  __syncthreads();

  // One-sided Jacobi on A = C^T: A V = U~ Sigma, U~ the eigenvectors of
  // S = B B^T and Sigma the singular values of B; the left vectors are the
  // normalised converged columns, so no rotation is accumulated.  (The
  // triangular factor makes this converge in about half the sweeps needed on
  // S itself.)
  if (split_jacobi<L, false>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
  double mu = 0.0;
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) mu = fma(t[ii], t[ii], mu);
  mu = sqrt(col_sum<L>(mu));   // singular value of B
  double inv_mu;
  {
    // directions at the rounding level of the largest carry no information
    // (their normalised columns would be noise): zero them
    double mmax = cv ? mu : 0.0;
    for (int o = 1; o < 64; o <<= 1) mmax = fmax(mmax, __shfl_xor(mmax, o, 64));
    inv_mu = (mu > 64.0 * EPS64 * mmax && mu > 0.0) ? 1.0 / mu : 0.0;
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) v[ii] = t[ii] * inv_mu;
  }
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
    if (h == 0 && rank < R) sig1[(size_t)k * R + rank] = mu;
    if (h == 0) sv[rank] = inv_mu;
  }
  __syncthreads();
  // Phi = Wh U~ (into Ss): the leading R columns give A_k; a power step
  // needs all L (its sketch matrix is P^T Phi Sigma^{-1} = the right singular
  // vectors of B, columns with a negligible singular value set to zero)
  const int nphi = omega_next ? L : R;
  for (int e = lane; e < L * nphi; e += 64) {
    const int a = e / nphi, r = e % nphi;
    double s = 0.0;
    for (int b = 0; b < L; ++b) s = fma(Ws[a * LD + b], Xs[b * LD + r], s);
    Ss[a * LD + r] = s;
  }
  __syncthreads();
  if (omega_next) {
    float* On = omega_next + (size_t)k * J * L;
    fetch(0);
    for (int jc = 0; jc < J; jc += CW) {
      stash();
      if (jc + CW < J) fetch(jc + CW);
      __syncthreads();
      v4d oacc[TRN][2];
#pragma unroll
      for (int x = 0; x < TRN; ++x)
#pragma unroll
        for (int y2 = 0; y2 < 2; ++y2) oacc[x][y2] = v4d{0.0, 0.0, 0.0, 0.0};
      chunk_atb<L, LD, CP, TRN>(Ss, Pc, L, oacc, lane);
#pragma unroll
      for (int tr = 0; tr < TRN; ++tr)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int l = 16 * tr + f64_row(lane, v), jj = 16 * tj + (lane & 15);
            if (l < L && jc + jj < J) On[(size_t)(jc + jj) * L + l] = (float)(oacc[tr][tj][v] * sv[l]);
          }
      __syncthreads();
    }
  }

  // C_k B_k = P^T Phi, written unsigned into the rows of M^T while lane
  // r < R finds the leading entry of row r (largest magnitude, first on
  // ties); the rows whose sign is negative are flipped afterwards (msgn)
  double bv = -1.0, bs = 0.0;
  double* Mk = Mt + (size_t)k * R * J;
  fetch(0);
  for (int jc = 0; jc < J; jc += CW) {
    stash();
    if (jc + CW < J) fetch(jc + CW);
    __syncthreads();
    v4d macc[TRN][2];
#pragma unroll
    for (int x = 0; x < TRN; ++x)
#pragma unroll
      for (int y2 = 0; y2 < 2; ++y2) macc[x][y2] = v4d{0.0, 0.0, 0.0, 0.0};
    chunk_atb<L, LD, CP, TRN>(Ss, Pc, R, macc, lane);
#pragma unroll
    for (int tr = 0; tr < TRN; ++tr)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * tr + f64_row(lane, v), jj = 16 * tj + (lane & 15);
          if (r < R) {
            const double m = macc[tr][tj][v];
            Mc[r * CP + jj] = m;
            if (jc + jj < J) Mk[(size_t)r * J + jc + jj] = m;
          }
        }
    __syncthreads();
    if (lane < R) {
      const int nj = (J - jc < CW) ? J - jc : CW;
      for (int jj = 0; jj < nj; ++jj) {
        const double m = Mc[lane * CP + jj];
        if (fabs(m) > bv) {
          bv = fabs(m);
          bs = m;
        }
      }
    }
  }
  if (lane < R) {
    sgn[lane] = (bs < 0.0) ? -1.0 : 1.0;
    msgn[(size_t)k * R + lane] = (bs < 0.0) ? -1.0f : 1.0f;
  }
  __syncthreads();
  for (int e = lane; e < L * R; e += 64) {
    const int a = e / R, r = e % R;
    Phi[(size_t)k * L * R + e] = sgn[r] * Ss[a * LD + r];
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl[slice_t[k]].warn, warn);   // the slice's tensor
}

template <int L>
hipError_t slice_fin_launch(int64_t K, int J, int R, const int32_t* slice_ptr, const int32_t* slice_list,
                            const double* partG, const double* partP, const double* partS, double* xnorm2,
                            double* Mt, double* Phi, double* sig1, float* omega_next, float* msgn, Ctl* ctl,
                            const int32_t* slice_t, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_fin<L>, dim3((unsigned)K), dim3(64), 0, s, (int)K, J, R, slice_ptr, slice_list,
                     partG, partP, partS, xnorm2, Mt, Phi, sig1, omega_next, msgn, ctl, slice_t);
  return hipGetLastError();
}

}  // namespace dpar2
