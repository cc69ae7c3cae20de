// Second-stage small kernels (Sec. III-B, Eq. 5, Alg. 1 applied to M),
// templated on the sketch width L2 and run by one 64-lane wave:
//   k_s2_orth  Q2 = orthonormal basis of span(Y2) (QR step), Y2 overwritten:
//              two whitening passes (CholeskyQR2), each Wh = R^{-1} from the
//              Cholesky factor of Y2^T Y2, or the eigen form V Lambda^{-1/2}
//              (directions below 64 eps lambda_max dropped) when a pivot is
//              below 1e-9 of the largest diagonal (e.g. M of exact low rank)
//   k_s2_evd   B2 B2^T = U2 Lambda U2^T (small SVD): Cholesky B2 B2^T = C^T C
//              and one-sided Jacobi on C^T, whose normalised columns are U2;
//              E = sqrt(Lambda_R), D = Q2 U2_R, U2_R E^{-1} and D^T D
#pragma once

#include "slice_impl.h"

namespace dpar2 {

template <int L>
__global__ __launch_bounds__(64) void k_s2_orth(int J, double* __restrict__ Yall, Ctl* ctlall) {
  double* __restrict__ Y = Yall + (size_t)blockIdx.x * J * L;   // one tensor per block
  Ctl* ctl = ctlall + blockIdx.x;
  constexpr int RM = SC<L>::RM, LH = SC<L>::LH, LD = SC<L>::LD;
  constexpr int TJ = 64;                       // rows of Y2 per LDS tile
  __shared__ double Ys[TJ * LD];
  __shared__ double Gs[L * LD], Ws[L * LD], row[L], rinv[L];
  const int lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const bool cv = c < L;
  unsigned warn = 0;
  // rows j0 .. j0 + nj - 1 of Y2 into Ys (TJ * L / 64 = L loads per lane,
  // issued together)
  auto stage = [&](int j0, int nj) {
    double yv[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int e = lane + 64 * u, jj = e / L;
      const double x = Y[(jj < nj) ? (size_t)(j0 + jj) * L + e % L : 0];
      yv[u] = (jj < nj) ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int e = lane + 64 * u;
      Ys[(e / L) * LD + e % L] = yv[u];
    }
  };
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    // Gram column c (own rows), Y2 streamed through LDS
    double t[LH], v[LH];
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      t[ii] = 0.0;
      v[ii] = (h * LH + ii == c) ? 1.0 : 0.0;
    }
    for (int j0 = 0; j0 < J; j0 += TJ) {
      const int nj = (J - j0 < TJ) ? J - j0 : TJ;
      stage(j0, nj);
      __syncthreads();
      if (cv) {
        // four rows per step, every LDS read of a step issued before its
        // multiply-adds (the sums still run over the rows in order); rows
        // a >= L read a valid entry and are cleared below
        auto rowacc = [&](int jj) {
          const double yc = Ys[jj * LD + c];
#pragma unroll
          for (int ii = 0; ii < LH; ++ii) {
            const int a = h * LH + ii;
            t[ii] = fma(Ys[jj * LD + (a < L ? a : L - 1)], yc, t[ii]);
          }
        };
        int jj = 0;
        for (; jj + 4 <= nj; jj += 4) {
          double yc[4], ya[4][LH];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            yc[u] = Ys[(jj + u) * LD + c];
#pragma unroll
            for (int ii = 0; ii < LH; ++ii) {
              const int a = h * LH + ii;
              ya[u][ii] = Ys[(jj + u) * LD + (a < L ? a : L - 1)];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int ii = 0; ii < LH; ++ii) t[ii] = fma(ya[u][ii], yc[u], t[ii]);
        }
        for (; jj < nj; ++jj) rowacc(jj);
      }
      __syncthreads();
    }
#pragma unroll
    for (int ii = 0; ii < LH; ++ii)
      if (h * LH + ii >= L) t[ii] = 0.0;
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      if (cv && a < L) Gs[a * LD + c] = t[ii];
    }
    __syncthreads();
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
    // Y2 <- Y2 Wh: lane (h, c) keeps column c of Wh and produces column c of
    // the rows h, h + H, ... of each LDS tile
    {
      constexpr int H = SC<L>::H;
      double w[L];
#pragma unroll
      for (int a = 0; a < L; ++a) w[a] = cv ? Ws[a * LD + c] : 0.0;
      for (int j0 = 0; j0 < J; j0 += TJ) {
        const int nj = (J - j0 < TJ) ? J - j0 : TJ;
        __syncthreads();
        stage(j0, nj);
        __syncthreads();
        if (cv) {
          // two rows per step, reads first
          int jj = h;
          for (; jj + H < nj; jj += 2 * H) {
            double y0[L], y1[L];
#pragma unroll
            for (int a = 0; a < L; ++a) {
              y0[a] = Ys[jj * LD + a];
              y1[a] = Ys[(jj + H) * LD + a];
            }
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int a = 0; a < L; ++a) {
              s0 = fma(y0[a], w[a], s0);
              s1 = fma(y1[a], w[a], s1);
            }
            Y[(size_t)(j0 + jj) * L + c] = s0;
            Y[(size_t)(j0 + jj + H) * L + c] = s1;
          }
          for (; jj < nj; jj += H) {
            double s0 = 0.0;
#pragma unroll
            for (int a = 0; a < L; ++a) s0 = fma(Ys[jj * LD + a], w[a], s0);
            Y[(size_t)(j0 + jj) * L + c] = s0;
          }
        }
      }
    }
    __syncthreads();
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl->warn, warn);
}

template <int L>
__global__ __launch_bounds__(64) void k_s2_evd(int J, int R, const double* __restrict__ S2all,
                                               const double* __restrict__ Q2all, double* __restrict__ Dall,
                                               double* __restrict__ Eall, double* __restrict__ U2all,
                                               double* __restrict__ small, Ctl* ctlall) {
  // one tensor per block
  const int tt = blockIdx.x;
  const double* __restrict__ S2 = S2all + (size_t)tt * (L * (L + 1) / 2);
  const double* __restrict__ Q2 = Q2all + (size_t)tt * J * L;
  double* __restrict__ D = Dall + (size_t)tt * J * R;
  double* __restrict__ E = Eall + (size_t)tt * R;
  double* __restrict__ U2s = U2all + (size_t)tt * L * R;
  double* __restrict__ DtD = small + (size_t)tt * SM_COUNT * R * R + SM_DTD * R * R;
  Ctl* ctl = ctlall + tt;
  constexpr int RM = SC<L>::RM, LH = SC<L>::LH, LD = SC<L>::LD;
  constexpr int NP = L * (L + 1) / 2;
  __shared__ double Ss[L * LD], Us[L * LD], Es[L], row[L], rinv[L];
  __shared__ double Ds[64 * LD];
  const int lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const bool cv = c < L;
  unsigned warn = 0;
  // B2 B2^T, packed upper-triangle pairs
  for (int pi = lane; pi < NP; pi += 64) {
    int a = 0, rem = pi;
    while (rem >= L - a) {
      rem -= L - a;
      ++a;
    }
    const int b = a + rem;
    const double s = S2[pi];
    Ss[a * LD + b] = s;
    Ss[b * LD + a] = s;
  }
  __syncthreads();
  double col[L];
#pragma unroll
  for (int i = 0; i < L; ++i) col[i] = (lane < L) ? Ss[i * LD + lane] : 0.0;
  double smax = 0.0;
  for (int a = 0; a < L; ++a) smax = fmax(smax, Ss[a * LD + a]);
  __syncthreads();
  lane_cholesky<L>(col, row, rinv, 1e-13 * smax);
  if (lane < L) {
#pragma unroll
    for (int i = 0; i < L; ++i) Ss[i * LD + lane] = col[i];
  }
  __syncthreads();
  double t[LH], v[LH];
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int b = h * LH + ii;
    t[ii] = (cv && b < L) ? Ss[c * LD + b] : 0.0;
  }
  if (split_jacobi<L, false>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
  double mu = 0.0;
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) mu = fma(t[ii], t[ii], mu);
  mu = sqrt(col_sum<L>(mu));   // singular value of B2
  double mmax = cv ? mu : 0.0;
  for (int o = 1; o < 64; o <<= 1) mmax = fmax(mmax, __shfl_xor(mmax, o, 64));
  const double inv = (mu > 64.0 * EPS64 * mmax && mu > 0.0) ? 1.0 / mu : 0.0;
  int rank = 0;
  for (int c2 = 0; c2 < L; ++c2) {
    const double m2 = __shfl(mu, c2, 64);
    if (m2 > mu || (m2 == mu && c2 < c)) ++rank;
  }
  if (cv) {
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      if (a < L) Us[a * LD + rank] = t[ii] * inv;
    }
    if (h == 0) Es[rank] = mu;
  }
  __syncthreads();
  if (lane < R) E[lane] = Es[lane];
  for (int e = lane; e < L * R; e += 64) {
    const int l = e / R, r = e % R;
    U2s[e] = Es[r] > 0.0 ? Us[l * LD + r] / Es[r] : 0.0;
  }
  // D = Q2 U2_R (J x R), 64 rows at a time; D^T D from the same values,
  // summed over the rows in order from a copy of each 64-row block in LDS
  constexpr int NE = (L * L + 63) / 64;
  double dtd[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) dtd[i] = 0.0;
  for (int j0 = 0; j0 < J; j0 += 64) {
    const int j = j0 + lane;
    if (j < J) {
      double q[L];
#pragma unroll
      for (int l = 0; l < L; ++l) q[l] = Q2[(size_t)j * L + l];
      for (int r = 0; r < R; ++r) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) s = fma(q[l], Us[l * LD + r], s);
        D[(size_t)j * R + r] = s;
        Ds[lane * LD + r] = s;
      }
    }
    __syncthreads();
    const int nj = (J - j0 < 64) ? J - j0 : 64;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = lane + 64 * i;
      if (e < R * R) {
        const int a = e / R, b = e % R;
        double s = dtd[i];
        for (int jj = 0; jj < nj; ++jj) s = fma(Ds[jj * LD + a], Ds[jj * LD + b], s);
        dtd[i] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = lane + 64 * i;
    if (e < R * R) DtD[e] = dtd[i];
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl->warn, warn);
}

// ---------------------------------------------------------------------------
// The same steps for long Y2 (J >= S2_WIDE_J): the J-long parts (the Gram of
// each whitening pass, Y2 <- Y2 Wh, D = Q2 U2_R and D^T D) are spread over
// one wave per 64 rows of each tensor; the L x L factorisations stay on one
// wave per tensor.  Partials of the 64-row blocks are summed in block order.
// ---------------------------------------------------------------------------

// part[t][b] = (rows 64 b .. 64 b + 63 of Y2)^T (same rows), L x L
template <int L>
__global__ __launch_bounds__(64) void k_s2_gram(int J, const double* __restrict__ Yall, double* __restrict__ part) {
  constexpr int LD = L + 1;
  __shared__ double Ys[64 * LD];
  const int b = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  const double* __restrict__ Y = Yall + (size_t)t * J * L;
  const int j0 = 64 * b, nj = (J - j0 < 64) ? J - j0 : 64;
  for (int e = lane; e < 64 * L; e += 64) {
    const int jj = e / L;
    Ys[jj * LD + e % L] = (jj < nj) ? Y[(size_t)(j0 + jj) * L + e % L] : 0.0;
  }
  __syncthreads();
  double* __restrict__ out = part + ((size_t)t * gridDim.x + b) * L * L;
  for (int e = lane; e < L * L; e += 64) {
    const int a = e / L, c = e % L;
    double sum = 0.0;
    for (int jj = 0; jj < 64; ++jj) sum = fma(Ys[jj * LD + a], Ys[jj * LD + c], sum);
    out[e] = sum;
  }
}

// out[t * ostride + e] = sum over b < nb (in order, four accumulators b mod 4
// combined pairwise) of part[(t * nb + b) * width + e]
static __global__ __launch_bounds__(64) void k_fixsum(int nb, int width, const double* __restrict__ part,
                                               double* __restrict__ out, int64_t ostride) {
  const int e = blockIdx.x * 64 + threadIdx.x, t = blockIdx.y;
  if (e >= width) return;
  const double* __restrict__ p = part + (size_t)t * nb * width + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = 0;
  for (; b + 4 <= nb; b += 4) {
    s0 += p[(size_t)b * width];
    s1 += p[(size_t)(b + 1) * width];
    s2 += p[(size_t)(b + 2) * width];
    s3 += p[(size_t)(b + 3) * width];
  }
  for (; b < nb; ++b) s0 += p[(size_t)b * width];
  out[(size_t)t * ostride + e] = (s0 + s1) + (s2 + s3);
}

// Whitening of one tensor from its Gram G (L x L): Wh = R^{-1} (Cholesky
// G = R^T R), or the eigen form when a pivot is below 1e-9 of the largest
// diagonal, as in k_s2_orth; one wave per tensor
template <int L>
__global__ __launch_bounds__(64) void k_s2_whiten(const double* __restrict__ Gall, double* __restrict__ Whall,
                                                  Ctl* ctlall) {
  constexpr int RM = SC<L>::RM, LH = SC<L>::LH, LD = SC<L>::LD;
  __shared__ double Gs[L * LD], Ws[L * LD], row[L], rinv[L];
  const int t = blockIdx.x, lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const bool cv = c < L;
  const double* __restrict__ G = Gall + (size_t)t * L * L;
  double* __restrict__ Wh = Whall + (size_t)t * L * L;
  unsigned warn = 0;
  for (int e = lane; e < L * L; e += 64) Gs[(e / L) * LD + e % L] = G[e];
  __syncthreads();
  double t_[LH], v[LH];
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int a = h * LH + ii;
    t_[ii] = (cv && a < L) ? Gs[a * LD + c] : 0.0;
    v[ii] = (a == c) ? 1.0 : 0.0;
  }
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
    if (lane < L) {
      double x[L];
#pragma unroll
      for (int i = L - 1; i >= 0; --i) {
        double sum = (i == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int j = i + 1; j < L; ++j) sum = fma(-Gs[i * LD + j], x[j], sum);
        x[i] = (i > lane) ? 0.0 : sum * rinv[i];
      }
#pragma unroll
      for (int i = 0; i < L; ++i) Ws[i * LD + lane] = x[i];
    }
  } else {
    if (split_jacobi<L, true>(t_, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
    double lam = 0.0;
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) lam = fma(t_[ii], t_[ii], lam);
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
  for (int e = lane; e < L * L; e += 64) Wh[e] = Ws[(e / L) * LD + e % L];
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctlall[t].warn, warn);
}

// Y2 <- Y2 Wh in place, one lane per row (its row read whole first), Wh of
// the tensor through scalar loads
template <int L>
__global__ __launch_bounds__(64) void k_s2_apply(int J, double* __restrict__ Yall, const double* __restrict__ Whall) {
  const int t = blockIdx.y, j = blockIdx.x * 64 + threadIdx.x;
  if (j >= J) return;
  double* __restrict__ y = Yall + ((size_t)t * J + j) * L;
  const double* __restrict__ Wh = Whall + (size_t)t * L * L;
  double yv[L];
#pragma unroll
  for (int a = 0; a < L; ++a) yv[a] = y[a];
#pragma unroll
  for (int c = 0; c < L; ++c) {
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < L; ++a) sum = fma(yv[a], Wh[a * L + c], sum);
    y[c] = sum;
  }
}

// Small SVD of B2 B2^T as in k_s2_evd, without D: E, U2_R E^{-1} (U2s) and
// U2_R itself (Us, L x R per tensor) for k_s2_dmat; one wave per tensor
template <int L>
__global__ __launch_bounds__(64) void k_s2_svd(int R, const double* __restrict__ S2all, double* __restrict__ Eall,
                                               double* __restrict__ U2all, double* __restrict__ Usall, Ctl* ctlall) {
  const int tt = blockIdx.x;
  const double* __restrict__ S2 = S2all + (size_t)tt * (L * (L + 1) / 2);
  double* __restrict__ E = Eall + (size_t)tt * R;
  double* __restrict__ U2s = U2all + (size_t)tt * L * R;
  double* __restrict__ Uout = Usall + (size_t)tt * L * L;
  Ctl* ctl = ctlall + tt;
  constexpr int RM = SC<L>::RM, LH = SC<L>::LH, LD = SC<L>::LD;
  constexpr int NP = L * (L + 1) / 2;
  __shared__ double Ss[L * LD], Us[L * LD], Es[L], row[L], rinv[L];
  const int lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const bool cv = c < L;
  unsigned warn = 0;
  for (int pi = lane; pi < NP; pi += 64) {
    int a = 0, rem = pi;
    while (rem >= L - a) {
      rem -= L - a;
      ++a;
    }
    const int b = a + rem;
    const double sv = S2[pi];
    Ss[a * LD + b] = sv;
    Ss[b * LD + a] = sv;
  }
  __syncthreads();
  double col[L];
#pragma unroll
  for (int i = 0; i < L; ++i) col[i] = (lane < L) ? Ss[i * LD + lane] : 0.0;
  double smax = 0.0;
  for (int a = 0; a < L; ++a) smax = fmax(smax, Ss[a * LD + a]);
  __syncthreads();
  lane_cholesky<L>(col, row, rinv, 1e-13 * smax);
  if (lane < L) {
#pragma unroll
    for (int i = 0; i < L; ++i) Ss[i * LD + lane] = col[i];
  }
  __syncthreads();
  double t[LH], v[LH];
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int b = h * LH + ii;
    t[ii] = (cv && b < L) ? Ss[c * LD + b] : 0.0;
  }
  if (split_jacobi<L, false>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
  double mu = 0.0;
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) mu = fma(t[ii], t[ii], mu);
  mu = sqrt(col_sum<L>(mu));
  double mmax = cv ? mu : 0.0;
  for (int o = 1; o < 64; o <<= 1) mmax = fmax(mmax, __shfl_xor(mmax, o, 64));
  const double inv = (mu > 64.0 * EPS64 * mmax && mu > 0.0) ? 1.0 / mu : 0.0;
  int rank = 0;
  for (int c2 = 0; c2 < L; ++c2) {
    const double m2 = __shfl(mu, c2, 64);
    if (m2 > mu || (m2 == mu && c2 < c)) ++rank;
  }
  if (cv) {
#pragma unroll
    for (int ii = 0; ii < LH; ++ii) {
      const int a = h * LH + ii;
      if (a < L) Us[a * LD + rank] = t[ii] * inv;
    }
    if (h == 0) Es[rank] = mu;
  }
  __syncthreads();
  if (lane < R) E[lane] = Es[lane];
  for (int e = lane; e < L * R; e += 64) {
    const int l = e / R, r = e % R;
    U2s[e] = Es[r] > 0.0 ? Us[l * LD + r] / Es[r] : 0.0;
    Uout[e] = Us[l * LD + r];
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl->warn, warn);
}

// D = Q2 U2_R (J x R) one lane per row (U2_R through scalar loads), and the
// 64-row block's partial of D^T D (R x R) from a copy of its rows in LDS
template <int L>
__global__ __launch_bounds__(64) void k_s2_dmat(int J, int R, const double* __restrict__ Q2all,
                                                const double* __restrict__ Usall, double* __restrict__ Dall,
                                                double* __restrict__ part) {
  constexpr int LD = L + 1;
  __shared__ double Ds[64 * LD];
  const int b = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  const int j = 64 * b + lane, nj = (J - 64 * b < 64) ? J - 64 * b : 64;
  const double* __restrict__ Us = Usall + (size_t)t * L * L;   // L x R
  if (j < J) {
    const double* __restrict__ q = Q2all + ((size_t)t * J + j) * L;
    double qv[L];
#pragma unroll
    for (int l = 0; l < L; ++l) qv[l] = q[l];
    double* __restrict__ D = Dall + ((size_t)t * J + j) * R;
    for (int r = 0; r < R; ++r) {
      double sum = 0.0;
#pragma unroll
      for (int l = 0; l < L; ++l) sum = fma(qv[l], Us[l * R + r], sum);
      D[r] = sum;
      Ds[lane * LD + r] = sum;
    }
  }
  __syncthreads();
  double* __restrict__ out = part + ((size_t)t * gridDim.x + b) * R * R;
  for (int e = lane; e < R * R; e += 64) {
    const int a = e / R, c = e % R;
    double sum = 0.0;
    for (int jj = 0; jj < nj; ++jj) sum = fma(Ds[jj * LD + a], Ds[jj * LD + c], sum);
    out[e] = sum;
  }
}

// which = 0: orthonormalise each tensor's Y2 in place; which = 1: small SVD
// of each B2 B2^T (packed pairs S2) and D, E, U2_R E^{-1}, D^T D; one block
// per tensor
// scratch (J >= S2_WIDE_J): s2_scratch_doubles(nt, J, L, R) doubles
template <int L>
hipError_t s2_small_launch(int nt, int which, int J, int R, double* Y2, const double* S2, double* D,
                           double* E, double* U2s, double* small, Ctl* ctl, double* scratch, hipStream_t s) {
  if (J < S2_WIDE_J) {
    if (which == 0)
      hipLaunchKernelGGL(k_s2_orth<L>, dim3((unsigned)nt), dim3(64), 0, s, J, Y2, ctl);
    else
      hipLaunchKernelGGL(k_s2_evd<L>, dim3((unsigned)nt), dim3(64), 0, s, J, R, S2, Y2, D, E, U2s, small, ctl);
    return hipGetLastError();
  }
  const int nb = (J + 63) / 64, M = L > R ? L : R;
  double* part = scratch;                             // nt x nb x M^2
  double* sq = part + (size_t)nt * nb * M * M;        // nt x L^2: the summed Gram
  double* wh = sq + (size_t)nt * L * L;               // nt x L^2: Wh, later U2_R
  const dim3 rows((unsigned)nb, (unsigned)nt);
  if (which == 0) {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_s2_gram<L>, rows, dim3(64), 0, s, J, Y2, part);
      hipLaunchKernelGGL(k_fixsum, dim3((unsigned)((L * L + 63) / 64), (unsigned)nt), dim3(64), 0, s, nb, L * L, part,
                         sq, (int64_t)L * L);
      hipLaunchKernelGGL(k_s2_whiten<L>, dim3((unsigned)nt), dim3(64), 0, s, sq, wh, ctl);
      hipLaunchKernelGGL(k_s2_apply<L>, rows, dim3(64), 0, s, J, Y2, wh);
    }
  } else {
    hipLaunchKernelGGL(k_s2_svd<L>, dim3((unsigned)nt), dim3(64), 0, s, R, S2, E, U2s, wh, ctl);
    hipLaunchKernelGGL(k_s2_dmat<L>, rows, dim3(64), 0, s, J, R, Y2, wh, D, part);
    hipLaunchKernelGGL(k_fixsum, dim3((unsigned)((R * R + 63) / 64), (unsigned)nt), dim3(64), 0, s, nb, R * R, part,
                       small + SM_DTD * R * R, (int64_t)SM_COUNT * R * R);
  }
  return hipGetLastError();
}

}  // namespace dpar2
