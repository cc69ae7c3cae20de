// PARAFAC2-ALS on the uncompressed slices (Alg. 2; the method DPar2 speeds
// up), templated on the rank R.  One iteration:
//
//   slab pass   Z'_k = X_k V (the first-stage slab kernel with the shared
//               sketch matrix V, rounded to float32), with the item partials
//               Z'^T Z' (R x R) and Z'^T X_k (R x J), exactly as the first
//               stage forms Y^T Y and Y^T X
//   slice       per slice k: T = S_k H^T, Z_k = X_k V S_k H^T = Z'_k T,
//               G = Z_k^T Z_k = T^T (Z'^T Z') T; the polar factor of Z_k is
//               Q_k = Z_k G^{-1/2} (G^{-1/2} from a Jacobi eigen-decomposition
//               of G), so Y_k = Q_k^T X_k = G^{-1/2} T^T (Z'^T X_k) (R x J,
//               stored); Theta_k = T G^{-1/2} (Q_k = Z'_k Theta_k, for U_k);
//               the slice's part of G1 = sum_k Y_k V S_k (H update)
//   H           H = G1 (W^T W * V^T V)^dagger, unit columns; H^T H
//   V pass      per block of slices, partial G2 = sum_k Y_k^T H S_k (J x R)
//   V           V = G2 (W^T W * H^T H)^dagger, unit columns; V^T V; the
//               float32 copy of V for the next slab pass;
//               (V^T V * H^T H)^dagger
//   W pass      per slice: G3(k, r) = H(:, r)^T Y_k V(:, r); W(k, :) =
//               G3(k, :) (V^T V * H^T H)^dagger; partials of W^T W and of the
//               error terms
//   error       e = sum_k ||X_k||^2 - 2 sum_{k,r} W(k,r) G3(k,r)
//                   + sum_k W(k,:) (H^T H * V^T V) W(k,:)^T
//               (= sum_k ||X_k - Q_k H S_k V^T||^2, as Q_k^T Q_k = I), stop rule
//
// Every kernel returns at once once the stop rule has fired (the slab pass
// through SlabArgs::skip).  Partial sums are per slice or per block and are
// reduced in a fixed order.
#pragma once

#include "als_impl.h"

namespace dpar2 {

constexpr int PL_CW = 32;        // columns of Z'^T X streamed per chunk

// Begin of a call: W^T W, V^T V from the factors, the float32 copy of V, the
// control block.  One block.
template <int R>
__global__ __launch_bounds__(256) void k_pl_begin(PlainArgs a) {
  constexpr int RR = R * R;
  const int tid = threadIdx.x;
  for (int e = tid; e < a.J * R; e += 256) a.om_next[e] = (float)a.V[e];
  for (int e = tid; e < RR; e += 256) {
    const int p = e / R, q = e % R;
    double w = 0.0, v = 0.0;
    for (int64_t k = 0; k < a.K; ++k) w = fma(a.W[k * R + p], a.W[k * R + q], w);
    for (int j = 0; j < a.J; ++j) v = fma(a.V[(size_t)j * R + p], a.V[(size_t)j * R + q], v);
    a.small[SM_WTW * RR + e] = w;
    a.small[SM_VTV * RR + e] = v;
  }
  if (tid == 0) {
    Ctl z;
    z.iters = 0;
    z.done = 0;
    z.base = 0;
    z.warn = 0;
    z.vc_valid = 0;
    z.bad = 0;
    z.e_prev = 0.0;
    z.e0 = 0.0;
    z.xnorm2 = 0.0;
    z.fit_true = 0.0;
    *a.ctl = z;
  }
}

// Start of an iteration: the slab pass reads the float32 V the previous
// iteration produced (om_cur keeps the one of the last pass that ran, for U).
static __global__ __launch_bounds__(256) void k_pl_commit(PlainArgs a, int n) {
  if (a.ctl->done) return;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) a.om_cur[e] = a.om_next[e];
}

// Per slice (one wave): G = T^T G' T, G^{-1/2}, Y_k, Theta_k, G1 part.
template <int R>
__global__ __launch_bounds__(64) void k_pl_slice(PlainArgs a) {
  constexpr int RM = SC<R>::RM, LH = SC<R>::LH, LD = R + 1, RR = R * R, CP = PL_CW + 1;
  __shared__ double Gp[R * LD], Ts[R * LD], Gs[R * LD], Ms[R * LD];
  __shared__ double Pc[R * CP], Yc[R * CP], Vc[PL_CW * LD];
  double* const Ws = Gp;   // eigenvectors, once G' is no longer needed
  __shared__ double lam[R];
  const int lane = threadIdx.x, c = lane % RM, h = lane / RM;
  const bool cv = c < R;
  const int64_t k = blockIdx.x;
  const int J = a.J;
  if (a.ctl->done) return;
  const int i0 = a.slice_ptr[k], i1 = a.slice_ptr[k + 1];
  unsigned warn = 0;
  // G' (summed over the slice's items), T = S_k H^T, ||X_k||^2
  for (int e = lane; e < RR; e += 64) {
    double s = 0.0;
    for (int q = i0; q < i1; ++q) s += a.partG[(size_t)a.slice_list[q] * RR + e];
    Gp[(e / R) * LD + e % R] = s;
    const int p = e / R, b = e % R;   // T[p][b] = W(k, p) H[b][p]
    Ts[p * LD + b] = a.W[k * R + p] * a.H[b * R + p];
  }
  if (lane == 0) {
    double s = 0.0;
    for (int q = i0; q < i1; ++q) s += a.partS[a.slice_list[q]];
    a.xnorm2[k] = s;
  }
  __syncthreads();
  // G = T^T G' T: first Ms = G' T, then Gs = T^T Ms
  for (int e = lane; e < RR; e += 64) {
    const int p = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(Gp[p * LD + i], Ts[i * LD + b], s);
    Ms[p * LD + b] = s;
  }
  __syncthreads();
  for (int e = lane; e < RR; e += 64) {
    const int p = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(Ts[i * LD + p], Ms[i * LD + b], s);
    Gs[p * LD + b] = s;
  }
  __syncthreads();
  // symmetric eigen-decomposition by one-sided Jacobi: G E = E Lambda
  double t[LH], v[LH];
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int r = h * LH + ii;
    t[ii] = (cv && r < R) ? 0.5 * (Gs[r * LD + c] + Gs[c * LD + r]) : 0.0;
    v[ii] = (cv && r == c) ? 1.0 : 0.0;
  }
  if (split_jacobi<R, true>(t, v, c, h) == JACOBI_SWEEPS) warn |= 0x1u;
  double l2 = 0.0;
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) l2 = fma(t[ii], t[ii], l2);
  const double l = sqrt(col_sum<R>(l2));   // eigenvalue (G is positive semidefinite)
  double lmax = cv ? l : 0.0;
  for (int o = 1; o < 64; o <<= 1) lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  const bool keep = cv && l > 64.0 * EPS64 * lmax && l > 0.0;
  if (cv && !keep) warn |= 0x2u;   // Z_k (numerically) rank deficient
  const double isq = keep ? 1.0 / sqrt(l) : 0.0;
#pragma unroll
  for (int ii = 0; ii < LH; ++ii) {
    const int r = h * LH + ii;
    if (cv && r < R) Ws[r * LD + c] = v[ii];   // eigenvector c in column c
  }
  if (cv && h == 0) lam[c] = isq;
  __syncthreads();
  // G^{-1/2} = E diag(isq) E^T (into Gs)
  for (int e = lane; e < RR; e += 64) {
    const int p = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(Ws[p * LD + i] * lam[i], Ws[b * LD + i], s);
    Gs[p * LD + b] = s;
  }
  __syncthreads();
  // M = G^{-1/2} T^T (Y_k = M Z'^T X_k) and Theta_k = T G^{-1/2} = M^T
  for (int e = lane; e < RR; e += 64) {
    const int p = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(Gs[p * LD + i], Ts[b * LD + i], s);
    Ms[p * LD + b] = s;
    a.theta[(size_t)k * RR + b * R + p] = s;
  }
  __syncthreads();
  // stream Z'^T X_k in chunks: Y_k chunk = M Pc, G1 part += Y chunk V chunk
  double g1[(RR + 63) / 64];
#pragma unroll
  for (int u = 0; u < (RR + 63) / 64; ++u) g1[u] = 0.0;
  double* Yk = a.Y + (size_t)k * R * J;
  for (int j0 = 0; j0 < J; j0 += PL_CW) {
    const int nj = (J - j0 < PL_CW) ? J - j0 : PL_CW;
    for (int e = lane; e < R * PL_CW; e += 64) {
      const int p = e / PL_CW, jj = e % PL_CW;
      double s = 0.0;
      if (jj < nj)
        for (int q = i0; q < i1; ++q) s += a.partP[((size_t)a.slice_list[q] * R + p) * J + j0 + jj];
      Pc[p * CP + jj] = s;
    }
    for (int e = lane; e < PL_CW * R; e += 64) {
      const int jj = e / R, r = e % R;
      Vc[jj * LD + r] = (jj < nj) ? a.V[(size_t)(j0 + jj) * R + r] : 0.0;
    }
    __syncthreads();
    for (int e = lane; e < R * PL_CW; e += 64) {
      const int p = e / PL_CW, jj = e % PL_CW;
      double s = 0.0;
      for (int i = 0; i < R; ++i) s = fma(Ms[p * LD + i], Pc[i * CP + jj], s);
      if (jj < nj) Yk[(size_t)p * J + j0 + jj] = s;
      Yc[p * CP + jj] = (jj < nj) ? s : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (RR + 63) / 64; ++u) {
      const int e = lane + 64 * u;
      if (e < RR) {
        const int p = e / R, r = e % R;
        double s = g1[u];
        for (int jj = 0; jj < nj; ++jj) s = fma(Yc[p * CP + jj], Vc[jj * LD + r], s);
        g1[u] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < (RR + 63) / 64; ++u) {
    const int e = lane + 64 * u;
    if (e < RR) a.g1p[(size_t)k * RR + e] = g1[u] * a.W[k * R + e % R];   // (Y_k V S_k)[p][r]
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&a.ctl->warn, warn);
}

// H = G1 (W^T W * V^T V)^dagger with unit columns; H^T H.  One block; G1 in
// the first R R entries of red, sum_k ||X_k||^2 after the 6 R R + 1st.
template <int R>
__global__ __launch_bounds__(EPI_THREADS) void k_pl_h(PlainArgs a) {
  constexpr int LD = RC<R>::LD, MR = RC<R>::MR, RR = R * R;
  __shared__ double G1[MR * LD], Gm[MR * LD], Gi[MR * LD], sT[MR * LD], sV[MR * LD], sg[MR];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  if (a.ctl->done) return;
  for (int e = tid; e < RR; e += EPI_THREADS) {
    G1[(e / R) * LD + e % R] = a.red[e];
    Gm[(e / R) * LD + e % R] = a.small[SM_WTW * RR + e] * a.small[SM_VTV * RR + e];
  }
  __syncthreads();
  const int capped = block_pinv<R>(Gm, Gi, sT, sV, sg, &sflag);
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int q = e / R, c = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(G1[q * LD + i], Gi[i * LD + c], s);
    sT[q * LD + c] = s;
  }
  __syncthreads();
  if (tid < R) {
    double s = 0.0;
    for (int q = 0; q < R; ++q) s = fma(sT[q * LD + tid], sT[q * LD + tid], s);
    s = sqrt(s);
    sg[tid] = (s < 1e-300) ? 1.0 : s;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int q = e / R, c = e % R;
    const double hv = sT[q * LD + c] / sg[c];
    a.H[e] = hv;
    G1[q * LD + c] = hv;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int q = e / R, c = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(G1[i * LD + q], G1[i * LD + c], s);
    a.small[SM_HTH * RR + e] = s;
  }
  if (tid == 0) {
    a.ctl->xnorm2 = a.red[RED_WIDTH * RR + 1];
    if (capped) atomicOr(&a.ctl->warn, 0x1u);
  }
}

// Partial G2 = sum_{k in block} Y_k^T H S_k (J x R); thread per column j.
template <int R>
__global__ __launch_bounds__(256) void k_pl_v(PlainArgs a) {
  constexpr int RR = R * R;
  __shared__ double sH[RR], sW[PL_VSLICES * R];
  const int tid = threadIdx.x, J = a.J;
  if (a.ctl->done) return;
  const int64_t k0 = (int64_t)blockIdx.x * PL_VSLICES;
  const int nk = (int)((a.K - k0 < PL_VSLICES) ? a.K - k0 : PL_VSLICES);
  for (int e = tid; e < RR; e += 256) sH[e] = a.H[e];
  for (int e = tid; e < nk * R; e += 256) sW[e] = a.W[k0 * R + e];
  __syncthreads();
  for (int j = (int)blockIdx.y * 256 + tid; j < J; j += (int)gridDim.y * 256) {
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int kk = 0; kk < nk; ++kk) {
      const double* Yk = a.Y + (size_t)(k0 + kk) * R * J;
      double y[R];
#pragma unroll
      for (int p = 0; p < R; ++p) y[p] = Yk[(size_t)p * J + j];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < R; ++p) s = fma(y[p], sH[p * R + r], s);
        acc[r] = fma(s, sW[kk * R + r], acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) a.g2p[((size_t)blockIdx.x * J + j) * R + r] = acc[r];
  }
}

// V = G2 (W^T W * H^T H)^dagger, unit columns; V^T V; float32 V for the next
// pass; H^T H * V^T V and (V^T V * H^T H)^dagger.  One block.
template <int R>
__global__ __launch_bounds__(EPI_THREADS) void k_pl_vupd(PlainArgs a) {
  constexpr int LD = RC<R>::LD, MR = RC<R>::MR, RR = R * R;
  __shared__ double Gm[MR * LD], Gi[MR * LD], sT[MR * LD], sV[MR * LD], sg[MR], nrm[MR], red[16];
  __shared__ int sflag;
  const int tid = threadIdx.x, J = a.J;
  if (a.ctl->done) return;
  for (int e = tid; e < RR; e += EPI_THREADS)
    Gm[(e / R) * LD + e % R] = a.small[SM_WTW * RR + e] * a.small[SM_HTH * RR + e];
  __syncthreads();
  int capped = block_pinv<R>(Gm, Gi, sT, sV, sg, &sflag);
  // raw V = G2 Gi, written to V; column norms
  double cn[R];
#pragma unroll
  for (int r = 0; r < R; ++r) cn[r] = 0.0;
  for (int j = tid; j < J; j += EPI_THREADS) {
    double g[R];
#pragma unroll
    for (int i = 0; i < R; ++i) g[i] = a.g2[(size_t)j * R + i];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) s = fma(g[i], Gi[i * LD + c], s);
      a.V[(size_t)j * R + c] = s;
      cn[c] = fma(s, s, cn[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const double s = block_sum(cn[c], red);
    if (tid == 0) nrm[c] = (sqrt(s) < 1e-300) ? 1.0 : sqrt(s);
  }
  __syncthreads();
  // normalise (each thread rescales the rows it wrote), float32 copy, V^T V
  double vt[RR <= 64 ? RR : 1];
  constexpr bool SMALLR = RR <= 64;
  if constexpr (SMALLR) {
#pragma unroll
    for (int e = 0; e < RR; ++e) vt[e] = 0.0;
  }
  for (int j = tid; j < J; j += EPI_THREADS) {
    double x[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      x[c] = a.V[(size_t)j * R + c] / nrm[c];
      a.V[(size_t)j * R + c] = x[c];
      a.om_next[(size_t)j * R + c] = (float)x[c];
    }
    if constexpr (SMALLR) {
#pragma unroll
      for (int p = 0; p < R; ++p)
#pragma unroll
        for (int q = 0; q < R; ++q) vt[p * R + q] = fma(x[p], x[q], vt[p * R + q]);
    }
  }
  __syncthreads();
  if constexpr (SMALLR) {
#pragma unroll
    for (int e = 0; e < RR; ++e) {
      const double s = block_sum(vt[e], red);
      if (tid == 0) sT[(e / R) * LD + e % R] = s;
    }
  } else {
    // larger ranks: one (p, q) entry per thread over all rows (V re-read)
    for (int e = tid; e < RR; e += EPI_THREADS) {
      const int p = e / R, q = e % R;
      double s = 0.0;
      for (int j = 0; j < J; ++j) s = fma(a.V[(size_t)j * R + p], a.V[(size_t)j * R + q], s);
      sT[p * LD + q] = s;
    }
  }
  __syncthreads();
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int p = e / R, q = e % R;
    const double vv = sT[p * LD + q], hh = a.small[SM_HTH * RR + e];
    a.small[SM_VTV * RR + e] = vv;
    a.small[SM_HV * RR + e] = vv * hh;
    Gm[p * LD + q] = vv * hh;
  }
  __syncthreads();
  capped |= block_pinv<R>(Gm, Gi, sT, sV, sg, &sflag);
  for (int e = tid; e < RR; e += EPI_THREADS) a.small[SM_G3INV * RR + e] = Gi[(e / R) * LD + e % R];
  if (tid == 0 && capped) atomicOr(&a.ctl->warn, 0x1u);
}

// Per slice (one wave): G3(k, :), the new W(k, :), partials of W^T W and the
// two error sums (RR + 2 per slice).
template <int R>
__global__ __launch_bounds__(64) void k_pl_w(PlainArgs a) {
  constexpr int LD = R + 1, RR = R * R, CP = PL_CW + 1;
  __shared__ double Yc[R * CP], Vc[PL_CW * LD], sH[RR], sG[RR], sHV[RR], yv[RR], g3[R], wn[R];
  const int lane = threadIdx.x, J = a.J;
  const int64_t k = blockIdx.x;
  if (a.ctl->done) return;
  for (int e = lane; e < RR; e += 64) {
    sH[e] = a.H[e];
    sG[e] = a.small[SM_G3INV * RR + e];
    sHV[e] = a.small[SM_HV * RR + e];
  }
  double acc[(RR + 63) / 64];
#pragma unroll
  for (int u = 0; u < (RR + 63) / 64; ++u) acc[u] = 0.0;
  const double* Yk = a.Y + (size_t)k * R * J;
  for (int j0 = 0; j0 < J; j0 += PL_CW) {
    const int nj = (J - j0 < PL_CW) ? J - j0 : PL_CW;
    __syncthreads();
    for (int e = lane; e < R * PL_CW; e += 64) {
      const int p = e / PL_CW, jj = e % PL_CW;
      Yc[p * CP + jj] = (jj < nj) ? Yk[(size_t)p * J + j0 + jj] : 0.0;
    }
    for (int e = lane; e < PL_CW * R; e += 64) {
      const int jj = e / R, r = e % R;
      Vc[jj * LD + r] = (jj < nj) ? a.V[(size_t)(j0 + jj) * R + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (RR + 63) / 64; ++u) {
      const int e = lane + 64 * u;
      if (e < RR) {
        const int p = e / R, r = e % R;
        double s = acc[u];
        for (int jj = 0; jj < nj; ++jj) s = fma(Yc[p * CP + jj], Vc[jj * LD + r], s);
        acc[u] = s;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < (RR + 63) / 64; ++u) {
    const int e = lane + 64 * u;
    if (e < RR) yv[e] = acc[u];   // (Y_k V)[p][r]
  }
  __syncthreads();
  if (lane < R) {   // G3(k, r) = H(:, r)^T (Y_k V)(:, r)
    double s = 0.0;
    for (int p = 0; p < R; ++p) s = fma(sH[p * R + lane], yv[p * R + lane], s);
    g3[lane] = s;
  }
  __syncthreads();
  if (lane < R) {
    double s = 0.0;
    for (int q = 0; q < R; ++q) s = fma(g3[q], sG[q * R + lane], s);
    wn[lane] = s;
    a.W[k * R + lane] = s;
  }
  __syncthreads();
  double* out = a.wp + (size_t)k * (RR + 2);
  for (int e = lane; e < RR; e += 64) out[e] = wn[e / R] * wn[e % R];
  if (lane == 0) {
    double ewg = 0.0, equad = 0.0;
    for (int r = 0; r < R; ++r) {
      ewg = fma(wn[r], g3[r], ewg);
      double q = 0.0;
      for (int s = 0; s < R; ++s) q = fma(sHV[r * R + s], wn[s], q);
      equad = fma(wn[r], q, equad);
    }
    out[RR] = ewg;
    out[RR + 1] = equad;
  }
}

// W^T W, e_t, stop rule.  One block; the summed W-pass partials at red + 2 R R.
template <int R>
__global__ __launch_bounds__(64) void k_pl_err(PlainArgs a) {
  constexpr int RR = R * R;
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  const double* s = a.red + 2 * RR;
  for (int e = threadIdx.x; e < RR; e += 64) a.small[SM_WTW * RR + e] = s[e];
  if (threadIdx.x == 0) {
    const double e = ctl->xnorm2 - 2.0 * s[RR] + s[RR + 1];
    const int it = ctl->iters;
    if (a.trace) a.trace[it - ctl->base] = e;
    ctl->iters = it + 1;
    if (a.tol >= 0.0 && it + 1 >= 2 && ctl->e_prev - e < a.tol * ctl->e_prev) ctl->done = 1;
    ctl->e_prev = e;
    ctl->fit_true = ctl->xnorm2 > 0.0 ? 1.0 - e / ctl->xnorm2 : 0.0;
  }
}

// Theta_k H (Q_k H = Z'_k Theta_k H = U_k), in place.  One block per slice.
template <int R>
__global__ __launch_bounds__(64) void k_pl_theta(PlainArgs a) {
  constexpr int RR = R * R;
  __shared__ double th[RR], sH[RR];
  const int64_t k = blockIdx.x;
  double* T = a.theta + (size_t)k * RR;
  for (int e = threadIdx.x; e < RR; e += 64) {
    th[e] = T[e];
    sH[e] = a.H[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < RR; e += 64) {
    const int p = e / R, q = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(th[p * R + i], sH[i * R + q], s);
    T[e] = s;
  }
}

// the launch sequence of one phase (0 begin, 1 iteration, 2 U output)
template <int R>
inline hipError_t plain_launch(int phase, const PlainArgs& a, const PlainLaunch& pl, hipStream_t s) {
  constexpr int RR = R * R;
  const int64_t K = a.K;
  const int J = a.J;
  hipError_t e;
  if (phase == 0) {   // begin
    hipLaunchKernelGGL(k_pl_begin<R>, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (phase == 2) {   // U output: Theta_k H
    hipLaunchKernelGGL(k_pl_theta<R>, dim3((unsigned)K), dim3(64), 0, s, a);
    return hipGetLastError();
  }
  const int n = J * R;
  hipLaunchKernelGGL(k_pl_commit, dim3((unsigned)std::min(64, (n + 255) / 256)), dim3(256), 0, s, a, n);
  if ((e = launch_slab(pl.slab, pl.dtype, pl.n_items, pl.vec, false, pl.wide, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl_slice<R>, dim3((unsigned)K), dim3(64), 0, s, a);
  if ((e = launch_segsum(1, nullptr, K, RR, RR, a.g1p, a.red, RR, s)) != hipSuccess) return e;
  if ((e = launch_segsum(1, nullptr, K, 1, 1, a.xnorm2, a.red + RED_WIDTH * RR + 1, 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl_h<R>, dim3(1), dim3(EPI_THREADS), 0, s, a);
  const unsigned nvb = (unsigned)((K + PL_VSLICES - 1) / PL_VSLICES);
  hipLaunchKernelGGL(k_pl_v<R>, dim3(nvb, (unsigned)((J + 255) / 256)), dim3(256), 0, s, a);
  if ((e = launch_segsum(1, nullptr, nvb, (int64_t)J * R, (int64_t)J * R, a.g2p, a.g2, (int64_t)J * R, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_pl_vupd<R>, dim3(1), dim3(EPI_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_pl_w<R>, dim3((unsigned)K), dim3(64), 0, s, a);
  if ((e = launch_segsum(1, nullptr, K, RR + 2, RR + 2, a.wp, a.red + 2 * RR, RR + 2, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pl_err<R>, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace dpar2
