// Compressed PARAFAC2-ALS iteration (Alg. 3 repeat loop, Secs. III-C..III-E).
//
// Per iteration (every kernel returns at once after the stop rule fired):
//   prep : record e of the previous iteration + stop test; W^T W, V^T V,
//          Bm = E D^T V
//   A    : per slice, T_k = F^(k) Bm S_k H^T (Eq. 8); one-sided Jacobi SVD
//          T_k = Z_k Sigma_k P_k^T (FP64, warm-started from the previous P_k);
//          Psi_k = Z_k P_k^T; M_k = P_k Z_k^T F^(k) = Psi_k^T F^(k) (the factor
//          of Y_k, Sec. III-D); G1 partial sum_k M_k Bm S_k (Lemma 1)
//   H    : H = G1 (W^T W * V^T V)^dagger, unit columns
//   B    : N partial sum_k M_k^T H S_k (Lemma 2: G2 = D E N)
//   V    : V = D E N (W^T W * H^T H)^dagger, unit columns; Bm' = E D^T V;
//          (V^T V * H^T H)^dagger
//   C    : G3(k,r) = H(:,r)^T M_k Bm'(:,r) (Lemma 3); W(k,:) = G3(k,:) (V^T V *
//          H^T H)^dagger (S_k = diag(W(k,:))); partials of W^T W and of the
//          error e = e0 - 2 sum W.G3 + sum_k W(k,:)(H^T H * V^T V)W(k,:)^T
// Per-slice kernels give each slice a group of RM lanes, lane j owning column
// j of the R x R matrices (rows in registers); partner columns of a Jacobi
// round are exchanged with cross-lane moves.
#include "internal.h"

namespace dpar2 {

constexpr int TPB = 128;   // threads of the per-slice kernels
constexpr double JACOBI_TOL = 1e-15;
constexpr int JACOBI_SWEEPS = 30;

template <int RM>
__global__ __launch_bounds__(TPB) void k_als_A(int K, int R, const double* __restrict__ F,
                                              const double* __restrict__ W, const double* __restrict__ H,
                                              const double* __restrict__ Bm, double* __restrict__ Pw,
                                              double* __restrict__ Psi, double* __restrict__ Mk,
                                              double* __restrict__ partA, Ctl* ctl) {
  if (ctl->done) return;
  constexpr int GPB = TPB / RM;
  __shared__ double sH[32 * 32], sB[32 * 32];
  __shared__ double sF[GPB * RM * RM], sZ[GPB * RM * RM], sP[GPB * RM * RM];
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  const int lane = tid & 63, gbase = lane & ~(RM - 1);
  const int RR = R * R;
  for (int e = tid; e < RR; e += TPB) {
    sH[e] = H[e];
    sB[e] = Bm[e];
  }
  double* F_ = sF + g * RM * RM;
  double* Z_ = sZ + g * RM * RM;
  double* P_ = sP + g * RM * RM;
  const int n = R + (R & 1);
  double acc[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) acc[a] = 0.0;
  unsigned warn = 0;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < K; base += (int64_t)gridDim.x * GPB) {
    const int64_t k = base + g;
    const bool live = (k < K) && (j < R);
    __syncthreads();
    if (k < K)
      for (int e = j; e < RR; e += RM) F_[(e / R) * RM + (e % R)] = F[(size_t)k * RR + e];
    __syncthreads();
    double wk[RM];
    double t[RM], v[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      wk[i] = (k < K && i < R) ? W[(size_t)k * R + i] : 0.0;
      v[i] = (live && i < R) ? Pw[(size_t)k * RR + i * R + j] : 0.0;
    }
    // t = F^(k) Bm diag(W_k) H^T p_j   (column j of T_k P_k)
    {
      double u[RM], x[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        double s = 0.0;
        if (a < R)
#pragma unroll
          for (int i = 0; i < RM; ++i)
            if (i < R) s += sH[i * R + a] * v[i];
        u[a] = s * wk[a];
      }
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        double s = 0.0;
        if (a < R)
#pragma unroll
          for (int i = 0; i < RM; ++i)
            if (i < R) s += sB[a * R + i] * u[i];
        x[a] = s;
      }
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        double s = 0.0;
        if (a < R)
#pragma unroll
          for (int i = 0; i < RM; ++i)
            if (i < R) s += F_[a * RM + i] * x[i];
        t[a] = live ? s : 0.0;
      }
    }
    // one-sided Jacobi on the columns of T_k P_k; v accumulates P_k
    int sweep;
    for (sweep = 0; sweep < JACOBI_SWEEPS; ++sweep) {
      int rotated = 0;
      for (int r = 0; r < n - 1; ++r) {
        const int pc = (j < n) ? rr_partner(j, r, n) : j;
        const int src = gbase + pc;
        double tp[RM], vp[RM];
        double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          tp[i] = __shfl(t[i], src, 64);
          vp[i] = __shfl(v[i], src, 64);
          aa += t[i] * t[i];
          bb += tp[i] * tp[i];
          ab += t[i] * tp[i];
        }
        const bool low = j < pc;
        const double alpha = low ? aa : bb, beta = low ? bb : aa;
        if (j < n && pc != j && ab != 0.0 && fabs(ab) > JACOBI_TOL * sqrt(alpha * beta)) {
          double c, s;
          jacobi_cs(alpha, beta, ab, &c, &s);
          rotated = 1;
          if (low) {
#pragma unroll
            for (int i = 0; i < RM; ++i) {
              t[i] = c * t[i] - s * tp[i];
              v[i] = c * v[i] - s * vp[i];
            }
          } else {
#pragma unroll
            for (int i = 0; i < RM; ++i) {
              t[i] = s * tp[i] + c * t[i];
              v[i] = s * vp[i] + c * v[i];
            }
          }
        }
      }
      if (!__any(rotated)) break;
    }
    if (sweep == JACOBI_SWEEPS) warn |= 0x1u;
    // Z column j = t / sigma_j ; P column j = v
    double sig = 0.0;
#pragma unroll
    for (int i = 0; i < RM; ++i) sig += t[i] * t[i];
    sig = sqrt(sig);
    double smax = sig;
    for (int o = 1; o < RM; o <<= 1) smax = fmax(smax, __shfl_xor(smax, o, 64));
    if (live && !(sig > 1e-14 * smax)) warn |= 0x2u;
    const double inv = (sig > 0.0) ? 1.0 / sig : 0.0;
    if (live) {
#pragma unroll
      for (int i = 0; i < RM; ++i)
        if (i < R) {
          Z_[i * RM + j] = t[i] * inv;
          P_[i * RM + j] = v[i];
          Pw[(size_t)k * RR + i * R + j] = v[i];
        }
    }
    __syncthreads();
    // Psi column j: Psi[a][j] = sum_c Z[a][c] P[j][c]
    double psi[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      double s = 0.0;
      if (a < R)
        for (int c = 0; c < R; ++c) s += Z_[a * RM + c] * P_[j * RM + c];
      psi[a] = s;
    }
    __syncthreads();
    if (live) {
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < R) {
          P_[a * RM + j] = psi[a];
          Psi[(size_t)k * RR + a * R + j] = psi[a];
        }
    }
    __syncthreads();
    // M_k column j = Psi^T F^(k)(:, j)
    double mcol[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      double s = 0.0;
      if (a < R)
        for (int i = 0; i < R; ++i) s += P_[i * RM + a] * F_[i * RM + j];
      mcol[a] = s;
    }
    if (live) {
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < R) {
          Z_[a * RM + j] = mcol[a];
          Mk[(size_t)k * RR + a * R + j] = mcol[a];
        }
    }
    __syncthreads();
    // G1 partial, column j: W(k,j) * M_k Bm(:, j)
    if (live) {
      const double wj = wk[j];
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        double s = 0.0;
        if (a < R)
          for (int i = 0; i < R; ++i) s += Z_[a * RM + i] * sB[i * R + j];
        acc[a] += wj * s;
      }
    }
  }
  // block partial of G1
  __syncthreads();
  if (j < R)
#pragma unroll
    for (int a = 0; a < RM; ++a)
      if (a < R) sZ[g * RM * RM + a * RM + j] = acc[a];
  __syncthreads();
  for (int e = tid; e < RR; e += TPB) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int gg = 0; gg < GPB; ++gg) s += sZ[gg * RM * RM + a * RM + b];
    partA[(size_t)blockIdx.x * RR + e] = s;
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl->warn, warn);
}

// N partial: sum_k M_k^T H diag(W_k)  (column j: W(k,j) M_k^T H(:,j))
template <int RM>
__global__ __launch_bounds__(TPB) void k_als_B(int K, int R, const double* __restrict__ Mk,
                                              const double* __restrict__ W, const double* __restrict__ H,
                                              double* __restrict__ partB, const Ctl* ctl) {
  if (ctl->done) return;
  constexpr int GPB = TPB / RM;
  __shared__ double sH[32 * 32];
  __shared__ double sM[GPB * RM * RM];
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  const int RR = R * R;
  for (int e = tid; e < RR; e += TPB) sH[e] = H[e];
  double* M_ = sM + g * RM * RM;
  double acc[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) acc[a] = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < K; base += (int64_t)gridDim.x * GPB) {
    const int64_t k = base + g;
    __syncthreads();
    if (k < K)
      for (int e = j; e < RR; e += RM) M_[(e / R) * RM + (e % R)] = Mk[(size_t)k * RR + e];
    __syncthreads();
    if (k < K && j < R) {
      const double wj = W[(size_t)k * R + j];
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        double s = 0.0;
        if (a < R)
          for (int i = 0; i < R; ++i) s += M_[i * RM + a] * sH[i * R + j];
        acc[a] += wj * s;
      }
    }
  }
  __syncthreads();
  if (j < R)
#pragma unroll
    for (int a = 0; a < RM; ++a)
      if (a < R) sM[g * RM * RM + a * RM + j] = acc[a];
  __syncthreads();
  for (int e = tid; e < RR; e += TPB) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int gg = 0; gg < GPB; ++gg) s += sM[gg * RM * RM + a * RM + b];
    partB[(size_t)blockIdx.x * RR + e] = s;
  }
}

// G3 rows, new W rows, and partials of W^T W, sum W.G3, sum W (HtH*VtV) W^T.
// With update == 0 only the W^T W partials of the given W are produced.
template <int RM>
__global__ __launch_bounds__(TPB) void k_als_C(int K, int R, int update, const double* __restrict__ Mk,
                                              double* __restrict__ W, const double* __restrict__ H,
                                              const double* __restrict__ Bm, const double* __restrict__ G3inv,
                                              const double* __restrict__ HV, double* __restrict__ partC,
                                              const Ctl* ctl) {
  if (update && ctl->done) return;
  constexpr int GPB = TPB / RM;
  __shared__ double sH[32 * 32], sB[32 * 32], sGi[32 * 32], sHV[32 * 32];
  __shared__ double sM[GPB * RM * RM];
  __shared__ double sRed[GPB * RM * 2];
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  const int lane = tid & 63, gbase = lane & ~(RM - 1);
  const int RR = R * R;
  if (update)
    for (int e = tid; e < RR; e += TPB) {
      sH[e] = H[e];
      sB[e] = Bm[e];
      sGi[e] = G3inv[e];
      sHV[e] = HV[e];
    }
  double* M_ = sM + g * RM * RM;
  double wtw[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) wtw[a] = 0.0;
  double ewg = 0.0, equad = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < K; base += (int64_t)gridDim.x * GPB) {
    const int64_t k = base + g;
    const bool live = (k < K) && (j < R);
    double wnew = 0.0;
    if (update) {
      __syncthreads();
      if (k < K)
        for (int e = j; e < RR; e += RM) M_[(e / R) * RM + (e % R)] = Mk[(size_t)k * RR + e];
      __syncthreads();
      double g3 = 0.0;
      if (live) {
        for (int a = 0; a < R; ++a) {
          double s = 0.0;
          for (int i = 0; i < R; ++i) s += M_[a * RM + i] * sB[i * R + j];
          g3 += sH[a * R + j] * s;
        }
      }
      for (int s = 0; s < RM; ++s) {
        const double gs = __shfl(g3, gbase + s, 64);
        if (s < R && live) wnew += gs * sGi[s * R + j];
      }
      if (live) {
        W[(size_t)k * R + j] = wnew;
        ewg += wnew * g3;
      }
      double q = 0.0;
      for (int s = 0; s < RM; ++s) {
        const double ws = __shfl(wnew, gbase + s, 64);
        if (s < R && live) q += sHV[j * R + s] * ws;
      }
      if (live) equad += wnew * q;
    } else {
      if (live) wnew = W[(size_t)k * R + j];
    }
#pragma unroll
    for (int s = 0; s < RM; ++s) {
      const double ws = __shfl(wnew, gbase + s, 64);
      if (live && s < R) wtw[s] += ws * wnew;
    }
  }
  __syncthreads();
  if (j < R)
#pragma unroll
    for (int a = 0; a < RM; ++a)
      if (a < R) sM[g * RM * RM + a * RM + j] = wtw[a];
  sRed[g * RM * 2 + j * 2] = ewg;
  sRed[g * RM * 2 + j * 2 + 1] = equad;
  __syncthreads();
  double* out = partC + (size_t)blockIdx.x * (RR + 2);
  for (int e = tid; e < RR; e += TPB) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int gg = 0; gg < GPB; ++gg) s += sM[gg * RM * RM + a * RM + b];
    out[e] = s;
  }
  if (tid < 2) {
    double s = 0.0;
    for (int i = 0; i < GPB * RM; ++i) s += sRed[i * 2 + tid];
    out[RR + tid] = s;
  }
}

// Finish the previous iteration (error, stop rule) and prepare this one.
__global__ __launch_bounds__(256) void k_als_prep(int nblkC, int J, int R, int finalize_only, double tol,
                                                  const double* __restrict__ partC, const double* __restrict__ V,
                                                  const double* __restrict__ D, const double* __restrict__ E,
                                                  double* __restrict__ small, double* __restrict__ trace,
                                                  Ctl* ctl) {
  __shared__ double red[16];
  __shared__ int s_done;
  const int tid = threadIdx.x;
  const int RR = R * R;
  double* WtW = small + SM_WTW * RR;
  for (int e = tid; e < RR; e += 256) {
    double s = 0.0;
    for (int b = 0; b < nblkC; ++b) s += partC[(size_t)b * (RR + 2) + e];
    WtW[e] = s;
  }
  double wg = 0.0, qd = 0.0;
  for (int b = tid; b < nblkC; b += 256) {
    wg += partC[(size_t)b * (RR + 2) + RR];
    qd += partC[(size_t)b * (RR + 2) + RR + 1];
  }
  wg = block_sum(wg, red);
  qd = block_sum(qd, red);
  if (tid == 0) {
    if (ctl->pending) {
      const double e = ctl->e0 - 2.0 * wg + qd;
      if (trace) trace[ctl->iters - ctl->base] = e;
      ctl->iters += 1;
      ctl->pending = 0;
      if (tol >= 0.0 && ctl->iters >= 2 && ctl->e_prev - e < tol * ctl->e_prev) ctl->done = 1;
      ctl->e_prev = e;
    }
    s_done = ctl->done;
  }
  __syncthreads();
  if (s_done || finalize_only) return;
  double* VtV = small + SM_VTV * RR;
  double* Bm = small + SM_BM * RR;
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0, t = 0.0;
    for (int jj = 0; jj < J; ++jj) {
      s += V[(size_t)jj * R + a] * V[(size_t)jj * R + b];
      t += D[(size_t)jj * R + a] * V[(size_t)jj * R + b];
    }
    VtV[e] = s;
    Bm[e] = E[a] * t;
  }
}

// H = G1 (W^T W * V^T V)^dagger with unit columns; H^T H.
__global__ __launch_bounds__(256) void k_als_H(int nblkA, int R, const double* __restrict__ partA,
                                               double* __restrict__ small, double* __restrict__ H,
                                               const Ctl* ctl) {
  if (ctl->done) return;
  constexpr int LD = 33;
  __shared__ double G1[32 * LD], Gm[32 * LD], Gi[32 * LD], U[32 * LD], cs[40], nrm[32];
  const int tid = threadIdx.x, RR = R * R;
  const double* WtW = small + SM_WTW * RR;
  const double* VtV = small + SM_VTV * RR;
  for (int e = tid; e < RR; e += 256) {
    double s = 0.0;
    for (int b = 0; b < nblkA; ++b) s += partA[(size_t)b * RR + e];
    G1[(e / R) * LD + e % R] = s;
    Gm[(e / R) * LD + e % R] = WtW[e] * VtV[e];
  }
  __syncthreads();
  block_spd_pinv(Gm, LD, Gi, U, R, cs);
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += G1[a * LD + i] * Gi[i * LD + b];
    U[a * LD + b] = s;
  }
  __syncthreads();
  if (tid < R) {
    double s = 0.0;
    for (int a = 0; a < R; ++a) s += U[a * LD + tid] * U[a * LD + tid];
    s = sqrt(s);
    nrm[tid] = (s < 1e-300) ? 1.0 : s;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    const double h = U[a * LD + b] / nrm[b];
    H[e] = h;
    G1[a * LD + b] = h;
  }
  __syncthreads();
  double* HtH = small + SM_HTH * RR;
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += G1[i * LD + a] * G1[i * LD + b];
    HtH[e] = s;
  }
}

// V = D E N (W^T W * H^T H)^dagger with unit columns; then V^T V, Bm = E D^T V,
// (V^T V * H^T H)^dagger and H^T H * V^T V.
__global__ __launch_bounds__(256) void k_als_V(int nblkB, int J, int R, const double* __restrict__ partB,
                                               const double* __restrict__ D, const double* __restrict__ E,
                                               double* __restrict__ small, double* __restrict__ V, Ctl* ctl) {
  if (ctl->done) return;
  constexpr int LD = 33;
  __shared__ double N[32 * LD], Gm[32 * LD], Gi[32 * LD], U[32 * LD], NE[32 * LD], cs[40], red[16];
  __shared__ double nrm[32];
  const int tid = threadIdx.x, RR = R * R;
  const double* WtW = small + SM_WTW * RR;
  const double* HtH = small + SM_HTH * RR;
  for (int e = tid; e < RR; e += 256) {
    double s = 0.0;
    for (int b = 0; b < nblkB; ++b) s += partB[(size_t)b * RR + e];
    N[(e / R) * LD + e % R] = s;
    Gm[(e / R) * LD + e % R] = WtW[e] * HtH[e];
  }
  __syncthreads();
  block_spd_pinv(Gm, LD, Gi, U, R, cs);
  // NE = diag(E) N Gi  (R x R), so V row j = D(j,:) NE
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += N[a * LD + i] * Gi[i * LD + b];
    NE[a * LD + b] = E[a] * s;
  }
  __syncthreads();
  double cn[32];
  for (int r = 0; r < R; ++r) cn[r] = 0.0;
  for (int jj = tid; jj < J; jj += 256) {
    for (int b = 0; b < R; ++b) {
      double s = 0.0;
      for (int a = 0; a < R; ++a) s += D[(size_t)jj * R + a] * NE[a * LD + b];
      V[(size_t)jj * R + b] = s;
      cn[b] += s * s;
    }
  }
  for (int b = 0; b < R; ++b) {
    const double t = block_sum(cn[b], red);
    if (tid == 0) nrm[b] = (sqrt(t) < 1e-300) ? 1.0 : sqrt(t);
  }
  __syncthreads();
  for (int jj = tid; jj < J; jj += 256)
    for (int b = 0; b < R; ++b) V[(size_t)jj * R + b] /= nrm[b];
  __syncthreads();
  double* VtV = small + SM_VTV * RR;
  double* Bm = small + SM_BM * RR;
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0, t = 0.0;
    for (int jj = 0; jj < J; ++jj) {
      s += V[(size_t)jj * R + a] * V[(size_t)jj * R + b];
      t += D[(size_t)jj * R + a] * V[(size_t)jj * R + b];
    }
    VtV[e] = s;
    Bm[e] = E[a] * t;
    Gm[a * LD + b] = s * HtH[e];
    small[SM_HV * RR + e] = s * HtH[e];
  }
  __syncthreads();
  block_spd_pinv(Gm, LD, Gi, U, R, cs);
  for (int e = tid; e < RR; e += 256) small[SM_G3INV * RR + e] = Gi[(e / R) * LD + e % R];
  if (tid == 0) ctl->pending = 1;
}

// Fitness partials: per slice tr(V S_k H^T Psi_k^T (C_k B_k)^T) and
// W(k,:)(H^T H * V^T V)W(k,:)^T.
__global__ __launch_bounds__(256) void k_fit_part(int K, int J, int R, const double* __restrict__ Mt,
                                                  const double* __restrict__ V, const double* __restrict__ H,
                                                  const double* __restrict__ W, const double* __restrict__ Psi,
                                                  const double* __restrict__ HV, double* __restrict__ fitp) {
  __shared__ double Q[32 * 33], sPsi[32 * 33], sH[32 * 33], red[16];
  const int tid = threadIdx.x, RR = R * R;
  for (int e = tid; e < RR; e += 256) sH[(e / R) * 33 + e % R] = H[e];
  double tr = 0.0, qd = 0.0;
  for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
      const int r = e / R, s = e % R;
      double acc = 0.0;
      for (int jj = 0; jj < J; ++jj) acc += Mt[((size_t)k * R + r) * J + jj] * V[(size_t)jj * R + s];
      Q[r * 33 + s] = acc;
      sPsi[r * 33 + s] = Psi[(size_t)k * RR + e];
    }
    __syncthreads();
    if (tid < R) {
      const int r = tid;
      const double wr = W[(size_t)k * R + r];
      double x = 0.0;
      for (int a = 0; a < R; ++a) {
        double y = 0.0;
        for (int b = 0; b < R; ++b) y += sPsi[b * 33 + a] * Q[b * 33 + r];
        x += sH[a * 33 + r] * y;
      }
      tr += wr * x;
      double q = 0.0;
      for (int s = 0; s < R; ++s) q += HV[r * R + s] * W[(size_t)k * R + s];
      qd += wr * q;
    }
  }
  tr = block_sum(tr, red);
  qd = block_sum(qd, red);
  if (tid == 0) {
    fitp[2 * blockIdx.x] = tr;
    fitp[2 * blockIdx.x + 1] = qd;
  }
}

__global__ __launch_bounds__(256) void k_fit_final(int nblk, const double* __restrict__ fitp,
                                                   double* __restrict__ fit, Ctl* ctl) {
  __shared__ double red[16];
  double tr = 0.0, qd = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    tr += fitp[2 * b];
    qd += fitp[2 * b + 1];
  }
  tr = block_sum(tr, red);
  qd = block_sum(qd, red);
  if (threadIdx.x == 0) {
    const double x2 = ctl->xnorm2;
    const double f = 1.0 - (x2 - 2.0 * tr + qd) / x2;
    ctl->fit_true = f;
    if (fit) *fit = f;
  }
}

// Theta_k = Phi_k Psi_k H (L x R) for the U output.
__global__ __launch_bounds__(256) void k_theta(int K, int L, int R, const double* __restrict__ Phi,
                                               const double* __restrict__ Psi, const double* __restrict__ H,
                                               double* __restrict__ theta) {
  __shared__ double sT[32 * 33];
  const int k = blockIdx.x, tid = threadIdx.x, RR = R * R;
  // T = Psi_k H
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += Psi[(size_t)k * RR + a * R + i] * H[i * R + b];
    sT[a * 33 + b] = s;
  }
  __syncthreads();
  for (int e = tid; e < L * R; e += 256) {
    const int l = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += Phi[(size_t)k * L * R + l * R + i] * sT[i * 33 + b];
    theta[(size_t)k * L * R + e] = s;
  }
}

__global__ void k_eye(int64_t K, int R, double* __restrict__ P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int RR = R * R;
  if (e >= K * RR) return;
  const int w = (int)(e % RR);
  P[e] = (w / R == w % R) ? 1.0 : 0.0;
}

__global__ void k_ctl_begin(Ctl* ctl) {
  ctl->base = ctl->iters;
}

// ---------------------------------------------------------------------------
static int rm_of(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : 32); }

#define DPAR2_RM_DISPATCH(RMV, KERNEL, GRID, ...)                                                  \
  do {                                                                                             \
    if (RMV == 8) hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(TPB), 0, s, __VA_ARGS__);               \
    else if (RMV == 16) hipLaunchKernelGGL(KERNEL<16>, GRID, dim3(TPB), 0, s, __VA_ARGS__);        \
    else hipLaunchKernelGGL(KERNEL<32>, GRID, dim3(TPB), 0, s, __VA_ARGS__);                       \
  } while (0)

struct AlsPtrs {
  Ctl* ctl;
  double *F, *D, *E, *Mt, *Psi, *Pw, *Mk, *small, *partA, *partB, *partC, *fitp, *Phi;
};
static AlsPtrs ptrs(const Layout& lay, char* ws) {
  AlsPtrs p;
  p.ctl = reinterpret_cast<Ctl*>(ws + lay.ctl);
  p.F = reinterpret_cast<double*>(ws + lay.F);
  p.D = reinterpret_cast<double*>(ws + lay.D);
  p.E = reinterpret_cast<double*>(ws + lay.E);
  p.Mt = reinterpret_cast<double*>(ws + lay.Mt);
  p.Psi = reinterpret_cast<double*>(ws + lay.Psi);
  p.Pw = reinterpret_cast<double*>(ws + lay.Pw);
  p.Mk = reinterpret_cast<double*>(ws + lay.Mk);
  p.small = reinterpret_cast<double*>(ws + lay.small);
  p.partA = reinterpret_cast<double*>(ws + lay.partA);
  p.partB = reinterpret_cast<double*>(ws + lay.partB);
  p.partC = reinterpret_cast<double*>(ws + lay.partC);
  p.fitp = reinterpret_cast<double*>(ws + lay.fitp);
  p.Phi = reinterpret_cast<double*>(ws + lay.Phi);
  return p;
}

int als_blocks(int64_t K, int R) {
  const int gpb = TPB / rm_of(R);
  int64_t nb = (K + gpb - 1) / gpb;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t launch_pw_identity(const Layout& lay, char* ws, hipStream_t s) {
  AlsPtrs p = ptrs(lay, ws);
  const int64_t n = lay.K * lay.R * lay.R;
  hipLaunchKernelGGL(k_eye, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lay.K, lay.R, p.Pw);
  return hipGetLastError();
}

hipError_t launch_als_begin(const Layout& lay, char* ws, const double* W, hipStream_t s) {
  AlsPtrs p = ptrs(lay, ws);
  const int rm = rm_of(lay.R);
  hipLaunchKernelGGL(k_ctl_begin, dim3(1), dim3(1), 0, s, p.ctl);
  DPAR2_RM_DISPATCH(rm, k_als_C, dim3(lay.nblkC), (int)lay.K, lay.R, 0, p.Mk, const_cast<double*>(W),
                    (const double*)nullptr, (const double*)nullptr, (const double*)nullptr,
                    (const double*)nullptr, p.partC, (const Ctl*)p.ctl);
  return hipGetLastError();
}

hipError_t launch_als_iteration(const Layout& lay, char* ws, double* H, double* V, double* W,
                                double* err_trace, double tol, hipStream_t s) {
  AlsPtrs p = ptrs(lay, ws);
  const int R = lay.R, RR = R * R, J = (int)lay.J;
  const int K = (int)lay.K;
  const int rm = rm_of(R);
  hipLaunchKernelGGL(k_als_prep, dim3(1), dim3(256), 0, s, lay.nblkC, J, R, 0, tol, p.partC, V, p.D, p.E,
                     p.small, err_trace, p.ctl);
  DPAR2_RM_DISPATCH(rm, k_als_A, dim3(lay.nblkA), K, R, p.F, W, H, p.small + SM_BM * RR, p.Pw, p.Psi,
                    p.Mk, p.partA, p.ctl);
  hipLaunchKernelGGL(k_als_H, dim3(1), dim3(256), 0, s, lay.nblkA, R, p.partA, p.small, H, p.ctl);
  DPAR2_RM_DISPATCH(rm, k_als_B, dim3(lay.nblkB), K, R, p.Mk, W, H, p.partB, p.ctl);
  hipLaunchKernelGGL(k_als_V, dim3(1), dim3(256), 0, s, lay.nblkB, J, R, p.partB, p.D, p.E, p.small, V,
                     p.ctl);
  DPAR2_RM_DISPATCH(rm, k_als_C, dim3(lay.nblkC), K, R, 1, p.Mk, W, H, p.small + SM_BM * RR,
                    p.small + SM_G3INV * RR, p.small + SM_HV * RR, p.partC, (const Ctl*)p.ctl);
  return hipGetLastError();
}

hipError_t launch_als_finalize(const Layout& lay, char* ws, double* err_trace, double tol,
                               hipStream_t s) {
  AlsPtrs p = ptrs(lay, ws);
  hipLaunchKernelGGL(k_als_prep, dim3(1), dim3(256), 0, s, lay.nblkC, (int)lay.J, lay.R, 1, tol, p.partC,
                     (const double*)nullptr, p.D, p.E, p.small, err_trace, p.ctl);
  return hipGetLastError();
}

hipError_t launch_fitness(const Layout& lay, char* ws, const double* H, const double* V,
                          const double* W, double* fit, hipStream_t s) {
  AlsPtrs p = ptrs(lay, ws);
  const int R = lay.R, RR = R * R;
  hipLaunchKernelGGL(k_fit_part, dim3(lay.nblkF), dim3(256), 0, s, (int)lay.K, (int)lay.J, R, p.Mt, V, H,
                     W, p.Psi, p.small + SM_HV * RR, p.fitp);
  hipLaunchKernelGGL(k_fit_final, dim3(1), dim3(256), 0, s, lay.nblkF, p.fitp, fit, p.ctl);
  return hipGetLastError();
}

hipError_t launch_theta(const Layout& lay, char* ws, const double* H, double* theta, hipStream_t s) {
  AlsPtrs p = ptrs(lay, ws);
  hipLaunchKernelGGL(k_theta, dim3((unsigned)lay.K), dim3(256), 0, s, (int)lay.K, lay.L, lay.R, p.Phi,
                     p.Psi, H, theta);
  return hipGetLastError();
}

}  // namespace dpar2
