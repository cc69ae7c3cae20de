// Compressed PARAFAC2-ALS iteration (Alg. 3 repeat loop, Secs. III-C..III-E),
// templated on the rank R so that every R x R loop is unrolled and the
// column exchanges of the Jacobi rounds are issued back to back.
//
// One iteration = six launches:
//   A     per slice: T_k = F^(k) Bm S_k H^T with Bm = E D^T V (Eq. 8);
//         one-sided Jacobi SVD T_k = Z_k Sigma_k P_k^T (FP64, warm-started
//         from the previous P_k); Psi_k = Z_k P_k^T; M_k = P_k Z_k^T F^(k) =
//         Psi_k^T F^(k) (the factor of Y_k, Sec. III-D); block partial of
//         G1 = sum_k M_k Bm S_k (Lemma 1)
//   Aepi  H = G1 (W^T W * V^T V)^dagger, unit columns; H^T H
//   B     block partial of N = sum_k M_k^T H S_k (Lemma 2: G2 = D E N)
//   Bepi  V = D E N (W^T W * H^T H)^dagger with unit columns, kept as
//         V = D VC (VC is R x R; V^T V = VC^T D^T D VC, D^T V = D^T D VC):
//         the loop never touches a J-long array; Bm = E D^T V;
//         (V^T V * H^T H)^dagger
//   C     G3(k,r) = H(:,r)^T M_k Bm(:,r) (Lemma 3); W(k,:) = G3(k,:)
//         (V^T V * H^T H)^dagger, S_k = diag(W(k,:)); block partials of
//         W^T W and of e = e0 - 2 sum W.G3 + sum_k W(k,:)(H^T H*V^T V)W(k,:)^T
//   Cepi  W^T W, e_t of Sec. III-E, stop rule
// Every kernel returns at once after the stop rule fired.  Per-slice work
// gives each slice a group of RM lanes, lane j owning column j of the R x R
// matrices (rows in registers).  Epilogues sum the block partials in a fixed
// order (bitwise reproducible).
#pragma once

#include "wave_linalg.h"

namespace dpar2 {

constexpr int EPI_THREADS = 256;

struct AlsArgs {
  int nt, J;
  int64_t K1;                      // slices of the tensor when nt == 1
  const TDesc* td;                 // per tensor: K, first slice, factors, trace, tol
  const Blk* blk;                  // iteration kernels: block -> (tensor, global slices)
  const Blk* blk0;                 // begin kernel: block -> (tensor, local rows)
  const double *F, *D, *E;         // F: global rows; D: nt x J x R; E: nt x R
  double *Pw, *Psi, *Mk;           // global slice index
  double* small;                   // nt x SM_COUNT x R R
  double *partA, *partB, *partC, *partBegin;   // one partial per block
  double* red;                     // nt x (6 R R + 2): partial sums per tensor
  Ctl* ctl;                        // nt
  const double* Mt;                // fitness: M^T (K R x J), rows C_k B_k
  double* fitp;                    // fitness: 2 partials per slice
};

// per-slice kernels: the block's tensor, its control block and small state.
// A single tensor's block table is GPB consecutive slices per block, so the
// block's range follows from its index without a table read first.
#define ALS_BLOCK_PROLOGUE(R_)                                         \
  Blk bk;                                                              \
  if (a.nt == 1) {                                                     \
    const int64_t s0_ = (int64_t)blockIdx.x * RC<R_>::GPB;             \
    const int64_t s1_ = s0_ + RC<R_>::GPB;                             \
    bk = Blk{0, (int32_t)s0_, (int32_t)(s1_ < a.K1 ? s1_ : a.K1), 0};  \
  } else {                                                             \
    bk = a.blk[blockIdx.x];                                            \
  }                                                                    \
  const int tt = bk.t;                                                 \
  const TDesc& td = a.td[tt];                                          \
  Ctl* ctl = a.ctl + tt;                                               \
  double* small = a.small + (size_t)tt * SM_COUNT * (R_) * (R_);
// (each kernel tests ctl->done itself, after issuing its first loads)
// epilogues: one block per tensor.  The inputs are read into registers
// (epi_fetch) before the stop flag is tested, so that both reads overlap.
#define ALS_EPI_PROLOGUE(R_)                                           \
  const int tt = blockIdx.x;                                           \
  const TDesc& td = a.td[tt];                                          \
  Ctl* ctl = a.ctl + tt;                                               \
  double* small = a.small + (size_t)tt * SM_COUNT * (R_) * (R_);       \
  double* red = a.red + (size_t)tt * (RED_WIDTH * (R_) * (R_) + 2);

// v[u] = src[threadIdx.x + u * EPI_THREADS] for the indices below n
template <int NU>
__device__ __forceinline__ void epi_fetch(const double* __restrict__ src, int n, double (&v)[NU]) {
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = threadIdx.x + u * EPI_THREADS;
    v[u] = (e < n) ? src[e] : 0.0;
  }
}

template <int R>
struct RC {
  static constexpr int N = R + (R & 1);                           // Jacobi players
  static constexpr int RM = pow2ceil(N) < 2 ? 2 : pow2ceil(N);    // lanes per slice
  // per-slice block (one slice per 64-lane block above R = 32: the per-slice
  // R x R matrices in LDS then take up to 100 KB)
  static constexpr int TPB = (R > 32) ? 64 : (R > 16) ? 128 : 256;
  static constexpr int GPB = TPB / RM;                            // slices per block
  static constexpr int RR = R * R;
  // R x R matrices of the epilogues in LDS: leading dimension and rows
  static constexpr int LD = (R > 32) ? R + 1 : 33;
  static constexpr int MR = (R > 32) ? R : 32;
};

// One-sided Jacobi (Hestenes) on the R columns held by a group of RM lanes:
// lane j holds column j of T in t[] and of the accumulated right rotation in
// v[].  Round-robin pairing; both lanes of a pair compute the same rotation
// from the same sums.  All lanes of the wave must call it.  Returns sweeps.
template <int R, bool WITHV = true>
__device__ inline int group_jacobi(double (&t)[R], double (&v)[R], int j, int gbase) {
  constexpr int N = RC<R>::N;
  int sweep;
  for (sweep = 0; sweep < JACOBI_SWEEPS; ++sweep) {
    int rotated = 0;
    int big = 0;   // some rotation had |a.b| / (|a| |b|) above 1e-7
    for (int r = 0; r < N - 1; ++r) {
      const int pc = (j < N) ? rr_partner(j, r, N) : j;
      const int src = gbase + pc;
      if constexpr (4 * R > 192) {
        // (t and the partner's whole column would take more than 192 of the
        // 256 vector registers) the partner's column in two halves, fetched
        // once for the sums and again for the rotation (both halves are
        // fetched before this lane changes them); the same sums in the same
        // order as below
        constexpr int HF = (R + 1) / 2;
        double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          double tp[HF];
#pragma unroll
          for (int i = 0; i < HF; ++i)
            if (hf * HF + i < R) tp[i] = __shfl(t[hf * HF + i], src, 64);
#pragma unroll
          for (int i = 0; i < HF; ++i)
            if (hf * HF + i < R) {
              aa = fma(t[hf * HF + i], t[hf * HF + i], aa);
              bb = fma(tp[i], tp[i], bb);
              ab = fma(t[hf * HF + i], tp[i], ab);
            }
        }
        const bool low = j < pc;
        const double alpha = low ? aa : bb, beta = low ? bb : aa;
        const double ab2 = ab * ab, ref = alpha * beta;
        const bool rot = j < N && pc != j && ab != 0.0 && ab2 > (JACOBI_TOL * JACOBI_TOL) * ref;
        double c = 1.0, sn = 0.0;
        if (rot) {
          big |= (ab2 > 1e-14 * ref) ? 1 : 0;
          jacobi_cs(alpha, beta, ab, &c, &sn);
          rotated = 1;
        }
        const double sa = low ? -sn : sn;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          double tp[HF];
#pragma unroll
          for (int i = 0; i < HF; ++i)
            if (hf * HF + i < R) tp[i] = __shfl(t[hf * HF + i], src, 64);
          if (rot) {
#pragma unroll
            for (int i = 0; i < HF; ++i)
              if (hf * HF + i < R) t[hf * HF + i] = fma(c, t[hf * HF + i], sa * tp[i]);
          }
        }
        if constexpr (WITHV) {
#pragma unroll
          for (int hf = 0; hf < 2; ++hf) {
            double vp[HF];
#pragma unroll
            for (int i = 0; i < HF; ++i)
              if (hf * HF + i < R) vp[i] = __shfl(v[hf * HF + i], src, 64);
            if (rot) {
#pragma unroll
              for (int i = 0; i < HF; ++i)
                if (hf * HF + i < R) v[hf * HF + i] = fma(c, v[hf * HF + i], sa * vp[i]);
            }
          }
        }
        continue;
      }
      double tp[R], vp[R];
#pragma unroll
      for (int i = 0; i < R; ++i) tp[i] = __shfl(t[i], src, 64);
      if constexpr (WITHV) {
#pragma unroll
        for (int i = 0; i < R; ++i) vp[i] = __shfl(v[i], src, 64);
      }
      double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        aa = fma(t[i], t[i], aa);
        bb = fma(tp[i], tp[i], bb);
        ab = fma(t[i], tp[i], ab);
      }
      const bool low = j < pc;
      const double alpha = low ? aa : bb, beta = low ? bb : aa;
      const double ab2 = ab * ab, ref = alpha * beta;
      if (j < N && pc != j && ab != 0.0 && ab2 > (JACOBI_TOL * JACOBI_TOL) * ref) {
        big |= (ab2 > 1e-14 * ref) ? 1 : 0;
        double c, s;
        jacobi_cs(alpha, beta, ab, &c, &s);
        rotated = 1;
        const double sa = low ? -s : s;   // low: c a - s b ; high: s a + c b = c b + s a
#pragma unroll
        for (int i = 0; i < R; ++i) t[i] = fma(c, t[i], sa * tp[i]);
        if constexpr (WITHV) {
#pragma unroll
          for (int i = 0; i < R; ++i) v[i] = fma(c, v[i], sa * vp[i]);
        }
      }
    }
    if (!__any(rotated)) break;
    if (!__any(big)) {   // largest |a.b| / (|a| |b|) below 1e-7: quadratic
      ++sweep;                     // convergence leaves nothing for another sweep
      break;
    }
  }
  return sweep;
}

// Inverse of a symmetric positive definite R x R matrix G (LDS, leading
// dimension RC<R>::LD) by Gauss-Jordan elimination without pivoting on
// [G | I], one lane per column (2R <= 64 lanes of wave 0; above R = 32 lane c
// holds both column c of G and column c of I).  Returns false (wave-uniform)
// when a pivot falls below 1e-13 max_i G_ii, i.e. when G is singular to
// working accuracy; the caller then takes the eigen-based pseudoinverse.
template <int R>
__device__ inline bool wave_spd_inverse(const double* G, double* Ginv) {
  constexpr int LD = RC<R>::LD;
  const int c = threadIdx.x;   // lane of wave 0
  double dmax = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) dmax = fmax(dmax, G[i * LD + i]);
  bool ok = dmax > 0.0;
  if constexpr (2 * R <= 64) {
    double col[R];
#pragma unroll
    for (int i = 0; i < R; ++i)
      col[i] = (c < R) ? G[i * LD + c] : ((c - R == i) ? 1.0 : 0.0);
#pragma unroll
    for (int p = 0; p < R; ++p) {
      double colp[R];
#pragma unroll
      for (int i = 0; i < R; ++i) colp[i] = __shfl(col[i], p, 64);
      const double piv = colp[p];
      ok = ok && (piv > 1e-13 * dmax);
      // a pivot that fails the test leaves garbage, discarded with ok = false
      const double f = col[p] * nr_rcp(piv);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (i != p) col[i] = fma(-colp[i], f, col[i]);
      col[p] = f;
    }
    if (c >= R && c < 2 * R)
#pragma unroll
      for (int i = 0; i < R; ++i) Ginv[i * LD + (c - R)] = col[i];
  } else {
    double col[R], idc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      col[i] = (c < R) ? G[i * LD + c] : 0.0;
      idc[i] = (c == i) ? 1.0 : 0.0;
    }
    for (int p = 0; p < R; ++p) {
      double colp[R];
#pragma unroll
      for (int i = 0; i < R; ++i) colp[i] = __shfl(col[i], p, 64);
      double piv = 0.0, cp = 0.0, ip = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (i == p) {
          piv = colp[i];
          cp = col[i];
          ip = idc[i];
        }
      ok = ok && (piv > 1e-13 * dmax);
      const double rp = nr_rcp(piv);
      const double f = cp * rp, g = ip * rp;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        col[i] = (i == p) ? f : fma(-colp[i], f, col[i]);
        idc[i] = (i == p) ? g : fma(-colp[i], g, idc[i]);
      }
    }
    if (c < R)
#pragma unroll
      for (int i = 0; i < R; ++i) Ginv[i * LD + c] = idc[i];
  }
  return ok;
}

// Moore-Penrose pseudoinverse of a symmetric positive semidefinite R x R
// matrix G (LDS, ld RC<R>::LD): one-sided Jacobi G P = T (columns t_j =
// lambda_j p_j), G^dagger = sum_j p_j t_j^T / lambda_j^2 over lambda_j > R eps
// lambda_max.  Wave 0 runs the Jacobi; sT, sV: LDS RC<R>::MR x RC<R>::LD; sg:
// RC<R>::MR doubles.
template <int R>
__device__ inline int jacobi_pinv(const double* G, double* Ginv, double* sT, double* sV, double* sg) {
  constexpr int RM = RC<R>::RM, LD = RC<R>::LD;
  int capped = 0;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, j = lane % RM, gbase = lane & ~(RM - 1);
    double t[R], v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      t[i] = (j < R) ? G[i * LD + j] : 0.0;
      v[i] = (i == j) ? 1.0 : 0.0;
    }
    capped = group_jacobi<R>(t, v, j, gbase) == JACOBI_SWEEPS;
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) s2 = fma(t[i], t[i], s2);
    if (lane < RM && j < R) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        sT[i * LD + j] = t[i];
        sV[i * LD + j] = v[i];
      }
      sg[j] = sqrt(s2);
    }
  }
  __syncthreads();
  double smax = 0.0;
  for (int i = 0; i < R; ++i) smax = fmax(smax, sg[i]);
  const double cut = (double)R * EPS64 * smax;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) {
      const double l = sg[i];
      if (l > cut) s += sV[a * LD + i] * sT[b * LD + i] / (l * l);
    }
    Ginv[a * LD + b] = s;
  }
  __syncthreads();
  return capped;
}

// Pseudoinverse of an SPD/PSD R x R LDS matrix: Gauss-Jordan when G is
// nonsingular to working accuracy (then G^dagger = G^{-1}), else Jacobi.
// Block-cooperative; returns 1 if a Jacobi fallback hit its sweep cap.
template <int R>
__device__ inline int block_pinv(const double* G, double* Ginv, double* sT, double* sV, double* sg,
                                 int* sflag) {
  if (threadIdx.x < 64) {
    const bool ok = wave_spd_inverse<R>(G, Ginv);
    if (threadIdx.x == 0) *sflag = ok ? 1 : 0;
  }
  __syncthreads();
  if (*sflag) return 0;
  return jacobi_pinv<R>(G, Ginv, sT, sV, sg);
}

// out[e] = sum_b part[b * stride + e] for e < width, summed in a fixed order
// by teams of T lanes (T a power of two, team inside one wave, as large as
// the block allows), eight independent loads in flight per lane.
__device__ inline void team_sum(const double* __restrict__ part, int nb, int stride, int width, double* out) {
  int T = 1;
  while (T < 64 && 2 * T * width <= (int)blockDim.x) T *= 2;
  const int team = threadIdx.x / T, sub = threadIdx.x % T;
  const int nteam = blockDim.x / T;
  for (int e = team; e < width; e += nteam) {
    double s[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] = 0.0;
    int b = sub;
    for (; b + 7 * T < nb; b += 8 * T) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += part[(size_t)(b + u * T) * stride + e];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u)
      if (b + u * T < nb) s[u] += part[(size_t)(b + u * T) * stride + e];
    double x = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    for (int o = T / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (sub == 0) out[e] = x;
  }
  __syncthreads();
}

// Group-column accumulators acc[] (lane j: column j) summed over the groups
// of the block into an R x R partial at `out` (global).
template <int R>
__device__ inline void block_partial_out(const double (&acc)[R], double* sred, double* out) {
  constexpr int RM = RC<R>::RM, GPB = RC<R>::GPB, TPB = RC<R>::TPB;
  const int g = threadIdx.x / RM, j = threadIdx.x % RM;
  __syncthreads();
  if (j < R)
#pragma unroll
    for (int a = 0; a < R; ++a) sred[g * R * R + a * R + j] = acc[a];
  __syncthreads();
  for (int e = threadIdx.x; e < R * R; e += TPB) {
    double s = 0.0;
    for (int gg = 0; gg < GPB; ++gg) s += sred[gg * R * R + e];
    out[e] = s;
  }
}

// Q-step of a wave with a (nearly) rank-deficient T_k (see k_als_A): t, v on
// entry hold column j of T_k P_prev and of P_prev.  On return t = z_j (unit
// columns, orthonormal within each slice's group) and v = p_j (orthonormal),
// T_k = Z Sigma P^T with the singular values below 1e-12 sigma_1 taken as 0
// and their z_j completed by Gram-Schmidt: each such column in turn (lowest
// index first) takes the unit vector e_i whose projection onto the columns
// kept so far is smallest (lowest i on ties) minus that projection,
// normalised.  Every lane of the wave calls it (shuffles only, no barrier).
template <int R>
__device__ inline void q_step_complete(const double* T_, bool live, int j, int gbase, double (&t)[R],
                                       double (&v)[R], unsigned& warn) {
  constexpr int RM = RC<R>::RM;
#pragma unroll
  for (int q = 0; q < R; ++q) t[q] = 0.0;
  if (live)
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int q = 0; q < R; ++q) t[q] = fma(T_[q * R + i], v[i], t[q]);
  if (group_jacobi<R, true>(t, v, j, gbase) == JACOBI_SWEEPS) warn |= 0x1u;
  double sig = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) sig = fma(t[i], t[i], sig);
  sig = sqrt(sig);
  double smax = sig;
  for (int o = 1; o < RM; o <<= 1) smax = fmax(smax, __shfl_xor(smax, o, 64));
  bool keep = live && sig > 1e-12 * smax;
  if (live && !keep) warn |= 0x2u;
  const double inv = keep ? 1.0 / sig : 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) t[i] *= inv;   // kept columns unit, the others zero
  // complete the zero columns one by one (the same steps on every group of
  // the wave; a group without such a column changes nothing)
  for (int d = 0; d < R; ++d) {
    const bool isdef = __shfl((int)(live && !keep), gbase + d, 64) != 0;
    // squared norms of the rows of the current Z (sum over the group's lanes)
    double rn[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double x = (j < R) ? t[i] * t[i] : 0.0;
      for (int o = 1; o < RM; o <<= 1) x += __shfl_xor(x, o, 64);
      rn[i] = x;
    }
    int is = 0;
#pragma unroll
    for (int i = 1; i < R; ++i)
      if (rn[i] < rn[is]) is = i;
    // w = e_is - Z Z^T e_is (the group's columns), then normalised
    double zi = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (i == is) zi = t[i];
    double w[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double x = (j < R) ? zi * t[i] : 0.0;
      for (int o = 1; o < RM; o <<= 1) x += __shfl_xor(x, o, 64);
      w[i] = ((i == is) ? 1.0 : 0.0) - x;
    }
    double wn = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) wn = fma(w[i], w[i], wn);
    const double wi = (wn > 0.0) ? 1.0 / sqrt(wn) : 0.0;
    if (isdef && j == d) {
#pragma unroll
      for (int i = 0; i < R; ++i) t[i] = w[i] * wi;
      keep = true;
    }
  }
}

// ---------------------------------------------------------------------------
// A: Q-step (Eq. 8), implicit Y_k, Lemma 1 partial
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(RC<R>::TPB) void k_als_A(AlsArgs a) {
  ALS_BLOCK_PROLOGUE(R)
  constexpr int RM = RC<R>::RM, GPB = RC<R>::GPB, TPB = RC<R>::TPB, RR = R * R;
  // above R = 32 (one slice per 64-lane block) H, Bm and F^(k) are read from
  // global memory where they are used and Z_k takes the place of T_k once
  // T_k has been read for the last time (one wave: its LDS accesses stay in
  // order), so that four blocks share a compute unit's LDS
  constexpr bool GO = R > 32;
  __shared__ double sH[GO ? 1 : RR], sB[GO ? 1 : RR];
  __shared__ double sF[GO ? 1 : GPB * RR], sZ[GO ? 1 : GPB * RR], sP[GPB * RR], sT[GPB * RR], sW[GPB * R];
  const int64_t K = bk.s1;   // slices bk.s0 .. bk.s1 - 1 (at most GPB)
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  const int lane = tid & 63, gbase = lane & ~(RM - 1);
  const double* Bm = small + SM_BM * RR;
  const double* Hs = GO ? td.H : sH;
  const double* Bs = GO ? Bm : sB;
  double* Fl = sF + g * RR;
  const double* F_ = GO ? a.F + (size_t)bk.s0 * RR : Fl;
  double* Z_ = (GO ? sT : sZ) + g * RR;
  double* P_ = sP + g * RR;
  double* T_ = sT + g * RR;
  double acc[R];
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = 0.0;
  unsigned warn = 0;
  {
    const int64_t base = bk.s0;
    const int64_t k = base + g;
    const bool live = (k < K) && (j < R);
    // every global read of the slice set-up is issued before the stop flag
    // is tested (one round of loads)
    constexpr int NS = GO ? 1 : (RR + TPB - 1) / TPB;
    double hv[NS], bv[NS];
    if constexpr (!GO) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int e = tid + TPB * u;
        hv[u] = (e < RR) ? td.H[e] : 0.0;
        bv[u] = (e < RR) ? Bm[e] : 0.0;
      }
    }
    constexpr int NF = (RR + RM - 1) / RM;   // loads issued together (clamped index)
    // F^(k) and the previous P_k (row-major, as flat arrays) and W(k, j):
    // through LDS, so that no R-long array is held across the set-up
    double fv[NF], pv[NF];
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int e = j + RM * u;
      const bool ok = k < K && e < RR;
      const double y = a.Pw[ok ? (size_t)k * RR + e : 0];
      pv[u] = ok ? y : 0.0;
      if constexpr (!GO) {
        const double x = a.F[ok ? (size_t)k * RR + e : 0];
        fv[u] = ok ? x : 0.0;
      }
    }
    const double wkj = live ? td.W[(size_t)(k - td.k0) * R + j] : 0.0;
    if (ctl->done) return;
    if constexpr (!GO) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int e = tid + TPB * u;
        if (e < RR) {
          sH[e] = hv[u];
          sB[e] = bv[u];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NF; ++u)
      if (j + RM * u < RR) {
        if constexpr (!GO) Fl[j + RM * u] = fv[u];
        P_[j + RM * u] = pv[u];
      }
    if (live) sW[g * R + j] = wkj;
    __syncthreads();
    // column j of T_k = F^(k) Bm diag(W(k,:)) H^T (Eq. 8)
    // (the small products below run their R sums side by side, each over
    // its index in ascending order)
    {
      double x[R];
#pragma unroll
      for (int i = 0; i < R; ++i) x[i] = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const double y = sW[g * R + i] * Hs[(live ? j : 0) * R + i];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = fma(Bs[q * R + i], y, x[q]);
      }
      if (live) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          double tq = 0.0;
#pragma unroll
          for (int i = 0; i < R; ++i) tq = fma(F_[q * R + i], x[i], tq);
          T_[q * R + j] = tq;
        }
      }
    }
    __syncthreads();
    // t = T_k p_j, p_j the warm start (column j of the previous P_k)
    double t[R], v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = live ? P_[i * R + j] : 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) t[q] = 0.0;
    if (live)
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) t[q] = fma(T_[q * R + i], v[i], t[q]);
    // T_k P V' = Z Sigma (one-sided Jacobi without accumulating V'); then
    // z_j = t / sigma_j and the new p_j = T_k^T z_j / sigma_j
    if (group_jacobi<R, false>(t, v, j, gbase) == JACOBI_SWEEPS) warn |= 0x1u;
    double sig = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) sig = fma(t[i], t[i], sig);
    sig = sqrt(sig);
    double smax = sig;
    for (int o = 1; o < RM; o <<= 1) smax = fmax(smax, __shfl_xor(smax, o, 64));
    if (__any(live && !(sig > 1e-12 * smax))) {
      // rare: some T_k of this wave is (nearly) rank deficient, so the polar
      // factor is not unique and z_j = t_j / sigma_j is undefined for a
      // vanishing sigma_j.  Redo the Jacobi accumulating the rotation
      // (P = P_prev V' stays orthogonal) and complete Z to an orthonormal
      // basis (q_step_complete), so that Psi_k = Z_k P_k^T is orthogonal.
      q_step_complete<R>(T_, live, j, gbase, t, v, warn);
    } else if (live) {
      const double inv = 1.0 / sig;
#pragma unroll
      for (int i = 0; i < R; ++i) t[i] *= inv;
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = 0.0;
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = fma(T_[q * R + i], t[q], v[i]);
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] *= inv;
    }
    if (live) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        Z_[i * R + j] = t[i];
        P_[i * R + j] = v[i];
        a.Pw[(size_t)k * RR + i * R + j] = v[i];
      }
    }
    __syncthreads();
    // Psi column j: Psi[q][j] = sum_c Z[q][c] P[j][c]
    double psi[R];
#pragma unroll
    for (int q = 0; q < R; ++q) psi[q] = 0.0;
    if (j < R)
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) psi[q] = fma(Z_[q * R + c], P_[j * R + c], psi[q]);
    __syncthreads();
    if (live) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        P_[q * R + j] = psi[q];
        a.Psi[(size_t)k * RR + q * R + j] = psi[q];
      }
    }
    __syncthreads();
    // M_k column j = Psi^T F^(k)(:, j)
    if (live) {
      double mcol[R];
#pragma unroll
      for (int q = 0; q < R; ++q) mcol[q] = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) mcol[q] = fma(P_[i * R + q], F_[i * R + j], mcol[q]);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        Z_[q * R + j] = mcol[q];
        a.Mk[(size_t)k * RR + q * R + j] = mcol[q];
      }
    }
    __syncthreads();
    // G1 partial, column j: W(k,j) * M_k Bm(:, j)
    if (live) {
      const double wj = wkj;
      double sq[R];
#pragma unroll
      for (int q = 0; q < R; ++q) sq[q] = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) sq[q] = fma(Z_[q * R + i], Bs[i * R + j], sq[q]);
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = fma(wj, sq[q], acc[q]);
    }
  }
  for (int o = 1; o < 64; o <<= 1) warn |= __shfl_xor((int)warn, o, 64);
  if (lane == 0 && warn) atomicOr(&ctl->warn, warn);
  block_partial_out<R>(acc, GO ? sT : sZ, a.partA + (size_t)blockIdx.x * RR);
}

// H = G1 (W^T W * V^T V)^dagger, unit columns; H^T H.
template <int R>
__global__ __launch_bounds__(EPI_THREADS) void k_als_A_epi(AlsArgs a, int nblk) {
  ALS_EPI_PROLOGUE(R)
  constexpr int LD = RC<R>::LD, MR = RC<R>::MR, RR = R * R;
  __shared__ double G1[MR * LD], Gm[MR * LD], Gi[MR * LD], sT[MR * LD], sV[MR * LD], sg[MR];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  (void)nblk;
  // G1 = the summed partials (one row of red), W^T W * V^T V
  constexpr int NU = (RR + EPI_THREADS - 1) / EPI_THREADS;
  double g1[NU], wtw[NU], vtv[NU];
  epi_fetch(red, RR, g1);
  epi_fetch(small + SM_WTW * RR, RR, wtw);
  epi_fetch(small + SM_VTV * RR, RR, vtv);
  if (ctl->done) return;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = tid + u * EPI_THREADS;
    if (e < RR) {
      G1[(e / R) * LD + e % R] = g1[u];
      Gm[(e / R) * LD + e % R] = wtw[u] * vtv[u];
    }
  }
  __syncthreads();
  const int capped = block_pinv<R>(Gm, Gi, sT, sV, sg, &sflag);
  for (int e = tid; e < RR; e += EPI_THREADS) {      // raw H = G1 Gi
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
    const double h = sT[q * LD + c] / sg[c];
    td.H[e] = h;
    G1[q * LD + c] = h;
  }
  __syncthreads();
  double* HtH = small + SM_HTH * RR;
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int q = e / R, c = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(G1[i * LD + q], G1[i * LD + c], s);
    HtH[e] = s;
  }
  if (tid == 0 && capped) atomicOr(&ctl->warn, 0x1u);
}

// ---------------------------------------------------------------------------
// B: Lemma 2 partials
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(RC<R>::TPB) void k_als_B(AlsArgs a) {
  ALS_BLOCK_PROLOGUE(R)
  (void)small;
  constexpr int RM = RC<R>::RM, GPB = RC<R>::GPB, TPB = RC<R>::TPB, RR = R * R;
  __shared__ double sH[RR];
  __shared__ double sM[GPB * RR];
  const int64_t K = bk.s1;
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  double* M_ = sM + g * RR;
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  {
    const int64_t base = bk.s0;
    const int64_t k = base + g;
    // H, M_k and W(k, j) read before the stop flag is tested
    constexpr int NS = (RR + TPB - 1) / TPB, NM = (RR + RM - 1) / RM;
    double hv[NS], mv[NM];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + TPB * u;
      hv[u] = (e < RR) ? td.H[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NM; ++u) {
      const int e = j + RM * u;
      mv[u] = (k < K && e < RR) ? a.Mk[(size_t)k * RR + e] : 0.0;
    }
    const double wj = (k < K && j < R) ? td.W[(size_t)(k - td.k0) * R + j] : 0.0;
    if (ctl->done) return;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + TPB * u;
      if (e < RR) sH[e] = hv[u];
    }
#pragma unroll
    for (int u = 0; u < NM; ++u) {
      const int e = j + RM * u;
      if (k < K && e < RR) M_[e] = mv[u];
    }
    __syncthreads();
    if (k < K && j < R) {
      double sq[R];
#pragma unroll
      for (int q = 0; q < R; ++q) sq[q] = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) sq[q] = fma(M_[i * R + q], sH[i * R + j], sq[q]);
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = fma(wj, sq[q], acc[q]);
    }
  }
  block_partial_out<R>(acc, sM, a.partB + (size_t)blockIdx.x * RR);
}

// V = D E N (W^T W * H^T H)^dagger with unit columns, held as V = D VC;
// V^T V, Bm = E D^T V, H^T H * V^T V, (V^T V * H^T H)^dagger.
template <int R>
__global__ __launch_bounds__(EPI_THREADS) void k_als_B_epi(AlsArgs a, int nblk) {
  ALS_EPI_PROLOGUE(R)
  constexpr int LD = RC<R>::LD, MR = RC<R>::MR, RR = R * R;
  __shared__ double N[MR * LD], Gm[MR * LD], Gi[MR * LD], sT[MR * LD], sV[MR * LD], sg[MR];
  __shared__ double DtD[RR], Et[R];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  (void)nblk;
  // N = the summed partials (second row of red), W^T W * H^T H, D^T D, E
  constexpr int NU = (RR + EPI_THREADS - 1) / EPI_THREADS;
  double nv[NU], wtw[NU], hth[NU], dtd[NU];
  epi_fetch(red + RR, RR, nv);
  epi_fetch(small + SM_WTW * RR, RR, wtw);
  epi_fetch(small + SM_HTH * RR, RR, hth);
  epi_fetch(small + SM_DTD * RR, RR, dtd);
  const double ev = (tid < R) ? a.E[(size_t)tt * R + tid] : 0.0;
  if (ctl->done) return;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = tid + u * EPI_THREADS;
    if (e < RR) {
      N[(e / R) * LD + e % R] = nv[u];
      Gm[(e / R) * LD + e % R] = wtw[u] * hth[u];
      DtD[e] = dtd[u];
    }
  }
  if (tid < R) Et[tid] = ev;
  __syncthreads();
  int capped = block_pinv<R>(Gm, Gi, sT, sV, sg, &sflag);
  // VC = diag(E) N Gi  (V = D VC before normalisation)
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int q = e / R, c = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(N[q * LD + i], Gi[i * LD + c], s);
    Gm[q * LD + c] = Et[q] * s;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += EPI_THREADS) {            // sT <- (D^T D) VC
    const int q = e / R, c = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(DtD[q * R + i], Gm[i * LD + c], s);
    sT[q * LD + c] = s;
  }
  __syncthreads();
  if (tid < R) {                                            // column norms of V
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(Gm[i * LD + tid], sT[i * LD + tid], s);
    s = sqrt(s > 0.0 ? s : 0.0);
    sg[tid] = (s < 1e-300) ? 1.0 : s;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += EPI_THREADS) {
    const int q = e / R, c = e % R;
    Gm[q * LD + c] /= sg[c];
    sT[q * LD + c] /= sg[c];
  }
  __syncthreads();
  double* VtV = small + SM_VTV * RR;
  double* Bm = small + SM_BM * RR;
  double* HV = small + SM_HV * RR;
  double* VC = small + SM_VC * RR;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = tid + u * EPI_THREADS;
    if (e >= RR) continue;
    const int q = e / R, c = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s = fma(Gm[i * LD + q], sT[i * LD + c], s);   // VC^T (D^T D) VC
    VtV[e] = s;
    Bm[e] = Et[q] * sT[q * LD + c];                                           // E D^T V
    HV[e] = s * hth[u];
    VC[e] = Gm[q * LD + c];
    N[q * LD + c] = s * hth[u];
  }
  __syncthreads();
  capped |= block_pinv<R>(N, Gi, sT, sV, sg, &sflag);
  for (int e = tid; e < RR; e += EPI_THREADS) small[SM_G3INV * RR + e] = Gi[(e / R) * LD + e % R];
  if (tid == 0) {
    ctl->vc_valid = 1;
    if (capped) atomicOr(&ctl->warn, 0x1u);
  }
}

// ---------------------------------------------------------------------------
// C: Lemma 3, W rows, error partials
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(RC<R>::TPB) void k_als_C(AlsArgs a) {
  ALS_BLOCK_PROLOGUE(R)
  constexpr int RM = RC<R>::RM, GPB = RC<R>::GPB, TPB = RC<R>::TPB, RR = R * R;
  // above R = 32 (one slice per block) the small state is read from global
  // memory where it is used, so that several blocks share a compute unit's LDS
  constexpr bool GO = R > 32;
  __shared__ double sH[GO ? 1 : RR], sB[GO ? 1 : RR], sGi[GO ? 1 : RR], sHV[GO ? 1 : RR];
  __shared__ double sM[GPB * RR];
  __shared__ double sRed[TPB * 2];
  const int64_t K = bk.s1;
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  const int lane = tid & 63, gbase = lane & ~(RM - 1);
  double* M_ = sM + g * RR;
  double wtw[R];
#pragma unroll
  for (int q = 0; q < R; ++q) wtw[q] = 0.0;
  double ewg = 0.0, equad = 0.0;
  {
    const int64_t base = bk.s0;
    const int64_t k = base + g;
    const bool live = (k < K) && (j < R);
    // the small state and M_k read before the stop flag is tested
    constexpr int NS = GO ? 1 : (RR + TPB - 1) / TPB, NM = (RR + RM - 1) / RM;
    double hv[NS], bv[NS], gv[NS], qv[NS], mv[NM];
    if constexpr (!GO) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int e = tid + TPB * u;
        const bool ok = e < RR;
        hv[u] = ok ? td.H[e] : 0.0;
        bv[u] = ok ? small[SM_BM * RR + e] : 0.0;
        gv[u] = ok ? small[SM_G3INV * RR + e] : 0.0;
        qv[u] = ok ? small[SM_HV * RR + e] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < NM; ++u) {
      const int e = j + RM * u;
      mv[u] = (k < K && e < RR) ? a.Mk[(size_t)k * RR + e] : 0.0;
    }
    if (ctl->done) return;
    if constexpr (!GO) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int e = tid + TPB * u;
        if (e < RR) {
          sH[e] = hv[u];
          sB[e] = bv[u];
          sGi[e] = gv[u];
          sHV[e] = qv[u];
        }
      }
    }
    const double* Hs = GO ? td.H : sH;
    const double* Bs = GO ? small + SM_BM * RR : sB;
    const double* Gis = GO ? small + SM_G3INV * RR : sGi;
    const double* HVs = GO ? small + SM_HV * RR : sHV;
#pragma unroll
    for (int u = 0; u < NM; ++u) {
      const int e = j + RM * u;
      if (k < K && e < RR) M_[e] = mv[u];
    }
    __syncthreads();
    double g3 = 0.0;
    if (live) {
      double sq[R];
#pragma unroll
      for (int q = 0; q < R; ++q) sq[q] = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) sq[q] = fma(M_[q * R + i], Bs[i * R + j], sq[q]);
#pragma unroll
      for (int q = 0; q < R; ++q) g3 = fma(Hs[q * R + j], sq[q], g3);
    }
    double gs[R];
#pragma unroll
    for (int s = 0; s < R; ++s) gs[s] = __shfl(g3, gbase + s, 64);
    double wnew = 0.0;
    if (live) {
#pragma unroll
      for (int s = 0; s < R; ++s) wnew = fma(gs[s], Gis[s * R + j], wnew);
      td.W[(size_t)(k - td.k0) * R + j] = wnew;
      ewg = fma(wnew, g3, ewg);
    }
    double ws[R];
#pragma unroll
    for (int s = 0; s < R; ++s) ws[s] = __shfl(wnew, gbase + s, 64);
    if (live) {
      double q2 = 0.0;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        q2 = fma(HVs[j * R + s], ws[s], q2);
        wtw[s] = fma(ws[s], wnew, wtw[s]);
      }
      equad = fma(wnew, q2, equad);
    }
  }
  __syncthreads();
  if (j < R)
#pragma unroll
    for (int q = 0; q < R; ++q) sM[g * RR + q * R + j] = wtw[q];
  sRed[tid * 2] = ewg;
  sRed[tid * 2 + 1] = equad;
  __syncthreads();
  double* out = a.partC + (size_t)blockIdx.x * (RR + 2);
  for (int e = tid; e < RR; e += TPB) {
    double s = 0.0;
    for (int gg = 0; gg < GPB; ++gg) s += sM[gg * RR + e];
    out[e] = s;
  }
  if (tid < 2) {
    double s = 0.0;
    for (int i = 0; i < TPB; ++i) s += sRed[i * 2 + tid];
    out[RR + tid] = s;
  }
}

// W^T W, e_t = e0 - 2 sum W.G3 + sum W (H^T H * V^T V) W^T, stop rule.
template <int R>
__global__ __launch_bounds__(EPI_THREADS) void k_als_C_epi(AlsArgs a, int nblk) {
  ALS_EPI_PROLOGUE(R)
  constexpr int RR = R * R;
  (void)nblk;
  // third row of red: W^T W and the two error sums
  constexpr int NU = (RR + 2 + EPI_THREADS - 1) / EPI_THREADS;
  double v[NU];
  epi_fetch(red + 2 * RR, RR + 2, v);
  // the stop rule's inputs, read by thread 0 in the same round of loads
  double ewg = 0.0, equad = 0.0, e0 = 0.0, eprev = 0.0, tol = -1.0;
  int32_t it = 0, base = 0;
  double* trace = nullptr;
  if (threadIdx.x == 0) {
    ewg = red[3 * RR];
    equad = red[3 * RR + 1];
    e0 = ctl->e0;
    eprev = ctl->e_prev;
    it = ctl->iters;
    base = ctl->base;
    trace = td.trace;
    tol = td.tol;
  }
  if (ctl->done) return;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = threadIdx.x + u * EPI_THREADS;
    if (e < RR) small[SM_WTW * RR + e] = v[u];
  }
  if (threadIdx.x == 0) {
    const double e = e0 - 2.0 * ewg + equad;
    if (trace) trace[it - base] = e;
    ctl->iters = it + 1;
    if (tol >= 0.0 && it + 1 >= 2 && eprev - e < tol * eprev) ctl->done = 1;
    ctl->e_prev = e;
  }
}

// ---------------------------------------------------------------------------
// Begin of a call: W^T W, V^T V and E D^T V of the factors given
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(RC<R>::TPB) void k_als_begin(AlsArgs a) {
  constexpr int RM = RC<R>::RM, GPB = RC<R>::GPB, RR = R * R;
  __shared__ double sM[GPB * RR];
  const Blk bk = a.blk0[blockIdx.x];   // local rows bk.s0 .. bk.s1 - 1 of tensor bk.t
  const TDesc& td = a.td[bk.t];
  const int64_t K = td.K, J = a.J;
  const double* Dt = a.D + (size_t)bk.t * J * R;
  const int tid = threadIdx.x, g = tid / RM, j = tid % RM;
  const int lane = tid & 63, gbase = lane & ~(RM - 1);
  double acc0[R], acc1[R], acc2[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc0[q] = acc1[q] = acc2[q] = 0.0;
  const int64_t rows = bk.s1;
  {
    const int64_t base = bk.s0;
    const int64_t k = base + g;
    const double w = (k < rows && k < K && j < R) ? td.W[(size_t)k * R + j] : 0.0;
    const double v = (k < rows && k < J && j < R) ? td.V[(size_t)k * R + j] : 0.0;
    const double d = (k < rows && k < J && j < R) ? Dt[(size_t)k * R + j] : 0.0;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const double ws = __shfl(w, gbase + s, 64);
      const double vs = __shfl(v, gbase + s, 64);
      const double ds = __shfl(d, gbase + s, 64);
      acc0[s] = fma(ws, w, acc0[s]);   // (W^T W)[s][j]
      acc1[s] = fma(vs, v, acc1[s]);   // (V^T V)[s][j]
      acc2[s] = fma(ds, v, acc2[s]);   // (D^T V)[s][j]
    }
  }
  double* out = a.partBegin + (size_t)blockIdx.x * 3 * RR;
  block_partial_out<R>(acc0, sM, out);
  block_partial_out<R>(acc1, sM, out + RR);
  block_partial_out<R>(acc2, sM, out + 2 * RR);
}

// reset_base: the start of a call (the trace of the call begins here); 0 when
// the begin step closes an iteration of the resumable mode
template <int R>
__global__ __launch_bounds__(EPI_THREADS) void k_als_begin_epi(AlsArgs a, int reset_base) {
  const int tt = blockIdx.x;
  Ctl* ctl = a.ctl + tt;
  double* small = a.small + (size_t)tt * SM_COUNT * R * R;
  const double* red = a.red + (size_t)tt * (RED_WIDTH * R * R + 2);
  const double* Et = a.E + (size_t)tt * R;
  constexpr int RR = R * R;
  __shared__ double tmp[3 * RR];
  team_sum(red + 3 * RR + 2, 1, 3 * RR, 3 * RR, tmp);
  for (int e = threadIdx.x; e < RR; e += EPI_THREADS) {
    small[SM_WTW * RR + e] = tmp[e];
    small[SM_VTV * RR + e] = tmp[RR + e];
    small[SM_BM * RR + e] = Et[e / R] * tmp[2 * RR + e];
  }
  if (threadIdx.x == 0) {
    if (reset_base) ctl->base = ctl->iters;
    ctl->vc_valid = 0;
  }
}

// ---------------------------------------------------------------------------
// Fitness partials (Sec. IV-A) per slice k: tr(V S_k H^T Psi_k^T (C_k B_k)^T)
// and W(k,:)(H^T H * V^T V)W(k,:)^T.  One lane per row r of C_k B_k (a row of
// M^T, read once): Q(r, :) = sum_j M^T(kR + r, j) V(j, :), j in order, the
// rows of V through scalar loads; then lane (k, r) forms its terms from
// column r of Q_k and the slice sums its R lanes in order.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(RC<R>::TPB) void k_fit_rows(AlsArgs a) {
  ALS_BLOCK_PROLOGUE(R)
  constexpr int GPB = RC<R>::GPB, TPB = RC<R>::TPB, RR = R * R;
  // above R = 32 (one slice per block) H, H^T H * V^T V and Psi_k are read
  // from global memory where they are used, so that several blocks share a
  // compute unit's LDS
  constexpr bool GO = R > 32;
  __shared__ double sQ[GPB * RR], sP[GO ? 1 : GPB * RR], sH[GO ? 1 : RR], sHV[GO ? 1 : RR], sW[GPB * R];
  __shared__ double sT[2 * TPB];
  (void)ctl;
  const int tid = threadIdx.x, g = tid / R, r = tid % R;
  const int J = a.J;
  const int64_t k = bk.s0 + g;
  const bool live = g < GPB && k < bk.s1;
  const double* __restrict__ mrow = a.Mt + (size_t)((live ? k : (int64_t)bk.s0) * R + (live ? r : 0)) * J;
  const double* __restrict__ V = td.V;
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  int j = 0;
  for (; j + 8 <= J; j += 8) {
    double m[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m[u] = mrow[j + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* __restrict__ vr = V + (size_t)(j + u) * R;
#pragma unroll
      for (int c = 0; c < R; ++c) acc[c] = fma(m[u], vr[c], acc[c]);
    }
  }
  for (; j < J; ++j) {
    const double m = mrow[j];
    const double* __restrict__ vr = V + (size_t)j * R;
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = fma(m, vr[c], acc[c]);
  }
  if constexpr (!GO) {
    for (int e = tid; e < RR; e += TPB) {
      sH[e] = td.H[e];
      sHV[e] = small[SM_HV * RR + e];
    }
    for (int e = tid; e < GPB * RR; e += TPB) {
      const int64_t kk = bk.s0 + e / RR;
      sP[e] = kk < bk.s1 ? a.Psi[(size_t)kk * RR + e % RR] : 0.0;
    }
  }
  const double* Hs = GO ? td.H : sH;
  const double* HVs = GO ? small + SM_HV * RR : sHV;
  for (int e = tid; e < GPB * R; e += TPB) {
    const int64_t kk = bk.s0 + e / R;
    sW[e] = kk < bk.s1 ? td.W[(size_t)(kk - td.k0) * R + e % R] : 0.0;
  }
  if (live) {
#pragma unroll
    for (int c = 0; c < R; ++c) sQ[g * RR + r * R + c] = acc[c];
  }
  __syncthreads();
  double tr = 0.0, qd = 0.0;
  if (live) {
    const double* Q = sQ + g * RR;
    const double* P = GO ? a.Psi + (size_t)k * RR : sP + g * RR;
    double x = 0.0;
    for (int aa = 0; aa < R; ++aa) {
      double y = 0.0;
      for (int b = 0; b < R; ++b) y += P[b * R + aa] * Q[b * R + r];
      x += Hs[aa * R + r] * y;
    }
    const double wr = sW[g * R + r];
    tr = wr * x;
    double q = 0.0;
    for (int s2 = 0; s2 < R; ++s2) q += HVs[r * R + s2] * sW[g * R + s2];
    qd = wr * q;
  }
  sT[2 * tid] = tr;
  sT[2 * tid + 1] = qd;
  __syncthreads();
  if (tid < GPB && bk.s0 + tid < bk.s1) {
    double t1 = 0.0, t2 = 0.0;
    for (int rr = 0; rr < R; ++rr) {
      t1 += sT[2 * (tid * R + rr)];
      t2 += sT[2 * (tid * R + rr) + 1];
    }
    a.fitp[2 * (bk.s0 + tid)] = t1;
    a.fitp[2 * (bk.s0 + tid) + 1] = t2;
  }
}

// Launches of one rank's kernels: phase 0 = begin (+epi) of a call, 1 = one
// iteration, 2 = the begin step that closes an iteration in the resumable
// mode (W^T W, V^T V, E D^T V from the factors, as at the start of a call),
// 3 = the fitness partials.
// nb, nb0: blocks of the iteration / begin per-slice kernels; seg, seg0: their
// per-tensor block offsets (device, nt + 1).
template <int R>
hipError_t als_launch(int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg, const int64_t* seg0,
                      hipStream_t s) {
  constexpr int TPB = RC<R>::TPB, RR = R * R;
  constexpr int64_t RW = RED_WIDTH * RR + 2;
  const int nt = a.nt;
  // each per-slice kernel writes one partial per block; the segmented column
  // sum reduces them per tensor (one load per thread) before the epilogues
  hipError_t e;
  if (phase == 3) {
    hipLaunchKernelGGL(k_fit_rows<R>, dim3(nb), dim3(TPB), 0, s, a);
  } else if (phase == 0 || phase == 2) {
    hipLaunchKernelGGL(k_als_begin<R>, dim3(nb0), dim3(TPB), 0, s, a);
    if ((e = launch_segsum(nt, seg0, nb0, 3 * RR, 3 * RR, a.partBegin, a.red + 3 * RR + 2, RW, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_als_begin_epi<R>, dim3(nt), dim3(EPI_THREADS), 0, s, a, phase == 0 ? 1 : 0);
  } else {
    hipLaunchKernelGGL(k_als_A<R>, dim3(nb), dim3(TPB), 0, s, a);
    if ((e = launch_segsum(nt, seg, nb, RR, RR, a.partA, a.red, RW, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_als_A_epi<R>, dim3(nt), dim3(EPI_THREADS), 0, s, a, 1);
    hipLaunchKernelGGL(k_als_B<R>, dim3(nb), dim3(TPB), 0, s, a);
    if ((e = launch_segsum(nt, seg, nb, RR, RR, a.partB, a.red + RR, RW, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_als_B_epi<R>, dim3(nt), dim3(EPI_THREADS), 0, s, a, 1);
    hipLaunchKernelGGL(k_als_C<R>, dim3(nb), dim3(TPB), 0, s, a);
    if ((e = launch_segsum(nt, seg, nb, RR + 2, RR + 2, a.partC, a.red + 2 * RR, RW, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_als_C_epi<R>, dim3(nt), dim3(EPI_THREADS), 0, s, a, 1);
  }
  return hipGetLastError();
}

}  // namespace dpar2
