// First-stage slab pass (Sec. III-B, Eq. 4; Alg. 1 applied to every slice).
//
// One pass over the slab computes, for every work item (a row range of one
// slice), the pieces of the randomized SVD that need the slab:
//   Y   = X Omega_1                (sketch step of Alg. 1; FP32 matrix cores)
//   G   = Y^T Y                    (Gram of the sketch; FP64 matrix cores)
//   P   = Y^T X                    (projection; FP64 matrix cores)
//   ss  = ||X||_F^2                (for the fitness of Sec. IV-A)
// With Y = Q Rc (Rc upper, Rc^T Rc = G) the matrix B = Q^T X of Alg. 1's projection step
// is Rc^{-T} P, so the slab is read exactly once.  Y is rounded to FP32 once
// and that same Y enters both G and P, whose products and sums are exact /
// FP64: the orthogonal projection onto span(Y) is then exact up to FP64
// rounding, and the R^{-T} solve does not amplify FP32 rounding.
//
// The same tile code, in its U variant, recomputes bitwise the same Y and
// writes U_k = Y_k Theta_k (Theta_k = Rc^{-1} U~ Z_k P_k^T H, L x R).
#include "internal.h"

namespace dpar2 {

template <int LT, int JT, bool VEC, bool UOUT>
__global__ __launch_bounds__(256) void k_sketch(
    const float* __restrict__ slab, int J, int L, int R, const float* __restrict__ omega1,
    const Item* __restrict__ items, double* __restrict__ partG, double* __restrict__ partP,
    double* __restrict__ partS, const double* __restrict__ theta, double* __restrict__ Uout) {
  constexpr int TM = SKETCH_TM;
  constexpr int JP = JT * 16;
  constexpr int XS = ((JP + 31) / 32) * 32 + 4;   // row stride: 16-byte reads of 8 rows hit 32 banks
  constexpr int LP = LT * 16;
  constexpr int YS = LP + 16;
  constexpr int NTP = LT * JT;                     // projection tiles (16 x 16, FP64)
  constexpr int NG = (LT == 1) ? 1 : 3;            // Gram tiles (upper triangle)
  constexpr int NTT = NTP + NG;
  constexpr int NPW = (NTT + 3) / 4;               // tiles per wave
  constexpr int NV = VEC ? (TM * JP / 4 + 255) / 256 : (TM * JP + 255) / 256;

  __shared__ __align__(16) float sX[TM * XS];
  __shared__ __align__(16) float sOm[LP * XS];
  __shared__ __align__(16) float sY[TM * YS];
  __shared__ double sred[8];
  __shared__ double sTh[UOUT ? 32 * 32 : 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const Item it = items[blockIdx.x];
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);

  for (int e = tid; e < LP * XS; e += 256) {
    const int n = e / XS, j = e % XS;
    sOm[e] = (n < L && j < J) ? omega1[(size_t)j * L + n] : 0.f;
  }
  for (int e = tid; e < TM * XS; e += 256) sX[e] = 0.f;
  if constexpr (UOUT) {
    for (int e = tid; e < L * R; e += 256) sTh[e] = theta[(size_t)it.slice * L * R + e];
  }

  // fixed (row, column) of every register slot of the tile copy
  const int nel = VEC ? (TM * J) / 4 : TM * J;
  int srow[NV], scol[NV];
#pragma unroll
  for (int s = 0; s < NV; ++s) {
    const int v = s * 256 + tid;
    if (v < nel) {
      const int e = VEC ? 4 * v : v;
      srow[s] = e / J;
      scol[s] = e % J;
    } else {
      srow[s] = TM;
      scol[s] = 0;
    }
  }
  typedef typename std::conditional<VEC, float4, float>::type slot_t;
  slot_t buf[NV];
  auto load_tile = [&](int t) {
    const float* base = slab + (size_t)(it.row0 + (int64_t)t * TM) * J;
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      if (srow[s] < nvalid) {
        if constexpr (VEC) buf[s] = *reinterpret_cast<const float4*>(base + (size_t)srow[s] * J + scol[s]);
        else buf[s] = base[(size_t)srow[s] * J + scol[s]];
      } else {
        if constexpr (VEC) buf[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        else buf[s] = 0.f;
      }
    }
  };

  double ss = 0.0;
  v4d pacc[NPW];
#pragma unroll
  for (int q = 0; q < NPW; ++q) pacc[q] = v4d{0.0, 0.0, 0.0, 0.0};

  if (ntiles > 0) load_tile(0);
  for (int t = 0; t < ntiles; ++t) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      if (srow[s] < TM) {
        if constexpr (VEC) {
          *reinterpret_cast<float4*>(&sX[srow[s] * XS + scol[s]]) = buf[s];
          if constexpr (!UOUT) {
            ss += (double)buf[s].x * buf[s].x + (double)buf[s].y * buf[s].y +
                  (double)buf[s].z * buf[s].z + (double)buf[s].w * buf[s].w;
          }
        } else {
          sX[srow[s] * XS + scol[s]] = buf[s];
          if constexpr (!UOUT) ss += (double)buf[s] * buf[s];
        }
      }
    }
    if (t + 1 < ntiles) load_tile(t + 1);
    __syncthreads();

    // Y rows 16w .. 16w+15 of this tile: (16 x J) . (J x LP) on FP32 matrix cores.
    // Each lane reads 4 consecutive columns; instruction m takes column
    // 4 lk + m of every 16-column group, and B reads the same permutation.
    v4f acc[LT];
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) acc[lt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jg = 0; jg < JT; ++jg) {
      const float4 xa = *reinterpret_cast<const float4*>(&sX[(16 * w + lr) * XS + jg * 16 + 4 * lk]);
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) {
        const float4 ob = *reinterpret_cast<const float4*>(&sOm[(lt * 16 + lr) * XS + jg * 16 + 4 * lk]);
        acc[lt] = mfma_f32(xa.x, ob.x, acc[lt]);
        acc[lt] = mfma_f32(xa.y, ob.y, acc[lt]);
        acc[lt] = mfma_f32(xa.z, ob.z, acc[lt]);
        acc[lt] = mfma_f32(xa.w, ob.w, acc[lt]);
      }
    }
#pragma unroll
    for (int lt = 0; lt < LT; ++lt)
#pragma unroll
      for (int v = 0; v < 4; ++v) sY[(16 * w + f32_row(lane, v)) * YS + lt * 16 + lr] = acc[lt][v];
    __syncthreads();

    if constexpr (UOUT) {
      const int64_t rem = nrows - (int64_t)t * TM;
      const int nvalid = rem < TM ? (int)rem : TM;
      for (int e = tid; e < nvalid * R; e += 256) {
        const int row = e / R, r = e % R;
        double u = 0.0;
        for (int l = 0; l < L; ++l) u += (double)sY[row * YS + l] * sTh[l * R + r];
        Uout[(size_t)(it.row0 + (int64_t)t * TM + row) * R + r] = u;
      }
    } else {
      // P += Y^T X and G += Y^T Y over the 64 rows of the tile, FP64.
#pragma unroll 4
      for (int kk = 0; kk < TM / 4; ++kk) {
        const int row = 4 * kk + lk;
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
          const int task = w + 4 * q;
          if (task < NTT) {
            double a, b;
            if (task < NTP) {
              const int lt = task / JT, jt = task % JT;
              a = (double)sY[row * YS + lt * 16 + lr];
              b = (double)sX[row * XS + jt * 16 + lr];
            } else {
              const int g = task - NTP;
              const int ga = (g == 2) ? 1 : 0, gb = (g == 0) ? 0 : 1;
              a = (double)sY[row * YS + ga * 16 + lr];
              b = (double)sY[row * YS + gb * 16 + lr];
            }
            pacc[q] = mfma_f64(a, b, pacc[q]);
          }
        }
      }
    }
  }

  if constexpr (!UOUT) {
    double* Pp = partP + (size_t)blockIdx.x * L * J;
    double* Gp = partG + (size_t)blockIdx.x * L * L;
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
      const int task = w + 4 * q;
      if (task < NTP) {
        const int lt = task / JT, jt = task % JT;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = lt * 16 + f64_row(lane, v), j = jt * 16 + lr;
          if (i < L && j < J) Pp[(size_t)i * J + j] = pacc[q][v];
        }
      } else if (task < NTT) {
        const int g = task - NTP;
        const int ga = (g == 2) ? 1 : 0, gb = (g == 0) ? 0 : 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = ga * 16 + f64_row(lane, v), j = gb * 16 + lr;
          if (i < L && j < L) {
            Gp[i * L + j] = pacc[q][v];
            if (ga != gb) Gp[j * L + i] = pacc[q][v];
          }
        }
      }
    }
    ss = block_sum(ss, sred);
    if (tid == 0) partS[blockIdx.x] = ss;
  }
}

// ---------------------------------------------------------------------------
// Slab pass with exact integer accumulation of the Gram and projection.
//
// Same tiles and the same FP32 sketch as k_sketch (so Y is bit-identical), but
// Y^T Y and Y^T X are formed on the int8 matrix cores: per 64-row tile, every
// column of Y and of X is scaled by a power of two so that its largest entry
// is below 2^22 and written as three balanced base-256 digits
// (q = d0 2^16 + d1 2^8 + d2, |d| <= 128); all nine digit products are
// summed exactly in int32 (one 16x16x64 instruction per digit pair covers the
// whole tile), combined exactly in FP64 and rescaled.  The only rounding is
// the 22-bit fixed-point representation of each column within its tile (at
// most 2^-22 of the column maximum); the tile sums then accumulate in FP64.
// The Gram is therefore the exact Gram of the represented Y, consistent with
// the projection: the whitening that follows amplifies any inconsistency
// between the two by the condition number of Y^T Y, so no digit product may
// be dropped.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4i mfma_i8(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// exponent e with |m| < 2^e (m >= 0); 0 for m == 0
__device__ __forceinline__ int col_exp(float m) {
  int e = 0;
  if (m > 0.f) frexpf(m, &e);
  return e;
}

// round(x 2^(22 - e)) for |x| < 2^e: the scaled value is exact in FP32 and
// |x 2^(22-e)| < 2^22, so adding 1.5 * 2^23 leaves the nearest integer (ties
// to even) in the low mantissa bits.
__device__ __forceinline__ int q22(float x, int e) {
  const float m = ldexpf(x, 22 - e) + 12582912.0f;
  return __float_as_int(m) - 0x4B400000;
}

// byte k of each of w0..w3 packed into one word (w0 in the low byte)
template <int K>
__device__ __forceinline__ uint32_t bytes_k(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
  constexpr uint32_t sel = 0x0c0c0000u | ((4u + K) << 8) | K;
  const uint32_t lo = __builtin_amdgcn_perm(w1, w0, sel);
  const uint32_t hi = __builtin_amdgcn_perm(w3, w2, sel);
  return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// Balanced base-256 digits of four values |q| <= 2^22, q = d0 2^16 + d1 2^8
// + d2 with |d| <= 128, packed as the byte planes p0 (d0), p1, p2.  With
// r = q - d2 (a multiple of 256) and r2 = r - 256 d1 (a multiple of 2^16),
// d2, d1 and d0 are the signed bytes 0, 1 and 2 of q, r and r2.
__device__ __forceinline__ void digits4(const int (&q)[4], uint32_t& p0, uint32_t& p1, uint32_t& p2) {
  uint32_t r[4], r2[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rv = q[v] - __builtin_amdgcn_sbfe(q[v], 0, 8);
    r[v] = (uint32_t)rv;
    r2[v] = (uint32_t)(rv - (__builtin_amdgcn_sbfe(rv, 8, 8) << 8));
  }
  p2 = bytes_k<0>((uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2], (uint32_t)q[3]);
  p1 = bytes_k<1>(r[0], r[1], r[2], r[3]);
  p0 = bytes_k<2>(r2[0], r2[1], r2[2], r2[3]);
}

template <int LT, int JT, bool VEC>
__global__ __launch_bounds__(256) void k_sketch_q(const float* __restrict__ slab, int J, int L,
                                                  const float* __restrict__ omega1,
                                                  const Item* __restrict__ items, double* __restrict__ partG,
                                                  double* __restrict__ partP, double* __restrict__ partS) {
  constexpr int TM = SKETCH_TM;
  constexpr int JP = JT * 16;
  constexpr int XS = ((JP + 31) / 32) * 32 + 4;
  constexpr int LP = LT * 16;
  constexpr int QW = 20;                           // dwords per digit-plane row (64 bytes + pad)
  constexpr int NTP = LT * JT;
  constexpr int NG = (LT == 1) ? 1 : 3;
  constexpr int NTT = NTP + NG;
  constexpr int NPW = (NTT + 3) / 4;
  constexpr int NV = VEC ? (TM * JP / 4 + 255) / 256 : (TM * JP + 255) / 256;

  __shared__ __align__(16) float sX[TM * XS];
  __shared__ __align__(16) float sOm[LP * XS];
  __shared__ __align__(16) uint32_t sXq[3 * JP * QW];
  __shared__ __align__(16) uint32_t sYq[3 * LP * QW];
  __shared__ float sXm[4 * JP];
  __shared__ float sYm[4 * LP];
  __shared__ int sXe[JP], sYe[LP];
  __shared__ double sred[8];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const Item it = items[blockIdx.x];
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);

  for (int e = tid; e < LP * XS; e += 256) {
    const int n = e / XS, j = e % XS;
    sOm[e] = (n < L && j < J) ? omega1[(size_t)j * L + n] : 0.f;
  }
  for (int e = tid; e < TM * XS; e += 256) sX[e] = 0.f;

  const int nel = VEC ? (TM * J) / 4 : TM * J;
  int srow[NV], scol[NV];
#pragma unroll
  for (int s = 0; s < NV; ++s) {
    const int v = s * 256 + tid;
    if (v < nel) {
      const int e = VEC ? 4 * v : v;
      srow[s] = e / J;
      scol[s] = e % J;
    } else {
      srow[s] = TM;
      scol[s] = 0;
    }
  }
  typedef typename std::conditional<VEC, float4, float>::type slot_t;
  slot_t buf[NV];
  auto load_tile = [&](int t) {
    const float* base = slab + (size_t)(it.row0 + (int64_t)t * TM) * J;
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      if (srow[s] < nvalid) {
        if constexpr (VEC) buf[s] = *reinterpret_cast<const float4*>(base + (size_t)srow[s] * J + scol[s]);
        else buf[s] = base[(size_t)srow[s] * J + scol[s]];
      } else {
        if constexpr (VEC) buf[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        else buf[s] = 0.f;
      }
    }
  };

  double ss = 0.0;
  v4d pacc[NPW];
#pragma unroll
  for (int q = 0; q < NPW; ++q) pacc[q] = v4d{0.0, 0.0, 0.0, 0.0};

  if (ntiles > 0) load_tile(0);
  for (int t = 0; t < ntiles; ++t) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      if (srow[s] < TM) {
        if constexpr (VEC) {
          *reinterpret_cast<float4*>(&sX[srow[s] * XS + scol[s]]) = buf[s];
          ss += (double)buf[s].x * buf[s].x + (double)buf[s].y * buf[s].y +
                (double)buf[s].z * buf[s].z + (double)buf[s].w * buf[s].w;
        } else {
          sX[srow[s] * XS + scol[s]] = buf[s];
          ss += (double)buf[s] * buf[s];
        }
      }
    }
    if (t + 1 < ntiles) load_tile(t + 1);
    __syncthreads();

    // Y rows 16w .. 16w+15 (FP32 matrix cores; identical to k_sketch)
    v4f acc[LT];
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) acc[lt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jg = 0; jg < JT; ++jg) {
      const float4 xa = *reinterpret_cast<const float4*>(&sX[(16 * w + lr) * XS + jg * 16 + 4 * lk]);
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) {
        const float4 ob = *reinterpret_cast<const float4*>(&sOm[(lt * 16 + lr) * XS + jg * 16 + 4 * lk]);
        acc[lt] = mfma_f32(xa.x, ob.x, acc[lt]);
        acc[lt] = mfma_f32(xa.y, ob.y, acc[lt]);
        acc[lt] = mfma_f32(xa.z, ob.z, acc[lt]);
        acc[lt] = mfma_f32(xa.w, ob.w, acc[lt]);
      }
    }
    // column maxima: Y per wave (16 rows), X per row quarter (16 rows)
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) {
      float m = fmaxf(fmaxf(fabsf(acc[lt][0]), fabsf(acc[lt][1])), fmaxf(fabsf(acc[lt][2]), fabsf(acc[lt][3])));
      m = fmaxf(m, __shfl_xor(m, 16, 64));
      m = fmaxf(m, __shfl_xor(m, 32, 64));
      if (lk == 0) sYm[w * LP + lt * 16 + lr] = m;
    }
    for (int task = tid; task < JP * 4; task += 256) {
      const int j = task % JP, q = task / JP;
      float m = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) m = fmaxf(m, fabsf(sX[(16 * q + r) * XS + j]));
      sXm[q * JP + j] = m;
    }
    __syncthreads();
    // digits of Y (transposed planes: [digit][column][row byte])
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) {
      const int col = lt * 16 + lr;
      const float m = fmaxf(fmaxf(sYm[col], sYm[LP + col]), fmaxf(sYm[2 * LP + col], sYm[3 * LP + col]));
      const int e = col_exp(m);
      int q[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) q[v] = q22(acc[lt][v], e);
      uint32_t p[3];
      digits4(q, p[0], p[1], p[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) sYq[(a * LP + col) * QW + 4 * w + lk] = p[a];
      if (w == 0 && lk == 0) sYe[col] = e;
    }
    // digits of X
    for (int task = tid; task < JP * 4; task += 256) {
      const int j = task % JP, q = task / JP;
      const float m = fmaxf(fmaxf(sXm[j], sXm[JP + j]), fmaxf(sXm[2 * JP + j], sXm[3 * JP + j]));
      const int e = col_exp(m);
      uint32_t pk[3][4];
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        int qv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) qv[v] = q22(sX[(16 * q + 4 * r4 + v) * XS + j], e);
        digits4(qv, pk[0][r4], pk[1][r4], pk[2][r4]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
        *reinterpret_cast<uint4*>(&sXq[(a * JP + j) * QW + 4 * q]) = make_uint4(pk[a][0], pk[a][1], pk[a][2], pk[a][3]);
      if (q == 0) sXe[j] = e;
    }
    __syncthreads();

    // exact digit products on the int8 matrix cores, one task per 16x16 tile
#pragma unroll
    for (int qi = 0; qi < NPW; ++qi) {
      const int task = w + 4 * qi;
      if (task < NTT) {
        int ca, cb;
        const uint32_t* Bp;
        const int* eb;
        if (task < NTP) {
          ca = (task / JT) * 16;
          cb = (task % JT) * 16;
          Bp = sXq;
          eb = sXe;
        } else {
          const int g = task - NTP;
          ca = (g == 2) ? 16 : 0;
          cb = (g == 0) ? 0 : 16;
          Bp = sYq;
          eb = sYe;
        }
        const int nb = (task < NTP) ? JP : LP;
        v4i A[3], B[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          A[a] = *reinterpret_cast<const v4i*>(&sYq[(a * LP + ca + lr) * QW + 4 * lk]);
          B[a] = *reinterpret_cast<const v4i*>(&Bp[(a * nb + cb + lr) * QW + 4 * lk]);
        }
        const v4i z = v4i{0, 0, 0, 0};
        v4i S0 = mfma_i8(A[0], B[0], z);
        v4i S1 = mfma_i8(A[0], B[1], z);
        S1 = mfma_i8(A[1], B[0], S1);
        v4i S2 = mfma_i8(A[0], B[2], z);
        S2 = mfma_i8(A[1], B[1], S2);
        S2 = mfma_i8(A[2], B[0], S2);
        v4i S3 = mfma_i8(A[1], B[2], z);
        S3 = mfma_i8(A[2], B[1], S3);
        const v4i S4 = mfma_i8(A[2], B[2], z);
        const int ecol = eb[cb + lr];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // |S0| <= 2^18, |S1| <= 2^20, |S3| <= 2^21, |S4| <= 2^20: the two
          // pairs combine exactly in int32, the total exactly in FP64 (< 2^52)
          const int hi = S0[v] * 256 + S1[v], lo = S3[v] * 256 + S4[v];
          const double val = fma((double)hi, 16777216.0, fma((double)S2[v], 65536.0, (double)lo));
          const int erow = sYe[ca + f32_row(lane, v)];
          pacc[qi][v] += ldexp(val, erow + ecol - 44);
        }
      }
    }
  }

  double* Pp = partP + (size_t)blockIdx.x * L * J;
  double* Gp = partG + (size_t)blockIdx.x * L * L;
#pragma unroll
  for (int qi = 0; qi < NPW; ++qi) {
    const int task = w + 4 * qi;
    if (task < NTP) {
      const int lt = task / JT, jt = task % JT;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = lt * 16 + f32_row(lane, v), j = jt * 16 + lr;
        if (i < L && j < J) Pp[(size_t)i * J + j] = pacc[qi][v];
      }
    } else if (task < NTT) {
      const int g = task - NTP;
      const int ga = (g == 2) ? 1 : 0, gb = (g == 0) ? 0 : 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ga * 16 + f32_row(lane, v), j = gb * 16 + lr;
        if (i < L && j < L) {
          Gp[i * L + j] = pacc[qi][v];
          if (ga != gb) Gp[j * L + i] = pacc[qi][v];
        }
      }
    }
  }
  ss = block_sum(ss, sred);
  if (tid == 0) partS[blockIdx.x] = ss;
}

bool sketch_supported(int J, int L) { return J >= 1 && J <= 256 && L >= 1 && L <= 32; }

static int jt_bucket(int J) {
  const int jt = (J + 15) / 16;
  const int b[] = {1, 2, 3, 4, 6, 8, 12, 16};
  for (int x : b)
    if (jt <= x) return x;
  return -1;
}

template <bool UOUT>
static hipError_t dispatch(const float* slab, int J, int L, int R, const float* omega1,
                           const Item* items, int64_t n_items, double* partG, double* partP,
                           double* partS, const double* theta, double* U, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const int lt = L <= 16 ? 1 : 2;
  const int jt = jt_bucket(J);
  const bool vec = (J % 4 == 0) && ((uintptr_t)slab % 16 == 0);
  dim3 grid((unsigned)n_items), block(256);
#define DPAR2_SK(LT_, JT_)                                                                         \
  if (lt == LT_ && jt == JT_) {                                                                    \
    if (vec)                                                                                       \
      hipLaunchKernelGGL((k_sketch<LT_, JT_, true, UOUT>), grid, block, 0, s, slab, J, L, R,     \
                         omega1, items, partG, partP, partS, theta, U);                            \
    else                                                                                           \
      hipLaunchKernelGGL((k_sketch<LT_, JT_, false, UOUT>), grid, block, 0, s, slab, J, L, R,    \
                         omega1, items, partG, partP, partS, theta, U);                            \
    return hipGetLastError();                                                                      \
  }
  DPAR2_SK(1, 1) DPAR2_SK(1, 2) DPAR2_SK(1, 3) DPAR2_SK(1, 4) DPAR2_SK(1, 6) DPAR2_SK(1, 8)
  DPAR2_SK(1, 12) DPAR2_SK(1, 16)
  DPAR2_SK(2, 1) DPAR2_SK(2, 2) DPAR2_SK(2, 3) DPAR2_SK(2, 4) DPAR2_SK(2, 6) DPAR2_SK(2, 8)
  DPAR2_SK(2, 12) DPAR2_SK(2, 16)
#undef DPAR2_SK
  return hipErrorInvalidValue;
}

hipError_t launch_sketch(const float* slab, int J, int L, const float* omega1, const Item* items,
                         int64_t n_items, double* partG, double* partP, double* partS,
                         hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const int lt = L <= 16 ? 1 : 2;
  const int jt = jt_bucket(J);
  const bool vec = (J % 4 == 0) && ((uintptr_t)slab % 16 == 0);
  dim3 grid((unsigned)n_items), block(256);
#define DPAR2_SQ(LT_, JT_)                                                                         \
  if (lt == LT_ && jt == JT_) {                                                                    \
    if (vec)                                                                                       \
      hipLaunchKernelGGL((k_sketch_q<LT_, JT_, true>), grid, block, 0, s, slab, J, L, omega1,     \
                         items, partG, partP, partS);                                              \
    else                                                                                           \
      hipLaunchKernelGGL((k_sketch_q<LT_, JT_, false>), grid, block, 0, s, slab, J, L, omega1,    \
                         items, partG, partP, partS);                                              \
    return hipGetLastError();                                                                      \
  }
  DPAR2_SQ(1, 1) DPAR2_SQ(1, 2) DPAR2_SQ(1, 3) DPAR2_SQ(1, 4) DPAR2_SQ(1, 6) DPAR2_SQ(1, 8)
  DPAR2_SQ(2, 1) DPAR2_SQ(2, 2) DPAR2_SQ(2, 3) DPAR2_SQ(2, 4) DPAR2_SQ(2, 6) DPAR2_SQ(2, 8)
#undef DPAR2_SQ
  return dispatch<false>(slab, J, L, 0, omega1, items, n_items, partG, partP, partS, nullptr,
                         nullptr, s);
}

hipError_t launch_output_U(const float* slab, int J, int L, int R, const float* omega1,
                           const Item* items, int64_t n_items, const double* theta, double* U,
                           hipStream_t s) {
  return dispatch<true>(slab, J, L, R, omega1, items, n_items, nullptr, nullptr, nullptr, theta,
                        U, s);
}

}  // namespace dpar2
