// First-stage slab pass (Sec. III-B, Eq. 4; Alg. 1 applied to every slice):
// the FP64-matrix-core variant for float32 slabs with 128 < J <= 256, and the
// dispatcher over all variants (the int8-exact kernel of sketch_impl.h serves
// J <= 128).
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
#include "sketch_impl.h"

namespace dpar2 {

template <int LT, int JT, bool VEC, bool UOUT>
__global__ __launch_bounds__(256) void k_sketch(SlabArgs a) {
  const int J = a.J, L = a.L, R = a.R;
  const Item* __restrict__ items = a.items;
  double* __restrict__ partG = a.partG;
  double* __restrict__ partP = a.partP;
  double* __restrict__ partS = a.partS;
  const double* __restrict__ theta = a.theta;
  double* __restrict__ Uout = a.U;
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
  if (a.skip && *a.skip) return;
  const Item it = items[blockIdx.x];
  const float* __restrict__ slab = static_cast<const float*>(a.td[it.pad].slab);
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);
  const float* __restrict__ omega1 = a.omega ? a.omega + (size_t)it.slice * J * L : a.td[it.pad].om1;

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

bool sketch_supported(int J, int L, int dtype) {
  (void)dtype;
  return width_supported(L) && J >= 1 && J <= MAX_J;
}

static int jt_bucket(int J) {
  const int jt = (J + 15) / 16;
  const int b[] = {1, 2, 3, 4, 6, 8, 12, 16};
  for (int x : b)
    if (jt <= x) return x;
  return -1;
}

// FP32 slabs with 128 < J <= 256: FP64 matrix-core Gram and projection
template <bool UOUT>
static hipError_t dispatch_wide(const SlabArgs& a, int64_t n_items, bool vec, hipStream_t s) {
  const int lt = a.L <= 16 ? 1 : 2;
  const int jt = jt_bucket(a.J);
  dim3 grid((unsigned)n_items), block(256);
#define DPAR2_SK(LT_, JT_)                                                                         \
  if (lt == LT_ && jt == JT_) {                                                                    \
    if (vec)                                                                                       \
      hipLaunchKernelGGL((k_sketch<LT_, JT_, true, UOUT>), grid, block, 0, s, a);                  \
    else                                                                                           \
      hipLaunchKernelGGL((k_sketch<LT_, JT_, false, UOUT>), grid, block, 0, s, a);                 \
    return hipGetLastError();                                                                      \
  }
  DPAR2_SK(1, 12) DPAR2_SK(1, 16) DPAR2_SK(2, 12) DPAR2_SK(2, 16)
#undef DPAR2_SK
  return hipErrorInvalidValue;
}

hipError_t slab_launch_f32(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s);
hipError_t slab_launch_bf16(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s);
hipError_t slab_launch_fp8(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s);

hipError_t launch_slab(const SlabArgs& a, int dtype, int64_t n_items, bool vec, bool uout, bool wide,
                       hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (wide || a.J > narrow_j_limit(dtype) || a.L > 32) return launch_slab_wide(a, dtype, n_items, vec, uout, s);
  if (a.J > 128) return uout ? dispatch_wide<true>(a, n_items, vec, s) : dispatch_wide<false>(a, n_items, vec, s);
  if (dtype == DPAR2_F32) return slab_launch_f32(a, n_items, vec, uout, s);
  if (dtype == DPAR2_BF16) return slab_launch_bf16(a, n_items, vec, uout, s);
  return slab_launch_fp8(a, n_items, vec, uout, s);
}

}  // namespace dpar2
