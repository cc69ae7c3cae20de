// Slab pass for wide slices (J above the narrow kernels' limit; Sec. III-B,
// Eq. 4, Alg. 1 applied to every slice), in two kernels:
//   k_wide_y  per work item: Y = X Omega tile by tile, the row of a tile
//             streamed through LDS in chunks of 128 columns (FP32 matrix cores
//             for float32 slabs, bf16 matrix cores with Omega rounded to bf16
//             otherwise; chunk sums added in FP64, Y rounded to FP32 once),
//             Y written to a row buffer, and ||X||_F^2; or, in the U variant,
//             U = Y Theta_k
//   k_wide_p  per (work item, 128-column chunk): P(:, chunk) = Y^T X(:, chunk)
//             and, for chunk 0, G = Y^T Y, on the FP64 matrix cores: the FP32
//             factors multiply exactly in FP64 and the sums are FP64, so G and
//             P are the Gram and projection of the same FP32 Y up to FP64
//             rounding (the property the whitening of the completion needs)
// The slab is read twice (once per kernel); Y adds 16 LT floats per row.
#include "sketch_impl.h"

namespace dpar2 {

constexpr int WJC = 128;        // columns per chunk
constexpr int WXS = WJC + 4;    // LDS row stride of an X chunk (floats)

template <int LT, bool VEC, int TIN, bool UOUT>
__global__ __launch_bounds__(256) void k_wide_y(SlabArgs a) {
  typedef typename In<TIN>::E E;
  typedef typename In<TIN>::V4 V4;
  const int J = a.J, L = a.L, R = a.R;
  constexpr int TM = SKETCH_TM, LP = LT * 16;
  constexpr int NV = VEC ? TM * WJC / 4 / 256 : TM * WJC / 256;
  constexpr int YS = LP + 1;
  __shared__ __align__(16) float sX[TM * WXS];
  __shared__ __align__(16) float sOm[LP * WXS];
  __shared__ float sYf[UOUT ? TM * YS : 1];
  __shared__ double sTh[UOUT ? 32 * 32 : 1];
  __shared__ double sred[8];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const Item it = a.items[blockIdx.x];
  const TDesc& td = a.td[it.pad];
  const E* __restrict__ slab = static_cast<const E*>(td.slab);
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);
  const int nchunks = (J + WJC - 1) / WJC;
  const float* __restrict__ omega = a.omega ? a.omega + (size_t)it.slice * J * L : td.om1;
  const float scale = (TIN == DPAR2_FP8_E4M3) ? td.scale[it.slice - td.k0] : 1.0f;
  if constexpr (UOUT) {
    for (int e = tid; e < L * R; e += 256) sTh[e] = a.theta[(size_t)it.slice * L * R + e];
  }

  double ss = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
    const E* base = slab + (size_t)(it.row0 + (int64_t)t * TM) * J;
    // each chunk's sum comes from the matrix cores in FP32 and is added in
    // FP64, so the rounding of Y does not grow with the number of chunks
    v4d ysum[LT];
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) ysum[lt] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < nchunks; ++c) {
      const int c0 = c * WJC;
      v4f acc[LT];
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) acc[lt] = v4f{0.f, 0.f, 0.f, 0.f};
      __syncthreads();
      for (int e = tid; e < LP * WXS; e += 256) {
        const int n = e / WXS, j = e % WXS;
        const float o = (n < L && j < WJC && c0 + j < J) ? omega[(size_t)(c0 + j) * L + n] : 0.f;
        sOm[e] = (TIN == DPAR2_F32) ? o : round_bf16(o);
      }
      // the chunk's loads are unrolled with clamped addresses so they issue together
      if constexpr (VEC) {
        V4 buf[NV];
#pragma unroll
        for (int s = 0; s < NV; ++s) {
          const int e = 4 * (s * 256 + tid), row = e / WJC, col = e % WJC;
          const bool ok = row < nvalid && c0 + col < J;
          const V4 x = *reinterpret_cast<const V4*>(base + (ok ? (size_t)row * J + c0 + col : 0));
          buf[s] = ok ? x : V4{};
        }
#pragma unroll
        for (int s = 0; s < NV; ++s) {
          const int e = 4 * (s * 256 + tid), row = e / WJC, col = e % WJC;
          const float4 x = to_f32x4<TIN>(buf[s], scale);
          *reinterpret_cast<float4*>(&sX[row * WXS + col]) = x;
          if constexpr (!UOUT) ss += (double)x.x * x.x + (double)x.y * x.y + (double)x.z * x.z + (double)x.w * x.w;
        }
      } else {
        E buf[NV];
#pragma unroll
        for (int s = 0; s < NV; ++s) {
          const int e = s * 256 + tid, row = e / WJC, col = e % WJC;
          const bool ok = row < nvalid && c0 + col < J;
          const E x = base[ok ? (size_t)row * J + c0 + col : 0];
          buf[s] = ok ? x : E{};
        }
#pragma unroll
        for (int s = 0; s < NV; ++s) {
          const int e = s * 256 + tid, row = e / WJC, col = e % WJC;
          const float x = to_f32<TIN>(buf[s], scale);
          sX[row * WXS + col] = x;
          if constexpr (!UOUT) ss += (double)x * x;
        }
      }
      __syncthreads();
      // Y rows 16w .. 16w+15 of this tile, this chunk's columns
      if constexpr (TIN == DPAR2_F32) {
#pragma unroll
        for (int jg = 0; jg < WJC / 16; ++jg) {
          const float4 xa = *reinterpret_cast<const float4*>(&sX[(16 * w + lr) * WXS + jg * 16 + 4 * lk]);
#pragma unroll
          for (int lt = 0; lt < LT; ++lt) {
            const float4 ob = *reinterpret_cast<const float4*>(&sOm[(lt * 16 + lr) * WXS + jg * 16 + 4 * lk]);
            acc[lt] = mfma_f32(xa.x, ob.x, acc[lt]);
            acc[lt] = mfma_f32(xa.y, ob.y, acc[lt]);
            acc[lt] = mfma_f32(xa.z, ob.z, acc[lt]);
            acc[lt] = mfma_f32(xa.w, ob.w, acc[lt]);
          }
        }
      } else {
#pragma unroll
        for (int kc = 0; kc < WJC / 32; ++kc) {
          const v8bf xa = bf16x8(&sX[(16 * w + lr) * WXS + kc * 32 + 8 * lk]);
#pragma unroll
          for (int lt = 0; lt < LT; ++lt) {
            const v8bf ob = bf16x8(&sOm[(lt * 16 + lr) * WXS + kc * 32 + 8 * lk]);
            acc[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, ob, acc[lt], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int lt = 0; lt < LT; ++lt)
#pragma unroll
        for (int v = 0; v < 4; ++v) ysum[lt][v] += (double)acc[lt][v];
    }
    if constexpr (!UOUT) {
      float* Yt = a.ybuf + (size_t)(td.rbase + it.row0 + (int64_t)t * TM) * LP;
#pragma unroll
      for (int lt = 0; lt < LT; ++lt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * w + f32_row(lane, v);
          if (row < nvalid) Yt[(size_t)row * LP + lt * 16 + lr] = (float)ysum[lt][v];
        }
    } else {
#pragma unroll
      for (int lt = 0; lt < LT; ++lt)
#pragma unroll
        for (int v = 0; v < 4; ++v) sYf[(16 * w + f32_row(lane, v)) * YS + lt * 16 + lr] = (float)ysum[lt][v];
      __syncthreads();
      for (int e = tid; e < nvalid * R; e += 256) {
        const int row = e / R, r = e % R;
        double u = 0.0;
        for (int l = 0; l < L; ++l) u += (double)sYf[row * YS + l] * sTh[l * R + r];
        a.U[(size_t)(it.row0 + (int64_t)t * TM + row) * R + r] = u;
      }
    }
  }
  if constexpr (!UOUT) {
    ss = block_sum(ss, sred);
    if (tid == 0) a.partS[blockIdx.x] = ss;
  }
}

template <int LT, int TIN>
__global__ __launch_bounds__(256) void k_wide_p(SlabArgs a) {
  typedef typename In<TIN>::E E;
  const int J = a.J, L = a.L;
  constexpr int TM = SKETCH_TM, LP = LT * 16, JT = WJC / 16;
  constexpr int YS = LP + 16;
  constexpr int NTP = LT * JT;                 // projection tiles (16 x 16, FP64)
  constexpr int NG = (LT == 1) ? 1 : 3;        // Gram tiles (upper triangle), chunk 0 only
  constexpr int NTT = NTP + NG;
  constexpr int NPW = (NTT + 3) / 4;           // tiles per wave
  constexpr int NV = TM * WJC / 256;
  __shared__ __align__(16) float sX[TM * WXS];
  __shared__ __align__(16) float sY[TM * YS];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t item = blockIdx.x;
  const int c0 = (int)blockIdx.y * WJC;
  const bool gram = blockIdx.y == 0;
  const Item it = a.items[item];
  const TDesc& td = a.td[it.pad];
  const E* __restrict__ slab = static_cast<const E*>(td.slab);
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);
  const float scale = (TIN == DPAR2_FP8_E4M3) ? td.scale[it.slice - td.k0] : 1.0f;
  const float* __restrict__ Yi = a.ybuf + (size_t)(td.rbase + it.row0) * LP;

  v4d pacc[NPW];
#pragma unroll
  for (int q = 0; q < NPW; ++q) pacc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < ntiles; ++t) {
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
    const E* base = slab + (size_t)(it.row0 + (int64_t)t * TM) * J;
    E buf[NV];
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const int e = s * 256 + tid, row = e / WJC, col = e % WJC;
      const bool ok = row < nvalid && c0 + col < J;
      const E x = base[ok ? (size_t)row * J + c0 + col : 0];
      buf[s] = ok ? x : E{};
    }
    __syncthreads();
    for (int e = tid; e < TM * LP; e += 256) {
      const int row = e / LP, l = e % LP;
      sY[row * YS + l] = row < nvalid ? Yi[(size_t)(t * TM + row) * LP + l] : 0.f;
    }
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const int e = s * 256 + tid, row = e / WJC, col = e % WJC;
      sX[row * WXS + col] = to_f32<TIN>(buf[s], scale);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TM / 4; ++kk) {
      const int row = 4 * kk + lk;
#pragma unroll
      for (int q = 0; q < NPW; ++q) {
        const int task = w + 4 * q;
        if (task < NTP) {
          const int lt = task / JT, jt = task % JT;
          pacc[q] = mfma_f64((double)sY[row * YS + lt * 16 + lr], (double)sX[row * WXS + jt * 16 + lr], pacc[q]);
        } else if (task < NTT && gram) {
          const int g = task - NTP;
          const int ga = (g == 2) ? 1 : 0, gb = (g == 0) ? 0 : 1;
          pacc[q] = mfma_f64((double)sY[row * YS + ga * 16 + lr], (double)sY[row * YS + gb * 16 + lr], pacc[q]);
        }
      }
    }
  }
  double* Pp = a.partP + (size_t)item * L * J;
  double* Gp = a.partG + (size_t)item * L * L;
#pragma unroll
  for (int q = 0; q < NPW; ++q) {
    const int task = w + 4 * q;
    if (task < NTP) {
      const int lt = task / JT, jt = task % JT;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = lt * 16 + f64_row(lane, v), j = c0 + jt * 16 + lr;
        if (i < L && j < J) Pp[(size_t)i * J + j] = pacc[q][v];
      }
    } else if (task < NTT && gram) {
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
}

template <int LT, int TIN>
static hipError_t wide_launch(const SlabArgs& a, int64_t n_items, bool vec, bool uout, hipStream_t s) {
  const dim3 g1((unsigned)n_items), blk(256);
  if (uout) {
    if (vec) hipLaunchKernelGGL((k_wide_y<LT, true, TIN, true>), g1, blk, 0, s, a);
    else hipLaunchKernelGGL((k_wide_y<LT, false, TIN, true>), g1, blk, 0, s, a);
    return hipGetLastError();
  }
  if (vec) hipLaunchKernelGGL((k_wide_y<LT, true, TIN, false>), g1, blk, 0, s, a);
  else hipLaunchKernelGGL((k_wide_y<LT, false, TIN, false>), g1, blk, 0, s, a);
  const dim3 g2((unsigned)n_items, (unsigned)((a.J + WJC - 1) / WJC));
  hipLaunchKernelGGL((k_wide_p<LT, TIN>), g2, blk, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_slab_wide(const SlabArgs& a, int dtype, int64_t n_items, bool vec, bool uout, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (a.L > 32 || a.J > MAX_J || (!uout && !a.ybuf)) return hipErrorInvalidValue;
  const bool l1 = a.L <= 16;
  if (dtype == DPAR2_F32) return l1 ? wide_launch<1, DPAR2_F32>(a, n_items, vec, uout, s)
                                    : wide_launch<2, DPAR2_F32>(a, n_items, vec, uout, s);
  if (dtype == DPAR2_BF16) return l1 ? wide_launch<1, DPAR2_BF16>(a, n_items, vec, uout, s)
                                     : wide_launch<2, DPAR2_BF16>(a, n_items, vec, uout, s);
  return l1 ? wide_launch<1, DPAR2_FP8_E4M3>(a, n_items, vec, uout, s)
            : wide_launch<2, DPAR2_FP8_E4M3>(a, n_items, vec, uout, s);
}

}  // namespace dpar2
