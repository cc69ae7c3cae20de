// Slab pass for wide slices (J above the narrow kernels' limit; Sec. III-B,
// Eq. 4, Alg. 1 applied to every slice), in two kernels:
//   k_wide_y  per work item: Y = X Omega tile by tile, the row of a tile
//             streamed through LDS in chunks of 128 columns (FP32 matrix cores
//             for float32 slabs, bf16 matrix cores with Omega rounded to bf16
//             otherwise; chunk sums added in FP64, Y rounded to FP32 once) and
//             ||X||_F^2; Y of each tile in 22-bit fixed point per column as
//             three int8 digit planes (written to the Y-digit buffer) and the
//             exact Gram Y^T Y from them on the int8 matrix cores; or, in the U
//             variant, U = Y Theta_k
//   k_wide_p  per (128-column chunk, work item): the chunk of X in 22-bit
//             fixed point per column of each tile as int8 digits, and the
//             exact P(:, chunk) = Y^T X(:, chunk) from the nine digit products
//             on the int8 matrix cores, combined in FP64 per tile
// The arithmetic is that of the whole-row pass (sketch_impl.h): Gram and
// projection are the exact products of the same rounded pair.  The slab is
// read twice (once per kernel).
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
  constexpr int QW = 20;                       // dwords per digit-plane row (64 bytes + pad)
  __shared__ __align__(16) uint32_t sYq[UOUT ? 4 : 3 * LP * QW];
  __shared__ float sYm[UOUT ? 1 : 4 * LP];
  __shared__ int sYe[UOUT ? 1 : LP];
  constexpr int NG = (LT == 1) ? 1 : 3;        // Gram tiles (upper triangle), waves 0 .. NG-1
  const size_t TB = wide_tile_bytes(L);
  v4d gacc = v4d{0.0, 0.0, 0.0, 0.0};

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (a.skip && *a.skip) return;
  const Item it = a.items[blockIdx.x];
  const TDesc& td = a.td[it.pad];
  const E* __restrict__ slab = static_cast<const E*>(td.slab);
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);
  const int nchunks = (J + WJC - 1) / WJC;
  const float* __restrict__ omega = a.omega ? a.omega + (size_t)it.slice * J * L : td.om1;
  const float scale = (TIN == DPAR2_FP8_E4M3) ? td.scale[it.slice - td.k0] : 1.0f;
  // FP32 matrix cores with Omega as given: float32 slabs, and the passes of a
  // power step (per-slice sketch matrices) for every dtype; otherwise bf16
  // matrix cores with Omega rounded to bf16
  const bool f32mm = (TIN == DPAR2_F32) || a.omega != nullptr;
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
        sOm[e] = f32mm ? o : round_bf16(o);
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
      if (f32mm) {
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
      // Y rounded to float32 once (rows past the tile's end are zero: their
      // X rows were loaded as zeros); column maxima per wave, then per tile
      float yv[LT][4];
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) yv[lt][v] = (float)ysum[lt][v];
        float m = fmaxf(fmaxf(fabsf(yv[lt][0]), fabsf(yv[lt][1])), fmaxf(fabsf(yv[lt][2]), fabsf(yv[lt][3])));
        m = fmaxf(m, __shfl_xor(m, 16, 64));
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        if (lk == 0) sYm[w * LP + lt * 16 + lr] = m;
      }
      __syncthreads();
      uint32_t* Yw = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(a.ybuf) + (size_t)(it.tslot + t) * TB);
      int* Yex = reinterpret_cast<int*>(Yw + 3 * LP * 16);
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) {
        const int col = lt * 16 + lr;
        const float m = fmaxf(fmaxf(sYm[col], sYm[LP + col]), fmaxf(sYm[2 * LP + col], sYm[3 * LP + col]));
        const int e = col_exp(m);
        float sc;
        const bool tiny = col_scale(e, sc);
        if (__builtin_amdgcn_ballot_w64(tiny)) {   // rare: taken only when a lane needs it
          const float pre = tiny ? 0x1p64f : 1.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) yv[lt][v] *= pre;
        }
        int q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = q22b(yv[lt][v], sc);
        uint32_t pw[3];
        digits4(q, pw[0], pw[1], pw[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          sYq[(d * LP + col) * QW + 4 * w + lk] = pw[d];
          Yw[(d * LP + col) * 16 + 4 * w + lk] = pw[d];
        }
        if (w == 0 && lk == 0) {
          sYe[col] = e;
          Yex[col] = e;
        }
      }
      __syncthreads();
      // exact Gram of the represented Y: nine digit products per 16 x 16 tile
      if (w < NG) {
        const int ca = (w == 2) ? 16 : 0, cb = (w == 0) ? 0 : 16;
        v4i A[3], B[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          A[d] = *reinterpret_cast<const v4i*>(&sYq[(d * LP + ca + lr) * QW + 4 * lk]);
          B[d] = *reinterpret_cast<const v4i*>(&sYq[(d * LP + cb + lr) * QW + 4 * lk]);
        }
        gacc = digit_tile_fma(A, B, sYe[cb + lr], sYe, ca, lane, gacc);
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
    if (w < NG) {
      double* Gp = a.partG + (size_t)blockIdx.x * L * L;
      const int ga = (w == 2) ? 1 : 0, gb = (w == 0) ? 0 : 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ga * 16 + f32_row(lane, v), j = gb * 16 + lr;
        if (i < L && j < L) {
          Gp[i * L + j] = gacc[v];
          if (ga != gb) Gp[j * L + i] = gacc[v];
        }
      }
    }
    ss = block_sum(ss, sred);
    if (tid == 0) a.partS[blockIdx.x] = ss;
  }
}

// P(:, chunk) = Y^T X(:, chunk) for one 128-column chunk of one work item:
// per tile, the chunk's columns in 22-bit fixed point (digits in LDS), the
// Y digits straight from the digit buffer, nine int8 products per 16 x 16
// output tile.  Thread (j, q): column j of the chunk, row quarters q and q + 2.
template <int LT, int TIN>
__global__ __launch_bounds__(256) void k_wide_p(SlabArgs a) {
  typedef typename In<TIN>::E E;
  const int J = a.J, L = a.L;
  constexpr int TM = SKETCH_TM, LP = LT * 16, JT = WJC / 16;
  constexpr int QW = 20;
  constexpr int NTP = LT * JT;                 // projection tiles (16 x 16)
  constexpr int NPW = NTP / 4;                 // tiles per wave
  __shared__ __align__(16) uint32_t sXq[3 * WJC * QW];
  __shared__ float sXm[4 * WJC];
  __shared__ int sXe[WJC];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (a.skip && *a.skip) return;
  const int nchunks = (J + WJC - 1) / WJC;
  const int64_t item = (int64_t)blockIdx.x / nchunks;   // the chunks of one item are consecutive blocks
  const int c0 = (int)(blockIdx.x % nchunks) * WJC;
  const Item it = a.items[item];
  const TDesc& td = a.td[it.pad];
  const E* __restrict__ slab = static_cast<const E*>(td.slab);
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);
  const float scale = (TIN == DPAR2_FP8_E4M3) ? td.scale[it.slice - td.k0] : 1.0f;
  const size_t TB = wide_tile_bytes(L);
  const int j = tid % WJC, q0 = tid / WJC;     // column and first row quarter
  const bool jok = c0 + j < J;

  // 32 values per thread: rows 16 q + r of column c0 + j, q = q0, q0 + 2
  E buf[2][16];
  auto load_tile = [&](int t) {
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
    // (slots out of range load the tile's first element, which exists)
    const E* base = slab + (size_t)(it.row0 + (int64_t)t * TM) * J;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 16 * (q0 + 2 * h) + r;
        const bool ok = jok && row < nvalid;
        const E x = base[ok ? (size_t)row * J + c0 + j : 0];
        buf[h][r] = ok ? x : E{};
      }
  };

  v4d pacc[NPW];
#pragma unroll
  for (int qi = 0; qi < NPW; ++qi) pacc[qi] = v4d{0.0, 0.0, 0.0, 0.0};
  if (ntiles > 0) load_tile(0);
  for (int t = 0; t < ntiles; ++t) {
    float xv[2][16];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float m = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        xv[h][r] = to_f32<TIN>(buf[h][r], scale);
        m = fmaxf(m, fabsf(xv[h][r]));
      }
      sXm[(q0 + 2 * h) * WJC + j] = m;
    }
    if (t + 1 < ntiles) load_tile(t + 1);
    __syncthreads();
    {
      const float m = fmaxf(fmaxf(sXm[j], sXm[WJC + j]), fmaxf(sXm[2 * WJC + j], sXm[3 * WJC + j]));
      const int e = col_exp(m);
      float sc;
      const bool tiny = col_scale(e, sc);
      if (__builtin_amdgcn_ballot_w64(tiny)) {   // rare: taken only when a lane needs it
        const float pre = tiny ? 0x1p64f : 1.0f;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 16; ++r) xv[h][r] *= pre;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t pk[3][4];
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          int qv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) qv[v] = q22b(xv[h][4 * r4 + v], sc);
          digits4(qv, pk[0][r4], pk[1][r4], pk[2][r4]);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
          *reinterpret_cast<uint4*>(&sXq[(d * WJC + j) * QW + 4 * (q0 + 2 * h)]) =
              make_uint4(pk[d][0], pk[d][1], pk[d][2], pk[d][3]);
      }
      if (q0 == 0) sXe[j] = e;
    }
    // Y digits of the tile from the digit buffer (16 bytes per lane and plane)
    const uint32_t* Yw =
        reinterpret_cast<const uint32_t*>(reinterpret_cast<const unsigned char*>(a.ybuf) + (size_t)(it.tslot + t) * TB);
    const int* Yex = reinterpret_cast<const int*>(Yw + 3 * LP * 16);
    __syncthreads();
#pragma unroll
    for (int qi = 0; qi < NPW; ++qi) {
      const int task = w + 4 * qi;
      const int ca = (task / JT) * 16, cb = (task % JT) * 16;
      v4i A[3], B[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        A[d] = *reinterpret_cast<const v4i*>(&Yw[(d * LP + ca + lr) * 16 + 4 * lk]);
        B[d] = *reinterpret_cast<const v4i*>(&sXq[(d * WJC + cb + lr) * QW + 4 * lk]);
      }
      pacc[qi] = digit_tile_fma(A, B, sXe[cb + lr], Yex, ca, lane, pacc[qi]);
    }
    __syncthreads();
  }
  double* Pp = a.partP + (size_t)item * L * J;
#pragma unroll
  for (int qi = 0; qi < NPW; ++qi) {
    const int task = w + 4 * qi;
    const int lt = task / JT, jt = task % JT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = lt * 16 + f32_row(lane, v), jj = c0 + jt * 16 + lr;
      if (i < L && jj < J) Pp[(size_t)i * J + jj] = pacc[qi][v];
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
  // chunks of one item in consecutive blocks: they read the item's Y digits
  // around the same time
  const dim3 g2((unsigned)(((a.J + WJC - 1) / WJC) * n_items));
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
