// Slab pass for wide slices (J above the narrow kernels' limit; Sec. III-B,
// Eq. 4, Alg. 1 applied to every slice), in two kernels:
//   k_wide_y  per work item: Y = X Omega tile by tile, the row of a tile
//             streamed through LDS in chunks of 128 columns, one chunk of X
//             and of Omega (read from L2 into registers) prefetched ahead;
//             each wave takes a 16-column tile of Y and a share of every
//             chunk's columns (FP32 matrix cores for float32 slabs, bf16
//             matrix cores with Omega rounded to bf16 otherwise; the waves'
//             chunk sums added in FP64 in a fixed order, Y rounded to FP32
//             once) and
//             ||X||_F^2; Y of each tile in 22-bit fixed point per column as
//             three int8 digit planes (written to the Y-digit buffer) and the
//             exact Gram Y^T Y from them on the int8 matrix cores; or, in the U
//             variant, U = Y Theta_k
//   k_wide_p  per (128-column chunk, work item): the chunk of X in 22-bit
//             fixed point per column of each tile as int8 digits (X and the
//             tile's Y digits prefetched one tile ahead), and the
//             exact P(:, chunk) = Y^T X(:, chunk) from the nine digit products
//             on the int8 matrix cores, combined in FP64 per tile
// The arithmetic is that of the whole-row pass (sketch_impl.h): Gram and
// projection are the exact products of the same rounded pair.  The slab is
// read twice (once per kernel).
#include "sketch_impl.h"

namespace dpar2 {

constexpr int WJC = 128;        // columns per chunk
constexpr int WXS = WJC + 4;    // LDS row stride of an X chunk (floats)

// Raw buffer loads: the resource covers n bytes from its base and a load at
// a byte offset at or past n returns zero, so the rows past a tile's end and
// masked slots need no clamped addresses (offsets are 32-bit registers and
// the base stays in scalar registers).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t OOB = 0x80000000u;   // an offset past every resource here (< 2^31 bytes)
__device__ __forceinline__ rsrc_t buf_rsrc(const void* p, uint32_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, 0x00020000);
}
// voff: per-lane byte offset; soff: a wave-uniform byte offset (scalar register)
template <typename T>
__device__ __forceinline__ T buf_load(rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float buf_load<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ uint16_t buf_load<uint16_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}
template <>
__device__ __forceinline__ uint8_t buf_load<uint8_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
}
template <>
__device__ __forceinline__ uint32_t buf_load<uint32_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
template <>
__device__ __forceinline__ uint2 buf_load<uint2>(rsrc_t r, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_uint2(v[0], v[1]);
}
template <>
__device__ __forceinline__ float4 buf_load<float4>(rsrc_t r, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

// Tile g of the upper triangle of the Gram, column by column: (0,0), (0,1),
// (1,1), (0,2), (1,2), (2,2), ...; gram_a is its row tile, gram_b its column
// tile.
__device__ __forceinline__ int gram_b(int g) {
  int b = 0;
  while (g > b) {
    g -= b + 1;
    ++b;
  }
  return b;
}
__device__ __forceinline__ int gram_a(int g) { return g - gram_b(g) * (gram_b(g) + 1) / 2; }

template <int LT, bool VEC, int TIN, bool UOUT>
__global__ __launch_bounds__(256, 2) void k_wide_y(SlabArgs a) {
  typedef typename In<TIN>::E E;
  typedef typename In<TIN>::V4 V4;
  const int J = a.J, L = a.L, R = a.R;
  constexpr int TM = SKETCH_TM, LP = LT * 16;
  constexpr int NV = VEC ? TM * WJC / 4 / 256 : TM * WJC / 256;
  constexpr int YS = LP + 1;
  // wave w: 16-column tile lt = w % LT of Y, and the share ks = w / LT of
  // every chunk's columns (KS shares); all 64 rows of the tile
  constexpr int KS = 4 / LT;
  constexpr int NJG = (WJC / 16) / KS;       // FP32 products: 16-column groups per wave
  constexpr int NKW = (WJC / 32) / KS;       // bf16 products: 32-column groups per wave
  constexpr int OB = 8 * LT;                 // Omega values per lane and chunk (= 4 NJG = 8 NKW)
  // sX holds a chunk of X, and at the end of a tile the KS partial sums of Y
  // (KS x 64 x LP doubles)
  static_assert(KS * TM * LP * 2 <= TM * WXS, "partial sums of Y must fit over the X chunk");
  __shared__ __align__(16) float sX[TM * WXS];
  __shared__ float sYf[UOUT ? TM * YS : 1];
  // Theta_k (L x R): above L = 32 at most 60 x 50 (the supported ranks and widths)
  __shared__ double sTh[UOUT ? (LT > 2 ? 60 * 50 : 32 * 32) : 1];
  __shared__ double sred[8];
  constexpr int QW = 20;                       // dwords per digit-plane row (64 bytes + pad)
  __shared__ __align__(16) uint32_t sYq[UOUT ? 4 : 3 * LP * QW];
  __shared__ float sYm[UOUT ? 1 : 4 * LP];
  __shared__ int sYe[UOUT ? 1 : LP];
  // Gram tiles (upper triangle, column by column: tile g = (ga, gb), ga <= gb),
  // tile g on wave g % 4
  constexpr int NG = LT * (LT + 1) / 2;
  constexpr int NGW = (NG + 3) / 4;            // tiles per wave
  const size_t TB = wide_tile_bytes(L);
  v4d gacc[NGW];
#pragma unroll
  for (int gi = 0; gi < NGW; ++gi) gacc[gi] = v4d{0.0, 0.0, 0.0, 0.0};
  double* sYp = reinterpret_cast<double*>(sX);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int lt = w % LT, ks = w / LT;
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

  // Prefetch of one chunk ahead: X of (tile, chunk) into xb, this wave's
  // Omega operands of the chunk into ob (straight from the J x L matrix, which
  // stays in L2; entries past J or L are zero).  FP32 products: lane (lr, lk)
  // holds Omega[c0 + 16 jg + 4 lk + i][16 lt + lr] for its groups jg = ks +
  // KS g; bf16 products: Omega[c0 + 32 kc + 8 lk + i][16 lt + lr] for kc = ks
  // + KS g.
  typedef typename std::conditional<VEC, V4, E>::type slot_t;
  slot_t xb[NV];
  float ob[OB];
  const int ncol = 16 * lt + lr;
  const rsrc_t om_r = buf_rsrc(omega, (uint32_t)((size_t)J * L * 4));
  constexpr int XRS = (VEC ? 4 : 1) * 256 / WJC;          // rows between a thread's slots
  const int xrow0 = (VEC ? 4 * tid : tid) / WJC, xcol = (VEC ? 4 * tid : tid) % WJC;
  auto load_step = [&](int t, int c) {
    const int c0 = c * WJC;
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
    // the tile's rows: loads of rows past its end return zero
    const rsrc_t xr = buf_rsrc(slab + (size_t)(it.row0 + (int64_t)t * TM) * J,
                               (uint32_t)((size_t)nvalid * J * sizeof(E)));
    // slot s: row xrow0 + s XRS, column xcol of the chunk; the per-slot part
    // of the offset is wave-uniform
    const uint32_t xoff = c0 + xcol < J ? (uint32_t)((xrow0 * J + c0 + xcol) * (int)sizeof(E)) : OOB;
#pragma unroll
    for (int s = 0; s < NV; ++s) xb[s] = buf_load<slot_t>(xr, xoff, (uint32_t)(s * XRS * J * (int)sizeof(E)));
    // Omega[k][ncol], k = kbase + kstep(g); k >= J lies past the end
    const int kbase = f32mm ? c0 + 16 * ks + 4 * lk : c0 + 32 * ks + 8 * lk;
    const uint32_t ooff = ncol < L ? (uint32_t)((kbase * L + ncol) * 4) : OOB;
#pragma unroll
    for (int g = 0; g < OB; ++g) {
      const int kstep = f32mm ? 16 * KS * (g / 4) + (g % 4) : 32 * KS * (g / 8) + (g % 8);
      ob[g] = buf_load<float>(om_r, ooff, (uint32_t)(kstep * L * 4));
    }
  };

  double ss = 0.0;
  v4d ysum[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) ysum[rb] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nsteps = ntiles * nchunks;
  if (nsteps > 0) load_step(0, 0);
  for (int step = 0; step < nsteps; ++step) {
    const int t = step / nchunks, c = step % nchunks;
    // every wave is done with sX (the previous chunk's products, or the
    // previous tile's partial sums of Y)
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const int e = VEC ? 4 * (s * 256 + tid) : s * 256 + tid, row = e / WJC, col = e % WJC;
      if constexpr (VEC) {
        const float4 x = to_f32x4<TIN>(xb[s], scale);
        *reinterpret_cast<float4*>(&sX[row * WXS + col]) = x;
        if constexpr (!UOUT) ss += (double)x.x * x.x + (double)x.y * x.y + (double)x.z * x.z + (double)x.w * x.w;
      } else {
        const float x = to_f32<TIN>(xb[s], scale);
        sX[row * WXS + col] = x;
        if constexpr (!UOUT) ss += (double)x * x;
      }
    }
    float oc[OB];
#pragma unroll
    for (int g = 0; g < OB; ++g) oc[g] = ob[g];
    if (step + 1 < nsteps) load_step((step + 1) / nchunks, (step + 1) % nchunks);
    __syncthreads();
    // this wave's share of the chunk: rows 16 rb .. 16 rb + 15, columns of
    // its groups, Y columns 16 lt .. 16 lt + 15; the chunk's FP32 sums are
    // added in FP64, so the rounding of Y does not grow with J
    v4f acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};
    if (f32mm) {
#pragma unroll
      for (int g = 0; g < NJG; ++g) {
        const int jg = ks + KS * g;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          const float4 xa = *reinterpret_cast<const float4*>(&sX[(16 * rb + lr) * WXS + jg * 16 + 4 * lk]);
          acc[rb] = mfma_f32(xa.x, oc[4 * g + 0], acc[rb]);
          acc[rb] = mfma_f32(xa.y, oc[4 * g + 1], acc[rb]);
          acc[rb] = mfma_f32(xa.z, oc[4 * g + 2], acc[rb]);
          acc[rb] = mfma_f32(xa.w, oc[4 * g + 3], acc[rb]);
        }
      }
    } else {
#pragma unroll
      for (int g = 0; g < NKW; ++g) {
        const int kc = ks + KS * g;
        v8bf obv;
#pragma unroll
        for (int i = 0; i < 8; ++i) obv[i] = (__bf16)oc[8 * g + i];   // nearest even
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          const v8bf xa = bf16x8(&sX[(16 * rb + lr) * WXS + kc * 32 + 8 * lk]);
          acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, obv, acc[rb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) ysum[rb][v] += (double)acc[rb][v];
    if (c + 1 < nchunks) continue;

    // --- end of tile t: Y from the KS partial sums, in a fixed order --------
    const int64_t rem = nrows - (int64_t)t * TM;
    const int nvalid = rem < TM ? (int)rem : TM;
    __syncthreads();   // sX is free
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sYp[(ks * TM + 16 * rb + f32_row(lane, v)) * LP + ncol] = ysum[rb][v];
      ysum[rb] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();
    // wave w now takes rows 16 w .. 16 w + 15 and every column of Y
    float yv[LT][4];
#pragma unroll
    for (int l2 = 0; l2 < LT; ++l2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * w + f32_row(lane, v);
        double y = 0.0;
#pragma unroll
        for (int k2 = 0; k2 < KS; ++k2) y += sYp[(k2 * TM + row) * LP + 16 * l2 + lr];
        yv[l2][v] = (float)y;   // Y rounded to float32 once
      }
    if constexpr (!UOUT) {
      // rows past the tile's end are zero (their X rows were loaded as
      // zeros); column maxima per wave, then per tile
#pragma unroll
      for (int l2 = 0; l2 < LT; ++l2) {
        float m = fmaxf(fmaxf(fabsf(yv[l2][0]), fabsf(yv[l2][1])), fmaxf(fabsf(yv[l2][2]), fabsf(yv[l2][3])));
        m = fmaxf(m, __shfl_xor(m, 16, 64));
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        if (lk == 0) sYm[w * LP + l2 * 16 + lr] = m;
      }
      __syncthreads();
      uint32_t* Yw = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(a.ybuf) + (size_t)(it.tslot + t) * TB);
      int* Yex = reinterpret_cast<int*>(Yw + 3 * LP * 16);
#pragma unroll
      for (int l2 = 0; l2 < LT; ++l2) {
        const int col = l2 * 16 + lr;
        const float m = fmaxf(fmaxf(sYm[col], sYm[LP + col]), fmaxf(sYm[2 * LP + col], sYm[3 * LP + col]));
        const int e = col_exp(m);
        float sc;
        const bool tiny = col_scale(e, sc);
        if (__builtin_amdgcn_ballot_w64(tiny)) {   // rare: taken only when a lane needs it
          const float pre = tiny ? 0x1p64f : 1.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) yv[l2][v] *= pre;
        }
        int q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = q22b(yv[l2][v], sc);
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
#pragma unroll
      for (int gi = 0; gi < NGW; ++gi) {
        const int g = w + 4 * gi;
        if (g < NG) {
          const int ca = 16 * gram_a(g), cb = 16 * gram_b(g);
          v4i A[3], B[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            A[d] = *reinterpret_cast<const v4i*>(&sYq[(d * LP + ca + lr) * QW + 4 * lk]);
            B[d] = *reinterpret_cast<const v4i*>(&sYq[(d * LP + cb + lr) * QW + 4 * lk]);
          }
          gacc[gi] = digit_tile_fma(A, B, sYe[cb + lr], sYe, ca, lane, gacc[gi]);
        }
      }
    } else {
#pragma unroll
      for (int l2 = 0; l2 < LT; ++l2)
#pragma unroll
        for (int v = 0; v < 4; ++v) sYf[(16 * w + f32_row(lane, v)) * YS + l2 * 16 + lr] = yv[l2][v];
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
    double* Gp = a.partG + (size_t)blockIdx.x * L * L;
#pragma unroll
    for (int gi = 0; gi < NGW; ++gi) {
      const int g = w + 4 * gi;
      if (g < NG) {
        const int ga = gram_a(g), gb = gram_b(g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = ga * 16 + f32_row(lane, v), j = gb * 16 + lr;
          if (i < L && j < L) {
            Gp[i * L + j] = gacc[gi][v];
            if (ga != gb) Gp[j * L + i] = gacc[gi][v];
          }
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
__global__ __launch_bounds__(256, 2) void k_wide_p(SlabArgs a) {
  typedef typename In<TIN>::E E;
  const int J = a.J, L = a.L;
  constexpr int TM = SKETCH_TM, LP = LT * 16, JT = WJC / 16;
  constexpr int QW = 20;
  constexpr int NTP = LT * JT;                 // projection tiles (16 x 16)
  constexpr int NPW = NTP / 4;                 // tiles per wave
  __shared__ __align__(16) uint32_t sXq[3 * WJC * QW];
  __shared__ float sXm[4 * WJC];
  __shared__ int sXe[WJC];
  // the tile's Y digits (rows padded to QW dwords) and column exponents,
  // prefetched from the digit buffer one tile ahead
  constexpr int NYQ = 3 * LP * 4;              // 16-byte words of the digit planes
  constexpr int NYW = NYQ + LP / 4;            // ... and of the exponents
  constexpr int NYR = (NYW + 255) / 256;       // per thread
  __shared__ __align__(16) uint32_t sYq[3 * LP * QW];
  __shared__ __align__(16) int sYe[LP];

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
    // the tile's rows: loads of rows past its end return zero
    const rsrc_t xr = buf_rsrc(slab + (size_t)(it.row0 + (int64_t)t * TM) * J,
                               (uint32_t)((size_t)nvalid * J * sizeof(E)));
    const uint32_t xoff = jok ? (uint32_t)((16 * q0 * J + c0 + j) * (int)sizeof(E)) : OOB;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[h][r] = buf_load<E>(xr, xoff, (uint32_t)((32 * h + r) * J * (int)sizeof(E)));
  };

  uint4 yb[NYR];
  auto load_y = [&](int t) {
    const uint4* Yw = reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(a.ybuf) +
                                                     (size_t)(it.tslot + t) * TB);
#pragma unroll
    for (int i = 0; i < NYR; ++i) {
      const int u = tid + 256 * i;
      yb[i] = Yw[u < NYW ? u : 0];
    }
  };

  v4d pacc[NPW];
#pragma unroll
  for (int qi = 0; qi < NPW; ++qi) pacc[qi] = v4d{0.0, 0.0, 0.0, 0.0};
  if (ntiles > 0) {
    load_tile(0);
    load_y(0);
  }
  for (int t = 0; t < ntiles; ++t) {
    // Y digits of tile t into LDS (the previous tile's products are done:
    // the barrier at the end of the loop)
#pragma unroll
    for (int i = 0; i < NYR; ++i) {
      const int u = tid + 256 * i;
      if (u < NYQ) *reinterpret_cast<uint4*>(&sYq[(u >> 2) * QW + 4 * (u & 3)]) = yb[i];
      else if (u < NYW) *reinterpret_cast<uint4*>(&sYe[4 * (u - NYQ)]) = yb[i];
    }
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
    if (t + 1 < ntiles) {
      load_tile(t + 1);
      load_y(t + 1);
    }
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
    __syncthreads();
#pragma unroll
    for (int qi = 0; qi < NPW; ++qi) {
      const int task = w + 4 * qi;
      const int ca = (task / JT) * 16, cb = (task % JT) * 16;
      v4i A[3], B[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        A[d] = *reinterpret_cast<const v4i*>(&sYq[(d * LP + ca + lr) * QW + 4 * lk]);
        B[d] = *reinterpret_cast<const v4i*>(&sXq[(d * WJC + cb + lr) * QW + 4 * lk]);
      }
      pacc[qi] = digit_tile_fma(A, B, sXe[cb + lr], sYe, ca, lane, pacc[qi]);
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
  if (a.L > 64 || a.J > MAX_J || (!uout && !a.ybuf)) return hipErrorInvalidValue;
  const int lt = wide_lt(a.L);
#define DPAR2_WL(TIN_)                                                     \
  return lt == 1 ? wide_launch<1, TIN_>(a, n_items, vec, uout, s)          \
       : lt == 2 ? wide_launch<2, TIN_>(a, n_items, vec, uout, s)          \
                 : wide_launch<4, TIN_>(a, n_items, vec, uout, s);
  if (dtype == DPAR2_F32) { DPAR2_WL(DPAR2_F32) }
  if (dtype == DPAR2_BF16) { DPAR2_WL(DPAR2_BF16) }
  DPAR2_WL(DPAR2_FP8_E4M3)
#undef DPAR2_WL
}

}  // namespace dpar2
