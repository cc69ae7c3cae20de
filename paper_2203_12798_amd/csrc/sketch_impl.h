// Slab pass on the int8 matrix cores (Sec. III-B, Eq. 4; Alg. 1 applied to
// every slice), templated on the input type and on the output:
//   Y  = X Omega                  (sketch step of Alg. 1 on the bf16 matrix
//                                  cores: float32 slabs as three-piece bf16
//                                  products with FP32-level error, bf16 / fp8
//                                  slabs exactly with Omega rounded to bf16)
//   G  = Y^T Y, P = Y^T X         (exact: int8 digit products, FP64 totals)
//   ss = ||X||_F^2
// or, in the U variant, the same Y (bit for bit) times Theta_k.  Omega is the
// shared Omega_1 (om_stride 0) or, after a power step, one J x L matrix per
// slice (om_stride J L).
//
// Exact integer accumulation of the Gram and projection: per 64-row tile,
// every column of Y and of X is scaled by a power of two so that its largest
// entry is below 2^22 and written as three balanced base-256 digits
// (q = d0 2^16 + d1 2^8 + d2, -128 <= d <= 127); all nine digit products are
// summed exactly in int32 (one 16x16x64 instruction per digit pair covers the
// whole tile), combined exactly in FP64 and rescaled.  The only rounding is
// the 22-bit fixed-point representation of each column within its tile (at
// most 2^-22 of the column maximum); the tile sums then accumulate in FP64.
// The Gram is therefore the exact Gram of the represented Y, consistent with
// the projection: the whitening that follows amplifies any inconsistency
// between the two by the condition number of Y^T Y, so no digit product may
// be dropped.
#pragma once

#include "internal.h"
#include "../../include/dpar2.h"

namespace dpar2 {


typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int TIN>
struct In;
template <>
struct In<DPAR2_F32> {
  typedef float E;
  typedef float4 V4;
};
template <>
struct In<DPAR2_BF16> {
  typedef uint16_t E;
  typedef uint2 V4;
};
template <>
struct In<DPAR2_FP8_E4M3> {
  typedef uint8_t E;
  typedef uint32_t V4;
};

// bf16 (bit pattern) to float: exact
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// OCP fp8 e4m3fn (bias 7, no infinities, S.1111.111 = NaN) to float: exact,
// on the conversion unit (one byte, or a pair of bytes per instruction)
typedef float v2f_cvt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float e4m3_to_f32(uint32_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

// round to the nearest bf16 value (ties to even), returned as float
__device__ __forceinline__ float round_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;   // inf / NaN unchanged
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

template <int TIN>
__device__ __forceinline__ float to_f32(typename In<TIN>::E x, float scale) {
  if constexpr (TIN == DPAR2_F32) return x;
  else if constexpr (TIN == DPAR2_BF16) return bf16_bits_to_f32(x);
  else return e4m3_to_f32(x) * scale;
}

template <int TIN>
__device__ __forceinline__ float4 to_f32x4(typename In<TIN>::V4 x, float scale) {
  if constexpr (TIN == DPAR2_F32) {
    return x;
  } else if constexpr (TIN == DPAR2_BF16) {
    return make_float4(bf16_bits_to_f32(x.x & 0xffffu), bf16_bits_to_f32(x.x >> 16),
                       bf16_bits_to_f32(x.y & 0xffffu), bf16_bits_to_f32(x.y >> 16));
  } else {
    const v2f_cvt lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)x, false);   // bytes 0, 1
    const v2f_cvt hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)x, true);    // bytes 2, 3
    return make_float4(lo[0] * scale, lo[1] * scale, hi[0] * scale, hi[1] * scale);
  }
}

// eight consecutive floats (bf16-representable) as a bf16 vector: exact
__device__ __forceinline__ v8bf bf16x8(const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v8bf r;
  r[0] = (__bf16)a.x;
  r[1] = (__bf16)a.y;
  r[2] = (__bf16)a.z;
  r[3] = (__bf16)a.w;
  r[4] = (__bf16)b.x;
  r[5] = (__bf16)b.y;
  r[6] = (__bf16)b.z;
  r[7] = (__bf16)b.w;
  return r;
}

// x = h + m + l exactly: h is x rounded to bf16 (nearest even), m the
// remainder rounded likewise and l what is left, which has at most 8
// significant bits.  Each subtraction is exact.  Pieces below the FP32 normal
// range may be flushed, so callers keep |x| >= 2^-100 where it matters.
// Two values per conversion instruction; a bf16 pair unpacks to floats by a
// shift (low half) and a mask (high half).
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a, b}, v2bf));
}

__device__ __forceinline__ void split3(const float (&x)[8], v8bf& h, v8bf& m, v8bf& l) {
  v4u hw, mw, lw;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float a = x[2 * i], b = x[2 * i + 1];
    const uint32_t ph = pk_bf16(a, b);
    const float ra = a - __uint_as_float(ph << 16), rb = b - __uint_as_float(ph & 0xffff0000u);
    const uint32_t pm = pk_bf16(ra, rb);
    const float sa = ra - __uint_as_float(pm << 16), sb = rb - __uint_as_float(pm & 0xffff0000u);
    hw[i] = ph;
    mw[i] = pm;
    lw[i] = pk_bf16(sa, sb);
  }
  h = __builtin_bit_cast(v8bf, hw);
  m = __builtin_bit_cast(v8bf, mw);
  l = __builtin_bit_cast(v8bf, lw);
}

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

// Column scale for the 22-bit fixed point: sc = 2^(22 - e) for |x| < 2^e.
// For e < -104 the power of two is beyond the FP32 range; the column's
// values are then multiplied by 2^64 first (exact: they are below 2^-104) and
// the scale lowered by the same amount.  Returns true when that pre-scale
// applies.
__device__ __forceinline__ bool col_scale(int e, float& sc) {
  const bool tiny = e < -104;
  sc = __int_as_float((127 + 22 - e - (tiny ? 64 : 0)) << 23);
  return tiny;
}

// round(x sc) + 0x808080 with sc from col_scale: x sc is exact (a power-of-two
// scaling within range) and |x sc| <= 2^22, so one fused multiply-add of
// 1.5 * 2^23 leaves the nearest integer (ties to even) in the low mantissa
// bits; the bias 0x808080 is folded into the same subtraction (see digits4).
__device__ __forceinline__ int q22b(float x, float sc) {
  const float m = fmaf(x, sc, 12582912.0f);
  return __float_as_int(m) - (0x4B400000 - 0x808080);
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
// + d2 with -128 <= d <= 127 (the representation is unique), packed as the
// signed byte planes p0 (d0), p1, p2.  Given u = q + 0x808080 (from q22b),
// 0 <= u < 2^24 and the unsigned bytes of u are the digits plus 128, so each
// plane is a byte of u with its top bit flipped.
__device__ __forceinline__ void digits4(const int (&u)[4], uint32_t& p0, uint32_t& p1, uint32_t& p2) {
  p2 = bytes_k<0>((uint32_t)u[0], (uint32_t)u[1], (uint32_t)u[2], (uint32_t)u[3]) ^ 0x80808080u;
  p1 = bytes_k<1>((uint32_t)u[0], (uint32_t)u[1], (uint32_t)u[2], (uint32_t)u[3]) ^ 0x80808080u;
  p0 = bytes_k<2>((uint32_t)u[0], (uint32_t)u[1], (uint32_t)u[2], (uint32_t)u[3]) ^ 0x80808080u;
}

// One 16 x 16 output tile of a digit-plane product over a 64-row tile:
// A[d], B[d] are this lane's 16 bytes (rows 16 lk .. 16 lk + 15) of digit
// plane d of its A column (ca + lr) and B column; the nine products are summed
// exactly in int32, combined exactly in FP64 and scaled by
// 2^(erow + ecol - 44), erow = erow_e[ca + row] and ecol = ecol_e the column
// exponents of the 22-bit fixed point; the result is added to acc (row
// f32_row(lane, v), column lane % 16).
__device__ __forceinline__ v4d digit_tile_fma(const v4i (&A)[3], const v4i (&B)[3], int ecol_e, const int* erow_e,
                                              int ca, int lane, v4d acc) {
  const v4i z = v4i{0, 0, 0, 0};
  const v4i S0 = mfma_i8(A[0], B[0], z);
  v4i S1 = mfma_i8(A[0], B[1], z);
  S1 = mfma_i8(A[1], B[0], S1);
  v4i S2 = mfma_i8(A[0], B[2], z);
  S2 = mfma_i8(A[1], B[1], S2);
  S2 = mfma_i8(A[2], B[0], S2);
  v4i S3 = mfma_i8(A[1], B[2], z);
  S3 = mfma_i8(A[2], B[1], S3);
  const v4i S4 = mfma_i8(A[2], B[2], z);
  // 2^(erow + ecol - 44) as an FP64 bit pattern (high word only); the
  // exponent stays within [-340, 212]
  const int ecol = (ecol_e - 44 + 1023) << 20;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // |S0| <= 2^18, |S1| <= 2^20, |S3| <= 2^21, |S4| <= 2^20: the two
    // pairs combine exactly in int32, the total exactly in FP64 (< 2^52)
    const int hi = S0[v] * 256 + S1[v], lo = S3[v] * 256 + S4[v];
    const double val = fma((double)hi, 16777216.0, fma((double)S2[v], 65536.0, (double)lo));
    const int erow = erow_e[ca + f32_row(lane, v)];
    acc[v] = fma(val, __hiloint2double((erow << 20) + ecol, 0), acc[v]);
  }
  return acc;
}

// SPL: Omega as three bf16 pieces (FP32-level products).  float32 slabs always;
// bf16 / fp8 slabs in the passes of a power step, whose per-slice sketch
// matrices are not rounded to bf16 (their X is bf16-exact: three products
// per chunk instead of six).
template <int LT, int JT, bool VEC, int TIN, bool UOUT, bool SPL>
__global__ __launch_bounds__(256) void k_sketch_q(SlabArgs a) {
  typedef typename In<TIN>::E E;
  const int J = a.J, L = a.L;
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

  constexpr int YS = LP + 1;                       // U variant: row stride of Y in LDS
  constexpr int QWORDS = 3 * JP * QW + 3 * LP * QW;
  constexpr int UWORDS = 2 * (TM * YS) + 2 * 32 * 32;
  __shared__ __align__(16) float sX[TM * XS];
  // Omega as three bf16 planes (split3), or as floats already rounded to bf16
  constexpr bool SPLIT = SPL;
  constexpr bool XSPLIT = (TIN == DPAR2_F32);      // X itself needs three pieces
  constexpr int NKC = (JT + 1) / 2;                // 32-column chunks
  constexpr int XSB = 32 * NKC + 8;                // bf16 row stride of the planes
  constexpr int PLANE = LP * XSB;
  __shared__ __align__(16) float sOm[SPLIT ? 4 : LP * XS];
  __shared__ __align__(16) __bf16 sOmb[SPLIT ? 3 * PLANE : 8];
  // digit planes, or in the U variant Y (FP32) and Theta_k (FP64)
  __shared__ __align__(16) uint32_t sQ[UOUT ? UWORDS : QWORDS];
  uint32_t* sXq = sQ;
  uint32_t* sYq = sQ + 3 * JP * QW;
  __shared__ float sXm[4 * JP];
  __shared__ float sYm[4 * LP];
  __shared__ int sXe[JP], sYe[LP];
  __shared__ double sred[8];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (a.skip && *a.skip) return;
  const Item it = a.items[blockIdx.x];
  const TDesc& td = a.td[it.pad];
  const E* __restrict__ slab = static_cast<const E*>(td.slab);
  const int64_t nrows = it.row1 - it.row0;
  const int ntiles = (int)((nrows + TM - 1) / TM);
  const float* __restrict__ omega = a.omega ? a.omega + (size_t)it.slice * J * L : td.om1;
  const float scale = (TIN == DPAR2_FP8_E4M3) ? td.scale[it.slice - td.k0] : 1.0f;

  // the low-precision inputs sketch on the bf16 matrix cores: Omega is
  // rounded to bf16 (nearest even) once, X is already bf16-representable
  if constexpr (SPLIT) {
    for (int e = tid; e < PLANE; e += 256) {
      const int n = e / XSB, j = e % XSB;
      const float o = (n < L && j < J) ? omega[(size_t)j * L + n] : 0.f;
      const __bf16 h = (__bf16)o;
      const float r = o - (float)h;
      const __bf16 m = (__bf16)r;
      sOmb[e] = h;
      sOmb[PLANE + e] = m;
      sOmb[2 * PLANE + e] = (__bf16)(r - (float)m);
    }
  } else {
    for (int e = tid; e < LP * XS; e += 256) {
      const int n = e / XS, j = e % XS;
      const float o = (n < L && j < J) ? omega[(size_t)j * L + n] : 0.f;
      sOm[e] = round_bf16(o);
    }
  }
  for (int e = tid; e < TM * XS; e += 256) sX[e] = 0.f;
  float* sYf = reinterpret_cast<float*>(sQ);                  // U variant: Y of the tile
  double* sTh = reinterpret_cast<double*>(sQ + 2 * TM * YS);  // U variant: Theta_k
  if constexpr (UOUT) {
    for (int e = tid; e < L * a.R; e += 256) sTh[e] = a.theta[(size_t)it.slice * L * a.R + e];
  }

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
  typedef typename std::conditional<VEC, typename In<TIN>::V4, E>::type slot_t;
  slot_t buf[NV];
  auto load_tile = [&](int t) {
    const E* base = slab + (size_t)(it.row0 + (int64_t)t * TM) * J;
    const int64_t rem = nrows - (int64_t)t * TM;
    if (rem >= TM) {
      // full tile: every row is in range; slots past the tile (srow = TM)
      // load its first element and are never stored
#pragma unroll
      for (int s = 0; s < NV; ++s) {
        const size_t off = srow[s] < TM ? (size_t)srow[s] * J + scol[s] : 0;
        if constexpr (VEC) buf[s] = *reinterpret_cast<const slot_t*>(base + off);
        else buf[s] = base[off];
      }
      return;
    }
    const int nvalid = (int)rem;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const bool ok = srow[s] < nvalid;
      const size_t off = ok ? (size_t)srow[s] * J + scol[s] : 0;
      if constexpr (VEC) {
        const slot_t x = *reinterpret_cast<const slot_t*>(base + off);
        buf[s] = ok ? x : slot_t{};
      } else {
        const E x = base[off];
        buf[s] = ok ? x : E{};
      }
    }
  };

  double ss = 0.0;
  v4d pacc[NPW];
#pragma unroll
  for (int q = 0; q < NPW; ++q) pacc[q] = v4d{0.0, 0.0, 0.0, 0.0};

  if (ntiles > 0) load_tile(0);
  // The tile loop needs no barrier at its top: sX, the only shared array
  // written before the first barrier of a tile, was last read in the
  // previous tile's sketch and column-maximum phase, and a barrier of that
  // tile already follows that phase.  This one orders the fills above before
  // the first tile.
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      if (srow[s] < TM) {
        if constexpr (VEC) {
          const float4 x = to_f32x4<TIN>(buf[s], scale);
          *reinterpret_cast<float4*>(&sX[srow[s] * XS + scol[s]]) = x;
          if constexpr (!UOUT)
            ss += (double)x.x * x.x + (double)x.y * x.y + (double)x.z * x.z + (double)x.w * x.w;
        } else {
          const float x = to_f32<TIN>(buf[s], scale);
          sX[srow[s] * XS + scol[s]] = x;
          if constexpr (!UOUT) ss += (double)x * x;
        }
      }
    }
    if (t + 1 < ntiles) load_tile(t + 1);
    __syncthreads();

    // Y rows 16w .. 16w+15 of this tile
    v4f acc[LT];
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) acc[lt] = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (SPLIT) {
      // FP32 products from the bf16 matrix cores: X and Omega are each split
      // into three bf16 pieces (split3) and the six piece products down to
      // 2^-16 relative are summed in FP32 (the three dropped ones lie below
      // 2^-25 of the product).  The leading product accumulates apart from
      // the five smaller ones.  Lane (lr, lk) holds columns 8 lk .. 8 lk + 7
      // of each 32-column chunk of row lr of X (A) and of Omega^T (B).
      float xr[NKC][8];
      float mx = 0.f;
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) {
        const float* p = &sX[(16 * w + lr) * XS + kc * 32 + 8 * lk];
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float4 b = *reinterpret_cast<const float4*>(p + 4);
        xr[kc][0] = a.x; xr[kc][1] = a.y; xr[kc][2] = a.z; xr[kc][3] = a.w;
        xr[kc][4] = b.x; xr[kc][5] = b.y; xr[kc][6] = b.z; xr[kc][7] = b.w;
#pragma unroll
        for (int i = 0; i < 8; ++i) mx = fmaxf(mx, fabsf(xr[kc][i]));
      }
      // a wave whose 16 rows are all below 2^-100 (and not all zero) works on
      // X 2^64 and scales Y back (both exact), so that no piece is subnormal
      const bool tiny = XSPLIT && __builtin_amdgcn_ballot_w64(mx >= 0x1p-100f) == 0 &&
                        __builtin_amdgcn_ballot_w64(mx > 0.f) != 0;
      if (tiny) {
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
          for (int i = 0; i < 8; ++i) xr[kc][i] *= 0x1p64f;
      }
      v4f lo[LT];
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) lo[lt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) {
        v8bf xh, xm, xl;
        if constexpr (XSPLIT) {
          split3(xr[kc], xh, xm, xl);
        } else {
          xh = bf16x8(xr[kc]);   // bf16 / fp8 rows are bf16-exact: one piece
        }
#pragma unroll
        for (int lt = 0; lt < LT; ++lt) {
          const __bf16* ob = &sOmb[(lt * 16 + lr) * XSB + kc * 32 + 8 * lk];
          const v8bf oh = *reinterpret_cast<const v8bf*>(ob);
          const v8bf om = *reinterpret_cast<const v8bf*>(ob + PLANE);
          const v8bf ol = *reinterpret_cast<const v8bf*>(ob + 2 * PLANE);
          acc[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, oh, acc[lt], 0, 0, 0);
          if constexpr (XSPLIT) {
            lo[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, oh, lo[lt], 0, 0, 0);
            lo[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xm, om, lo[lt], 0, 0, 0);
          }
          lo[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ol, lo[lt], 0, 0, 0);
          if constexpr (XSPLIT) lo[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xm, oh, lo[lt], 0, 0, 0);
          lo[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, om, lo[lt], 0, 0, 0);
        }
      }
#pragma unroll
      for (int lt = 0; lt < LT; ++lt) {
        acc[lt] += lo[lt];
        if (tiny) acc[lt] *= 0x1p-64f;
      }
    } else {
      // bf16 matrix cores, 32 columns per instruction: lane (lr, lk) holds
      // columns 8 lk .. 8 lk + 7 of the chunk for A (row lr of X) and B
      // (row lr of Omega^T); the products are exact, the sums FP32
#pragma unroll
      for (int kc = 0; kc < (JT + 1) / 2; ++kc) {
        const v8bf xa = bf16x8(&sX[(16 * w + lr) * XS + kc * 32 + 8 * lk]);
#pragma unroll
        for (int lt = 0; lt < LT; ++lt) {
          const v8bf ob = bf16x8(&sOm[(lt * 16 + lr) * XS + kc * 32 + 8 * lk]);
          acc[lt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, ob, acc[lt], 0, 0, 0);
        }
      }
    }
    if constexpr (UOUT) {
      // U rows of this tile: U = Y Theta_k (FP64 products of the FP32 Y)
#pragma unroll
      for (int lt = 0; lt < LT; ++lt)
#pragma unroll
        for (int v = 0; v < 4; ++v) sYf[(16 * w + f32_row(lane, v)) * YS + lt * 16 + lr] = acc[lt][v];
      __syncthreads();
      const int64_t rem = nrows - (int64_t)t * TM;
      const int nvalid = rem < TM ? (int)rem : TM;
      for (int e = tid; e < nvalid * a.R; e += 256) {
        const int row = e / a.R, r = e % a.R;
        double u = 0.0;
        for (int l = 0; l < L; ++l) u += (double)sYf[row * YS + l] * sTh[l * a.R + r];
        a.U[(size_t)(it.row0 + (int64_t)t * TM + row) * a.R + r] = u;
      }
      continue;
    }
    // column maxima: Y per wave (16 rows), X per row quarter (16 rows)
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) {
      float m = fmaxf(fmaxf(fabsf(acc[lt][0]), fabsf(acc[lt][1])), fmaxf(fabsf(acc[lt][2]), fabsf(acc[lt][3])));
      m = fmaxf(m, __shfl_xor(m, 16, 64));
      m = fmaxf(m, __shfl_xor(m, 32, 64));
      if (lk == 0) sYm[w * LP + lt * 16 + lr] = m;
    }
    // each thread keeps the 16 values of its column quarters for the digits
    constexpr int NXT = (JP * 4 + 255) / 256;
    float xv[NXT][16];
#pragma unroll
    for (int k = 0; k < NXT; ++k) {
      const int task = tid + 256 * k;
      if (task < JP * 4) {
        const int j = task % JP, q = task / JP;
        float m = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          xv[k][r] = sX[(16 * q + r) * XS + j];
          m = fmaxf(m, fabsf(xv[k][r]));
        }
        sXm[q * JP + j] = m;
      }
    }
    __syncthreads();
    // digits of Y (transposed planes: [digit][column][row byte])
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
        for (int v = 0; v < 4; ++v) acc[lt][v] *= pre;
      }
      int q[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) q[v] = q22b(acc[lt][v], sc);
      uint32_t p[3];
      digits4(q, p[0], p[1], p[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) sYq[(a * LP + col) * QW + 4 * w + lk] = p[a];
      if (w == 0 && lk == 0) sYe[col] = e;
    }
    // digits of X
#pragma unroll
    for (int k = 0; k < NXT; ++k) {
      const int task = tid + 256 * k;
      if (task < JP * 4) {
        const int j = task % JP, q = task / JP;
        const float m = fmaxf(fmaxf(sXm[j], sXm[JP + j]), fmaxf(sXm[2 * JP + j], sXm[3 * JP + j]));
        const int e = col_exp(m);
        float sc;
        const bool tiny = col_scale(e, sc);
        if (__builtin_amdgcn_ballot_w64(tiny)) {   // rare: taken only when a lane needs it
          const float pre = tiny ? 0x1p64f : 1.0f;
#pragma unroll
          for (int r = 0; r < 16; ++r) xv[k][r] *= pre;
        }
        uint32_t pk[3][4];
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          int qv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) qv[v] = q22b(xv[k][4 * r4 + v], sc);
          digits4(qv, pk[0][r4], pk[1][r4], pk[2][r4]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
          *reinterpret_cast<uint4*>(&sXq[(a * JP + j) * QW + 4 * q]) =
              make_uint4(pk[a][0], pk[a][1], pk[a][2], pk[a][3]);
        if (q == 0) sXe[j] = e;
      }
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
        pacc[qi] = digit_tile_fma(A, B, eb[cb + lr], sYe, ca, lane, pacc[qi]);
      }
    }
  }

  if constexpr (UOUT) return;
  double* Pp = a.partP + (size_t)blockIdx.x * L * J;
  double* Gp = a.partG + (size_t)blockIdx.x * L * L;
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
  if (tid == 0) a.partS[blockIdx.x] = ss;
}


// Launch for J <= 128 (JT <= 8); returns hipErrorInvalidValue otherwise.
// SPL: see k_sketch_q (float32 slabs always split Omega; bf16 / fp8 slabs in
// the passes of a power step).
template <int TIN, bool UOUT, bool SPL>
hipError_t slab_launch(const SlabArgs& a, int64_t n_items, bool vec, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const int lt = a.L <= 16 ? 1 : 2;
  const int jt0 = (a.J + 15) / 16;
  const int jt = jt0 <= 4 ? jt0 : (jt0 <= 6 ? 6 : (jt0 <= 8 ? 8 : -1));
  dim3 grid((unsigned)n_items), block(256);
#define DPAR2_SQ(LT_, JT_)                                                                          \
  if (lt == LT_ && jt == JT_) {                                                                     \
    if (vec)                                                                                        \
      hipLaunchKernelGGL((k_sketch_q<LT_, JT_, true, TIN, UOUT, SPL>), grid, block, 0, s, a);       \
    else                                                                                            \
      hipLaunchKernelGGL((k_sketch_q<LT_, JT_, false, TIN, UOUT, SPL>), grid, block, 0, s, a);      \
    return hipGetLastError();                                                                       \
  }
  DPAR2_SQ(1, 1) DPAR2_SQ(1, 2) DPAR2_SQ(1, 3) DPAR2_SQ(1, 4) DPAR2_SQ(1, 6) DPAR2_SQ(1, 8)
  DPAR2_SQ(2, 1) DPAR2_SQ(2, 2) DPAR2_SQ(2, 3) DPAR2_SQ(2, 4) DPAR2_SQ(2, 6) DPAR2_SQ(2, 8)
#undef DPAR2_SQ
  return hipErrorInvalidValue;
}

}  // namespace dpar2
