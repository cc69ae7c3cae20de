// Second-stage compression (Sec. III-B, Eq. 5): randomized SVD (Alg. 1) of
// M = ||_k C_k B_k (J x KR), held transposed as M^T (KR x J, FP64):
//   Y2 = M Omega_2                      (J x L2)
//   Q2 = orthonormal basis of span(Y2)  (QR step of Alg. 1; FP64, stage2_impl.h)
//   B2 = Q2^T M                         (L2 x KR, stored as B2^T)
//   B2 B2^T = U2 Lambda U2^T            (small SVD of Alg. 1, stage2_impl.h)
//   D = Q2 U2_R,  E = sqrt(Lambda_R),  F = B2^T U2_R E^{-1}   (KR x R)
// and the constant part e0 = sum_k ||F^(k) E D^T||_F^2 of the iteration error.
#include "internal.h"

namespace dpar2 {

// Omega_2 as FP64, one row of L2 values per row of M^T (global row order),
// into `dst` (the B2t buffer, free until the projection writes it)
__global__ __launch_bounds__(256) void k_om2d(int L2, int R, int64_t rows, const TDesc* __restrict__ td,
                                              const int32_t* __restrict__ slice_t, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * L2) return;
  const int64_t row = e / L2;
  const TDesc& d = td[slice_t[row / R]];
  dst[e] = (double)d.om2[(row - (int64_t)d.k0 * R) * L2 + e % L2];
}

// partial Y2 over one chunk of rows of M^T (all of one tensor), one wave
// per 64 columns, one lane per column j (each row of M^T read once,
// coalesced), the chunk's rows of Omega_2 (FP64) through scalar loads, the
// rows in order: Y2p[c][j][l] = sum_rows Mt[row][j] Omega2[row][l]
template <int L2>
__global__ __launch_bounds__(64) void k_s2_y(int J, const Chunk* __restrict__ ychunks, const double* __restrict__ Mt,
                                             const double* __restrict__ om2d, double* __restrict__ Y2p) {
  const int c = blockIdx.x;
  const int j = blockIdx.y * 64 + threadIdx.x;
  const Chunk ch = ychunks[c];
  const int jc = j < J ? j : 0;   // lanes past J read column 0 and store nothing
  double acc[L2];
#pragma unroll
  for (int l = 0; l < L2; ++l) acc[l] = 0.0;
  const double* __restrict__ mp = Mt + jc;
  int64_t r = ch.r0;
  for (; r + 8 <= ch.r1; r += 8) {
    double m[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m[u] = mp[(size_t)(r + u) * J];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* __restrict__ o = om2d + (size_t)(r + u) * L2;
#pragma unroll
      for (int l = 0; l < L2; ++l) acc[l] = fma(m[u], o[l], acc[l]);
    }
  }
  for (; r < ch.r1; ++r) {
    const double m = mp[(size_t)r * J];
    const double* __restrict__ o = om2d + (size_t)r * L2;
#pragma unroll
    for (int l = 0; l < L2; ++l) acc[l] = fma(m, o[l], acc[l]);
  }
  if (j < J) {
    double* __restrict__ out = Y2p + ((size_t)c * J + j) * L2;
#pragma unroll
    for (int l = 0; l < L2; ++l) out[l] = acc[l];
  }
}

// out[t * ostride + e] = sum over b of part[b * stride + e], b over [0, n1)
// (n1 >= 0) or over [seg[t], seg[t+1]): one thread per e (the partials of
// consecutive e are read together), the b in order into eight accumulators
// (b mod 8) combined pairwise.  For wide sums over few partials.
__global__ __launch_bounds__(256) void k_colsum(const int64_t* __restrict__ seg, int64_t n1, int64_t stride,
                                                int64_t width, const double* __restrict__ part,
                                                double* __restrict__ out, int64_t ostride) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y;
  if (e >= width) return;
  const int64_t b0 = n1 >= 0 ? 0 : seg[t], nb = n1 >= 0 ? n1 : seg[t + 1] - b0;
  const double* __restrict__ p = part + (size_t)b0 * stride + e;
  double sv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) sv[u] = 0.0;
  int64_t b = 0;
  for (; b + 8 <= nb; b += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) sv[u] += p[(size_t)(b + u) * stride];
  }
  for (int u = 0; b < nb; ++b, ++u) sv[u] += p[(size_t)b * stride];
  out[(size_t)t * ostride + e] = ((sv[0] + sv[1]) + (sv[2] + sv[3])) + ((sv[4] + sv[5]) + (sv[6] + sv[7]));
}

// out[t * ostride + e] = sum over b in [seg[t], seg[t+1]) of part[b * stride + e]:
// one block per (e, t); the threads split b (four independent accumulators
// each) and combine in a fixed order.
__global__ __launch_bounds__(256) void k_segsum(const int64_t* __restrict__ seg, int64_t n1, int64_t stride,
                                                const double* __restrict__ part, double* __restrict__ out,
                                                int64_t ostride) {
  __shared__ double red[16];
  const int64_t e = blockIdx.x;
  const int t = blockIdx.y, tid = threadIdx.x;
  const int64_t b0 = n1 >= 0 ? 0 : seg[t], nb = n1 >= 0 ? n1 : seg[t + 1] - b0;
  const double* p = part + (size_t)b0 * stride + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t q = tid;
  for (; q + 768 < nb; q += 1024) {
    s0 += p[(size_t)q * stride];
    s1 += p[(size_t)(q + 256) * stride];
    s2 += p[(size_t)(q + 512) * stride];
    s3 += p[(size_t)(q + 768) * stride];
  }
  for (; q < nb; q += 256) s0 += p[(size_t)q * stride];
  const double x = block_sum((s0 + s1) + (s2 + s3), red);
  if (tid == 0) out[(size_t)t * ostride + e] = x;
}

// B2^T rows of one chunk: B2t[row][l] = sum_j Mt[row][j] Q2[j][l] (Q2 of the
// chunk's tensor, FP64 J x L2, its rows through scalar loads), one lane per
// row of M^T, j in order; then the chunk's partial of B2 B2^T (upper
// triangle, pairs a <= b row-major), its rows through LDS 64 at a time.
template <int L2>
__global__ __launch_bounds__(256) void k_s2_b(int J, const Chunk* __restrict__ chunks, const double* __restrict__ Mt,
                                              const double* __restrict__ Q2all, double* __restrict__ B2t,
                                              double* __restrict__ S2p) {
  constexpr int LP = L2 + 1, NPAIR = L2 * (L2 + 1) / 2, NQ = (NPAIR + 255) / 256;
  __shared__ double sB[64 * LP];
  const int tid = threadIdx.x;
  const Chunk ch = chunks[blockIdx.x];
  const int64_t row = ch.r0 + tid;
  const bool ok = row < ch.r1;
  const double* __restrict__ mrow = Mt + (size_t)(ok ? row : ch.r0) * J;
  const double* __restrict__ Q2 = Q2all + (size_t)ch.t * J * L2;
  double acc[L2];
#pragma unroll
  for (int l = 0; l < L2; ++l) acc[l] = 0.0;
  int j = 0;
  for (; j + 8 <= J; j += 8) {
    double m[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m[u] = mrow[j + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* __restrict__ q = Q2 + (size_t)(j + u) * L2;
#pragma unroll
      for (int l = 0; l < L2; ++l) acc[l] = fma(m[u], q[l], acc[l]);
    }
  }
  for (; j < J; ++j) {
    const double m = mrow[j];
    const double* __restrict__ q = Q2 + (size_t)j * L2;
#pragma unroll
    for (int l = 0; l < L2; ++l) acc[l] = fma(m, q[l], acc[l]);
  }
  if (ok) {
#pragma unroll
    for (int l = 0; l < L2; ++l) B2t[(size_t)row * L2 + l] = acc[l];
  }
  // pair indices of this thread
  int pa[NQ], pb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    int pi = tid + 256 * q, a = 0;
    if (pi >= NPAIR) pi = 0;
    while (pi >= L2 - a) {
      pi -= L2 - a;
      ++a;
    }
    pa[q] = a;
    pb[q] = a + pi;
  }
  double sacc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) sacc[q] = 0.0;
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if ((tid >> 6) == w) {
#pragma unroll
      for (int l = 0; l < L2; ++l) sB[(tid & 63) * LP + l] = ok ? acc[l] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int rr = 0; rr < 64; ++rr) s = fma(sB[rr * LP + pa[q]], sB[rr * LP + pb[q]], s);
      sacc[q] += s;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int pi = tid + 256 * q;
    if (pi < NPAIR) S2p[(size_t)blockIdx.x * NPAIR + pi] = sacc[q];
  }
}

// launches of k_s2_y and k_s2_b for the group's L2
static hipError_t s2_stream_launch(int which, int L2, int J, int64_t nchunks, const Chunk* chunks,
                                   const double* Mt, const double* aux, double* out1, double* out2, hipStream_t s) {
  switch (L2) {
#define DPAR2_S2(N_)                                                                                          \
  case N_:                                                                                                    \
    if (which == 0)                                                                                           \
      hipLaunchKernelGGL(k_s2_y<N_>, dim3((unsigned)nchunks, (unsigned)((J + 63) / 64)), dim3(64), 0, s,    \
                         J, chunks, Mt, aux, out1);                                                           \
    else                                                                                                      \
      hipLaunchKernelGGL(k_s2_b<N_>, dim3((unsigned)nchunks), dim3(256), 0, s, J, chunks, Mt, aux, out1,    \
                         out2);                                                                               \
    return hipGetLastError();
    DPAR2_S2(1) DPAR2_S2(2) DPAR2_S2(3) DPAR2_S2(4) DPAR2_S2(5) DPAR2_S2(6) DPAR2_S2(7) DPAR2_S2(8)
    DPAR2_S2(9) DPAR2_S2(10) DPAR2_S2(11) DPAR2_S2(12) DPAR2_S2(13) DPAR2_S2(14) DPAR2_S2(15) DPAR2_S2(16)
    DPAR2_S2(17) DPAR2_S2(18) DPAR2_S2(19) DPAR2_S2(20) DPAR2_S2(21) DPAR2_S2(22) DPAR2_S2(23) DPAR2_S2(24)
    DPAR2_S2(25) DPAR2_S2(26) DPAR2_S2(27) DPAR2_S2(28) DPAR2_S2(29) DPAR2_S2(30) DPAR2_S2(31) DPAR2_S2(32)
    DPAR2_S2(40) DPAR2_S2(50) DPAR2_S2(60)
#undef DPAR2_S2
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_segsum(int nt, const int64_t* seg, int64_t n1, int64_t stride, int64_t width,
                         const double* part, double* out, int64_t ostride, hipStream_t s) {
  if (width <= 0 || nt <= 0) return hipSuccess;
  if (nt != 1) n1 = -1;
  hipLaunchKernelGGL(k_segsum, dim3((unsigned)width, (unsigned)nt), dim3(256), 0, s, seg, n1, stride, part, out,
                     ostride);
  return hipGetLastError();
}

hipError_t s2_small_dispatch_1(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                               double* D, double* E, double* U2s, double* small, Ctl* ctl, double* scratch,
                               hipStream_t s);
hipError_t s2_small_dispatch_2(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                               double* D, double* E, double* U2s, double* small, Ctl* ctl, double* scratch,
                               hipStream_t s);
hipError_t s2_small_dispatch_3(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                               double* D, double* E, double* U2s, double* small, Ctl* ctl, double* scratch,
                               hipStream_t s);

// orthonormalisation of Y2 (which = 0) or the small SVD and D, E (which = 1),
// one block per tensor
static hipError_t s2_small(int nt, int L2, int which, int J, int R, double* Y2, const double* S2, double* D,
                           double* E, double* U2s, double* small, Ctl* ctl, double* scratch, hipStream_t s) {
  if (L2 <= 16) return s2_small_dispatch_1(nt, L2, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
  if (L2 <= 32) return s2_small_dispatch_2(nt, L2, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
  return s2_small_dispatch_3(nt, L2, which, J, R, Y2, S2, D, E, U2s, small, ctl, scratch, s);
}

// F = B2^T (U2_R E^{-1}) over one chunk (U2 of the chunk's tensor) and the
// chunk's partial of F^T F.  BIG: L2 up to 60 and R up to 50, else both up to
// 32.
template <bool BIG>
__global__ __launch_bounds__(256) void k_s2_f(int L2, int R, const Chunk* __restrict__ chunks,
                                              const double* __restrict__ B2t, const double* __restrict__ U2all,
                                              double* __restrict__ F, double* __restrict__ FtFp) {
  constexpr int LDF = BIG ? 51 : 33;
  __shared__ double sU[BIG ? 60 * 50 : 32 * 32];
  __shared__ double sF[256 * LDF];
  const int tid = threadIdx.x;
  const Chunk ch = chunks[blockIdx.x];
  const double* U2s = U2all + (size_t)ch.t * L2 * R;
  for (int e = tid; e < L2 * R; e += 256) sU[e] = U2s[e];
  __syncthreads();
  const int64_t row = ch.r0 + tid;
  const bool ok = row < ch.r1;
  for (int r = 0; r < R; ++r) {
    double s = 0.0;
    if (ok)
      for (int l = 0; l < L2; ++l) s += B2t[(size_t)row * L2 + l] * sU[l * R + r];
    sF[tid * LDF + r] = s;
    if (ok) F[(size_t)row * R + r] = s;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += sF[i * LDF + a] * sF[i * LDF + b];
    FtFp[(size_t)blockIdx.x * R * R + e] = s;
  }
}

// e0 = sum_{r,s} E_r E_s (F^T F)_{rs} (D^T D)_{rs} (Sec. III-E constant term),
// one block per tensor
__global__ __launch_bounds__(64) void k_s2_final(int R, const double* __restrict__ small,
                                                 const double* __restrict__ Eall, Ctl* ctlall) {
  const int lane = threadIdx.x, t = blockIdx.x, RR = R * R;
  const double* FtF = small + (size_t)t * SM_COUNT * RR + SM_FTF * RR;
  const double* DtD = small + (size_t)t * SM_COUNT * RR + SM_DTD * RR;
  const double* E = Eall + (size_t)t * R;
  Ctl* ctl = ctlall + t;
  double e0 = 0.0;
  for (int e = lane; e < R * R; e += 64) {
    const int a = e / R, c = e % R;
    e0 += E[a] * E[c] * FtF[e] * DtD[e];
  }
  for (int o = 1; o < 64; o <<= 1) e0 += __shfl_xor(e0, o, 64);
  if (lane == 0) {
    ctl->e0 = e0;
    // a NaN or Inf anywhere in the slab makes sum_k ||X_k||^2 non-finite
    // (squares of finite float32 values cannot overflow in FP64): flag the
    // tensor and skip its iteration
    if (!isfinite(ctl->xnorm2)) {
      ctl->bad = 1;
      ctl->done = 1;
      ctl->warn |= 0x4u;
    }
  }
}

hipError_t launch_stage2(const Layout& lay, char* ws, hipStream_t s) {
  const int J = (int)lay.J, L2 = lay.L2, R = lay.R, nt = lay.nt;
  Ctl* ctl = reinterpret_cast<Ctl*>(ws + lay.ctl);
  const TDesc* td = reinterpret_cast<const TDesc*>(ws + lay.tdesc);
  const Chunk* chunks = reinterpret_cast<const Chunk*>(ws + lay.chunks);
  const Chunk* ychunks = reinterpret_cast<const Chunk*>(ws + lay.ychunks);
  const int64_t* seg_ychunk = reinterpret_cast<const int64_t*>(ws + lay.seg_ychunk);
  const int32_t* slice_t = reinterpret_cast<const int32_t*>(ws + lay.slice_t);
  const int64_t* seg_chunk = reinterpret_cast<const int64_t*>(ws + lay.seg_chunk);
  const int64_t* seg_slice = reinterpret_cast<const int64_t*>(ws + lay.seg_slice);
  double* Mt = reinterpret_cast<double*>(ws + lay.Mt);
  double* Y2p = reinterpret_cast<double*>(ws + lay.Y2p);
  double* Y2 = reinterpret_cast<double*>(ws + lay.Y2);
  double* B2t = reinterpret_cast<double*>(ws + lay.B2t);
  double* S2p = reinterpret_cast<double*>(ws + lay.S2p);
  double* S2 = reinterpret_cast<double*>(ws + lay.S2);
  double* U2s = reinterpret_cast<double*>(ws + lay.U2);
  double* s2s = reinterpret_cast<double*>(ws + lay.s2s);
  double* D = reinterpret_cast<double*>(ws + lay.D);
  double* E = reinterpret_cast<double*>(ws + lay.E);
  double* F = reinterpret_cast<double*>(ws + lay.F);
  double* FtFp = reinterpret_cast<double*>(ws + lay.FtFp);
  double* small = reinterpret_cast<double*>(ws + lay.small);
  const double* xnorm2 = reinterpret_cast<const double*>(ws + lay.xnorm2);
  const int RR = R * R, npairs = L2 * (L2 + 1) / 2;
  const int64_t cstride = sizeof(Ctl) / sizeof(double);
  hipError_t e;
  // Omega_2 in FP64 (in the B2t buffer until the projection), Y2 = M Omega_2
  // per chunk, summed per tensor
  const int64_t KR = lay.K * R;
  hipLaunchKernelGGL(k_om2d, dim3((unsigned)((KR * L2 + 255) / 256)), dim3(256), 0, s, L2, R, KR, td, slice_t, B2t);
  if ((e = s2_stream_launch(0, L2, J, lay.n2y, ychunks, Mt, B2t, Y2p, nullptr, s)) != hipSuccess) return e;
  {
    // wide Y2: one thread per entry over the partials; narrow: one block per
    // entry, its threads over the partials
    const int64_t width = (int64_t)J * L2;
    if (width >= 8192)
      hipLaunchKernelGGL(k_colsum, dim3((unsigned)((width + 255) / 256), (unsigned)nt), dim3(256), 0, s, seg_ychunk,
                         nt == 1 ? lay.n2y : (int64_t)-1, width, width, Y2p, Y2, width);
    else if ((e = launch_segsum(nt, seg_ychunk, lay.n2y, width, width, Y2p, Y2, width, s)) != hipSuccess)
      return e;
  }
  if ((e = s2_small(nt, L2, 0, J, R, Y2, nullptr, D, E, U2s, small, ctl, s2s, s)) != hipSuccess) return e;
  if ((e = s2_stream_launch(1, L2, J, lay.n2, chunks, Mt, Y2, B2t, S2p, s)) != hipSuccess) return e;
  if ((e = launch_segsum(nt, seg_chunk, lay.n2, npairs, npairs, S2p, S2, npairs, s)) != hipSuccess) return e;
  // sum_k ||X_k||^2 of each tensor into its control block
  if ((e = launch_segsum(nt, seg_slice, lay.K, 1, 1, xnorm2, &ctl->xnorm2, cstride, s)) != hipSuccess) return e;
  if ((e = s2_small(nt, L2, 1, J, R, Y2, S2, D, E, U2s, small, ctl, s2s, s)) != hipSuccess) return e;
  if (L2 > 32)
    hipLaunchKernelGGL(k_s2_f<true>, dim3((unsigned)lay.n2), dim3(256), 0, s, L2, R, chunks, B2t, U2s, F, FtFp);
  else
    hipLaunchKernelGGL(k_s2_f<false>, dim3((unsigned)lay.n2), dim3(256), 0, s, L2, R, chunks, B2t, U2s, F, FtFp);
  if ((e = launch_segsum(nt, seg_chunk, lay.n2, RR, RR, FtFp, small + SM_FTF * RR, (int64_t)SM_COUNT * RR, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_s2_final, dim3((unsigned)nt), dim3(64), 0, s, R, small, E, ctl);
  return hipGetLastError();
}

}  // namespace dpar2
