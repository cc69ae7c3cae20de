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

// partial Y2 over one chunk of rows of M^T (all of one tensor):
// Y2p[c][j][l] = sum_rows Mt[row][j] * Omega2[row][l]
__global__ __launch_bounds__(256) void k_s2_y(int J, int L2, int R, const TDesc* __restrict__ td,
                                              const Chunk* __restrict__ chunks, const double* __restrict__ Mt,
                                              double* __restrict__ Y2p) {
  __shared__ double sM[64 * 64];
  __shared__ float sO[64 * 32];
  const int c = blockIdx.x, jb = blockIdx.y, tid = threadIdx.x;
  const int jl = tid & 63, l0 = tid >> 6;
  const int j = jb * 64 + jl;
  double acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  const Chunk ch = chunks[c];
  const int64_t r0 = ch.r0, r1 = ch.r1;
  // Omega_2 of the chunk's tensor, indexed by its local row of M^T
  const float* __restrict__ om2 = td[ch.t].om2 - (size_t)td[ch.t].k0 * R * L2;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)((r1 - rb) < 64 ? (r1 - rb) : 64);
    __syncthreads();
    // staging loads are unrolled with clamped indices so they issue together
    {
      double mv[16];
      float ov[8];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, rr = e / 64, jj = e % 64;
        const bool ok = rr < nr && jb * 64 + jj < J;
        const double x = Mt[ok ? (size_t)(rb + rr) * J + jb * 64 + jj : 0];
        mv[u] = ok ? x : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u, rr = e / 32, ll = e % 32;
        const bool ok = rr < nr && ll < L2;
        const float x = om2[(ok ? (size_t)(rb + rr) : (size_t)r0) * L2 + (ok ? ll : 0)];
        ov[u] = ok ? x : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) sM[tid + 256 * u] = mv[u];
#pragma unroll
      for (int u = 0; u < 8; ++u) sO[tid + 256 * u] = ov[u];
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const double m = sM[rr * 64 + jl];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += (double)sO[rr * 32 + l0 + 4 * q] * m;
    }
  }
  if (j < J)
    for (int q = 0; q < 8; ++q) {
      const int l = l0 + 4 * q;
      if (l < L2) Y2p[((size_t)c * J + j) * L2 + l] = acc[q];
    }
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
// chunk's tensor), plus the chunk's partial of B2 B2^T.
__global__ __launch_bounds__(256) void k_s2_b(int J, int L2, const Chunk* __restrict__ chunks,
                                              const double* __restrict__ Mt, const double* __restrict__ Q2all,
                                              double* __restrict__ B2t, double* __restrict__ S2p) {
  __shared__ double sM[64 * 65];
  __shared__ double sQ[64 * 32];
  __shared__ double sB[64 * 33];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int rl = tid >> 2, lg = tid & 3;
  const int npairs = L2 * (L2 + 1) / 2;
  double sacc[3] = {0.0, 0.0, 0.0};
  const Chunk ch = chunks[c];
  const int64_t r0 = ch.r0, r1 = ch.r1;
  const double* __restrict__ Q2 = Q2all + (size_t)ch.t * J * L2;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)((r1 - rb) < 64 ? (r1 - rb) : 64);
    double acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int jc = 0; jc < J; jc += 64) {
      __syncthreads();
      {
        double mv[16], qv[8];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = tid + 256 * u, rr = e / 64, jj = e % 64;
          const bool ok = rr < nr && jc + jj < J;
          const double x = Mt[ok ? (size_t)(rb + rr) * J + jc + jj : 0];
          mv[u] = ok ? x : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = tid + 256 * u, jj = e / 32, ll = e % 32;
          const bool ok = jc + jj < J && ll < L2;
          const double x = Q2[ok ? (size_t)(jc + jj) * L2 + ll : 0];
          qv[u] = ok ? x : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = tid + 256 * u;
          sM[(e / 64) * 65 + e % 64] = mv[u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) sQ[tid + 256 * u] = qv[u];
      }
      __syncthreads();
      for (int jj = 0; jj < 64; ++jj) {
        const double m = sM[rl * 65 + jj];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] += m * sQ[jj * 32 + lg + 4 * q];
      }
    }
    __syncthreads();
    for (int q = 0; q < 8; ++q) {
      const int l = lg + 4 * q;
      if (l < L2) {
        sB[rl * 33 + l] = (rl < nr) ? acc[q] : 0.0;
        if (rl < nr) B2t[(size_t)(rb + rl) * L2 + l] = acc[q];
      }
    }
    __syncthreads();
    for (int q = 0; q < 3; ++q) {
      const int pi = tid + 256 * q;
      if (pi < npairs) {
        int a = 0, rem = pi;
        while (rem >= L2 - a) { rem -= L2 - a; ++a; }
        const int b = a + rem;
        double s = 0.0;
        for (int rr = 0; rr < nr; ++rr) s += sB[rr * 33 + a] * sB[rr * 33 + b];
        sacc[q] += s;
      }
    }
  }
  for (int q = 0; q < 3; ++q) {
    const int pi = tid + 256 * q;
    if (pi < npairs) S2p[(size_t)c * npairs + pi] = sacc[q];
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
                               double* D, double* E, double* U2s, double* small, Ctl* ctl, hipStream_t s);
hipError_t s2_small_dispatch_2(int nt, int L2, int which, int J, int R, double* Y2, const double* S2,
                               double* D, double* E, double* U2s, double* small, Ctl* ctl, hipStream_t s);

// orthonormalisation of Y2 (which = 0) or the small SVD and D, E (which = 1),
// one block per tensor
static hipError_t s2_small(int nt, int L2, int which, int J, int R, double* Y2, const double* S2, double* D,
                           double* E, double* U2s, double* small, Ctl* ctl, hipStream_t s) {
  if (L2 <= 16) return s2_small_dispatch_1(nt, L2, which, J, R, Y2, S2, D, E, U2s, small, ctl, s);
  return s2_small_dispatch_2(nt, L2, which, J, R, Y2, S2, D, E, U2s, small, ctl, s);
}

// F = B2^T (U2_R E^{-1}) over one chunk (U2 of the chunk's tensor) and the
// chunk's partial of F^T F.
__global__ __launch_bounds__(256) void k_s2_f(int L2, int R, const Chunk* __restrict__ chunks,
                                              const double* __restrict__ B2t, const double* __restrict__ U2all,
                                              double* __restrict__ F, double* __restrict__ FtFp) {
  __shared__ double sU[32 * 32];
  __shared__ double sF[256 * 33];
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
    sF[tid * 33 + r] = s;
    if (ok) F[(size_t)row * R + r] = s;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += sF[i * 33 + a] * sF[i * 33 + b];
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
  const int64_t* seg_chunk = reinterpret_cast<const int64_t*>(ws + lay.seg_chunk);
  const int64_t* seg_slice = reinterpret_cast<const int64_t*>(ws + lay.seg_slice);
  double* Mt = reinterpret_cast<double*>(ws + lay.Mt);
  double* Y2p = reinterpret_cast<double*>(ws + lay.Y2p);
  double* Y2 = reinterpret_cast<double*>(ws + lay.Y2);
  double* B2t = reinterpret_cast<double*>(ws + lay.B2t);
  double* S2p = reinterpret_cast<double*>(ws + lay.S2p);
  double* S2 = reinterpret_cast<double*>(ws + lay.S2);
  double* U2s = reinterpret_cast<double*>(ws + lay.U2);
  double* D = reinterpret_cast<double*>(ws + lay.D);
  double* E = reinterpret_cast<double*>(ws + lay.E);
  double* F = reinterpret_cast<double*>(ws + lay.F);
  double* FtFp = reinterpret_cast<double*>(ws + lay.FtFp);
  double* small = reinterpret_cast<double*>(ws + lay.small);
  const double* xnorm2 = reinterpret_cast<const double*>(ws + lay.xnorm2);
  const int RR = R * R, npairs = L2 * (L2 + 1) / 2;
  const int64_t cstride = sizeof(Ctl) / sizeof(double);
  hipError_t e;
  hipLaunchKernelGGL(k_s2_y, dim3((unsigned)lay.n2, (unsigned)((J + 63) / 64)), dim3(256), 0, s, J, L2, R,
                     td, chunks, Mt, Y2p);
  if ((e = launch_segsum(nt, seg_chunk, lay.n2, (int64_t)J * L2, (int64_t)J * L2, Y2p, Y2, (int64_t)J * L2, s)) !=
      hipSuccess)
    return e;
  if ((e = s2_small(nt, L2, 0, J, R, Y2, nullptr, D, E, U2s, small, ctl, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_s2_b, dim3((unsigned)lay.n2), dim3(256), 0, s, J, L2, chunks, Mt, Y2, B2t, S2p);
  if ((e = launch_segsum(nt, seg_chunk, lay.n2, npairs, npairs, S2p, S2, npairs, s)) != hipSuccess) return e;
  // sum_k ||X_k||^2 of each tensor into its control block
  if ((e = launch_segsum(nt, seg_slice, lay.K, 1, 1, xnorm2, &ctl->xnorm2, cstride, s)) != hipSuccess) return e;
  if ((e = s2_small(nt, L2, 1, J, R, Y2, S2, D, E, U2s, small, ctl, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_s2_f, dim3((unsigned)lay.n2), dim3(256), 0, s, L2, R, chunks, B2t, U2s, F, FtFp);
  if ((e = launch_segsum(nt, seg_chunk, lay.n2, RR, RR, FtFp, small + SM_FTF * RR, (int64_t)SM_COUNT * RR, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_s2_final, dim3((unsigned)nt), dim3(64), 0, s, R, small, E, ctl);
  return hipGetLastError();
}

}  // namespace dpar2
