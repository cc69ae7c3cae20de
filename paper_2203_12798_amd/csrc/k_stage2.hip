// Second-stage compression (Sec. III-B, Eq. 5): randomized SVD (Alg. 1) of
// M = ||_k C_k B_k (J x KR), held transposed as M^T (KR x J, FP64):
//   Y2 = M Omega_2                      (J x L2)
//   Q2 = orthonormal basis of span(Y2)  (QR step of Alg. 1; FP64)
//   B2 = Q2^T M                         (L2 x KR, stored as B2^T)
//   B2 B2^T = U2 Lambda U2^T            (small SVD of Alg. 1)
//   D = Q2 U2_R,  E = sqrt(Lambda_R),  F = B2^T U2_R E^{-1}   (KR x R)
// and the constant part e0 = sum_k ||F^(k) E D^T||_F^2 of the iteration error.
#include "internal.h"

namespace dpar2 {

// partial Y2^T over a chunk of STAGE2_CHUNK rows of M^T:
// Y2p[c][l][j] = sum_rows Omega2[row][l] * Mt[row][j]
__global__ __launch_bounds__(256) void k_s2_y(int64_t KR, int J, int L2, const float* __restrict__ om2,
                                              const double* __restrict__ Mt, double* __restrict__ Y2p) {
  __shared__ double sM[64 * 64];
  __shared__ float sO[64 * 32];
  const int c = blockIdx.x, jb = blockIdx.y, tid = threadIdx.x;
  const int jl = tid & 63, l0 = tid >> 6;
  const int j = jb * 64 + jl;
  double acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  const int64_t r0 = (int64_t)c * STAGE2_CHUNK;
  const int64_t r1 = (r0 + STAGE2_CHUNK < KR) ? r0 + STAGE2_CHUNK : KR;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)((r1 - rb) < 64 ? (r1 - rb) : 64);
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
      const int rr = e / 64, jj = e % 64;
      sM[e] = (rr < nr && jb * 64 + jj < J) ? Mt[(size_t)(rb + rr) * J + jb * 64 + jj] : 0.0;
    }
    for (int e = tid; e < 64 * 32; e += 256) {
      const int rr = e / 32, ll = e % 32;
      sO[e] = (rr < nr && ll < L2) ? om2[(size_t)(rb + rr) * L2 + ll] : 0.f;
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
      if (l < L2) Y2p[((size_t)c * L2 + l) * J + j] = acc[q];
    }
}

// Y2[j][l] = sum_c Y2p[c][l][j]
__global__ void k_s2_y_reduce(int64_t n2, int J, int L2, const double* __restrict__ Y2p,
                              double* __restrict__ Y2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * L2) return;
  const int j = e / L2, l = e % L2;
  double s = 0.0;
  for (int64_t c = 0; c < n2; ++c) s += Y2p[((size_t)c * L2 + l) * J + j];
  Y2[e] = s;
}

// Orthonormal basis of span(Y2) in place (Y2 <- Q2), by two whitening passes
// (eigen-based CholeskyQR2: the second pass restores orthogonality to FP64
// rounding; dropped directions become zero columns).
__global__ __launch_bounds__(256) void k_s2_cqr2(int J, int L2, double* __restrict__ Y, Ctl* ctl) {
  constexpr int LD = 33;
  __shared__ double G[32 * LD], Wh[32 * LD], V[32 * LD], cs[40];
  const int tid = threadIdx.x;
  const int npairs = L2 * (L2 + 1) / 2;
  int capped = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int pi = tid; pi < npairs; pi += 256) {
      int a = 0, rem = pi;
      while (rem >= L2 - a) { rem -= L2 - a; ++a; }
      const int b = a + rem;
      double s = 0.0;
      for (int j = 0; j < J; ++j) s += Y[(size_t)j * L2 + a] * Y[(size_t)j * L2 + b];
      G[a * LD + b] = s;
      G[b * LD + a] = s;
    }
    __syncthreads();
    capped |= block_whiten(G, LD, L2, Wh, V, cs);
    for (int j = tid; j < J; j += 256) {
      double y[32];
      for (int l = 0; l < L2; ++l) y[l] = Y[(size_t)j * L2 + l];
      for (int b = 0; b < L2; ++b) {
        double v = 0.0;
        for (int a = 0; a < L2; ++a) v += y[a] * Wh[a * LD + b];
        Y[(size_t)j * L2 + b] = v;
      }
    }
    __syncthreads();
  }
  if (tid == 0 && capped) atomicOr(&ctl->warn, 0x1u);
}

// B2^T rows of one chunk: B2t[row][l] = sum_j Mt[row][j] Q2[j][l], plus the
// chunk's partial of B2 B2^T.
__global__ __launch_bounds__(256) void k_s2_b(int64_t KR, int J, int L2, const double* __restrict__ Mt,
                                              const double* __restrict__ Q2, double* __restrict__ B2t,
                                              double* __restrict__ S2p) {
  __shared__ double sM[64 * 65];
  __shared__ double sQ[64 * 32];
  __shared__ double sB[64 * 33];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int rl = tid >> 2, lg = tid & 3;
  const int npairs = L2 * (L2 + 1) / 2;
  double sacc[3] = {0.0, 0.0, 0.0};
  const int64_t r0 = (int64_t)c * STAGE2_CHUNK;
  const int64_t r1 = (r0 + STAGE2_CHUNK < KR) ? r0 + STAGE2_CHUNK : KR;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)((r1 - rb) < 64 ? (r1 - rb) : 64);
    double acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int jc = 0; jc < J; jc += 64) {
      __syncthreads();
      for (int e = tid; e < 64 * 64; e += 256) {
        const int rr = e / 64, jj = e % 64;
        sM[rr * 65 + jj] = (rr < nr && jc + jj < J) ? Mt[(size_t)(rb + rr) * J + jc + jj] : 0.0;
      }
      for (int e = tid; e < 64 * 32; e += 256) {
        const int jj = e / 32, ll = e % 32;
        sQ[e] = (jc + jj < J && ll < L2) ? Q2[(size_t)(jc + jj) * L2 + ll] : 0.0;
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

// EVD of B2 B2^T, then D, E, the L2 x R map U2_R E^{-1}, D^T D, and the
// total ||X||^2.
__global__ __launch_bounds__(256) void k_s2_evd(int64_t n2, int64_t K, int J, int L2, int R,
                                                const double* __restrict__ S2p, const double* __restrict__ Q2,
                                                const double* __restrict__ xnorm2, double* __restrict__ D,
                                                double* __restrict__ E, double* __restrict__ U2s,
                                                double* __restrict__ DtD, Ctl* ctl) {
  constexpr int LD = 33;
  __shared__ double S[32 * LD], U[32 * LD], cs[40], red[16], sD[1];
  __shared__ int perm[32];
  const int tid = threadIdx.x;
  const int npairs = L2 * (L2 + 1) / 2;
  for (int pi = tid; pi < npairs; pi += 256) {
    int a = 0, rem = pi;
    while (rem >= L2 - a) { rem -= L2 - a; ++a; }
    const int b = a + rem;
    double s = 0.0;
    for (int64_t c = 0; c < n2; ++c) s += S2p[(size_t)c * npairs + pi];
    S[a * LD + b] = s;
    S[b * LD + a] = s;
  }
  double xs = 0.0;
  for (int64_t k = tid; k < K; k += 256) xs += xnorm2[k];
  xs = block_sum(xs, red);
  if (tid == 0) ctl->xnorm2 = xs;
  __syncthreads();
  const int capped = block_sym_evd(S, LD, U, L2, cs);
  block_sort_desc(S, LD, L2, perm);
  if (tid < R) {
    const double lam = S[perm[tid] * LD + perm[tid]];
    E[tid] = sqrt(lam > 0.0 ? lam : 0.0);
  }
  __syncthreads();
  for (int e = tid; e < L2 * R; e += 256) {
    const int l = e / R, r = e % R;
    const double er = E[r];
    U2s[e] = er > 0.0 ? U[l * LD + perm[r]] / er : 0.0;
  }
  for (int e = tid; e < J * R; e += 256) {
    const int j = e / R, r = e % R;
    double s = 0.0;
    for (int l = 0; l < L2; ++l) s += Q2[(size_t)j * L2 + l] * U[l * LD + perm[r]];
    D[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int j = 0; j < J; ++j) s += D[(size_t)j * R + a] * D[(size_t)j * R + b];
    DtD[e] = s;
  }
  if (tid == 0 && capped) atomicOr(&ctl->warn, 0x1u);
}

// F = B2^T (U2_R E^{-1}) and per-block partials of F^T F.
__global__ __launch_bounds__(256) void k_s2_f(int64_t KR, int L2, int R, const double* __restrict__ B2t,
                                              const double* __restrict__ U2s, double* __restrict__ F,
                                              double* __restrict__ FtFp) {
  __shared__ double sU[32 * 32];
  __shared__ double sF[256 * 33];
  const int tid = threadIdx.x;
  for (int e = tid; e < L2 * R; e += 256) sU[e] = U2s[e];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 256 + tid;
  for (int r = 0; r < R; ++r) {
    double s = 0.0;
    if (row < KR)
      for (int l = 0; l < L2; ++l) s += B2t[(size_t)row * L2 + l] * sU[l * R + r];
    sF[tid * 33 + r] = s;
    if (row < KR) F[(size_t)row * R + r] = s;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += sF[i * 33 + a] * sF[i * 33 + b];
    FtFp[(size_t)blockIdx.x * R * R + e] = s;
  }
}

// F^T F and e0 = sum_{r,s} E_r E_s (F^T F)_{rs} (D^T D)_{rs}.
__global__ __launch_bounds__(256) void k_s2_final(int nblk, int R, const double* __restrict__ FtFp,
                                                  const double* __restrict__ E, const double* __restrict__ DtD,
                                                  double* __restrict__ FtF, Ctl* ctl) {
  __shared__ double red[16];
  const int tid = threadIdx.x;
  double e0 = 0.0;
  for (int e = tid; e < R * R; e += 256) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += FtFp[(size_t)b * R * R + e];
    FtF[e] = s;
    const int a = e / R, c = e % R;
    e0 += E[a] * E[c] * s * DtD[e];
  }
  e0 = block_sum(e0, red);
  if (tid == 0) ctl->e0 = e0;
}

hipError_t launch_stage2(const Layout& lay, char* ws, const float* omega2, hipStream_t s) {
  const int64_t KR = lay.K * lay.R;
  const int J = (int)lay.J, L2 = lay.L2, R = lay.R;
  Ctl* ctl = reinterpret_cast<Ctl*>(ws + lay.ctl);
  double* Mt = reinterpret_cast<double*>(ws + lay.Mt);
  double* Y2p = reinterpret_cast<double*>(ws + lay.Y2p);
  double* Y2 = reinterpret_cast<double*>(ws + lay.Y2);
  double* B2t = reinterpret_cast<double*>(ws + lay.B2t);
  double* S2p = reinterpret_cast<double*>(ws + lay.S2p);
  double* U2s = reinterpret_cast<double*>(ws + lay.U2);
  double* D = reinterpret_cast<double*>(ws + lay.D);
  double* E = reinterpret_cast<double*>(ws + lay.E);
  double* F = reinterpret_cast<double*>(ws + lay.F);
  double* FtFp = reinterpret_cast<double*>(ws + lay.FtFp);
  double* small = reinterpret_cast<double*>(ws + lay.small);
  const double* xnorm2 = reinterpret_cast<const double*>(ws + lay.xnorm2);
  const int RR = R * R;
  hipLaunchKernelGGL(k_s2_y, dim3((unsigned)lay.n2, (unsigned)((J + 63) / 64)), dim3(256), 0, s, KR, J,
                     L2, omega2, Mt, Y2p);
  hipLaunchKernelGGL(k_s2_y_reduce, dim3((unsigned)((J * L2 + 255) / 256)), dim3(256), 0, s, lay.n2,
                     J, L2, Y2p, Y2);
  hipLaunchKernelGGL(k_s2_cqr2, dim3(1), dim3(256), 0, s, J, L2, Y2, ctl);
  hipLaunchKernelGGL(k_s2_b, dim3((unsigned)lay.n2), dim3(256), 0, s, KR, J, L2, Mt, Y2, B2t, S2p);
  hipLaunchKernelGGL(k_s2_evd, dim3(1), dim3(256), 0, s, lay.n2, lay.K, J, L2, R, S2p, Y2, xnorm2, D,
                     E, U2s, small + SM_DTD * RR, ctl);
  const unsigned nbf = (unsigned)((KR + 255) / 256);
  hipLaunchKernelGGL(k_s2_f, dim3(nbf), dim3(256), 0, s, KR, L2, R, B2t, U2s, F, FtFp);
  hipLaunchKernelGGL(k_s2_final, dim3(1), dim3(256), 0, s, (int)nbf, R, FtFp, E, small + SM_DTD * RR,
                     small + SM_FTF * RR, ctl);
  return hipGetLastError();
}

}  // namespace dpar2
