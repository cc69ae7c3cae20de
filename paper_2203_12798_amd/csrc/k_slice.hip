// Per-slice completion of the first-stage randomized SVD (Alg. 1 lines 3-6 for
// every X_k, Eq. 4), from the FP64 partial sums of the slab pass:
//   Y_k^T Y_k = V Lambda V^T,  Wh = V Lambda^{-1/2}  (Q_k = Y_k Wh, line 3;
//               directions with negligible lambda are dropped, so a rank-
//               deficient sketch still yields an orthonormal basis)
//   B_k     = Q_k^T X_k = Wh^T P_k,  P_k = Y_k^T X_k           (line 4)
//   B_k B_k^T = Wh^T (P_k P_k^T) Wh = U~ Lambda~ U~^T          (line 5)
//   sigma   = sqrt(lambda~[:R]),  C_k B_k = B_k^T U~_R = P_k^T Phi_k,
//   Phi_k   = Wh U~_R          (so A_k = Y_k Phi_k = Q_k U~_R, line 6)
// Output: block k of M = ||_k C_k B_k, stored as rows kR..kR+R-1 of M^T
// (R x J), the A_k recipe Phi_k (L x R), sigma_k and ||X_k||^2.
// Sign gauge: each column of C_k B_k is signed so that its largest-magnitude
// entry is positive (first one on ties).
#include "internal.h"

namespace dpar2 {

__global__ __launch_bounds__(256) void k_slice_finish(
    int J, int L, int R, const int32_t* __restrict__ slice_ptr,
    const int32_t* __restrict__ slice_list, const double* __restrict__ partG,
    const double* __restrict__ partP, const double* __restrict__ partS,
    double* __restrict__ xnorm2, double* __restrict__ Mt, double* __restrict__ Phi,
    double* __restrict__ sig1, Ctl* ctl) {
  constexpr int LD = 33;
  __shared__ double G[32 * LD], S[32 * LD], U[32 * LD], T[32 * LD];
  __shared__ double Pc[32 * LD];
  __shared__ double cs[40], red[16];
  __shared__ int perm[32];
  __shared__ double colmax[32];
  __shared__ int colarg[32];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int i0 = slice_ptr[k], i1 = slice_ptr[k + 1];

  for (int e = tid; e < L * L; e += 256) {
    double g = 0.0;
    for (int ii = i0; ii < i1; ++ii) g += partG[(size_t)slice_list[ii] * L * L + e];
    G[(e / L) * LD + (e % L)] = g;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int ii = i0; ii < i1; ++ii) s += partS[slice_list[ii]];
    xnorm2[k] = s;
  }

  // S' = P P^T (upper triangle pairs), P streamed in chunks of 32 columns
  const int npairs = L * (L + 1) / 2;
  double sacc[3] = {0.0, 0.0, 0.0};
  for (int jc = 0; jc < J; jc += 32) {
    __syncthreads();
    for (int e = tid; e < L * 32; e += 256) {
      const int l = e / 32, c = e % 32;
      double p = 0.0;
      if (jc + c < J)
        for (int ii = i0; ii < i1; ++ii) p += partP[(size_t)slice_list[ii] * L * J + (size_t)l * J + jc + c];
      Pc[l * LD + c] = p;
    }
    __syncthreads();
    for (int q = 0; q < 3; ++q) {
      const int pi = tid + 256 * q;
      if (pi < npairs) {
        int a = 0, rem = pi;
        while (rem >= L - a) { rem -= L - a; ++a; }
        const int b = a + rem;
        double s = 0.0;
        for (int c = 0; c < 32; ++c) s += Pc[a * LD + c] * Pc[b * LD + c];
        sacc[q] += s;
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < 3; ++q) {
    const int pi = tid + 256 * q;
    if (pi < npairs) {
      int a = 0, rem = pi;
      while (rem >= L - a) { rem -= L - a; ++a; }
      const int b = a + rem;
      S[a * LD + b] = sacc[q];
      S[b * LD + a] = sacc[q];
    }
  }
  __syncthreads();

  // Wh (in T): Y Wh is an orthonormal basis Q of span(Y) (Alg. 1 line 3)
  const int capped0 = block_whiten(G, LD, L, T, U, cs);
  // B B^T = Wh^T (P P^T) Wh with B = Q^T X = Wh^T P (Alg. 1 line 4)
  for (int e = tid; e < L * L; e += 256) {
    const int a = e / L, b = e % L;
    double v = 0.0;
    for (int i = 0; i < L; ++i) v += S[a * LD + i] * T[i * LD + b];
    G[a * LD + b] = v;
  }
  __syncthreads();
  for (int e = tid; e < L * L; e += 256) {
    const int a = e / L, b = e % L;
    double v = 0.0;
    for (int i = 0; i < L; ++i) v += T[i * LD + a] * G[i * LD + b];
    S[a * LD + b] = v;
  }
  __syncthreads();
  for (int e = tid; e < L * L; e += 256) {
    const int a = e / L, b = e % L;
    if (a < b) {
      const double m = 0.5 * (S[a * LD + b] + S[b * LD + a]);
      S[a * LD + b] = m;
      S[b * LD + a] = m;
    }
  }
  __syncthreads();

  // B B^T = U~ Lambda U~^T (Alg. 1 line 5)
  const int capped = block_sym_evd(S, LD, U, L, cs) | capped0;
  block_sort_desc(S, LD, L, perm);

  // Phi = Wh U~_R (in G), sigma = sqrt(lambda_R)
  for (int e = tid; e < L * R; e += 256) {
    const int l = e / R, r = e % R;
    double v = 0.0;
    for (int i = 0; i < L; ++i) v += T[l * LD + i] * U[i * LD + perm[r]];
    G[l * LD + r] = v;
  }
  if (tid < R) {
    const double lam = S[perm[tid] * LD + perm[tid]];
    sig1[(size_t)k * R + tid] = sqrt(lam > 0.0 ? lam : 0.0);
  }
  __syncthreads();

  // C_k B_k = P^T Phi ; columns written as rows of M^T, then sign-fixed
  double* Mk = Mt + (size_t)k * R * J;
  for (int e = tid; e < R * J; e += 256) {
    const int r = e / J, j = e % J;
    double m = 0.0;
    for (int l = 0; l < L; ++l) {
      double p = 0.0;
      for (int ii = i0; ii < i1; ++ii) p += partP[(size_t)slice_list[ii] * L * J + (size_t)l * J + j];
      m += G[l * LD + r] * p;
    }
    Mk[(size_t)r * J + j] = m;
  }
  __syncthreads();
  if (tid < R) {
    double best = -1.0;
    int arg = 0;
    for (int j = 0; j < J; ++j) {
      const double v = fabs(Mk[(size_t)tid * J + j]);
      if (v > best) { best = v; arg = j; }
    }
    colmax[tid] = Mk[(size_t)tid * J + arg];
    colarg[tid] = arg;
  }
  __syncthreads();
  for (int e = tid; e < R * J; e += 256) {
    const int r = e / J, j = e % J;
    if (colmax[r] < 0.0) Mk[(size_t)r * J + j] = -Mk[(size_t)r * J + j];
  }
  for (int e = tid; e < L * R; e += 256) {
    const int l = e / R, r = e % R;
    Phi[(size_t)k * L * R + e] = (colmax[r] < 0.0) ? -G[l * LD + r] : G[l * LD + r];
  }
  if (tid == 0) {
    unsigned bits = 0;
    if (capped) bits |= 0x1u;
    if (bits) atomicOr(&ctl->warn, bits);
  }
}

hipError_t launch_slice_finish(int64_t K, int J, int L, int R, const int32_t* slice_ptr,
                               const int32_t* slice_list, const double* partG,
                               const double* partP, const double* partS, double* xnorm2,
                               double* Mt, double* Phi, double* sig1, Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_slice_finish, dim3((unsigned)K), dim3(256), 0, s, J, L, R, slice_ptr,
                     slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1, ctl);
  return hipGetLastError();
}

}  // namespace dpar2
