// Learned warm start for the iteration of Alg. 3: a set encoder reads the
// compressed representation of Sec. III-B (M ~ D E F^T) and proposes the
// starting H, V, W.  Kernels:
//   k_warm_feat     per-slice tokens: the upper triangle of
//                   R Phi_k / e_mean, Phi_k = (F^(k) E s)^T (F^(k) E s),
//                   s the signs that make the largest-magnitude entry of each
//                   column of D positive, e_mean = ||E||^2 / K
//   k_warm_targets  converged factors in one gauge (unit columns of H and V,
//                   V~ = D'^T V signed by its largest entry, W columns with a
//                   non-negative sum, components by decreasing ||W(:, r)||):
//                   H^T H, V~ and W / sqrt(e_mean / R)
//   k_warm_apply    H = predicted H, V = D' V~, W = predicted W sqrt(e_mean/R)
//   k_warm_fwd      per tensor: two ReLU layers (width 128) per token, mean
//                   pooling, heads H, V~ (pooled) and W(k, :) ([token; pooled])
//   k_warm_bwd      gradient of ||H^T H - T_H||^2/R^2 + ||V~ - T_V||^2/R^2 +
//                   sum_k ||W_k - T_W,k||^2/(K R), one partial per tensor
//   k_warm_gsum     sum of the per-tensor partials in a fixed order
//   k_warm_adam     Adam (Kingma & Ba) with bias correction
// Network arithmetic is FP32; features and targets are formed in FP64.
#include <algorithm>

#include "internal.h"

namespace dpar2 {

constexpr int WW = WARM_WIDTH;   // hidden width

__host__ __device__ WarmLayout warm_layout(int R) {
  WarmLayout w;
  w.F = R * (R + 1) / 2;
  const int RR = R * R;
  int at = 0;
  w.W1 = at; at += WW * w.F;
  w.b1 = at; at += WW;
  w.W2 = at; at += WW * WW;
  w.b2 = at; at += WW;
  w.WH = at; at += RR * WW;
  w.bH = at; at += RR;
  w.WV = at; at += RR * WW;
  w.bV = at; at += RR;
  w.Ww = at; at += R * 2 * WW;
  w.bw = at; at += R;
  w.P = at;
  return w;
}

// signs of D's columns (largest-magnitude entry positive, lowest index on
// ties) into s[0..R), and e_mean = ||E||^2 / K into *em; threads r < R
__device__ void basis_signs(int J, int R, int64_t K, const double* __restrict__ D, const double* __restrict__ E,
                            double* s, double* em) {
  const int r = threadIdx.x;
  if (r < R) {
    double best = -1.0, v = 1.0;
    for (int j = 0; j < J; ++j) {
      const double x = D[(size_t)j * R + r];
      if (fabs(x) > best) {
        best = fabs(x);
        v = x;
      }
    }
    s[r] = v < 0.0 ? -1.0 : 1.0;
  }
  if (r == 0) {
    double e = 0.0;
    for (int i = 0; i < R; ++i) e += E[i] * E[i];
    *em = e / (double)K;
  }
}

constexpr int FEAT_SLICES = 16;   // slices per block of k_warm_feat

__global__ __launch_bounds__(256) void k_warm_feat(int64_t K, int J, int R, const double* __restrict__ F,
                                                   const double* __restrict__ E, const double* __restrict__ D,
                                                   float* __restrict__ tok) {
  __shared__ double s[32], em;
  basis_signs(J, R, K, D, E, s, &em);
  __syncthreads();
  const int NF = R * (R + 1) / 2;
  const int64_t k0 = (int64_t)blockIdx.x * FEAT_SLICES;
  const double scale = (double)R / em;
  for (int e = threadIdx.x; e < FEAT_SLICES * NF; e += 256) {
    const int64_t k = k0 + e / NF;
    if (k >= K) break;
    int q = e % NF, a = 0;
    while (q >= R - a) {   // pair index -> (a, b), a <= b, row-major upper triangle
      q -= R - a;
      ++a;
    }
    const int b = a + q;
    const double* Fk = F + (size_t)k * R * R;
    double acc = 0.0;
    for (int i = 0; i < R; ++i) acc += Fk[i * R + a] * Fk[i * R + b];
    tok[(size_t)k * NF + e % NF] = (float)(acc * E[a] * E[b] * s[a] * s[b] * scale);
  }
}

__global__ __launch_bounds__(256) void k_warm_targets(int64_t K, int J, int R, const double* __restrict__ D,
                                                      const double* __restrict__ E, const double* __restrict__ H,
                                                      const double* __restrict__ V, const double* __restrict__ W,
                                                      float* __restrict__ tH, float* __restrict__ tV,
                                                      float* __restrict__ tW) {
  __shared__ double s[32], em, nH[32], nV[32], fV[32], fH[32], nW[32], Vt[32 * 32];
  __shared__ int perm[32];
  const int tid = threadIdx.x;
  basis_signs(J, R, K, D, E, s, &em);
  if (tid < R) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < R; ++i) a += H[i * R + tid] * H[i * R + tid];
    for (int j = 0; j < J; ++j) b += V[(size_t)j * R + tid] * V[(size_t)j * R + tid];
    nH[tid] = a > 0.0 ? sqrt(a) : 1.0;
    nV[tid] = b > 0.0 ? sqrt(b) : 1.0;
  }
  __syncthreads();
  // V~ = D'^T V / ||V(:, r)||
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, r = e % R;
    double acc = 0.0;
    for (int j = 0; j < J; ++j) acc += D[(size_t)j * R + i] * V[(size_t)j * R + r];
    Vt[e] = acc * s[i] / nV[r];
  }
  __syncthreads();
  if (tid < R) {
    const int r = tid;
    double best = -1.0, v = 1.0;
    for (int i = 0; i < R; ++i) {
      const double x = Vt[i * R + r];
      if (fabs(x) > best) {
        best = fabs(x);
        v = x;
      }
    }
    fV[r] = v < 0.0 ? -1.0 : 1.0;
    double sum = 0.0, sq = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      const double w = W[(size_t)k * R + r];
      sum += w;
      sq += w * w;
    }
    const double c = nH[r] * nV[r];
    fH[r] = (sum * c * fV[r] < 0.0) ? -1.0 : 1.0;
    nW[r] = c * sqrt(sq);
  }
  __syncthreads();
  if (tid < R) {   // rank by decreasing ||W(:, r)||, lower index first on ties
    int pos = 0;
    for (int q = 0; q < R; ++q) pos += (nW[q] > nW[tid] || (nW[q] == nW[tid] && q < tid)) ? 1 : 0;
    perm[pos] = tid;
  }
  __syncthreads();
  const double wscale = 1.0 / sqrt(em / (double)R);
  for (int e = tid; e < R * R; e += 256) {
    const int a = e / R, b = e % R, pa = perm[a], pb = perm[b];
    double acc = 0.0;
    for (int i = 0; i < R; ++i) acc += H[i * R + pa] * H[i * R + pb];
    tH[e] = (float)(acc * fH[pa] * fH[pb] / (nH[pa] * nH[pb]));
    tV[e] = (float)(Vt[a * R + pb] * fV[pb]);   // row a of V~, component b
  }
  for (int64_t e = tid; e < K * R; e += 256) {
    const int a = (int)(e % R), pa = perm[a];
    const int64_t k = e / R;
    tW[e] = (float)(W[(size_t)k * R + pa] * nH[pa] * nV[pa] * fV[pa] * fH[pa] * wscale);
  }
}

__global__ __launch_bounds__(256) void k_warm_apply(int64_t K, int J, int R, const double* __restrict__ D,
                                                    const double* __restrict__ E, const float* __restrict__ pH,
                                                    const float* __restrict__ pV, const float* __restrict__ pW,
                                                    double* __restrict__ H, double* __restrict__ V,
                                                    double* __restrict__ W) {
  __shared__ double s[32], em;
  basis_signs(J, R, K, D, E, s, &em);
  __syncthreads();
  const int64_t nV = (int64_t)J * R, nW = K * R, RR = R * R;
  const double ws = sqrt(em / (double)R);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < RR + nV + nW; e += (int64_t)gridDim.x * 256) {
    if (e < RR) {
      H[e] = (double)pH[e];
    } else if (e < RR + nV) {
      const int64_t q = e - RR;
      const int j = (int)(q / R), r = (int)(q % R);
      double acc = 0.0;
      for (int i = 0; i < R; ++i) acc += D[(size_t)j * R + i] * s[i] * (double)pV[i * R + r];
      V[q] = acc;
    } else {
      const int64_t q = e - RR - nV;
      W[q] = (double)pW[q] * ws;
    }
  }
}

// act rows (one per token): [Z1 | Z2 | dA2 | dA1], WW floats each
constexpr int ACT = 4 * WW;

__global__ __launch_bounds__(256) void k_warm_fwd(int R, const int32_t* __restrict__ tok_off,
                                                  const float* __restrict__ tok, const float* __restrict__ th,
                                                  float* __restrict__ act, float* __restrict__ pH,
                                                  float* __restrict__ pV, float* __restrict__ pW) {
  __shared__ float sp[WW];
  const WarmLayout L = warm_layout(R);
  const int b = blockIdx.x, tid = threadIdx.x, RR = R * R, NF = L.F;
  const int t0 = tok_off[b], K = tok_off[b + 1] - t0;
  const float* x = tok + (size_t)t0 * NF;
  float* A = act + (size_t)t0 * ACT;
  for (int e = tid; e < K * WW; e += 256) {
    const int k = e / WW, u = e % WW;
    float acc = th[L.b1 + u];
    const float* w = th + L.W1 + u * NF;
    for (int f = 0; f < NF; ++f) acc = fmaf(w[f], x[(size_t)k * NF + f], acc);
    A[(size_t)k * ACT + u] = fmaxf(acc, 0.f);
  }
  __syncthreads();
  for (int e = tid; e < K * WW; e += 256) {
    const int k = e / WW, u = e % WW;
    float acc = th[L.b2 + u];
    const float* w = th + L.W2 + u * WW;
    const float* z = A + (size_t)k * ACT;
    for (int v = 0; v < WW; ++v) acc = fmaf(w[v], z[v], acc);
    A[(size_t)k * ACT + WW + u] = fmaxf(acc, 0.f);
  }
  __syncthreads();
  if (tid < WW) {
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc += A[(size_t)k * ACT + WW + tid];
    sp[tid] = acc / (float)K;
  }
  __syncthreads();
  for (int e = tid; e < 2 * RR; e += 256) {
    const int i = e % RR;
    const bool h = e < RR;
    const float* w = th + (h ? L.WH : L.WV) + i * WW;
    float acc = th[(h ? L.bH : L.bV) + i];
    for (int u = 0; u < WW; ++u) acc = fmaf(w[u], sp[u], acc);
    (h ? pH : pV)[(size_t)b * RR + i] = acc;
  }
  for (int e = tid; e < K * R; e += 256) {
    const int k = e / R, r = e % R;
    const float* w = th + L.Ww + r * 2 * WW;
    const float* z = A + (size_t)k * ACT + WW;
    float acc = th[L.bw + r];
    for (int u = 0; u < WW; ++u) acc = fmaf(w[u], z[u], acc);
    for (int u = 0; u < WW; ++u) acc = fmaf(w[WW + u], sp[u], acc);
    pW[(size_t)(t0 + k) * R + r] = acc;
  }
}

__device__ float block_sum_f(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float t = 0.f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

__global__ __launch_bounds__(256) void k_warm_bwd(int R, const int32_t* __restrict__ tok_off,
                                                  const float* __restrict__ tok, const float* __restrict__ th,
                                                  float* __restrict__ act, const float* __restrict__ pH,
                                                  const float* __restrict__ pV, const float* __restrict__ pW,
                                                  const float* __restrict__ tH, const float* __restrict__ tV,
                                                  const float* __restrict__ tW, float* __restrict__ gpart,
                                                  float* __restrict__ lpart) {
  __shared__ float sp[WW], sdp[WW], sdG[32 * 32], sdH[32 * 32], sdV[32 * 32], swsum[32], red[4];
  const WarmLayout L = warm_layout(R);
  const int b = blockIdx.x, tid = threadIdx.x, RR = R * R, NF = L.F;
  const int t0 = tok_off[b], K = tok_off[b + 1] - t0;
  const float* x = tok + (size_t)t0 * NF;
  float* A = act + (size_t)t0 * ACT;
  const float* Hp = pH + (size_t)b * RR;
  const float* Vp = pV + (size_t)b * RR;
  const float* TH = tH + (size_t)b * RR;
  const float* TV = tV + (size_t)b * RR;
  const float* Wp = pW + (size_t)t0 * R;
  const float* TW = tW + (size_t)t0 * R;
  float* g = gpart + (size_t)b * L.P;
  const float cw = 2.f / (float)(K * R), ch = 2.f / (float)RR;
  // pooled vector, dG, dV, sum_k dW_k and the three loss terms
  float lh = 0.f, lv = 0.f, lw = 0.f;
  if (tid < WW) {
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc += A[(size_t)k * ACT + WW + tid];
    sp[tid] = acc / (float)K;
  }
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, c = e % R;
    float G = 0.f;
    for (int i = 0; i < R; ++i) G = fmaf(Hp[i * R + a], Hp[i * R + c], G);
    const float d = G - TH[e];
    sdG[e] = ch * d;
    lh += d * d;
    const float dv = Vp[e] - TV[e];
    sdV[e] = ch * dv;
    lv += dv * dv;
  }
  if (tid < R) {
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc += cw * (Wp[k * R + tid] - TW[k * R + tid]);
    swsum[tid] = acc;
  }
  for (int e = tid; e < K * R; e += 256) {
    const float d = Wp[e] - TW[e];
    lw += d * d;
  }
  __syncthreads();
  // dL/dH = H (dG + dG^T)
  for (int e = tid; e < RR; e += 256) {
    const int i = e / R, a = e % R;
    float acc = 0.f;
    for (int c = 0; c < R; ++c) acc = fmaf(Hp[i * R + c], sdG[a * R + c] + sdG[c * R + a], acc);
    sdH[e] = acc;
  }
  __syncthreads();
  // head gradients and dL/dp
  for (int e = tid; e < RR * WW; e += 256) {
    const int i = e / WW, u = e % WW;
    g[L.WH + e] = sdH[i] * sp[u];
    g[L.WV + e] = sdV[i] * sp[u];
  }
  for (int e = tid; e < RR; e += 256) {
    g[L.bH + e] = sdH[e];
    g[L.bV + e] = sdV[e];
  }
  for (int e = tid; e < R * WW; e += 256) {
    const int r = e / WW, u = e % WW;
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc = fmaf(cw * (Wp[k * R + r] - TW[k * R + r]), A[(size_t)k * ACT + WW + u], acc);
    g[L.Ww + r * 2 * WW + u] = acc;
    g[L.Ww + r * 2 * WW + WW + u] = swsum[r] * sp[u];
  }
  if (tid < R) g[L.bw + tid] = swsum[tid];
  if (tid < WW) {
    const int u = tid;
    float acc = 0.f;
    for (int i = 0; i < RR; ++i) acc = fmaf(th[L.WH + i * WW + u], sdH[i], acc);
    for (int i = 0; i < RR; ++i) acc = fmaf(th[L.WV + i * WW + u], sdV[i], acc);
    for (int r = 0; r < R; ++r) acc = fmaf(th[L.Ww + r * 2 * WW + WW + u], swsum[r], acc);
    sdp[u] = acc;
  }
  __syncthreads();
  // dA2 = (Ww[:, :WW]^T dW_k + dp / K) * [Z2 > 0]
  for (int e = tid; e < K * WW; e += 256) {
    const int k = e / WW, u = e % WW;
    float acc = sdp[u] / (float)K;
    for (int r = 0; r < R; ++r) acc = fmaf(th[L.Ww + r * 2 * WW + u], cw * (Wp[k * R + r] - TW[k * R + r]), acc);
    A[(size_t)k * ACT + 2 * WW + u] = A[(size_t)k * ACT + WW + u] > 0.f ? acc : 0.f;
  }
  __syncthreads();
  // layer-2 gradients; dA1 = (W2^T dA2) * [Z1 > 0]
  for (int e = tid; e < WW * WW; e += 256) {
    const int u = e / WW, v = e % WW;
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc = fmaf(A[(size_t)k * ACT + 2 * WW + u], A[(size_t)k * ACT + v], acc);
    g[L.W2 + e] = acc;
  }
  if (tid < WW) {
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc += A[(size_t)k * ACT + 2 * WW + tid];
    g[L.b2 + tid] = acc;
  }
  for (int e = tid; e < K * WW; e += 256) {
    const int k = e / WW, v = e % WW;
    float acc = 0.f;
    for (int u = 0; u < WW; ++u) acc = fmaf(th[L.W2 + u * WW + v], A[(size_t)k * ACT + 2 * WW + u], acc);
    A[(size_t)k * ACT + 3 * WW + v] = A[(size_t)k * ACT + v] > 0.f ? acc : 0.f;
  }
  __syncthreads();
  // layer-1 gradients
  for (int e = tid; e < WW * NF; e += 256) {
    const int v = e / NF, f = e % NF;
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc = fmaf(A[(size_t)k * ACT + 3 * WW + v], x[(size_t)k * NF + f], acc);
    g[L.W1 + e] = acc;
  }
  if (tid < WW) {
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc += A[(size_t)k * ACT + 3 * WW + tid];
    g[L.b1 + tid] = acc;
  }
  lh = block_sum_f(lh, red);
  lv = block_sum_f(lv, red);
  lw = block_sum_f(lw, red);
  if (tid == 0) {
    lpart[b * 3 + 0] = lh / (float)RR;
    lpart[b * 3 + 1] = lv / (float)RR;
    lpart[b * 3 + 2] = lw / (float)(K * R);
  }
}

__global__ __launch_bounds__(256) void k_warm_gsum(int n, int P, const float* __restrict__ gpart,
                                                   float* __restrict__ grad) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= P) return;
  float acc = 0.f;
  for (int b = 0; b < n; ++b) acc += gpart[(size_t)b * P + e];
  grad[e] = acc;
}

__global__ __launch_bounds__(256) void k_warm_adam(int P, float* __restrict__ th, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, float lr,
                                                   float b1, float b2, float eps, float c1, float c2,
                                                   float scale) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= P) return;
  const float gr = grad[e] * scale;
  const float mm = b1 * m[e] + (1.f - b1) * gr;
  const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
  m[e] = mm;
  v[e] = vv;
  th[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// --- launchers ---------------------------------------------------------------

hipError_t launch_warm_feat(int64_t K, int J, int R, const double* F, const double* E, const double* D, float* tok,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_warm_feat, dim3((unsigned)((K + FEAT_SLICES - 1) / FEAT_SLICES)), dim3(256), 0, s, K, J, R,
                     F, E, D, tok);
  return hipGetLastError();
}

hipError_t launch_warm_targets(int64_t K, int J, int R, const double* D, const double* E, const double* H,
                               const double* V, const double* W, float* tH, float* tV, float* tW, hipStream_t s) {
  hipLaunchKernelGGL(k_warm_targets, dim3(1), dim3(256), 0, s, K, J, R, D, E, H, V, W, tH, tV, tW);
  return hipGetLastError();
}

hipError_t launch_warm_apply(int64_t K, int J, int R, const double* D, const double* E, const float* pH,
                             const float* pV, const float* pW, double* H, double* V, double* W, hipStream_t s) {
  const int64_t n = (int64_t)R * R + (int64_t)J * R + K * R;
  const unsigned blocks = (unsigned)std::min<int64_t>(256, (n + 255) / 256);
  hipLaunchKernelGGL(k_warm_apply, dim3(blocks), dim3(256), 0, s, K, J, R, D, E, pH, pV, pW, H, V, W);
  return hipGetLastError();
}

hipError_t launch_warm_forward(int R, int n, const int32_t* tok_off, const float* tok, const float* theta,
                               float* act, float* pH, float* pV, float* pW, hipStream_t s) {
  hipLaunchKernelGGL(k_warm_fwd, dim3((unsigned)n), dim3(256), 0, s, R, tok_off, tok, theta, act, pH, pV, pW);
  return hipGetLastError();
}

hipError_t launch_warm_backward(int R, int n, const int32_t* tok_off, const float* tok, const float* theta,
                                float* act, const float* pH, const float* pV, const float* pW, const float* tH,
                                const float* tV, const float* tW, float* gpart, float* grad, float* loss,
                                hipStream_t s) {
  const int P = warm_layout(R).P;
  hipLaunchKernelGGL(k_warm_bwd, dim3((unsigned)n), dim3(256), 0, s, R, tok_off, tok, theta, act, pH, pV, pW, tH,
                     tV, tW, gpart, loss);
  hipLaunchKernelGGL(k_warm_gsum, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, n, P, gpart, grad);
  return hipGetLastError();
}

hipError_t launch_warm_adam(int R, float* theta, const float* grad, float* m, float* v, int step, float lr,
                            float b1, float b2, float eps, float scale, hipStream_t s) {
  const int P = warm_layout(R).P;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_warm_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, theta, grad, m, v, lr, b1,
                     b2, eps, c1, c2, scale);
  return hipGetLastError();
}

}  // namespace dpar2
