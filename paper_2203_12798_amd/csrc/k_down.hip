// Post-processing of DPar2's factors (Sec. IV-E): feature correlations from
// V, slice similarities from U_k (Eq. 9), top-k ranking, and the random walk
// with restart on the similarity graph (Eqs. 10-11).  All FP64.
#include "internal.h"

namespace dpar2 {

constexpr int DT = 32;   // output tile (rows and columns) of the pairwise kernels

// C[a][b] = sum_r da[r] db[r] / sqrt(ssa ssb), d the centred rows of V; rows
// of zero variance give 0.  Block = a 32 x 32 tile of C; R <= MAX_RANK.
__global__ __launch_bounds__(256) void k_pcc(int64_t J, int R, const double* __restrict__ V,
                                             double* __restrict__ C) {
  constexpr int RP = MAX_RANK + 1;
  __shared__ double A[DT][RP], B[DT][RP], ssA[DT], ssB[DT];
  const int tid = threadIdx.x;
  const int64_t a0 = (int64_t)blockIdx.y * DT, b0 = (int64_t)blockIdx.x * DT;
  // thread t < 64 centres row t % 32 of side t / 32
  if (tid < 2 * DT) {
    const int side = tid / DT, i = tid % DT;
    const int64_t row = (side ? b0 : a0) + i;
    double (*M)[RP] = side ? B : A;
    double* ss = side ? ssB : ssA;
    if (row < J) {
      double m = 0.0;
      for (int r = 0; r < R; ++r) m += V[row * R + r];
      m /= R;
      double s = 0.0;
      for (int r = 0; r < R; ++r) {
        const double d = V[row * R + r] - m;
        M[i][r] = d;
        s += d * d;
      }
      ss[i] = s;
    } else {
      for (int r = 0; r < R; ++r) M[i][r] = 0.0;
      ss[i] = 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < DT * DT; e += 256) {
    const int i = e / DT, j = e % DT;
    const int64_t a = a0 + i, b = b0 + j;
    if (a >= J || b >= J) continue;
    double v = 0.0;
    if (ssA[i] > 0.0 && ssB[j] > 0.0) {
      double s = 0.0;
      for (int r = 0; r < R; ++r) s += A[i][r] * B[j][r];
      v = s / sqrt(ssA[i] * ssB[j]);
    }
    C[a * J + b] = v;
  }
}

// S[i][j] = exp(-gamma sum (u_i - u_j)^2) over the M = I R entries of the
// slices idx[i], idx[j] (rows off[idx] .. of U), streamed in chunks of SCH
// entries through LDS.  Block = a 64 x 64 tile of S; thread (ti, tj) = (t /
// 16, t % 16) holds the 4 x 4 entries (ti + 16 a, tj + 16 b), each summed over
// the entries in order.
constexpr int ST = 64;    // output tile (rows and columns) of the similarity
constexpr int SCH = 32;   // entries per chunk
__global__ __launch_bounds__(256) void k_sim(int n, int64_t M, int R, const int64_t* __restrict__ off,
                                             const int32_t* __restrict__ idx, const double* __restrict__ U,
                                             double gamma, double* __restrict__ S) {
  __shared__ double A[ST][SCH + 1], B[ST][SCH + 1];
  __shared__ const double* pa[ST];
  __shared__ const double* pb[ST];
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int i0 = blockIdx.y * ST, j0 = blockIdx.x * ST;
  if (tid < 2 * ST) {
    const int side = tid / ST, t = tid % ST, s = (side ? j0 : i0) + t;
    const double* p = (s < n) ? U + off[idx[s]] * R : nullptr;
    if (side) pb[t] = p;
    else pa[t] = p;
  }
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t m0 = 0; m0 < M; m0 += SCH) {
    const int nm = (M - m0 < SCH) ? (int)(M - m0) : SCH;
    __syncthreads();
    for (int e = tid; e < ST * SCH; e += 256) {
      const int t = e / SCH, c = e % SCH;
      A[t][c] = (pa[t] && c < nm) ? pa[t][m0 + c] : 0.0;
      B[t][c] = (pb[t] && c < nm) ? pb[t][m0 + c] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < nm; ++c) {
      double x[4], y[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        x[a] = A[ti + 16 * a][c];
        y[a] = B[tj + 16 * a][c];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double d = x[a] - y[b];
          acc[a][b] = fma(d, d, acc[a][b]);
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + ti + 16 * a, j = j0 + tj + 16 * b;
      if (i < n && j < n) S[(size_t)i * n + j] = exp(-gamma * acc[a][b]);
    }
}

// Order of the ranking: larger value first, then lower index; NaN ranks
// below every number.
__device__ __forceinline__ bool ahead(double va, int ia, double vb, int ib) {
  const bool na = va != va, nb = vb != vb;
  if (na != nb) return nb;
  if (!na && va != vb) return va > vb;
  return ia < ib;
}

// k rounds, each the best entry ranked after the previous pick.  One block.
__global__ __launch_bounds__(1024) void k_topk(const double* __restrict__ v, int n, int exclude, int k,
                                               int32_t* __restrict__ out) {
  __shared__ double sv[16];
  __shared__ int si[16];
  __shared__ double pv;
  __shared__ int pi;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int round = 0; round < k; ++round) {
    double bv = 0.0;
    int bi = -1;
    for (int i = tid; i < n; i += 1024) {
      if (i == exclude) continue;
      const double x = v[i];
      if (round > 0 && !ahead(pv, pi, x, i)) continue;   // at or ahead of the last pick
      if (bi < 0 || ahead(x, i, bv, bi)) {
        bv = x;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (oi >= 0 && (bi < 0 || ahead(ov, oi, bv, bi))) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      sv[w] = bv;
      si[w] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = 0.0;
      int ib = -1;
      for (int q = 0; q < 16; ++q)
        if (si[q] >= 0 && (ib < 0 || ahead(sv[q], si[q], b, ib))) {
          b = sv[q];
          ib = si[q];
        }
      out[round] = ib;
      pv = b;
      pi = ib;
    }
    __syncthreads();
  }
}

// d[i] = sum_{j != i} S[i][j]; r = q (e_target).  One block per row.
__global__ __launch_bounds__(256) void k_rwr_init(const double* __restrict__ S, int n, int target,
                                                  double* __restrict__ d, double* __restrict__ r) {
  __shared__ double red[16];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256)
    if (j != i) s += S[(size_t)i * n + j];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    d[i] = s;
    r[i] = (i == target) ? 1.0 : 0.0;
  }
}

// w[i] = r[i] / d[i] (0 for a node without edges)
__global__ __launch_bounds__(256) void k_rwr_w(const double* __restrict__ r, const double* __restrict__ d, int n,
                                               double* __restrict__ w) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) w[i] = d[i] > 0.0 ? r[i] / d[i] : 0.0;
}

// r_new[j] = (1 - c) sum_{i != j} S[i][j] w[i] + c q[j]: one block per 16
// columns; thread t takes column 16 b + t % 16 and every 64th row from row
// t / 16 (a wave reads 16 consecutive entries of 4 rows), and the 64 row-group
// sums of a column are added in a fixed order.
__global__ __launch_bounds__(1024) void k_rwr_step(const double* __restrict__ S, const double* __restrict__ w, int n,
                                                   int target, double c, double* __restrict__ rn) {
  __shared__ double part[64][17];
  const int tid = threadIdx.x, cl = tid & 15, g = tid >> 4;
  const int j = blockIdx.x * 16 + cl;
  double s0 = 0.0, s1 = 0.0;
  if (j < n) {
    int i = g;
    for (; i + 64 < n; i += 128) {
      s0 += (i == j) ? 0.0 : S[(size_t)i * n + j] * w[i];
      s1 += (i + 64 == j) ? 0.0 : S[(size_t)(i + 64) * n + j] * w[i + 64];
    }
    if (i < n) s0 += (i == j) ? 0.0 : S[(size_t)i * n + j] * w[i];
  }
  part[g][cl] = s0 + s1;
  __syncthreads();
  if (g == 0 && j < n) {
    double s = 0.0;
    for (int q = 0; q < 64; ++q) s += part[q][cl];
    rn[j] = (1.0 - c) * s + ((j == target) ? c : 0.0);
  }
}

hipError_t launch_pcc(int64_t J, int R, const double* V, double* C, hipStream_t s) {
  const unsigned t = (unsigned)((J + DT - 1) / DT);
  hipLaunchKernelGGL(k_pcc, dim3(t, t), dim3(256), 0, s, J, R, V, C);
  return hipGetLastError();
}

hipError_t launch_similarity(int n, int64_t M, int R, const int64_t* off, const int32_t* idx, const double* U,
                             double gamma, double* S, hipStream_t s) {
  const unsigned t = (unsigned)((n + ST - 1) / ST);
  hipLaunchKernelGGL(k_sim, dim3(t, t), dim3(256), 0, s, n, M, R, off, idx, U, gamma, S);
  return hipGetLastError();
}

hipError_t launch_topk(const double* v, int n, int exclude, int k, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, v, n, exclude, k, out);
  return hipGetLastError();
}

hipError_t launch_rwr(const double* S, int n, int target, double c, int iters, double* r, double* work,
                      hipStream_t s) {
  double* d = work;
  double* w = work + n;
  double* tmp = work + 2 * (size_t)n;
  // ping-pong so that the last step lands in r
  double* cur = (iters % 2 == 0) ? r : tmp;
  double* nxt = (iters % 2 == 0) ? tmp : r;
  hipLaunchKernelGGL(k_rwr_init, dim3((unsigned)n), dim3(256), 0, s, S, n, target, d, cur);
  const unsigned nb = (unsigned)((n + 255) / 256);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_rwr_w, dim3(nb), dim3(256), 0, s, cur, d, n, w);
    hipLaunchKernelGGL(k_rwr_step, dim3((unsigned)((n + 15) / 16)), dim3(1024), 0, s, S, w, n, target, c, nxt);
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  return hipGetLastError();
}

}  // namespace dpar2
