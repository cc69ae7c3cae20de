// Launch sequencing of the compressed ALS iteration (the rank-templated
// kernels are in als_impl.h, instantiated by k_als_r*.hip), the write-back of
// V, the fitness of Sec. IV-A from the compressed factors, and the U recipe.
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_1(int R, int phase, const AlsArgs& a, hipStream_t s);
hipError_t als_dispatch_2(int R, int phase, const AlsArgs& a, hipStream_t s);
hipError_t als_dispatch_3(int R, int phase, const AlsArgs& a, hipStream_t s);
hipError_t als_dispatch_4(int R, int phase, const AlsArgs& a, hipStream_t s);

static hipError_t als_dispatch(int R, int phase, const AlsArgs& a, hipStream_t s) {
  if (R <= 8) return als_dispatch_1(R, phase, a, s);
  if (R <= 16) return als_dispatch_2(R, phase, a, s);
  if (R <= 24) return als_dispatch_3(R, phase, a, s);
  return als_dispatch_4(R, phase, a, s);
}

// V = D VC, written when a call ends after at least one V update.
__global__ void k_als_vmat(int J, int R, const double* __restrict__ D, const double* __restrict__ small,
                           double* __restrict__ V, const Ctl* ctl) {
  if (!ctl->vc_valid) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * R) return;
  const int jj = e / R, c = e % R, RR = R * R;
  const double* VC = small + SM_VC * RR;
  double s = 0.0;
  for (int i = 0; i < R; ++i) s += D[(size_t)jj * R + i] * VC[i * R + c];
  V[e] = s;
}

// Fitness partials: per slice tr(V S_k H^T Psi_k^T (C_k B_k)^T) and
// W(k,:)(H^T H * V^T V)W(k,:)^T.
__global__ __launch_bounds__(256) void k_fit_part(int K, int J, int R, const double* __restrict__ Mt,
                                                  const double* __restrict__ V, const double* __restrict__ H,
                                                  const double* __restrict__ W, const double* __restrict__ Psi,
                                                  const double* __restrict__ HV, double* __restrict__ fitp) {
  __shared__ double Q[32 * 33], sPsi[32 * 33], sH[32 * 33], red[16];
  const int tid = threadIdx.x, RR = R * R;
  for (int e = tid; e < RR; e += 256) sH[(e / R) * 33 + e % R] = H[e];
  double tr = 0.0, qd = 0.0;
  for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
      const int r = e / R, s = e % R;
      double acc = 0.0;
      for (int jj = 0; jj < J; ++jj) acc += Mt[((size_t)k * R + r) * J + jj] * V[(size_t)jj * R + s];
      Q[r * 33 + s] = acc;
      sPsi[r * 33 + s] = Psi[(size_t)k * RR + e];
    }
    __syncthreads();
    if (tid < R) {
      const int r = tid;
      const double wr = W[(size_t)k * R + r];
      double x = 0.0;
      for (int a = 0; a < R; ++a) {
        double y = 0.0;
        for (int b = 0; b < R; ++b) y += sPsi[b * 33 + a] * Q[b * 33 + r];
        x += sH[a * 33 + r] * y;
      }
      tr += wr * x;
      double q = 0.0;
      for (int s = 0; s < R; ++s) q += HV[r * R + s] * W[(size_t)k * R + s];
      qd += wr * q;
    }
  }
  tr = block_sum(tr, red);
  qd = block_sum(qd, red);
  if (tid == 0) {
    fitp[2 * blockIdx.x] = tr;
    fitp[2 * blockIdx.x + 1] = qd;
  }
}

__global__ __launch_bounds__(256) void k_fit_final(int nblk, const double* __restrict__ fitp,
                                                   double* __restrict__ fit, Ctl* ctl) {
  __shared__ double red[16];
  double tr = 0.0, qd = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    tr += fitp[2 * b];
    qd += fitp[2 * b + 1];
  }
  tr = block_sum(tr, red);
  qd = block_sum(qd, red);
  if (threadIdx.x == 0) {
    const double x2 = ctl->xnorm2;
    const double f = 1.0 - (x2 - 2.0 * tr + qd) / x2;
    ctl->fit_true = f;
    if (fit) *fit = f;
  }
}

// Theta_k = Phi_k Psi_k H (L x R) for the U output.
__global__ __launch_bounds__(256) void k_theta(int K, int L, int R, const double* __restrict__ Phi,
                                               const double* __restrict__ Psi, const double* __restrict__ H,
                                               double* __restrict__ theta) {
  __shared__ double sT[32 * 33];
  const int k = blockIdx.x, tid = threadIdx.x, RR = R * R;
  // T = Psi_k H
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += Psi[(size_t)k * RR + a * R + i] * H[i * R + b];
    sT[a * 33 + b] = s;
  }
  __syncthreads();
  for (int e = tid; e < L * R; e += 256) {
    const int l = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += Phi[(size_t)k * L * R + l * R + i] * sT[i * 33 + b];
    theta[(size_t)k * L * R + e] = s;
  }
}

__global__ void k_eye(int64_t K, int R, double* __restrict__ P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int RR = R * R;
  if (e >= K * RR) return;
  const int w = (int)(e % RR);
  P[e] = (w / R == w % R) ? 1.0 : 0.0;
}

int als_blocks(int64_t K, int R) {
  (void)R;
  int64_t nb = K;   // upper bound on blocks of any per-slice kernel (one slice per group)
  if (nb > RED_MAXBLK) nb = RED_MAXBLK;
  if (nb < 1) nb = 1;
  return (int)nb;
}

static AlsArgs make_args(const Layout& lay, char* ws, double* H, double* V, double* W, double* trace,
                         double tol) {
  AlsArgs a;
  a.K = (int)lay.K;
  a.J = (int)lay.J;
  a.F = reinterpret_cast<const double*>(ws + lay.F);
  a.D = reinterpret_cast<const double*>(ws + lay.D);
  a.E = reinterpret_cast<const double*>(ws + lay.E);
  a.H = H;
  a.V = V;
  a.W = W;
  a.Pw = reinterpret_cast<double*>(ws + lay.Pw);
  a.Psi = reinterpret_cast<double*>(ws + lay.Psi);
  a.Mk = reinterpret_cast<double*>(ws + lay.Mk);
  a.small = reinterpret_cast<double*>(ws + lay.small);
  a.partA = reinterpret_cast<double*>(ws + lay.partA);
  a.partB = reinterpret_cast<double*>(ws + lay.partB);
  a.partC = reinterpret_cast<double*>(ws + lay.partC);
  a.partBegin = reinterpret_cast<double*>(ws + lay.partBegin);
  a.red = reinterpret_cast<double*>(ws + lay.red);
  a.trace = trace;
  a.tol = tol;
  a.ctl = reinterpret_cast<Ctl*>(ws + lay.ctl);
  return a;
}

hipError_t launch_pw_identity(const Layout& lay, char* ws, hipStream_t s) {
  double* Pw = reinterpret_cast<double*>(ws + lay.Pw);
  const int64_t n = lay.K * lay.R * lay.R;
  hipLaunchKernelGGL(k_eye, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lay.K, lay.R, Pw);
  return hipGetLastError();
}

hipError_t launch_als_begin(const Layout& lay, char* ws, double* H, double* V, double* W, hipStream_t s) {
  return als_dispatch(lay.R, 0, make_args(lay, ws, H, V, W, nullptr, -1.0), s);
}

hipError_t launch_als_iteration(const Layout& lay, char* ws, double* H, double* V, double* W,
                                double* err_trace, double tol, hipStream_t s) {
  return als_dispatch(lay.R, 1, make_args(lay, ws, H, V, W, err_trace, tol), s);
}

hipError_t launch_als_end(const Layout& lay, char* ws, double* V, hipStream_t s) {
  const int n = (int)(lay.J * lay.R);
  hipLaunchKernelGGL(k_als_vmat, dim3((n + 255) / 256), dim3(256), 0, s, (int)lay.J, lay.R,
                     reinterpret_cast<const double*>(ws + lay.D), reinterpret_cast<const double*>(ws + lay.small),
                     V, reinterpret_cast<const Ctl*>(ws + lay.ctl));
  return hipGetLastError();
}

hipError_t launch_fitness(const Layout& lay, char* ws, const double* H, const double* V,
                          const double* W, double* fit, hipStream_t s) {
  const int R = lay.R, RR = R * R;
  const double* small = reinterpret_cast<const double*>(ws + lay.small);
  double* fitp = reinterpret_cast<double*>(ws + lay.fitp);
  hipLaunchKernelGGL(k_fit_part, dim3(lay.nblkF), dim3(256), 0, s, (int)lay.K, (int)lay.J, R,
                     reinterpret_cast<const double*>(ws + lay.Mt), V, H, W,
                     reinterpret_cast<const double*>(ws + lay.Psi), small + SM_HV * RR, fitp);
  hipLaunchKernelGGL(k_fit_final, dim3(1), dim3(256), 0, s, lay.nblkF, fitp, fit,
                     reinterpret_cast<Ctl*>(ws + lay.ctl));
  return hipGetLastError();
}

hipError_t launch_theta(const Layout& lay, char* ws, const double* H, double* theta, hipStream_t s) {
  hipLaunchKernelGGL(k_theta, dim3((unsigned)lay.K), dim3(256), 0, s, (int)lay.K, lay.L, lay.R,
                     reinterpret_cast<const double*>(ws + lay.Phi),
                     reinterpret_cast<const double*>(ws + lay.Psi), H, theta);
  return hipGetLastError();
}

}  // namespace dpar2
