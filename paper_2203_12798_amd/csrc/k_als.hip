// Launch sequencing of the compressed ALS iteration (the rank-templated
// kernels are in als_impl.h, instantiated by k_als_r*.hip), the write-back of
// V, the fitness of Sec. IV-A from the compressed factors, and the U recipe.
// Every launch covers a whole group of tensors (one for the single-tensor
// entry points).
#include "als_impl.h"

namespace dpar2 {

hipError_t als_dispatch_1(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s);
hipError_t als_dispatch_2(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s);
hipError_t als_dispatch_3(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s);
hipError_t als_dispatch_4(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s);
hipError_t als_dispatch_5(int R, int phase, const AlsArgs& a, int nb, int nb0, const int64_t* seg,
                          const int64_t* seg0, hipStream_t s);

int als_slices_per_block(int R) {
  const int n = R + (R & 1);
  int rm = 1;
  while (rm < n) rm *= 2;
  if (rm < 2) rm = 2;
  return (R > 32 ? 64 : R > 16 ? 128 : 256) / rm;   // RC<R>::GPB
}

// V = D VC for each tensor whose V was updated during the call.
__global__ void k_als_vmat(int J, int R, const TDesc* __restrict__ td, const double* __restrict__ Dall,
                           const double* __restrict__ small, const Ctl* __restrict__ ctl) {
  const int t = blockIdx.y;
  if (!ctl[t].vc_valid) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * R) return;
  const int jj = e / R, c = e % R, RR = R * R;
  const double* VC = small + (size_t)t * SM_COUNT * RR + SM_VC * RR;
  const double* D = Dall + (size_t)t * J * R;
  double s = 0.0;
  for (int i = 0; i < R; ++i) s += D[(size_t)jj * R + i] * VC[i * R + c];
  td[t].V[e] = s;
}

// fitness of each tensor from its summed partials (fits: nt x 2)
__global__ void k_fit_final(int nt, const double* __restrict__ fits, double* __restrict__ fit, Ctl* ctl) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const double x2 = ctl[t].xnorm2;
  const double f = 1.0 - (x2 - 2.0 * fits[2 * t] + fits[2 * t + 1]) / x2;
  ctl[t].fit_true = f;
  if (fit && t == 0) *fit = f;
}

// Theta_k = Phi_k Psi_k H (L x R) for the U output (single tensor).
__global__ __launch_bounds__(256) void k_theta(int K, int L, int R, const double* __restrict__ Phi,
                                               const double* __restrict__ Psi, const double* __restrict__ H,
                                               double* __restrict__ theta) {
  constexpr int LD = MAX_RANK + 1;
  __shared__ double sT[MAX_RANK * LD];
  const int k = blockIdx.x, tid = threadIdx.x, RR = R * R;
  // T = Psi_k H
  for (int e = tid; e < RR; e += 256) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += Psi[(size_t)k * RR + a * R + i] * H[i * R + b];
    sT[a * LD + b] = s;
  }
  __syncthreads();
  for (int e = tid; e < L * R; e += 256) {
    const int l = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += Phi[(size_t)k * L * R + l * R + i] * sT[i * LD + b];
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

static AlsArgs make_args(const Layout& lay, char* ws) {
  AlsArgs a;
  a.nt = lay.nt;
  a.J = (int)lay.J;
  a.K1 = lay.K;
  a.td = reinterpret_cast<const TDesc*>(ws + lay.tdesc);
  a.blk = reinterpret_cast<const Blk*>(ws + lay.blk);
  a.blk0 = reinterpret_cast<const Blk*>(ws + lay.blk0);
  a.F = reinterpret_cast<const double*>(ws + lay.F);
  a.D = reinterpret_cast<const double*>(ws + lay.D);
  a.E = reinterpret_cast<const double*>(ws + lay.E);
  a.Pw = reinterpret_cast<double*>(ws + lay.Pw);
  a.Psi = reinterpret_cast<double*>(ws + lay.Psi);
  a.Mk = reinterpret_cast<double*>(ws + lay.Mk);
  a.small = reinterpret_cast<double*>(ws + lay.small);
  a.partA = reinterpret_cast<double*>(ws + lay.partA);
  a.partB = reinterpret_cast<double*>(ws + lay.partB);
  a.partC = reinterpret_cast<double*>(ws + lay.partC);
  a.partBegin = reinterpret_cast<double*>(ws + lay.partBegin);
  a.red = reinterpret_cast<double*>(ws + lay.red);
  a.ctl = reinterpret_cast<Ctl*>(ws + lay.ctl);
  a.Mt = reinterpret_cast<const double*>(ws + lay.Mt);
  a.fitp = reinterpret_cast<double*>(ws + lay.fitp);
  return a;
}

static hipError_t als_dispatch(const Layout& lay, char* ws, int phase, hipStream_t s) {
  const AlsArgs a = make_args(lay, ws);
  const int64_t* seg = reinterpret_cast<const int64_t*>(ws + lay.seg_blk);
  const int64_t* seg0 = reinterpret_cast<const int64_t*>(ws + lay.seg_blk0);
  const int R = lay.R;
  if (R <= 8) return als_dispatch_1(R, phase, a, lay.nblk, lay.nblk0, seg, seg0, s);
  if (R <= 16) return als_dispatch_2(R, phase, a, lay.nblk, lay.nblk0, seg, seg0, s);
  if (R <= 24) return als_dispatch_3(R, phase, a, lay.nblk, lay.nblk0, seg, seg0, s);
  if (R <= 32) return als_dispatch_4(R, phase, a, lay.nblk, lay.nblk0, seg, seg0, s);
  return als_dispatch_5(R, phase, a, lay.nblk, lay.nblk0, seg, seg0, s);
}

hipError_t launch_pw_identity(const Layout& lay, char* ws, hipStream_t s) {
  double* Pw = reinterpret_cast<double*>(ws + lay.Pw);
  const int64_t n = lay.K * lay.R * lay.R;
  hipLaunchKernelGGL(k_eye, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lay.K, lay.R, Pw);
  return hipGetLastError();
}

hipError_t launch_als_begin(const Layout& lay, char* ws, hipStream_t s) { return als_dispatch(lay, ws, 0, s); }

hipError_t launch_als_iteration(const Layout& lay, char* ws, hipStream_t s) {
  hipError_t e = als_dispatch(lay, ws, 1, s);
  if (e != hipSuccess || !lay.det) return e;
  // resumable mode: end the iteration in the state a new call starts from
  if ((e = launch_als_end(lay, ws, s)) != hipSuccess) return e;
  return als_dispatch(lay, ws, 2, s);
}

hipError_t launch_als_end(const Layout& lay, char* ws, hipStream_t s) {
  const int n = (int)(lay.J * lay.R);
  hipLaunchKernelGGL(k_als_vmat, dim3((n + 255) / 256, (unsigned)lay.nt), dim3(256), 0, s, (int)lay.J, lay.R,
                     reinterpret_cast<const TDesc*>(ws + lay.tdesc), reinterpret_cast<const double*>(ws + lay.D),
                     reinterpret_cast<const double*>(ws + lay.small), reinterpret_cast<const Ctl*>(ws + lay.ctl));
  return hipGetLastError();
}

hipError_t launch_fitness(const Layout& lay, char* ws, double* fit, hipStream_t s) {
  double* fitp = reinterpret_cast<double*>(ws + lay.fitp);
  double* fits = fitp + 2 * lay.K;   // nt x 2 sums after the K per-slice partials
  hipError_t e = als_dispatch(lay, ws, 3, s);
  if (e != hipSuccess) return e;
  e = launch_segsum(lay.nt, reinterpret_cast<const int64_t*>(ws + lay.seg_slice), lay.K, 2, 2, fitp, fits, 2, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fit_final, dim3((unsigned)((lay.nt + 63) / 64)), dim3(64), 0, s, lay.nt, fits, fit,
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
