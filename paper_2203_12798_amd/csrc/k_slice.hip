// Per-slice completion of the first-stage randomized SVD (QR, projection and
// small-SVD steps of Alg. 1 for every X_k, Eq. 4), from the FP64 partial sums
// of the slab pass, G = Y_k^T Y_k and P_k = Y_k^T X_k:
//   G = R^T R (Cholesky), Wh = R^{-1}        (Q_k = Y_k Wh, the QR step; when a
//               pivot is negligible the eigen form Wh = V Lambda^{-1/2} over the
//               eigenvalues kept is used, so a rank-deficient sketch still
//               yields an orthonormal basis)
//   B_k     = Q_k^T X_k = Wh^T P_k                               (projection)
//   B_k B_k^T = Wh^T (P_k P_k^T) Wh = U~ Lambda~ U~^T            (small SVD, by
//               one-sided Jacobi on the Cholesky factor of B_k B_k^T)
//   sigma   = sqrt(lambda~[:R]),  C_k B_k = B_k^T U~_R = P_k^T Phi_k,
//   Phi_k   = Wh U~_R          (so A_k = Y_k Phi_k = Q_k U~_R)
// Output: block k of M = ||_k C_k B_k, stored as rows kR..kR+R-1 of M^T
// (R x J), the A_k recipe Phi_k (L x R), sigma_k and ||X_k||^2; warnings go
// to the control block of the slice's tensor.
// Sign gauge: each column of C_k B_k is signed so that its largest-magnitude
// entry is positive (first one on ties): the completion writes the columns
// unsigned with their signs in msgn (K x R), k_msign then flips the rows of M^T
// with a negative sign.
#include "internal.h"

namespace dpar2 {

hipError_t slice_dispatch_1(int L, int64_t K, int J, int R, const int32_t* slice_ptr,
                            const int32_t* slice_list, const double* partG, const double* partP,
                            const double* partS, double* xnorm2, double* Mt, double* Phi, double* sig1,
                            float* omega_next, float* msgn, Ctl* ctl, const int32_t* slice_t, hipStream_t s);
hipError_t slice_dispatch_2(int L, int64_t K, int J, int R, const int32_t* slice_ptr,
                            const int32_t* slice_list, const double* partG, const double* partP,
                            const double* partS, double* xnorm2, double* Mt, double* Phi, double* sig1,
                            float* omega_next, float* msgn, Ctl* ctl, const int32_t* slice_t, hipStream_t s);
hipError_t slice_dispatch_3(int L, int64_t K, int J, int R, const int32_t* slice_ptr,
                            const int32_t* slice_list, const double* partG, const double* partP,
                            const double* partS, double* xnorm2, double* Mt, double* Phi, double* sig1,
                            float* omega_next, float* msgn, Ctl* ctl, const int32_t* slice_t, hipStream_t s);

// Rows kR + r of M^T whose column of C_k B_k takes a negative sign: one block
// per row, the rows with a positive sign return at once.
__global__ __launch_bounds__(256) void k_msign(int J, const float* __restrict__ msgn, double* __restrict__ Mt) {
  const int64_t row = blockIdx.x;
  if (msgn[row] > 0.f) return;
  double* m = Mt + row * J;
  for (int j = threadIdx.x; j < J; j += 256) m[j] = -m[j];
}

hipError_t launch_slice_finish(int64_t K, int J, int L, int R, const int32_t* slice_ptr,
                               const int32_t* slice_list, const double* partG,
                               const double* partP, const double* partS, double* xnorm2,
                               double* Mt, double* Phi, double* sig1, float* omega_next, float* msgn, Ctl* ctl,
                               const int32_t* slice_t, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const hipError_t e =
      L <= 16   ? slice_dispatch_1(L, K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1,
                                   omega_next, msgn, ctl, slice_t, s)
      : L <= 32 ? slice_dispatch_2(L, K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1,
                                   omega_next, msgn, ctl, slice_t, s)
                : slice_dispatch_3(L, K, J, R, slice_ptr, slice_list, partG, partP, partS, xnorm2, Mt, Phi, sig1,
                                   omega_next, msgn, ctl, slice_t, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_msign, dim3((unsigned)(K * R)), dim3(256), 0, s, J, msgn, Mt);
  return hipGetLastError();
}

}  // namespace dpar2
