// Precision-based stopping of the inner block CG: the alternative to a fixed
// number of inner iterations that Sec. 3 sets aside, built for comparison.
// A block (per right-hand side) stops after the first iteration whose
// residual norm is at most tol times its initial one: from then on its step
// length is zero, so its iterate and residual stay as they are while the
// batched kernels keep running for the other blocks.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mspcg {

// stop: [nblocks * nrhs][2] = {initial rho, stopped flag}; scal as for the
// block scalars ([rho, alpha, beta, pad] per (block, rhs)).
//   mode 0 (after the initial rho): record it, clear the flag
//   mode 1 (after alpha):           stopped blocks take alpha = 0
//   mode 2 (after rho_new):         set the flag once rho_new <= tol^2 rho_0
__global__ void __launch_bounds__(256) k_inner_stop(int mode, int n, double tol2, double *scal, double *stop) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double *sc = scal + (size_t)i * kScal;
  double *st = stop + 2 * (size_t)i;
  if (mode == 0) {
    st[0] = sc[0];
    st[1] = 0.0;
  } else if (mode == 1) {
    if (st[1] != 0.0) sc[1] = 0.0;
  } else if (st[1] == 0.0 && sc[0] <= tol2 * st[0]) {
    st[1] = 1.0;
  }
}

hipError_t inner_stop(int mode, int nblocks, int nrhs, double tol, double *scal, double *stop, hipStream_t st) {
  const int n = nblocks * nrhs;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inner_stop, dim3((n + 255) / 256), dim3(256), 0, st, mode, n, tol * tol, scal, stop);
  return hipGetLastError();
}

}  // namespace mspcg
