// FP64 (complex128 field) instantiation of the propagation kernels, plus the
// precision-independent control kernels.
#include "gmm_launch_impl.hpp"
template struct gmm::Launch<double>;

namespace gmm {

// Fixed-order reduction of the partial sums and the stopping decision.
__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ partials, int nblocks, Ctrl* ctrl,
                                                     double tol, int fixed_iters, int max_iter) {
  if (skip_iteration(ctrl)) return;
  __shared__ double red[2][256];
  double d = 0.0, s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    d += partials[2 * b];
    s += partials[2 * b + 1];
  }
  red[0][threadIdx.x] = d;
  red[1][threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double eps = red[1][0] > 0.0 ? sqrt(red[0][0] / red[1][0]) : 0.0;
    const int it = ctrl->iters + 1;
    ctrl->eps = eps;
    ctrl->iters = it;
    if (!isfinite(eps)) {
      ctrl->status = 2;
      ctrl->done = 1;
    } else if (fixed_iters > 0) {
      if (it >= fixed_iters) ctrl->done = 1;
    } else if (eps < tol) {
      ctrl->done = 1;
    } else if (it >= max_iter) {
      ctrl->status = 1;
      ctrl->done = 1;
    }
  }
}

__global__ void k_ctrl_reset(Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->eps = 0.0;
    ctrl->iters = 0;
    ctrl->done = 0;
    ctrl->status = 0;
    ctrl->pad = 0;
  }
}


hipError_t launch_norm_final(const double* partials, int nblocks, Ctrl* ctrl, double tol, int fixed_iters,
                             int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, partials, nblocks, ctrl, tol, fixed_iters, max_iter);
  return hipGetLastError();
}
hipError_t launch_ctrl_reset(Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, ctrl);
  return hipGetLastError();
}
}  // namespace gmm
