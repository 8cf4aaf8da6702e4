// FP64 (complex128 field) instantiation of the propagation kernels, plus the
// precision-independent control kernels.
#include "gmm_launch_impl.hpp"
template struct gmm::Launch<double>;

namespace gmm {

// Fixed-order reduction of the partial sums and the stopping decision: thread
// t adds partials t, t + 256, ... in order, each wave reduces its 64 sums by a
// butterfly of lane shuffles (the same pairing every launch: deterministic),
// and thread 0 adds the four wave sums in wave order after one barrier.  With
// `host` (pinned host memory mapped for the device), thread 0 also stores the
// updated control block there, so the host reads it once the launch is done
// instead of queueing a copy after every iteration.
__device__ __forceinline__ void norm_final_block(const double* __restrict__ partials, int nblocks, Ctrl* ctrl,
                                                 Ctrl* host, double tol, int fixed_iters, int max_iter) {
  __shared__ double wsum[2][4];
  double d = 0.0, s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    d += partials[2 * b];
    s += partials[2 * b + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d += __shfl_xor(d, o);
    s += __shfl_xor(s, o);
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[0][threadIdx.x >> 6] = d;
    wsum[1][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double dn = (wsum[0][0] + wsum[0][1]) + (wsum[0][2] + wsum[0][3]);
    const double sn = (wsum[1][0] + wsum[1][1]) + (wsum[1][2] + wsum[1][3]);
    // a non-finite sum means a non-finite field value: report it (eps = NaN), never as converged
    const double eps = (!isfinite(dn) || !isfinite(sn)) ? __builtin_nan("") : sn > 0.0 ? sqrt(dn / sn) : 0.0;
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
    if (host != nullptr) *host = *ctrl;
  }
}

__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ partials, int nblocks, Ctrl* ctrl,
                                                     Ctrl* host, double tol, int fixed_iters, int max_iter) {
  if (skip_iteration(ctrl)) return;
  norm_final_block(partials, nblocks, ctrl, host, tol, fixed_iters, max_iter);
}

// One block per slot of a batched round.
__global__ __launch_bounds__(256) void k_norm_final_b(const BatchSlot* __restrict__ slots, int nblocks, double tol,
                                                       int fixed_iters, int max_iter) {
  const BatchSlot d = slots[blockIdx.x];
  norm_final_block(d.partials, nblocks, d.ctrl, d.ctrl_host, tol, fixed_iters, max_iter);
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
                             int max_iter, hipStream_t s, Ctrl* host) {
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, partials, nblocks, ctrl, host, tol, fixed_iters,
                     max_iter);
  return hipGetLastError();
}
// k_gain_matrix: the per-sub-step matrix of the linear-in-A terms of Sec. III.F,
//   Mg_pl = g_p (delta_pl - inv_Isat sum_mn S^R_plmn Phi_mn)   (g != nullptr)
//         + K_pl                                                (K != nullptr)
// with Phi = dt * (sum of the C partials, fixed order) and K_pl = i Q_lp the
// linear mode coupling.  grid (N, count): block (p, j) forms row p; wave w
// takes l = w, w + 4, ..., its lanes split the (m, n) sum, and a fixed-order
// shuffle reduction closes it.
__global__ __launch_bounds__(256) void k_gain_matrix(const cplx<double>* __restrict__ part, int C,
                                                     const cplx<double>* __restrict__ SR,
                                                     const double* __restrict__ g, double inv_Isat, double dt,
                                                     const cplx<double>* __restrict__ K,
                                                     cplx<double>* __restrict__ Mg, int N, const Ctrl* ctrl) {
  if (skip_iteration(ctrl)) return;
  __shared__ cplx<double> sPhi[kGainNmax * kGainNmax];
  const int tid = threadIdx.x, p = blockIdx.x, jj = blockIdx.y, NN = N * N;
  const int lane = tid & 63, wave = tid >> 6;
  const bool sat = g != nullptr && inv_Isat != 0.0;
  if (sat) {
    for (int q = tid; q < NN; q += 256) {
      double re = 0.0, im = 0.0;
      for (int c = 0; c < C; ++c) {
        const cplx<double> v = part[((size_t)jj * C + c) * NN + q];
        re += v.re;
        im += v.im;
      }
      sPhi[q] = cplx<double>{re * dt, im * dt};
    }
  }
  __syncthreads();
  for (int l = wave; l < N; l += 4) {
    double re = 0.0, im = 0.0;
    if (sat) {
      const cplx<double>* srow = SR + ((size_t)p * N + l) * NN;   // S^R_plmn, (m, n) contiguous
      for (int mn = lane; mn < NN; mn += 64) {
        const cplx<double> a = srow[mn], b = sPhi[mn];
        re += a.re * b.re - a.im * b.im;
        im += a.re * b.im + a.im * b.re;
      }
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
      }
    }
    if (lane == 0) {
      const int q = p * N + l;
      cplx<double> m = K != nullptr ? K[q] : cplx<double>{0.0, 0.0};
      if (g != nullptr) {
        const double d = p == l ? 1.0 : 0.0;
        m.re += g[p] * (d - inv_Isat * re);
        m.im -= g[p] * inv_Isat * im;
      }
      Mg[(size_t)jj * NN + q] = m;
    }
  }
}

hipError_t launch_gain_matrix(const cplx<double>* part, int C, const cplx<double>* SR, const double* g,
                              double inv_Isat, double dt, const cplx<double>* K, cplx<double>* Mg, int N, int count,
                              const Ctrl* ctrl, hipStream_t s) {
  if (N > kGainNmax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gain_matrix, dim3(N, count), dim3(256), 0, s, part, C, SR, g, inv_Isat, dt, K, Mg, N, ctrl);
  return hipGetLastError();
}
// Zero fill of a device buffer (a kernel, so that a captured graph records no memset node).
__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* __restrict__ p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes % 4) return hipErrorInvalidValue;
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, words);
  return hipGetLastError();
}

hipError_t launch_norm_final_b(const BatchSlot* slots, int nslots, int nblocks, double tol, int fixed_iters,
                               int max_iter, hipStream_t s) {
  if (nslots < 1) return hipSuccess;
  hipLaunchKernelGGL(k_norm_final_b, dim3(nslots), dim3(256), 0, s, slots, nblocks, tol, fixed_iters, max_iter);
  return hipGetLastError();
}

hipError_t launch_ctrl_reset(Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, ctrl);
  return hipGetLastError();
}
}  // namespace gmm
