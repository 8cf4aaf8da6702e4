// Wide rank-r route (complex64 fields, up to 55 modes).
//
// The packed coupling matrix S^ of the pair products (Np = N(N+1)/2 rows, the
// Kerr and Raman sums of Eq. (1) with S^K = S^R real and symmetric) factors as
// S^ = U V, U [Np][r], V [r][Np], r its numerical rank (190 for the 55
// Hermite-Gauss modes of ten groups, against Np = 1540).  One evaluation of
// the bracket of Eq. (1), per sub-step field A_j(t):
//   B_Q(t)  = Re(A_m A_n^*) for the pairs Q = (m <= n)          k_pairs_wide
//   Y       = V B                                                library GEMM
//   Y'      = g * Y on the r rows (blended Raman filter g)       convolution kernels
//   C       = U Y'                                               library GEMM
//   NL_p(t) = sum_l C_(p,l)(t) A_l(t)                            k_fold_wide
// (S^ (g * B) = U (g * (V B)): the filter acts on time, S^ on the pair index.)
// The two products are plain GEMMs over Nt x count columns and go to rocBLAS;
// the pair products, the bf16 splits and the fold (the parts that touch the
// fields) are kernels here.
//   BF16X3: X W is computed as X^hi W^hi + X^lo W^hi + X^hi W^lo with bf16
//   hi/lo splits and FP32 accumulation: one product over the stacked inner
//   index [X^hi | X^lo] against [W^hi ; W^hi], then X^hi W^lo added to it.
//   FP32: one SGEMM per product.
// Layouts (row-major, time contiguous; one block of rows per sub-step j):
//   B   : BF16 two planes [j][2][Np][Nt] bf16 (hi, lo); FP32 [j][Np][Nt]
//   Y   : [j][RQ][Nt] FP32, rows >= r zero (V is zero there)
//   Y'  : BF16 two planes [j][2][RQ][Nt] bf16; FP32 [j][RQ][Nt]
//   C   : [j][Np][Nt] FP32
#include <rocblas/rocblas.h>

#include "gmm_launch_impl.hpp"

namespace gmm {

__device__ __forceinline__ void bf16_split1(float x, uint16_t& hi, uint16_t& lo) {
  const __bf16 h = (__bf16)x;  // round to nearest even
  const __bf16 l = (__bf16)(x - (float)h);
  hi = __builtin_bit_cast(uint16_t, h);
  lo = __builtin_bit_cast(uint16_t, l);
}

// B_Q(t) = Re(A_m A_n^*) = Re A_m Re A_n + Im A_m Im A_n for Q = n (n + 1) / 2 + m,
// m <= n < N.  One thread per sample t of one sub-step (grid (Nt / 256, count)).
// NMAX >= N fixes the unrolled pair list; fields of modes N..NMAX-1 are not read.
template <int NMAX, bool BF16>
__global__ __launch_bounds__(256) void k_pairs_wide(const cplx<float>* __restrict__ A, void* __restrict__ Bout, int N,
                                                    int Np, int Nt, const Ctrl* ctrl) {
  if (skip_iteration(ctrl)) return;
  const int t = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  const cplx<float>* Aj = A + (size_t)j * N * Nt + t;
  cplx<float> a[NMAX];
#pragma unroll
  for (int l = 0; l < NMAX; ++l) a[l] = l < N ? Aj[(size_t)l * Nt] : cplx<float>{0.f, 0.f};
  static_for<0, NMAX>([&](auto nc) {
    constexpr int n = decltype(nc)::value;
    if (n < N) {
      static_for<0, n + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        constexpr int Q = n * (n + 1) / 2 + m;
        const float b = a[m].re * a[n].re + a[m].im * a[n].im;
        if constexpr (BF16) {
          uint16_t h, l;
          bf16_split1(b, h, l);
          uint16_t* hp = reinterpret_cast<uint16_t*>(Bout) + (size_t)j * 2 * Np * Nt + (size_t)Q * Nt + t;
          hp[0] = h;
          hp[(size_t)Np * Nt] = l;
        } else {
          reinterpret_cast<float*>(Bout)[((size_t)j * Np + Q) * Nt + t] = b;
        }
      });
    }
  });
}

// FP32 rows [count][rows][Nt] -> bf16 planes [count][2][rows][Nt] (hi, lo), two elements a thread.
__global__ __launch_bounds__(256) void k_split_rows(const float* __restrict__ Y, uint32_t* __restrict__ P,
                                                    size_t per_pair, const Ctrl* ctrl) {
  if (skip_iteration(ctrl)) return;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;  // element pair within one sub-step
  if (e >= per_pair) return;
  const size_t j = blockIdx.y;
  const float2 x = reinterpret_cast<const float2*>(Y)[j * per_pair + e];
  uint32_t h, l;
  bf16_split2(x.x, x.y, h, l);
  P[(2 * j) * per_pair + e] = h;
  P[(2 * j + 1) * per_pair + e] = l;
}

// NL_p(t) = sum_l C_(p,l)(t) A_l(t) over the pairs in triangular order: pair
// (m <= n) adds C A_n to NL_m and, for m != n, C A_m to NL_n.  One thread per
// sample; it reads A_l(t) of its sample for every l before writing any NL_p(t),
// so NL overwrites A in place.
template <int NMAX>
__global__ __launch_bounds__(256) void k_fold_wide(const float* __restrict__ C, cplx<float>* A_NL, int N, int Np,
                                                   int Nt, const Ctrl* ctrl) {
  if (skip_iteration(ctrl)) return;
  const int t = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  cplx<float>* Aj = A_NL + (size_t)j * N * Nt + t;
  const float* Cj = C + (size_t)j * Np * Nt + t;
  cplx<float> a[NMAX], nl[NMAX];
#pragma unroll
  for (int l = 0; l < NMAX; ++l) {
    a[l] = l < N ? Aj[(size_t)l * Nt] : cplx<float>{0.f, 0.f};
    nl[l] = cplx<float>{0.f, 0.f};
  }
  static_for<0, NMAX>([&](auto nc) {
    constexpr int n = decltype(nc)::value;
    if (n < N) {
      static_for<0, n + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        const float c = Cj[(size_t)(n * (n + 1) / 2 + m) * Nt];
        nl[m].re += c * a[n].re;
        nl[m].im += c * a[n].im;
        if constexpr (m != n) {
          nl[n].re += c * a[m].re;
          nl[n].im += c * a[m].im;
        }
      });
    }
  });
#pragma unroll
  for (int p = 0; p < NMAX; ++p)
    if (p < N) Aj[(size_t)p * Nt] = nl[p];
}

namespace {
// smallest instantiated NMAX >= N (triangular mode counts of 3..10 groups), 0 if none
int wide_nmax(int N) {
  for (int v : {6, 10, 15, 21, 28, 36, 45, 55})
    if (N <= v) return v;
  return 0;
}
}  // namespace

int wide_max_modes() { return 55; }

hipError_t launch_pairs_wide(bool bf16, const cplx<float>* A, void* Bout, int N, int Np, int Nt, int count,
                             const Ctrl* ctrl, hipStream_t s) {
  if (count < 1) return hipSuccess;
  if (Nt % 256) return hipErrorInvalidValue;
  const dim3 grid(Nt / 256, count);
#define GMM_WIDE_CASE(NM)                                                                                     \
  case NM:                                                                                                    \
    if (bf16)                                                                                                 \
      hipLaunchKernelGGL((k_pairs_wide<NM, true>), grid, dim3(256), 0, s, A, Bout, N, Np, Nt, ctrl);          \
    else                                                                                                      \
      hipLaunchKernelGGL((k_pairs_wide<NM, false>), grid, dim3(256), 0, s, A, Bout, N, Np, Nt, ctrl);         \
    return hipGetLastError();
  switch (wide_nmax(N)) {
    GMM_WIDE_CASE(6)
    GMM_WIDE_CASE(10)
    GMM_WIDE_CASE(15)
    GMM_WIDE_CASE(21)
    GMM_WIDE_CASE(28)
    GMM_WIDE_CASE(36)
    GMM_WIDE_CASE(45)
    GMM_WIDE_CASE(55)
    default:
      return hipErrorInvalidValue;
  }
#undef GMM_WIDE_CASE
}

hipError_t launch_fold_wide(const float* C, cplx<float>* A_NL, int N, int Np, int Nt, int count, const Ctrl* ctrl,
                            hipStream_t s) {
  if (count < 1) return hipSuccess;
  if (Nt % 256) return hipErrorInvalidValue;
  const dim3 grid(Nt / 256, count);
#define GMM_WIDE_CASE(NM)                                                                       \
  case NM:                                                                                      \
    hipLaunchKernelGGL((k_fold_wide<NM>), grid, dim3(256), 0, s, C, A_NL, N, Np, Nt, ctrl);     \
    return hipGetLastError();
  switch (wide_nmax(N)) {
    GMM_WIDE_CASE(6)
    GMM_WIDE_CASE(10)
    GMM_WIDE_CASE(15)
    GMM_WIDE_CASE(21)
    GMM_WIDE_CASE(28)
    GMM_WIDE_CASE(36)
    GMM_WIDE_CASE(45)
    GMM_WIDE_CASE(55)
    default:
      return hipErrorInvalidValue;
  }
#undef GMM_WIDE_CASE
}

hipError_t launch_split_rows(const float* Y, void* planes, int rows, int Nt, int count, const Ctrl* ctrl,
                             hipStream_t s) {
  if (count < 1) return hipSuccess;
  const size_t per_pair = (size_t)rows * Nt / 2;
  hipLaunchKernelGGL(k_split_rows, dim3((unsigned)((per_pair + 255) / 256), count), dim3(256), 0, s, Y,
                     (uint32_t*)planes, per_pair, ctrl);
  return hipGetLastError();
}

// Column-major view of one sub-step: X [k rows][m = Nt] row-major is the m x k
// operand with leading dimension m; W [n][k] row-major is the k x n operand
// with leading dimension k; the result [n][m] row-major is m x n, ldc = m.
hipError_t wide_gemm(void* handle, bool bf16, int m, int n, int k, const void* X, const void* Wst, const void* Wlo,
                     float* out, int count, hipStream_t s) {
  if (count < 1) return hipSuccess;
  rocblas_handle h = (rocblas_handle)handle;
  if (rocblas_set_stream(h, s) != rocblas_status_success) return hipErrorInvalidHandle;
  const float one = 1.f, zero = 0.f;
  rocblas_status st;
  if (bf16) {
    // [X^hi | X^lo] (m x 2k, the two planes of a sub-step) . [W^hi ; W^hi] (2k x n)
    st = (rocblas_gemm_strided_batched_ex)(h, rocblas_operation_none, rocblas_operation_none, m, n, 2 * k, &one, X,
                                           rocblas_datatype_bf16_r, m, (rocblas_stride)2 * k * m, Wst,
                                           rocblas_datatype_bf16_r, 2 * k, 0, &zero, out, rocblas_datatype_f32_r, m,
                                           (rocblas_stride)n * m, out, rocblas_datatype_f32_r, m,
                                           (rocblas_stride)n * m, count, rocblas_datatype_f32_r,
                                           rocblas_gemm_algo_standard, 0, 0);
    // + X^hi (m x k) . W^lo (k x n)
    if (st == rocblas_status_success)
      st = (rocblas_gemm_strided_batched_ex)(h, rocblas_operation_none, rocblas_operation_none, m, n, k, &one, X,
                                             rocblas_datatype_bf16_r, m, (rocblas_stride)2 * k * m, Wlo,
                                             rocblas_datatype_bf16_r, k, 0, &one, out, rocblas_datatype_f32_r, m,
                                             (rocblas_stride)n * m, out, rocblas_datatype_f32_r, m,
                                             (rocblas_stride)n * m, count, rocblas_datatype_f32_r,
                                             rocblas_gemm_algo_standard, 0, 0);
  } else {
    st = rocblas_sgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, m, n, k, &one,
                                       (const float*)X, m, (rocblas_stride)k * m, (const float*)Wst, k, 0, &zero, out,
                                       m, (rocblas_stride)n * m, count);
  }
  return st == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

int wide_blas_create(void** handle) {
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return -1;
  *handle = h;
  return 0;
}

void wide_blas_destroy(void* handle) {
  if (handle) (void)rocblas_destroy_handle((rocblas_handle)handle);
}

}  // namespace gmm
