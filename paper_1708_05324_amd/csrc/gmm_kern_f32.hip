// FP32 (complex64 field) instantiation of the propagation kernels.
#include "gmm_launch_impl.hpp"
template struct gmm::Launch<float>;

namespace gmm {

hipError_t launch_pairs_bf16(int logn, bool raman, const cplx<float>* A, uint32_t* Bhi, uint32_t* Blo,
                             const int2* pairs, int N, int Np, int count, const cplx<float>* Gs,
                             const cplx<float>* tw, const Ctrl* ctrl, hipStream_t s) {
  using T = float;
  constexpr int KB = kBf16Kpad / 8;
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, 4>;
    const int total = (Np + 1) / 2 * count;
    dim3 grid(8 * ((total + 7) / 8));
    if (raman)
      hipLaunchKernelGGL((k_pairs_bf16<LOGN, true>), grid, dim3(S::THREADS), 0, s, A, Bhi, Blo, pairs, N, Np, count,
                         KB, Gs, tw, ctrl);
    else
      hipLaunchKernelGGL((k_pairs_bf16<LOGN, false>), grid, dim3(S::THREADS), 0, s, A, Bhi, Blo, pairs, N, Np,
                         count, KB, Gs, tw, ctrl);
  });
  return hipGetLastError();
}

template <int RT, int KPAD>
static int contract_bf16_blocks() {
  static int blocks = 0;
  if (blocks == 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_contract_bf16<RT, KPAD>, 256,
                                                     ContractBf16Shape<RT, KPAD>::lds_bytes()) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    blocks = per_cu * device_cus();
  }
  return blocks;
}

hipError_t launch_contract_bf16(int rt, int kpad, const void* Shi, const void* Slo, const uint32_t* Bhi,
                                const uint32_t* Blo, cplx<float>* A_NL, const int* pidx, int N, int Nt, int count,
                                const Ctrl* ctrl, hipStream_t s) {
  const int ntiles = count * (Nt / 64);
#define GMM_BF_CASE(R, KP)                                                                                        \
  if (rt == R && kpad == KP) {                                                                                    \
    const int nb = std::min(ntiles, contract_bf16_blocks<R, KP>());                                               \
    hipLaunchKernelGGL((k_contract_bf16<R, KP>), dim3(nb), dim3(256), (ContractBf16Shape<R, KP>::lds_bytes()), s, \
                       (const uint4*)Shi, (const uint4*)Slo, (const uint4*)Bhi, (const uint4*)Blo, A_NL, pidx, N, \
                       Nt, ntiles, ctrl);                                                                         \
    return hipGetLastError();                                                                                     \
  }
  GMM_BF_CASE(1, 128)
  GMM_BF_CASE(2, 128)
  GMM_BF_CASE(1, 64)
  GMM_BF_CASE(2, 64)
#undef GMM_BF_CASE
  return hipErrorInvalidValue;
}

template <int RPAD, bool BF16>
static int contract_cols_blocks() {
  static int blocks = 0;
  if (blocks == 0) {
    constexpr size_t lds = ColShape<RPAD, BF16>::lds_bytes();
    if (lds > 65536 && hipFuncSetAttribute((const void*)k_contract_cols<RPAD, BF16>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_contract_cols<RPAD, BF16>, 256, lds) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    blocks = per_cu * device_cus();
  }
  return blocks;
}

hipError_t launch_contract_cols(int rpad, bool bf16, const void* Ua, const void* Ub, const void* Ya, const void* Yb,
                                cplx<float>* A_NL, int N, int kv, int Nt, int count, const Ctrl* ctrl,
                                hipStream_t s) {
  const int ntiles = count * (Nt / 64);
#define GMM_COL_CASE(RP, BF)                                                                                  \
  if (rpad == RP && bf16 == BF) {                                                                             \
    const int cap = contract_cols_blocks<RP, BF>();                                                          \
    if (cap < 1) return hipErrorInvalidConfiguration;                                                        \
    const int nb = std::min((ntiles + 3) / 4, cap);                                                          \
    hipLaunchKernelGGL((k_contract_cols<RP, BF>), dim3(nb), dim3(256), (ColShape<RP, BF>::lds_bytes()), s, Ua, \
                       Ub, Ya, Yb, A_NL, N, kv, Nt, ntiles, ctrl);                                           \
    return hipGetLastError();                                                                                 \
  }
  GMM_COL_CASE(64, true)
  GMM_COL_CASE(128, true)
  GMM_COL_CASE(64, false)
  GMM_COL_CASE(128, false)
#undef GMM_COL_CASE
  return hipErrorInvalidValue;
}

template <int RQ, int KP, bool BF16>
static int project_cols_blocks() {
  static int blocks = 0;
  if (blocks == 0) {
    constexpr size_t lds = ProjShape<RQ, KP, BF16>::lds_bytes();
    if (lds > 65536 && hipFuncSetAttribute((const void*)k_project_cols<RQ, KP, BF16>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_project_cols<RQ, KP, BF16>, 256,
                                                     lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    blocks = per_cu * device_cus();
  }
  return blocks;
}

hipError_t launch_project_cols(int rq, int kpad, bool bf16, const void* Va, const void* Vb, const cplx<float>* A,
                               float* Y, int N, int Nt, int count, const Ctrl* ctrl, hipStream_t s) {
  const int ntiles = count * (Nt / 64);
#define GMM_PC_CASE(RQ, KP, BF)                                                                                 \
  if (rq == RQ && kpad == KP && bf16 == BF) {                                                                   \
    const int cap = project_cols_blocks<RQ, KP, BF>();                                                         \
    if (cap < 1) return hipErrorInvalidConfiguration;                                                          \
    const int nb = std::min((ntiles + 3) / 4, cap);                                                            \
    hipLaunchKernelGGL((k_project_cols<RQ, KP, BF>), dim3(nb), dim3(256), (ProjShape<RQ, KP, BF>::lds_bytes()), \
                       s, Va, Vb, A, Y, N, Nt, ntiles, ctrl);                                                  \
    return hipGetLastError();                                                                                   \
  }
#define GMM_PC_RQ(RQ) GMM_PC_CASE(RQ, 64, true) GMM_PC_CASE(RQ, 128, true) GMM_PC_CASE(RQ, 64, false) \
  GMM_PC_CASE(RQ, 128, false)
  GMM_PC_RQ(16)
  GMM_PC_RQ(32)
  GMM_PC_RQ(48)
  GMM_PC_RQ(64)
#undef GMM_PC_RQ
#undef GMM_PC_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_conv_bf16(int logn, const float* Y, uint32_t* Bhi, uint32_t* Blo, int R, int RQ, int count,
                            const cplx<float>* Gs, const cplx<float>* tw, const Ctrl* ctrl, hipStream_t s) {
  using T = float;
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, 4, kConvLogR<LOGN, true>>;
    const int total = (R + 1) / 2 * count;
    dim3 grid(8 * ((total + 7) / 8));
    hipLaunchKernelGGL((k_conv<float, LOGN, true>), grid, dim3(S::THREADS), 0, s, Y, nullptr, Bhi, Blo, R, RQ,
                       count, 32, Gs, tw, ctrl);
  });
  return hipGetLastError();
}

}  // namespace gmm
