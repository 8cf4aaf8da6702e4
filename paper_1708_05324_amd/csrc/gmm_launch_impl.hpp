// Definitions of the Launch<T> members; included once per precision.
#pragma once
#include "gmm_kernels.hpp"
#include "gmm_launch.hpp"

#include <algorithm>

namespace gmm {

template <typename T>
constexpr int max_logn() { return sizeof(T) == 8 ? 14 : 15; }

#define GMM_LOGN_SWITCH(logn, ...)                    \
  switch (logn) {                                     \
    case 8: { constexpr int LOGN = 8; __VA_ARGS__; } break;   \
    case 9: { constexpr int LOGN = 9; __VA_ARGS__; } break;   \
    case 10: { constexpr int LOGN = 10; __VA_ARGS__; } break; \
    case 11: { constexpr int LOGN = 11; __VA_ARGS__; } break; \
    case 12: { constexpr int LOGN = 12; __VA_ARGS__; } break; \
    case 13: { constexpr int LOGN = 13; __VA_ARGS__; } break; \
    case 14: { constexpr int LOGN = 14; __VA_ARGS__; } break; \
    case 15: {                                         \
      if constexpr (max_logn<T>() >= 15) {             \
        constexpr int LOGN = max_logn<T>();            \
        __VA_ARGS__;                                   \
      } else {                                         \
        return hipErrorInvalidValue;                   \
      }                                                \
    } break;                                           \
    default: return hipErrorInvalidValue;              \
  }

template <typename T>
bool Launch<T>::supports_logn(int logn) {
  return logn >= 8 && logn <= max_logn<T>();
}

template <typename T>
hipError_t Launch<T>::fft_rows(int logn, int sign, const cplx<T>* in, cplx<T>* out, T scale, int rows,
                               const cplx<T>* tw, hipStream_t s) {
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T)>;
    if (sign < 0)
      hipLaunchKernelGGL((k_fft_rows<T, LOGN, -1>), dim3(rows), dim3(S::THREADS), 0, s, in, out, scale, tw);
    else
      hipLaunchKernelGGL((k_fft_rows<T, LOGN, +1>), dim3(rows), dim3(S::THREADS), 0, s, in, out, scale, tw);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::phase_table(cplx<T>* E, const double* coef, int nb, int N, int nt, int rows, double dz,
                                  double domega, hipStream_t s, int j0) {
  const long total = (long)rows * N * nt;
  hipLaunchKernelGGL((k_phase_table<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, E, coef, nb, N, nt,
                     total, dz, domega, j0);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::phase_table_lam(cplx<T>* E, const double* lam, int N, int nt, int rows, double dz,
                                      hipStream_t s, int j0) {
  const long total = (long)rows * N * nt;
  hipLaunchKernelGGL((k_phase_table_lam<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, E, lam, N, nt,
                     total, dz, j0);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::mode_mix(bool back, const cplx<T>* src, long src_jrows, cplx<T>* dst, const cplx<T>* U,
                               const cplx<T>* E, int j0, int N, int nt, int count, const Ctrl* ctrl, hipStream_t s) {
  constexpr int W = mix_width<T>();  // frequencies per block
  if (N < 1 || N > kGainNmax || nt % W || count < 1) return hipErrorInvalidValue;
  const size_t lds = mix_lds_bytes<T>(N);
  const int lds_max = (int)mix_lds_bytes<T>(kGainNmax);
  if (back) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_mode_mix<T, true>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_mode_mix<T, true>), dim3(nt / W), dim3(256), lds, s, src, src_jrows, dst, U, E, j0, N, nt,
                       count, ctrl);
  } else {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_mode_mix<T, false>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_mode_mix<T, false>), dim3(nt / W), dim3(256), lds, s, src, src_jrows, dst, U, E, j0, N, nt,
                       count, ctrl);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::conv_os(const T* Y, T* Yout, int R, int RQ, int count, int Nt, int Lh, int V,
                              const cplx<T>* Gf, const cplx<T>* twf, const Ctrl* ctrl, hipStream_t s) {
  using S = FftShape<kOsLogF, (int)sizeof(T), 4>;
  if (Lh < 1 || V < 1 || Lh - 1 + V > S::N || Nt < S::N || (Nt & (Nt - 1))) return hipErrorInvalidValue;
  const int nseg = (Nt + V - 1) / V, total = nseg * ((R + 1) / 2) * count;
  hipLaunchKernelGGL((k_conv_os<T, false>), dim3(8 * ((total + 7) / 8)), dim3(S::THREADS), 0, s, Y, Yout, nullptr,
                     nullptr, R, RQ, count, 32, Nt, Lh, V, nseg, Gf, twf, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pairs_os(const cplx<T>* A, T* Bp, const int2* pairs, int N, int Np, int count, int Nt, int Lh,
                               int V, const cplx<T>* Gf, const cplx<T>* twf, const Ctrl* ctrl, hipStream_t s) {
  using S = FftShape<kOsLogF, (int)sizeof(T), 4>;
  if (Lh < 1 || V < 1 || Lh - 1 + V > S::N || Nt < S::N || (Nt & (Nt - 1))) return hipErrorInvalidValue;
  const int nseg = (Nt + V - 1) / V, total = nseg * ((Np + 1) / 2) * count;
  hipLaunchKernelGGL((k_pairs_os<T, false>), dim3(8 * ((total + 7) / 8)), dim3(S::THREADS), 0, s, A, Bp, nullptr,
                     nullptr, pairs, N, Np, count, 0, Nt, Lh, V, nseg, Gf, twf, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::phase_to_time(int logn, const cplx<T>* psi, long psi_jrows, cplx<T>* A, const cplx<T>* E,
                                    int N, int count, int j0, const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s) {
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T)>;
    hipLaunchKernelGGL((k_phase_to_time<T, LOGN>), dim3(N, count), dim3(S::THREADS), 0, s, psi, psi_jrows, A, E, j0,
                       tw, ctrl);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pairs(int logn, bool raman, const cplx<T>* A, T* Bp, const int2* pairs, int N, int Np,
                            int count, const cplx<T>* Gs, const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s) {
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T)>;
    const int total = (Np + 1) / 2 * count;
    dim3 grid(8 * ((total + 7) / 8));
    if (raman)
      hipLaunchKernelGGL((k_pairs<T, LOGN, true>), grid, dim3(S::THREADS), 0, s, A, Bp, pairs, N, Np, count, Gs, tw,
                         ctrl);
    else
      hipLaunchKernelGGL((k_pairs<T, LOGN, false>), grid, dim3(S::THREADS), 0, s, A, Bp, pairs, N, Np, count, Gs, tw,
                         ctrl);
  });
  return hipGetLastError();
}

template <typename T, int RT, int KPAD>
int contract_reg_blocks() {
  static int blocks = 0;
  if (blocks == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_contract_reg<T, RT, KPAD>, 256,
                                                     contract_reg_lds<RT, T>()) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    blocks = per_cu * cus;
  }
  return blocks;
}

inline int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
  }
  return cus;
}

template <typename T>
hipError_t Launch<T>::contract(int rt, int kpad, const T* ST, const T* Bp, cplx<T>* A_NL, const int* pidx, int N,
                               int kv, int Nt, int count, const Ctrl* ctrl, hipStream_t s, int blocks_per_cu) {
  const int ntiles = count * (Nt / 64);
#define GMM_RT_REG(R, KP)                                                                                   \
  if (rt == R && (kpad == KP || (kpad == 0 && KP == 64 * R))) {                                              \
    int cap = contract_reg_blocks<T, R, KP>();                                                               \
    if (blocks_per_cu > 0) cap = std::min(cap, blocks_per_cu * device_cus());                                \
    const int nb = std::min(ntiles, cap);                                                                    \
    hipLaunchKernelGGL((k_contract_reg<T, R, KP>), dim3(nb), dim3(256), (contract_reg_lds<R, T>()), s, ST, Bp, \
                       A_NL, pidx, N, kv, Nt, ntiles, ctrl);                                                 \
    return hipGetLastError();                                                                                \
  }
  GMM_RT_REG(1, 64)
  GMM_RT_REG(2, 128)
  GMM_RT_REG(2, 64)
#undef GMM_RT_REG
  if (kpad != 0) return hipErrorInvalidValue;
  dim3 grid(ntiles);
  switch (rt) {
#define GMM_RT_CASE(R)                                                                                         \
  case R: {                                                                                                    \
    constexpr size_t lds = ContractShape<R>::template lds_bytes<T>();                                          \
    if constexpr (lds > 65536) {                                                                               \
      static const hipError_t attr = hipFuncSetAttribute((const void*)k_contract<T, R>,                        \
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (attr != hipSuccess) return attr;                                                                     \
    }                                                                                                          \
    hipLaunchKernelGGL((k_contract<T, R>), grid, dim3(256), lds, s, ST, Bp, A_NL, pidx, N, kv, Nt, ctrl);      \
  } break;
    GMM_RT_CASE(3)
    GMM_RT_CASE(4)
#undef GMM_RT_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::project(int rq, int kp, const T* VT, const cplx<T>* A, T* Y, const int2* pairs, int N, int Np,
                              int Nt, int count, const Ctrl* ctrl, hipStream_t s) {
  const int ntiles = count * (Nt / 64);
  const int nb = std::min(ntiles, 2 * device_cus());
#define GMM_PROJ(RQ, KP)                                                                                     \
  if (rq == RQ && kp == KP) {                                                                                 \
    hipLaunchKernelGGL((k_project<T, RQ, KP>), dim3(nb), dim3(256), (project_lds<T, RQ, KP>()), s, VT, A, Y,  \
                       pairs, N, Np, Nt, ntiles, ctrl);                                                       \
    return hipGetLastError();                                                                                 \
  }
#define GMM_PROJ_K(RQ) GMM_PROJ(RQ, 64) GMM_PROJ(RQ, 128) GMM_PROJ(RQ, 192) GMM_PROJ(RQ, 256)
  GMM_PROJ_K(16)
  GMM_PROJ_K(32)
  GMM_PROJ_K(48)
  GMM_PROJ_K(64)
#undef GMM_PROJ_K
#undef GMM_PROJ
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t Launch<T>::conv(int logn, const T* Y, T* Yout, int R, int RQ, int count, const cplx<T>* Gs,
                           const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s) {
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T), kConvLogR<LOGN, false>>;
    const int total = (R + 1) / 2 * count;
    dim3 grid(8 * ((total + 7) / 8));
    hipLaunchKernelGGL((k_conv<T, LOGN, false>), grid, dim3(S::THREADS), 0, s, Y, Yout, nullptr, nullptr, R, RQ,
                       count, 0, Gs, tw, ctrl);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::spectral_out(int logn, const cplx<T>* in, cplx<T>* out, const cplx<T>* E, int N, int count,
                                   int j0, double domega, double gscale, double inv_omega0, int shock,
                                   const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s) {
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T), kSpectralLogR<LOGN>, true>;
    hipLaunchKernelGGL((k_spectral_out<T, LOGN>), dim3(N, count), dim3(S::THREADS), 0, s, in, out, E, j0, domega,
                       gscale, inv_omega0, shock, tw, ctrl);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::trapz(const cplx<T>* psi0, const cplx<T>* I0, const cplx<T>* I, cplx<T>* psi,
                            cplx<T>* I0_keep, int first, int M, long nn, T dz, double* partials, const Ctrl* ctrl,
                            hipStream_t s, const cplx<T>* E, const cplx<double>* Em64, cplx<T>* psi0_keep,
                            Ctrl* reset) {
  if (E != nullptr)
    hipLaunchKernelGGL((k_trapz_lab<T>), dim3(trapz_blocks(nn)), dim3(256), 0, s, psi0, I0, I, psi, I0_keep, E, Em64,
                       first, M, nn, dz, partials, ctrl, psi0_keep, reset);
  else if (psi0_keep != nullptr || reset != nullptr)
    return hipErrorInvalidValue;  // the start field is a separate kept copy in the psi frame
  else
    hipLaunchKernelGGL((k_trapz<T>), dim3(trapz_blocks(nn)), dim3(256), 0, s, psi0, I0, I, psi, I0_keep, first, M,
                       nn, dz, partials, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::close(const cplx<T>* src, cplx<T>* dst, const cplx<T>* Em, long nn, Ctrl* ctrl,
                            hipStream_t s, const cplx<double>* Em64) {
  hipLaunchKernelGGL((k_close<T>), dim3(trapz_blocks(nn)), dim3(256), 0, s, src, dst, Em, Em64, nn, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pairs_dense(int logn, bool raman, const cplx<T>* A, T* Bd, const int2* pairs, int N, int Np,
                                  int count, int KD, const cplx<T>* Hr, const cplx<T>* tw, const Ctrl* ctrl,
                                  hipStream_t s) {
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T)>;
    const int total = Np * count;
    dim3 grid(8 * ((total + 7) / 8));
    if (raman)
      hipLaunchKernelGGL((k_pairs_dense<T, LOGN, true>), grid, dim3(S::THREADS), 0, s, A, Bd, pairs, N, Np, count,
                         KD, Hr, tw, ctrl);
    else
      hipLaunchKernelGGL((k_pairs_dense<T, LOGN, false>), grid, dim3(S::THREADS), 0, s, A, Bd, pairs, N, Np, count,
                         KD, Hr, tw, ctrl);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::contract_dense(const T* G, const T* Bd, cplx<T>* A_NL, int N, int KD, int rows_pad, int Nt,
                                     int count, const Ctrl* ctrl, hipStream_t s) {
  const size_t lds = (size_t)64 * 64 * sizeof(T) + (size_t)2 * N * 64 * sizeof(cplx<T>);
  if (lds > 65536) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_contract_dense<T>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)contract_dense_lds<T>(22));
    if (attr != hipSuccess) return attr;
  }
  hipLaunchKernelGGL((k_contract_dense<T>), dim3(count * (Nt / 64)), dim3(256), lds, s, G, Bd, A_NL, N, KD,
                     rows_pad, Nt, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pair_integrals(const cplx<T>* A, cplx<double>* part, int N, int Nt, int count,
                                     const Ctrl* ctrl, hipStream_t s) {
  if (N > kGainNmax || Nt % kGainChunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_pair_integrals<T>), dim3(gain_partials(Nt), count), dim3(256), 0, s, A, part, N, Nt, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::gain_add(const cplx<T>* psi, long psi_jrows, const cplx<T>* E, int j0,
                               const cplx<double>* Mg, cplx<T>* out, int N, int Nt, int count, const Ctrl* ctrl,
                               hipStream_t s) {
  if (N > kGainNmax || Nt % 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gain_add<T>), dim3(Nt / 256, count), dim3(256), 0, s, psi, psi_jrows, E, j0, Mg, out, N, Nt,
                     ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::rk4ip_stage(int stage, cplx<T>* At, cplx<T>* AI, cplx<T>* k1, const cplx<T>* k2,
                                  const cplx<T>* k3, const cplx<T>* k4, cplx<T>* X, const cplx<T>* Eh, T h, long nn,
                                  hipStream_t s) {
  hipLaunchKernelGGL((k_rk4ip_stage<T>), dim3(trapz_blocks(nn)), dim3(256), 0, s, stage, At, AI, k1, k2, k3, k4, X,
                     Eh, h, nn);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::spec_sums(const cplx<T>* At, int nt, long nn, double domega, double omega0, double* partials,
                                hipStream_t s) {
  hipLaunchKernelGGL((k_spec_sums<T>), dim3(trapz_blocks(nn)), dim3(256), 0, s, At, nt, nn, domega, omega0,
                     partials);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::finish_H(const cplx<double>* H, cplx<T>* Gs, int nt, double fR, hipStream_t s) {
  hipLaunchKernelGGL((k_finish_H<T>), dim3((nt + 255) / 256), dim3(256), 0, s, H, Gs, nt, fR);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::phase_to_time_b(int logn, const BatchRow* rows, const cplx<T>* psi0, const cplx<T>* psi,
                                      const cplx<T>* E, cplx<T>* A, int N, int R, int M, const cplx<T>* tw, int lab,
                                      hipStream_t s) {
  if (R < 1) return hipSuccess;
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T)>;
    hipLaunchKernelGGL((k_phase_to_time_b<T, LOGN>), dim3(N, R), dim3(S::THREADS), 0, s, rows, psi0, psi, E, A, M,
                       tw, lab);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::spectral_out_b(int logn, const BatchRow* rows, cplx<T>* W, const cplx<T>* E, int N, int R,
                                     int M, double domega, double gscale, double inv_omega0, int shock,
                                     const cplx<T>* tw, int lab, hipStream_t s) {
  if (R < 1) return hipSuccess;
  GMM_LOGN_SWITCH(logn, {
    using S = FftShape<LOGN, (int)sizeof(T), kSpectralLogR<LOGN>, true>;
    hipLaunchKernelGGL((k_spectral_out_b<T, LOGN>), dim3(N, R), dim3(S::THREADS), 0, s, rows, W, E, M, domega, gscale,
                       inv_omega0, shock, tw, lab);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::trapz_b(const BatchSlot* slots, int nslots, long nn, hipStream_t s) {
  if (nslots < 1) return hipSuccess;
  hipLaunchKernelGGL((k_trapz_b<T>), dim3(trapz_blocks(nn), nslots), dim3(256), 0, s, slots, nn);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::close_b(const BatchSlot* slots, int nslots, long nn, hipStream_t s) {
  if (nslots < 1) return hipSuccess;
  hipLaunchKernelGGL((k_close_b<T>), dim3(trapz_blocks(nn), nslots), dim3(256), 0, s, slots, nn);
  return hipGetLastError();
}

}  // namespace gmm
