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

// k_contract_dense_bf16: the general-route product C = G B followed by the
// complex fold NL_p = sum_l C_pl A_l, for BF16X3 plans (up to 15 modes, so at
// most 29 blocks of 16 output rows).  G is split into bf16 hi/lo on the host
// ([rows_pad][KD32], K padded with zeros); B is split on the fly from the FP32
// pair rows; products hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16.
//
// One block of 8 waves owns 128 columns; wave w owns columns 16 w .. 16 w + 15
// and every output row, so its accumulators (32 blocks of 16 x 16) stay in
// registers for the whole K loop and B is read once.  Each 32-wide K slice of G
// (hi and lo, all rows) is staged in LDS once per block and read by all eight
// waves: G leaves L2 once per 128 columns.  The 16-byte chunks of a G row are
// XOR-swizzled by bits 1-2 of the row so that eight consecutive lanes of a
// 128-bit LDS read hit distinct banks.  After the K loop the accumulators pass
// through LDS in pieces of 64 rows and are folded into NL (thread (t, g) owns
// the modes p = g mod 4, fixed summation order).  NL overwrites A.
constexpr int kDenseCols = 128, kDenseRB = 29;
constexpr size_t kDenseSlice = (size_t)kDenseRB * 16 * 64;  // bytes of one plane (hi or lo) of one K slice
constexpr size_t kDenseGBytes = 4 * kDenseSlice;              // two slices (double buffer), hi and lo each

__global__ __launch_bounds__(512) void k_contract_dense_bf16(const uint4* __restrict__ Ghi,
                                                             const uint4* __restrict__ Glo,
                                                             const float* __restrict__ Bd, cplx<float>* A_NL, int N,
                                                             int KD, int KD32, int nrb, int Nt, const Ctrl* ctrl) {
  if (skip_iteration(ctrl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* sG = smem_raw;                                          // [2 slices][hi, lo][kDenseRB * 16][64 B]
  float* sC = reinterpret_cast<float*>(smem_raw);                        // [64][128], aliases sG after the K loop
  cplx<float>* sA = reinterpret_cast<cplx<float>*>(smem_raw + kDenseGBytes);  // [N][128]
  cplx<float>* sNL = sA + N * kDenseCols;                                // [N][128]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int tiles_per_j = Nt / kDenseCols;
  const int jj = blockIdx.x / tiles_per_j, t0 = (blockIdx.x - jj * tiles_per_j) * kDenseCols;
  cplx<float>* Aj = A_NL + (size_t)jj * N * Nt + t0;
  const float* Bj = Bd + (size_t)jj * KD * Nt + t0 + 16 * wave + lr;
  for (int i = tid; i < N * kDenseCols; i += 512) {
    sA[i] = Aj[(size_t)(i >> 7) * Nt + (i & 127)];
    sNL[i] = cplx<float>{0.f, 0.f};
  }
  const int KC = KD32 / 8;            // 16-byte chunks per G row
  const int nitems = nrb * 16 * 8;    // (row, chunk) items of one K slice: 4 hi + 4 lo chunks per row
  // fill item it = tid + 512 i: row = it >> 3, plane (hi 0, lo 1) = (it >> 2) & 1, chunk c = it & 3; the
  // thread's global offset and LDS offset are the same for every slice (plus 4 ks chunks, plus the slice)
  const uint4* gsrc[8];
  int gdst[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int it = min(tid + 512 * i, nitems - 1), row = it >> 3, c = it & 3, plane = (it >> 2) & 1;
    gsrc[i] = (plane ? Glo : Ghi) + (size_t)row * KC + c;
    gdst[i] = tid + 512 * i < nitems ? plane * (int)kDenseSlice + row * 64 + ((c ^ (row >> 1)) & 3) * 16 : -1;
  }
  floatx4 acc[kDenseRB];
#pragma unroll
  for (int rb = 0; rb < kDenseRB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  uint4 g0, g1, g2, g3, g4, g5, g6, g7;
  float x[8];
#define GMM_DENSE_LOAD(ks)                                                                          \
  g0 = gsrc[0][4 * (ks)]; g1 = gsrc[1][4 * (ks)]; g2 = gsrc[2][4 * (ks)]; g3 = gsrc[3][4 * (ks)];   \
  g4 = gsrc[4][4 * (ks)]; g5 = gsrc[5][4 * (ks)]; g6 = gsrc[6][4 * (ks)]; g7 = gsrc[7][4 * (ks)];
#define GMM_DENSE_STORE(buf)                                                                        \
  {                                                                                                 \
    unsigned char* d = sG + (buf) * 2 * kDenseSlice;                                                \
    const uint4 gv[8] = {g0, g1, g2, g3, g4, g5, g6, g7};                                          \
    _Pragma("unroll") for (int i = 0; i < 8; ++i) if (gdst[i] >= 0)                                 \
        *reinterpret_cast<uint4*>(d + gdst[i]) = gv[i];                                            \
  }
  const int nks = KD32 / 32;
  GMM_DENSE_LOAD(0);
#pragma unroll
  for (int e = 0; e < 8; ++e) x[e] = 8 * lk + e < KD ? Bj[(size_t)(8 * lk + e) * Nt] : 0.f;
  GMM_DENSE_STORE(0);
  __syncthreads();
  const int swz = ((lk ^ (lr >> 1)) & 3) * 16;  // swizzled chunk lk of row 16 rb + lr
  for (int ks = 0; ks < nks; ++ks) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) bf16_split2(x[2 * e], x[2 * e + 1], h[e], l[e]);
    const bf16x8 bh = __builtin_bit_cast(bf16x8, uint4{h[0], h[1], h[2], h[3]});
    const bf16x8 bl = __builtin_bit_cast(bf16x8, uint4{l[0], l[1], l[2], l[3]});
    if (ks + 1 < nks) {  // next slice of G and of B in flight during this slice's products
      GMM_DENSE_LOAD(ks + 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * (ks + 1) + 8 * lk + e;
        x[e] = k < KD ? Bj[(size_t)k * Nt] : 0.f;
      }
    }
    const unsigned char* src = sG + (ks & 1) * 2 * kDenseSlice + swz;
    static_for<0, kDenseRB>([&](auto rbc) {
      constexpr int RB = decltype(rbc)::value;
      if (RB < nrb) {
        const int off = (16 * RB + lr) * 64;
        const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(src + off));
        const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(src + kDenseSlice + off));
        acc[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[RB], 0, 0, 0);
        acc[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[RB], 0, 0, 0);
        acc[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[RB], 0, 0, 0);
      }
    });
    if (ks + 1 < nks) GMM_DENSE_STORE((ks + 1) & 1);  // the other buffer, last read before the previous barrier
    __syncthreads();
  }
#undef GMM_DENSE_LOAD
#undef GMM_DENSE_STORE
  // fold: accumulator register i of lane (lr, lk) in row block rb is row 16 rb + 4 lk + i
  const int NN = N * N, col = tid & 127, g = tid >> 7;
  static_for<0, (kDenseRB + 3) / 4>([&](auto qc) {
    constexpr int Q = decltype(qc)::value;  // rows 64 Q .. 64 Q + 63
    if (4 * Q < nrb) {
      __syncthreads();  // the K loop (first piece) or the previous fold has finished with the LDS
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 * Q + j < kDenseRB)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            sC[(16 * j + 4 * lk + i) * kDenseCols + 16 * wave + lr] = acc[min(4 * Q + j, kDenseRB - 1)][i];
      __syncthreads();
      // pairs pl = p N + l of this piece, walked with (p, l) carried (wave-uniform, no division in the loop)
      const int r2end = min(32, NN - 32 * Q);
      int p = (32 * Q) / N, l = 32 * Q - p * N;
      for (int r2 = 0; r2 < r2end; ++r2) {
        if ((p & 3) == g) {
          const float cr = sC[(2 * r2) * kDenseCols + col], ci = sC[(2 * r2 + 1) * kDenseCols + col];
          const cplx<float> a = sA[l * kDenseCols + col];
          cplx<float>& o = sNL[p * kDenseCols + col];
          o.re += cr * a.re - ci * a.im;
          o.im += cr * a.im + ci * a.re;
        }
        if (++l == N) l = 0, ++p;
      }
    }
  });
  __syncthreads();
  for (int i = tid; i < N * kDenseCols; i += 512) Aj[(size_t)(i >> 7) * Nt + (i & 127)] = sNL[i];
}

hipError_t launch_contract_dense_bf16(const void* Ghi, const void* Glo, const float* Bd, cplx<float>* A_NL, int N,
                                      int KD, int KD32, int rows_pad, int Nt, int count, const Ctrl* ctrl,
                                      hipStream_t s) {
  const int nrb = (2 * N * N + 15) / 16;
  if (N > 15 || KD32 % 32 || KD > KD32 || nrb > kDenseRB || rows_pad < 16 * nrb || Nt % kDenseCols) return hipErrorInvalidValue;
  const size_t lds = kDenseGBytes + (size_t)2 * N * kDenseCols * sizeof(cplx<float>);
  static const hipError_t attr =
      hipFuncSetAttribute((const void*)k_contract_dense_bf16, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(kDenseGBytes + (size_t)2 * 15 * kDenseCols * sizeof(cplx<float>)));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_contract_dense_bf16, dim3(count * (Nt / kDenseCols)), dim3(512), lds, s, (const uint4*)Ghi,
                     (const uint4*)Glo, Bd, A_NL, N, KD, KD32, nrb, Nt, ctrl);
  return hipGetLastError();
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
