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

template <int RPAD, bool BF16, int CB>
static int contract_cols_blocks() {
  static int blocks = 0;
  if (blocks == 0) {
    constexpr size_t lds = ColShape<RPAD, BF16>::lds_bytes();
    const void* fn = (const void*)k_contract_cols<RPAD, BF16, CB>;
    if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    blocks = per_cu * device_cus();
  }
  return blocks;
}

hipError_t launch_contract_cols(int rpad, bool bf16, const void* Ua, const void* Ub, const void* Ya, const void* Yb,
                                cplx<float>* A_NL, int N, int kv, int Nt, int count, const Ctrl* ctrl,
                                hipStream_t s, int blocks_per_cu, int col_blocks) {
#define GMM_COL_CASE(RP, BF, CB)                                                                               \
  if (rpad == RP && bf16 == BF && col_blocks == CB) {                                                          \
    const int ntiles = count * ((Nt + 16 * CB - 1) / (16 * CB));                                               \
    int cap = contract_cols_blocks<RP, BF, CB>();                                                              \
    if (cap < 1) return hipErrorInvalidConfiguration;                                                          \
    if (blocks_per_cu > 0) cap = std::min(cap, blocks_per_cu * device_cus());                                  \
    const int nb = std::min((ntiles + 3) / 4, cap);                                                            \
    hipLaunchKernelGGL((k_contract_cols<RP, BF, CB>), dim3(nb), dim3(256), (ColShape<RP, BF>::lds_bytes()), s, \
                       Ua, Ub, Ya, Yb, A_NL, N, kv, Nt, ntiles, ctrl);                                         \
    return hipGetLastError();                                                                                  \
  }
  GMM_COL_CASE(64, true, 4)
  GMM_COL_CASE(128, true, 4)
  GMM_COL_CASE(64, false, 4)
  GMM_COL_CASE(128, false, 4)
  GMM_COL_CASE(64, true, 3)
  GMM_COL_CASE(128, true, 3)
  GMM_COL_CASE(64, false, 3)
  GMM_COL_CASE(128, false, 3)
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
// One block of 4 waves owns 128 columns; wave w owns columns 32 w .. 32 w + 31
// (two blocks of 16) and every output row, so its accumulators (2 x 29 tiles of
// 16 x 16) stay in registers for the whole K loop and B is read once.  Each
// 32-wide K slice of G (hi and lo, all rows) is copied straight from global
// memory into LDS once per block (double-buffered: the next slice is in flight
// during the products) and every fragment read from LDS feeds both column
// blocks.  The 16-byte
// chunks of a G row are XOR-swizzled by bits 1-2 of the row so that eight
// consecutive lanes of a 128-bit LDS read hit distinct banks.  After the K loop
// the accumulators pass through LDS in pieces of 64 rows (32 pairs pl) and are
// folded into NL: thread (t, g) sums C_pl A_l over pairs 16 g .. 16 g + 15 of
// each piece in registers and adds each mode's partial to its own NL partial
// (fixed summation order, no atomics); NL = partial 0 + partial 1 overwrites A.
//
// Cost at 15 modes (2^14 samples, 128 columns a block): the products, the
// fragment reads from LDS, the G slices out of L2 and the fold take comparable
// shares; one wave per SIMD (232 accumulator registers) leaves little latency
// hiding.
constexpr int kDenseCols = 128, kDenseRB = 29, kDenseThreads = 256;  // kDenseRB: row blocks at 15 modes
constexpr size_t kDenseSlice = (size_t)kDenseRB * 16 * 64;    // bytes of one plane (hi or lo) of one K slice
constexpr size_t kDenseGBytes = 4 * kDenseSlice;                // two slices (double buffer), hi and lo each
static_assert(kDenseRB * 16 == kDenseGRows, "G hi/lo rows as allocated by the plan");
constexpr int kDenseCS = kDenseCols + 4;                         // row stride of a C piece (floats)
constexpr int kDenseAR = (15 * kDenseCols + kDenseThreads - 1) / kDenseThreads;  // A elements per thread
constexpr size_t kDenseFoldA = (size_t)64 * kDenseCS * sizeof(float);           // A tile offset in the fold
static_assert(kDenseFoldA + (size_t)3 * 15 * kDenseCols * sizeof(cplx<float>) <= kDenseGBytes,
              "the fold buffers fit in the G region");

template <int NRB>  // row blocks of 16 computed (the rows beyond 2 N^2 are zero in G)
__global__ __launch_bounds__(kDenseThreads) void k_contract_dense_bf16(const uint4* __restrict__ Ghi,
                                                                       const uint4* __restrict__ Glo,
                                                                       const float* __restrict__ Bd,
                                                                       cplx<float>* A_NL, int N, int KD, int KD32,
                                                                       int Nt, const Ctrl* ctrl) {
  if (skip_iteration(ctrl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // K loop: the G slices.  Fold: C piece [64][kDenseCS], A tile [N][128], two NL partials [N][128] (one per
  // half of each piece's pairs), all inside the G region once the K loop is over.
  unsigned char* sG = smem_raw;                                          // [2 slices][hi, lo][kDenseRB * 16][64 B]
  float* sC = reinterpret_cast<float*>(smem_raw);
  cplx<float>* sA = reinterpret_cast<cplx<float>*>(smem_raw + kDenseFoldA);
  cplx<float>* sNL0 = sA + N * kDenseCols;
  cplx<float>* sNL1 = sNL0 + N * kDenseCols;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int tiles_per_j = Nt / kDenseCols;
  const int jj = blockIdx.x / tiles_per_j, t0 = (blockIdx.x - jj * tiles_per_j) * kDenseCols;
  cplx<float>* Aj = A_NL + (size_t)jj * N * Nt + t0;
  const float* Bj = Bd + (size_t)jj * KD * Nt + t0 + 32 * wave + lr;
  cplx<float> areg[kDenseAR];  // this thread's share of the A tile, held through the K loop
#pragma unroll
  for (int r = 0; r < kDenseAR; ++r) {
    const int i = tid + kDenseThreads * r;
    if (i < N * kDenseCols) areg[r] = Aj[(size_t)(i >> 7) * Nt + (i & 127)];
  }
  // staging of a K slice: straight from global memory into LDS (global_load_lds_dwordx4: lane i of a wave
  // writes bytes 16 i .. 16 i + 15 of a 1 KB LDS block).  Unit u = 2 rb + plane (hi 0, lo 1) is rows
  // 16 rb .. 16 rb + 15 of one plane; lane i fills row 16 rb + i / 4 at swizzled position i % 4, i.e. it
  // loads chunk (i % 4) ^ ((row >> 1) % 4) = (i % 4) ^ ((i / 8) % 4) of that row.
  const int KC = KD32 / 8;  // 16-byte chunks per G row
  constexpr int nunits = 2 * NRB;
  const size_t lane_src = (size_t)(lane >> 2) * KC + ((lane & 3) ^ ((lane >> 3) & 3));
  auto stage = [&](int ks, int buf) {
    for (int u = wave; u < nunits; u += 4) {
      const int rb = u >> 1, plane = u & 1;
      const uint4* src = (plane ? Glo : Ghi) + (size_t)16 * rb * KC + 4 * ks + lane_src;
      unsigned char* dst = sG + (size_t)buf * 2 * kDenseSlice + (size_t)plane * kDenseSlice + (size_t)rb * 1024;
      __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  floatx4 acc0[NRB], acc1[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) acc0[rb] = acc1[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  float x0[8], x1[8];
  const int nks = KD32 / 32;
  stage(0, 0);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 8 * lk + e;
    x0[e] = k < KD ? Bj[(size_t)k * Nt] : 0.f;
    x1[e] = k < KD ? Bj[(size_t)k * Nt + 16] : 0.f;
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's LDS fills have landed
  __syncthreads();
  const int swz = ((lk ^ (lr >> 1)) & 3) * 16;  // swizzled chunk lk of row 16 rb + lr
  for (int ks = 0; ks < nks; ++ks) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) bf16_split2(x0[2 * e], x0[2 * e + 1], h[e], l[e]);
    const bf16x8 bh0 = __builtin_bit_cast(bf16x8, uint4{h[0], h[1], h[2], h[3]});
    const bf16x8 bl0 = __builtin_bit_cast(bf16x8, uint4{l[0], l[1], l[2], l[3]});
#pragma unroll
    for (int e = 0; e < 4; ++e) bf16_split2(x1[2 * e], x1[2 * e + 1], h[e], l[e]);
    const bf16x8 bh1 = __builtin_bit_cast(bf16x8, uint4{h[0], h[1], h[2], h[3]});
    const bf16x8 bl1 = __builtin_bit_cast(bf16x8, uint4{l[0], l[1], l[2], l[3]});
    if (ks + 1 < nks) {  // next slice of G (into the other buffer, last read before the previous barrier)
      stage(ks + 1, (ks + 1) & 1);  // and of B in flight during this slice's products
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * (ks + 1) + 8 * lk + e;
        x0[e] = k < KD ? Bj[(size_t)k * Nt] : 0.f;
        x1[e] = k < KD ? Bj[(size_t)k * Nt + 16] : 0.f;
      }
    }
    const unsigned char* src = sG + (ks & 1) * 2 * kDenseSlice + swz;
    // row blocks in groups of 4: the fragments of group q + 1 are read while the products of group q issue
    // (the scheduling barrier keeps the compiler from hoisting every fragment read of the slice at once)
    constexpr int GR = 4, NG = (NRB + GR - 1) / GR;
    bf16x8 fh[2][GR], fl[2][GR];
    static_for<0, NG + 1>([&](auto qc) {
      constexpr int Q = decltype(qc)::value;
      if constexpr (Q < NG) {
        static_for<0, GR>([&](auto jc) {
          constexpr int J = decltype(jc)::value, RB = GR * Q + J;
          if constexpr (RB < NRB) {
            const int off = (16 * RB + lr) * 64;
            fh[Q & 1][J] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(src + off));
            fl[Q & 1][J] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(src + kDenseSlice + off));
          }
        });
      }
      if constexpr (Q > 0) {
        static_for<0, GR>([&](auto jc) {
          constexpr int J = decltype(jc)::value, RB = GR * (Q - 1) + J;
          if constexpr (RB < NRB) {
            const bf16x8 ah = fh[(Q - 1) & 1][J], al = fl[(Q - 1) & 1][J];
            acc0[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh0, acc0[RB], 0, 0, 0);
            acc1[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh1, acc1[RB], 0, 0, 0);
            acc0[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl0, acc0[RB], 0, 0, 0);
            acc1[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl1, acc1[RB], 0, 0, 0);
            acc0[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh0, acc0[RB], 0, 0, 0);
            acc1[RB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh1, acc1[RB], 0, 0, 0);
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      }
    });
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's fills of the next slice have landed
    __syncthreads();
  }
  // fold: accumulator register i of lane (lr, lk) in row block rb is row 16 rb + 4 lk + i
#pragma unroll
  for (int r = 0; r < kDenseAR; ++r) {
    const int i = tid + kDenseThreads * r;
    if (i < N * kDenseCols) {
      sA[i] = areg[r];
      sNL0[i] = sNL1[i] = cplx<float>{0.f, 0.f};
    }
  }
  const int NN = N * N, col = tid & 127, g = tid >> 7;
  cplx<float>* myNL = g ? sNL1 : sNL0;
  static_for<0, (NRB + 3) / 4>([&](auto qc) {
    constexpr int Q = decltype(qc)::value;  // rows 64 Q .. 64 Q + 63: pairs pl = 32 Q .. 32 Q + 31
    if (32 * Q < NN) {
      __syncthreads();  // the previous piece's fold (or the K loop) has finished with the LDS
      static_for<0, 4>([&](auto jc) {
        constexpr int J = decltype(jc)::value;
        if constexpr (4 * Q + J < NRB) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            sC[(16 * J + 4 * lk + i) * kDenseCS + 32 * wave + lr] = acc0[4 * Q + J][i];
            sC[(16 * J + 4 * lk + i) * kDenseCS + 32 * wave + 16 + lr] = acc1[4 * Q + J][i];
          }
        }
      });
      __syncthreads();
      // thread (t, g) takes pairs pl = 32 Q + 16 g .. + 15 = p N + l in order, summing C_pl A_l in registers
      // and adding each mode's partial sum to its own NL partial when p changes or the range ends
      const int pl0 = 32 * Q + 16 * g, cnt = min(16, NN - pl0);
      if (cnt > 0) {
        int p = pl0 / N, l = pl0 - p * N;
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if (r < cnt) {
            const int r2 = 16 * g + r;
            const float cr = sC[(2 * r2) * kDenseCS + col], ci = sC[(2 * r2 + 1) * kDenseCS + col];
            const cplx<float> a = sA[l * kDenseCols + col];
            sr += cr * a.re - ci * a.im;
            si += cr * a.im + ci * a.re;
            if (++l == N || r + 1 == cnt) {
              myNL[p * kDenseCols + col].re += sr;
              myNL[p * kDenseCols + col].im += si;
              sr = si = 0.f;
              if (l == N) l = 0, ++p;
            }
          }
        }
      }
    }
  });
  __syncthreads();
  for (int i = tid; i < N * kDenseCols; i += kDenseThreads) {
    const cplx<float> a = sNL0[i], b = sNL1[i];
    Aj[(size_t)(i >> 7) * Nt + (i & 127)] = cplx<float>{a.re + b.re, a.im + b.im};
  }
}

template <int NRB>
hipError_t launch_dense_bf16_nrb(const void* Ghi, const void* Glo, const float* Bd, cplx<float>* A_NL, int N, int KD,
                                 int KD32, int Nt, int count, const Ctrl* ctrl, hipStream_t s) {
  const size_t lds = kDenseGBytes;
  static const hipError_t attr = hipFuncSetAttribute(
      (const void*)k_contract_dense_bf16<NRB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDenseGBytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_contract_dense_bf16<NRB>), dim3(count * (Nt / kDenseCols)), dim3(kDenseThreads), lds, s,
                     (const uint4*)Ghi, (const uint4*)Glo, Bd, A_NL, N, KD, KD32, Nt, ctrl);
  return hipGetLastError();
}

// G hi/lo must hold kDenseRB * 16 rows (zero beyond 2 N^2) of KD32 bf16 each.
hipError_t launch_contract_dense_bf16(const void* Ghi, const void* Glo, const float* Bd, cplx<float>* A_NL, int N,
                                      int KD, int KD32, int Nt, int count, const Ctrl* ctrl, hipStream_t s) {
  if (N > 15 || KD32 % 32 || KD > KD32 || Nt % kDenseCols) return hipErrorInvalidValue;
  const int rows = 2 * N * N;
  if (rows <= 128) return launch_dense_bf16_nrb<8>(Ghi, Glo, Bd, A_NL, N, KD, KD32, Nt, count, ctrl, s);
  if (rows <= 256) return launch_dense_bf16_nrb<16>(Ghi, Glo, Bd, A_NL, N, KD, KD32, Nt, count, ctrl, s);
  return launch_dense_bf16_nrb<kDenseRB>(Ghi, Glo, Bd, A_NL, N, KD, KD32, Nt, count, ctrl, s);
}

hipError_t launch_conv_os(const float* Y, float* Yout, uint32_t* Bhi, uint32_t* Blo, int R, int RQ, int count,
                          int Nt, int Lh, int V, const cplx<float>* Gf, const cplx<float>* twf, const Ctrl* ctrl,
                          hipStream_t s) {
  using S = FftShape<kOsLogF, 4, 4>;
  if (Lh < 1 || V < 1 || Lh - 1 + V > S::N || Nt < S::N || (Nt & (Nt - 1))) return hipErrorInvalidValue;
  const int nseg = (Nt + V - 1) / V, total = nseg * ((R + 1) / 2) * count;
  const dim3 grid(8 * ((total + 7) / 8));
  if (Bhi != nullptr)
    hipLaunchKernelGGL((k_conv_os<float, true>), grid, dim3(S::THREADS), 0, s, Y, nullptr, Bhi, Blo, R, RQ, count, 32,
                       Nt, Lh, V, nseg, Gf, twf, ctrl);
  else
    hipLaunchKernelGGL((k_conv_os<float, false>), grid, dim3(S::THREADS), 0, s, Y, Yout, nullptr, nullptr, R, RQ,
                       count, 32, Nt, Lh, V, nseg, Gf, twf, ctrl);
  return hipGetLastError();
}

hipError_t launch_pairs_os(const cplx<float>* A, float* Bp, uint32_t* Bhi, uint32_t* Blo, const int2* pairs, int N,
                           int Np, int count, int Nt, int Lh, int V, const cplx<float>* Gf, const cplx<float>* twf,
                           const Ctrl* ctrl, hipStream_t s) {
  using S = FftShape<kOsLogF, 4, 4>;
  if (Lh < 1 || V < 1 || Lh - 1 + V > S::N || Nt < S::N || (Nt & (Nt - 1)) || (Bhi != nullptr && Np > kBf16Kpad))
    return hipErrorInvalidValue;
  const int nseg = (Nt + V - 1) / V, total = nseg * ((Np + 1) / 2) * count;
  const dim3 grid(8 * ((total + 7) / 8));
  if (Bhi != nullptr)
    hipLaunchKernelGGL((k_pairs_os<float, true>), grid, dim3(S::THREADS), 0, s, A, nullptr, Bhi, Blo, pairs, N, Np, count,
                       kBf16Kpad / 8, Nt, Lh, V, nseg, Gf, twf, ctrl);
  else
    hipLaunchKernelGGL((k_pairs_os<float, false>), grid, dim3(S::THREADS), 0, s, A, Bp, nullptr, nullptr, pairs, N, Np, count,
                       kBf16Kpad / 8, Nt, Lh, V, nseg, Gf, twf, ctrl);
  return hipGetLastError();
}

// k_pairs_dense_os: k_pairs_dense by overlap-save segments (short h_R,
// complex64 fields): item (sub-step, pair, segment); the block forms
// B_mn = A_m A_n^* at its segment's input samples (indices mod Nt), writes the
// x, y rows at the valid outputs, then filters the segment (Gf = DFT_{+}(w) / F,
// w the truncated normalised h_R) and writes xr, yr.
__global__ __launch_bounds__((FftShape<kOsLogF, 4, 4>::THREADS)) void k_pairs_dense_os(
    const cplx<float>* __restrict__ A, float* __restrict__ Bd, const int2* __restrict__ pairs, int N, int Np,
    int count, int KD, int Nt, int Lh, int V, int nseg, const cplx<float>* __restrict__ Gf,
    const cplx<float>* __restrict__ twf, const Ctrl* ctrl) {
  using S = FftShape<kOsLogF, 4, 4>;
  if (skip_iteration(ctrl)) return;
  __shared__ __align__(16) float lds[S::LDS_ELEMS];
  const int w = xcd_local_index(blockIdx.x, gridDim.x >> 3, nseg * Np * count);
  if (w < 0) return;
  const int tid = threadIdx.x;
  const int blk = w / nseg, seg = w - blk * nseg;
  const int jj = blk / Np, Q = blk - jj * Np;
  const int2 mn = pairs[Q];
  const cplx<float>* am = A + ((size_t)jj * N + mn.x) * Nt;
  const cplx<float>* an = A + ((size_t)jj * N + mn.y) * Nt;
  float* out = Bd + (size_t)jj * KD * Nt;
  const int t0 = seg * V, base = t0 - (Lh - 1);
  cplx<float> z[S::R];
#pragma unroll
  for (int i = 0; i < S::R; ++i) {
    const int t = (base + tid + i * S::THREADS) & (Nt - 1);
    const cplx<float> x = am[t], y = an[t];
    z[i] = {x.re * y.re + x.im * y.im, x.im * y.re - x.re * y.im};  // A_m conj(A_n)
    const int o = tid + i * S::THREADS - (Lh - 1);
    if (o >= 0 && o < V && t0 + o < Nt) {
      out[(size_t)Q * Nt + t0 + o] = z[i].re;
      out[(size_t)(Np + Q) * Nt + t0 + o] = z[i].im;
    }
  }
  block_fft<S, float, +1>(z, lds, tid, twf);
#pragma unroll
  for (int i = 0; i < S::R; ++i) z[i] = cmul(z[i], Gf[tid + i * S::THREADS]);
  block_fft<S, float, -1>(z, lds, tid, twf);
#pragma unroll
  for (int i = 0; i < S::R; ++i) {
    const int o = tid + i * S::THREADS - (Lh - 1);
    const int t = t0 + o;
    if (o < 0 || o >= V || t >= Nt) continue;
    out[(size_t)(2 * Np + Q) * Nt + t] = z[i].re;
    out[(size_t)(3 * Np + Q) * Nt + t] = z[i].im;
  }
}

hipError_t launch_pairs_dense_os(const cplx<float>* A, float* Bd, const int2* pairs, int N, int Np, int count, int KD,
                                 int Nt, int Lh, int V, const cplx<float>* Gf, const cplx<float>* twf,
                                 const Ctrl* ctrl, hipStream_t s) {
  using S = FftShape<kOsLogF, 4, 4>;
  if (Lh < 1 || V < 1 || Lh - 1 + V > S::N || Nt < S::N || (Nt & (Nt - 1)) || KD < 4 * Np) return hipErrorInvalidValue;
  const int nseg = (Nt + V - 1) / V, total = nseg * Np * count;
  const dim3 grid(8 * ((total + 7) / 8));
  hipLaunchKernelGGL(k_pairs_dense_os, grid, dim3(S::THREADS), 0, s, A, Bd, pairs, N, Np, count, KD, Nt, Lh, V, nseg,
                     Gf, twf, ctrl);
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
