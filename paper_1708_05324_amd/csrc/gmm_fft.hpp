// Block-wide complex FFT for one row of length N = 2^LOGN (8 <= LOGN <= 15).
//
// Design (gfx950): one workgroup owns one row.  Each thread keeps R = 32 points
// (FP32 rows of 2^10 and more; 16 otherwise) in registers, does a radix-R butterfly per pass entirely in
// registers, and the passes exchange data through LDS in Stockham (self-
// sorting) order, so no bit-reversal pass is ever needed.  An FP32 2^14 row
// takes three passes [32, 16, 32] and two LDS exchanges.  An exchange moves
// the real and then the imaginary parts through N scalars of LDS (+ 1/16
// padding), which keeps an FP64 2^14 row inside the 160 KB LDS and lets two
// FP32 rows share a CU; a WIDE FP32 row (one per CU) moves N complex values
// in one round, one LDS access per point and direction.
//
// The pass schedule is [R, rem, R, ..., R]: first and last passes both have
// radix R, so the register of the i-th point is i*THREADS + tid both on entry
// and on exit.  Element-wise work before (phase factors, pair products) and
// after (spectral filters, shock factor) is done in registers on that layout,
// and a forward transform can feed an inverse one without touching LDS.
//
// SIGN = -1:  X_k = sum_j x_j exp(-2 pi i jk/N)   (numpy fft)
// SIGN = +1:  X_k = sum_j x_j exp(+2 pi i jk/N)   (numpy ifft times N)
#pragma once
#include "gmm_common.hpp"

namespace gmm {

// WIDE_: the row may take the LDS of a whole CU (one block per CU): an FP32 row
// of up to 2^14 points then goes through LDS as N complex values in one round
// (2 N scalars + 1/16 padding, 139 KB at 2^14) instead of its real and
// imaginary parts one after the other.
template <int LOGN_, int ELEM_BYTES, int MAX_LOGR = 5, bool WIDE_ = false>
struct FftShape {
  static constexpr int LOGN = LOGN_;
  static constexpr int N = 1 << LOGN;
  static constexpr bool WIDE = WIDE_ && ELEM_BYTES == 4 && LOGN <= 14;
  // 32 points per thread for FP32 rows of 2^10 and more; 16 for FP64 rows
  // (32 complex doubles would need 128 VGPRs for the data alone).
  static constexpr int LOGR = (ELEM_BYTES == 4 && LOGN >= 10 && MAX_LOGR >= 5) ? 5 : 4;
  static constexpr int R = 1 << LOGR;
  static constexpr int THREADS = N / R;
  static constexpr int NFULL = LOGN / LOGR;
  static constexpr int REM = LOGN % LOGR;
  static constexpr int NPASS = NFULL + (REM ? 1 : 0);
  static constexpr int LDS_ELEMS = (WIDE ? 2 : 1) * (N + (N >> 4));  // one padding slot per 16 points
  static constexpr int logp(int i) { return (i == 1 && REM) ? REM : LOGR; }
  static constexpr int log_stride(int i) {
    int s = 0;
    for (int k = 0; k < i; ++k) s += logp(k);
    return s;
  }
  static_assert(LOGN >= 8 && LOGN <= 15, "row length must be 2^8 .. 2^15");
};


// cos/sin of 2*pi*m/32, m = 0..31, from the first-octant table by symmetry.
__device__ __forceinline__ constexpr double c32_table(int r) {
  return r == 0 ? 1.0
       : r == 1 ? 0.98078528040323043
       : r == 2 ? 0.92387953251128674
       : r == 3 ? 0.83146961230254524
       : r == 4 ? 0.70710678118654752
       : r == 5 ? 0.55557023301960218
       : r == 6 ? 0.38268343236508977
       : r == 7 ? 0.19509032201612826
       : 0.0;
}

template <typename T, int SIGN>
__device__ __forceinline__ cplx<T> root32(int m) {  // exp(SIGN * 2 pi i m / 32)
  int q = (m >> 3) & 3, r = m & 7;
  double c, s;
  if (q == 0) { c = c32_table(r); s = c32_table(8 - r); }
  else if (q == 1) { c = -c32_table(8 - r); s = c32_table(r); }
  else if (q == 2) { c = -c32_table(r); s = -c32_table(8 - r); }
  else { c = c32_table(8 - r); s = -c32_table(r); }
  return {(T)c, (T)(SIGN * s)};
}

// In-register DFT of P points (natural order in and out), decimation in
// frequency with compile-time twiddles; the final bit reversal is a register
// renaming once unrolled.
template <typename T, int P, int SIGN>
__device__ __forceinline__ void dft_reg(cplx<T>* u) {
#pragma unroll
  for (int span = P / 2; span >= 1; span >>= 1) {
#pragma unroll
    for (int start = 0; start < P; start += 2 * span) {
#pragma unroll
      for (int k = 0; k < span; ++k) {
        cplx<T> a = u[start + k], b = u[start + k + span];
        u[start + k] = cadd(a, b);
        cplx<T> d = csub(a, b);
        const int m = k * (P / (2 * span));  // twiddle exponent in units of 1/P
        if (m == 0) {
          u[start + k + span] = d;
        } else if (4 * m == P) {  // exp(SIGN*i*pi/2) = SIGN*i
          u[start + k + span] = SIGN > 0 ? cplx<T>{-d.im, d.re} : cplx<T>{d.im, -d.re};
        } else {
          u[start + k + span] = cmul(d, root32<T, SIGN>(m * (32 / P)));
        }
      }
    }
  }
  cplx<T> tmp[P];
#pragma unroll
  for (int i = 0; i < P; ++i) tmp[i] = u[i];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    int r = 0;
#pragma unroll
    for (int b = 0, x = i; (1 << b) < P; ++b, x >>= 1) r = (r << 1) | (x & 1);
    u[r] = tmp[i];
  }
}

// Twiddle bases of pass I for this thread: wp[b][e] = W^(2^e k_b), with
// W = exp(SIGN 2 pi i / (Ns P)) and k_b = (tid + b THREADS) mod Ns; the pass
// multiplies them along the set bits of q to form W^(q k_b).  Loaded one pass
// ahead so their latency overlaps the LDS exchange.
template <class S, int I, typename T, int SIGN>
struct PassTwiddles {
  static constexpr int LP = S::logp(I), P = 1 << LP, B = S::R / P;
  static constexpr int LNS = S::log_stride(I), NS = 1 << LNS;
  static constexpr bool USED = NS > 1;
  cplx<T> wp[USED ? B : 1][USED ? LP : 1];
  __device__ __forceinline__ void load(int tid, const cplx<T>* __restrict__ tw) {
    if constexpr (USED) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int k = (tid + b * S::THREADS) & (NS - 1);
#pragma unroll
        for (int e = 0; e < LP; ++e) {
          wp[b][e] = tw[(k << e) << (S::LOGN - LNS - LP)];  // table holds exp(-2 pi i m / N)
          if (SIGN > 0) wp[b][e].im = -wp[b][e].im;
        }
      }
    }
  }
};

// One Stockham pass: butterflies read at j + q*N/P, write at
// (j / Ns) * Ns * P + j % Ns + q * Ns, with twiddles exp(SIGN 2 pi i q (j % Ns) / (Ns P)).
template <class S, int I, typename T, int SIGN>
__device__ __forceinline__ void fft_pass_compute(cplx<T> (&v)[S::R], const PassTwiddles<S, I, T, SIGN>& tws) {
  constexpr int LP = S::logp(I), P = 1 << LP, B = S::R / P;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (PassTwiddles<S, I, T, SIGN>::USED) {
#pragma unroll
      for (int q = 1; q < P; ++q) {
        cplx<T> w = {T(1), T(0)};
        bool first = true;
#pragma unroll
        for (int e = 0; e < LP; ++e)
          if (q & (1 << e)) {
            w = first ? tws.wp[b][e] : cmul(w, tws.wp[b][e]);
            first = false;
          }
        v[b * P + q] = cmul(v[b * P + q], w);
      }
    }
    dft_reg<T, P, SIGN>(&v[b * P]);
  }
}

// LDS padding of the exchange after pass I: one slot every 2^s points with
// s = max(log2 P_I, 4), so the stride-P (or run-of-Ns) writes of the pass fall
// on distinct banks; never more than N / 16 extra slots.
template <class S, int I>
__device__ __forceinline__ int lds_pad_x(int i) {
  constexpr int LP = S::logp(I);
  constexpr int SH = LP > 4 ? LP : 4;
  return i + (i >> SH);
}

// Exchange after pass I of a WIDE row: every point of pass I's output is
// written to LDS as one complex value, then pass I+1's inputs are read.
template <class S, int I, typename T>
__device__ __forceinline__ void fft_exchange_wide(cplx<T> (&v)[S::R], T* lds, int tid) {
  constexpr int LP = S::logp(I), P = 1 << LP, B = S::R / P;
  constexpr int LNS = S::log_stride(I), NS = 1 << LNS;
  constexpr int LP2 = S::logp(I + 1), P2 = 1 << LP2, B2 = S::R / P2;
  cplx<T>* c = reinterpret_cast<cplx<T>*>(lds);
  __syncthreads();  // the previous exchange has been read
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + b * S::THREADS;
    const int base = ((j >> LNS) << (LNS + LP)) + (j & (NS - 1));
#pragma unroll
    for (int q = 0; q < P; ++q) c[lds_pad_x<S, I>(base + (q << LNS))] = v[b * P + q];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B2; ++b) {
    const int j = tid + b * S::THREADS;
#pragma unroll
    for (int q = 0; q < P2; ++q) v[b * P2 + q] = c[lds_pad_x<S, I>(j + q * (S::N / P2))];
  }
}

// Exchange after pass I of other rows: the real and imaginary parts go through
// LDS one after the other (N scalars each).
template <class S, int I, typename T, bool IMAG>
__device__ __forceinline__ void fft_exchange_component(cplx<T> (&v)[S::R], T* lds, int tid) {
  constexpr int LP = S::logp(I), P = 1 << LP, B = S::R / P;
  constexpr int LNS = S::log_stride(I), NS = 1 << LNS;
  constexpr int LP2 = S::logp(I + 1), P2 = 1 << LP2, B2 = S::R / P2;
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + b * S::THREADS;
    const int base = ((j >> LNS) << (LNS + LP)) + (j & (NS - 1));
#pragma unroll
    for (int q = 0; q < P; ++q)
      lds[lds_pad_x<S, I>(base + (q << LNS))] = IMAG ? v[b * P + q].im : v[b * P + q].re;
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B2; ++b) {
    const int j = tid + b * S::THREADS;
#pragma unroll
    for (int q = 0; q < P2; ++q) {
      T x = lds[lds_pad_x<S, I>(j + q * (S::N / P2))];
      if (IMAG) v[b * P2 + q].im = x; else v[b * P2 + q].re = x;
    }
  }
}

template <class S, int I, typename T>
__device__ __forceinline__ void fft_exchange(cplx<T> (&v)[S::R], T* lds, int tid) {
  if constexpr (S::WIDE) {
    fft_exchange_wide<S, I, T>(v, lds, tid);
  } else {
    fft_exchange_component<S, I, T, false>(v, lds, tid);
    fft_exchange_component<S, I, T, true>(v, lds, tid);
  }
}

template <class S, int I, typename T, int SIGN>
__device__ __forceinline__ void fft_passes(cplx<T> (&v)[S::R], T* lds, int tid, const cplx<T>* __restrict__ tw,
                                           const PassTwiddles<S, I, T, SIGN>& tws) {
  fft_pass_compute<S, I, T, SIGN>(v, tws);
  if constexpr (I + 1 < S::NPASS) {
    PassTwiddles<S, I + 1, T, SIGN> next;
    next.load(tid, tw);
    fft_exchange<S, I, T>(v, lds, tid);
    fft_passes<S, I + 1, T, SIGN>(v, lds, tid, tw, next);
  }
}

// Full transform of the row held in v (v[i] = x[tid + i*THREADS]) in place.
// `lds` must hold S::LDS_ELEMS scalars of type T, 16-byte aligned.  All threads must call it.
template <class S, typename T, int SIGN>
__device__ __forceinline__ void block_fft(cplx<T> (&v)[S::R], T* lds, int tid, const cplx<T>* __restrict__ tw) {
  PassTwiddles<S, 0, T, SIGN> first;  // pass 0 has Ns = 1: no twiddles
  fft_passes<S, 0, T, SIGN>(v, lds, tid, tw, first);
}

}  // namespace gmm
