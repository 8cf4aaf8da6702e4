// Shared device-side types for the GMMNLSE propagation kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmm {

// Control block of one large step, written by the norm kernel, read by the
// guarded kernels of later (speculatively queued) iterations and by the host.
struct Ctrl {
  double eps;
  int iters;
  int done;    // 1: no more iterations (converged, fixed count reached, or failed)
  int status;  // 0 ok, 1 max_iter reached without eps < tol, 2 non-finite eps
  int pad;
};


// Batched rounds (see the batched kernels): one row of a round, and the per-slot part.
struct BatchRow {
  int slot;  // slot index
  int src;   // source iterate: -1 = the slot's psi_0, else its sub-step row (j - 1)
  int ej;    // sub-step j of the phase factor exp(D_w j dz) (row of the slot's table)
  int pad;
};

// Per-slot part of a batched iteration (trapezoid, norm) or large-step close.
struct BatchSlot {
  const void* psi0;   // [N][Nt] psi(z0)
  const void* I0;     // I_0: the round's row of sub-step 0 (first iteration) or the slot's kept copy
  const void* I;      // the round's first row of sub-step 1
  void* psi;          // [M][N][Nt] sub-step iterates (close: its row m - 1 is the source)
  void* I0_keep;      // [N][Nt] kept I_0
  void* dst;          // close: psi(z0 + m dz) goes here (the slot's psi_0)
  const void* Em;     // close: exp(D_w m dz) row of the slot's table (NULL: lab-frame iterates, a copy)
  const void* E;      // trapezoid with lab-frame storage: the slot's table [M + 1][N][Nt] (NULL: psi frame)
  const void* Em64;   // trapezoid: exp(D_w M dz) [N][Nt] in FP64 for a full large step of single-precision fields
                      // (the sub-step that ends the step multiplies in FP64), else NULL
  double* partials;   // [trapz_blocks(N Nt)][2] FP64 partial sums of the norm
  Ctrl* ctrl;         // the slot's control block
  Ctrl* ctrl_host;    // its mirror in pinned host memory (device-visible address), stored by the norm
  double dz;
  int first, m;
};

// Most modes the saturating-gain kernels take (their N x N matrices sit in LDS),
// and the samples per partial sum of the pair integrals.
constexpr int kGainNmax = 22;
// Segment length (log2) of the overlap-save Raman convolution.
constexpr int kOsLogF = 11;
constexpr int kGainChunkHost = 128;
// Partial sums per sub-step of the pair integrals: 64 (or Nt / 128 for short windows).
inline int gain_partials(int nt) { return nt / kGainChunkHost < 64 ? nt / kGainChunkHost : 64; }

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cplx<double> cwiden(cplx<T> a) { return {(double)a.re, (double)a.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cround(cplx<double> a) { return {(T)a.re, (T)a.im}; }

// exp(i*phase) with the phase first folded into [-pi, pi] in double precision,
// then evaluated in the field precision T.
template <typename T>
__device__ __forceinline__ cplx<T> expi_reduced(double phase);
template <>
__device__ __forceinline__ cplx<double> expi_reduced<double>(double phase) {
  const double twopi = 6.283185307179586476925286766559;
  double r = phase - twopi * rint(phase * (1.0 / twopi));
  double s, c;
  sincos(r, &s, &c);
  return {c, s};
}
template <>
__device__ __forceinline__ cplx<float> expi_reduced<float>(double phase) {
  const double twopi = 6.283185307179586476925286766559;
  float r = (float)(phase - twopi * rint(phase * (1.0 / twopi)));
  float s, c;
  sincosf(r, &s, &c);
  return {c, s};
}

// Angular frequency of spectral bin k on an nt-point grid: 2*pi*fftfreq(nt, dt).
__device__ __forceinline__ double omega_of(int k, int nt, double domega) {
  return (double)(k < nt / 2 ? k : k - nt) * domega;
}

}  // namespace gmm
