// Host-side launchers of the propagation kernels, one explicit instantiation
// per field precision (gmm_kern_f32.hip, gmm_kern_f64.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace gmm {

template <typename T>
struct cplx;
struct Ctrl;
struct BatchRow;
struct BatchSlot;

template <typename T>
struct Launch {
  static bool supports_logn(int logn);
  static hipError_t fft_rows(int logn, int sign, const cplx<T>* in, cplx<T>* out, T scale, int rows,
                             const cplx<T>* tw, hipStream_t s);
  // E[j][p][k] = exp(i (beta_p(w_k) - beta_0) j dz), j < rows
  static hipError_t phase_table(cplx<T>* E, const double* coef, int nb, int N, int nt, int rows, double dz,
                                double domega, hipStream_t s, int j0 = 0);
  // Eigenbasis table of the coupled linear operator: E[j][q][k] = exp(i lam_q(w_k) j dz), j < rows
  static hipError_t phase_table_lam(cplx<T>* E, const double* lam, int N, int nt, int rows, double dz,
                                    hipStream_t s, int j0 = 0);
  // back = false: dst = U (E .* src); back = true: dst = conj(E) .* (U^H src), per frequency (E may be null)
  static hipError_t mode_mix(bool back, const cplx<T>* src, long src_jrows, cplx<T>* dst, const cplx<T>* U,
                             const cplx<T>* E, int j0, int N, int nt, int count, const Ctrl* ctrl, hipStream_t s);
  // Overlap-save Raman convolution in the field precision (rows out): rank-r rows Y -> Yout, and the packed
  // route's pair rows from the fields A -> Bp [count][Np][Nt]; Gf / twf the 2^kOsLogF-point filter and twiddles
  static hipError_t conv_os(const T* Y, T* Yout, int R, int RQ, int count, int Nt, int Lh, int V,
                            const cplx<T>* Gf, const cplx<T>* twf, const Ctrl* ctrl, hipStream_t s);
  static hipError_t pairs_os(const cplx<T>* A, T* Bp, const int2* pairs, int N, int Np, int count, int Nt, int Lh,
                             int V, const cplx<T>* Gf, const cplx<T>* twf, const Ctrl* ctrl, hipStream_t s);
  static hipError_t phase_to_time(int logn, const cplx<T>* psi, long psi_jrows, cplx<T>* A, const cplx<T>* E, int N,
                                  int count, int j0, const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s);
  static hipError_t pairs(int logn, bool raman, const cplx<T>* A, T* Bp, const int2* pairs, int N, int Np,
                          int count, const cplx<T>* Gs, const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s);
  // kpad = 0: packed matrix with K = Rpad (kv = Np rows per sub-step); kpad = 64: rank factor U (kv = RQ).
  // blocks_per_cu > 0: at most that many blocks per CU for the persistent variants (0: as many as fit)
  static hipError_t contract(int rt, int kpad, const T* ST, const T* Bp, cplx<T>* A_NL, const int* pidx, int N,
                             int kv, int Nt, int count, const Ctrl* ctrl, hipStream_t s, int blocks_per_cu = 0);
  static hipError_t project(int rq, int kp, const T* VT, const cplx<T>* A, T* Y, const int2* pairs, int N, int Np,
                            int Nt, int count, const Ctrl* ctrl, hipStream_t s);
  static hipError_t conv(int logn, const T* Y, T* Yout, int R, int RQ, int count, const cplx<T>* Gs,
                         const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s);
  static hipError_t spectral_out(int logn, const cplx<T>* in, cplx<T>* out, const cplx<T>* E, int N, int count,
                                 int j0, double domega, double gscale, double inv_omega0, int shock,
                                 const cplx<T>* tw, const Ctrl* ctrl, hipStream_t s);
  // E != nullptr: lab-frame iterates (the phase table [M + 1][N][Nt] is applied inside the trapezoid);
  // Em64 != nullptr (with E): exp(D M dz) in FP64 for the sub-step that ends the large step;
  // psi0_keep / reset (with E, first iteration): psi0 is the previous step's last iterate, copied to psi0_keep,
  // and the control block `reset` is cleared for the new large step
  static hipError_t trapz(const cplx<T>* psi0, const cplx<T>* I0, const cplx<T>* I, cplx<T>* psi, cplx<T>* I0_keep,
                          int first, int M, long nn, T dz, double* partials, const Ctrl* ctrl, hipStream_t s,
                          const cplx<T>* E = nullptr, const cplx<double>* Em64 = nullptr,
                          cplx<T>* psi0_keep = nullptr, Ctrl* reset = nullptr);
  // dst = Em .* src (Em = nullptr: a copy; Em64 != nullptr: the factor and product in FP64); with ctrl, also
  // resets the control block for the next large step
  static hipError_t close(const cplx<T>* src, cplx<T>* dst, const cplx<T>* Em, long nn, Ctrl* ctrl, hipStream_t s,
                          const cplx<double>* Em64 = nullptr);
  // General-tensor route: pair rows [count][KD][Nt] (x, y and, with Raman, xr, yr), then C = G B and NL.
  static hipError_t pairs_dense(int logn, bool raman, const cplx<T>* A, T* Bd, const int2* pairs, int N, int Np,
                                int count, int KD, const cplx<T>* Hr, const cplx<T>* tw, const Ctrl* ctrl,
                                hipStream_t s);
  static hipError_t contract_dense(const T* G, const T* Bd, cplx<T>* A_NL, int N, int KD, int rows_pad, int Nt,
                                   int count, const Ctrl* ctrl, hipStream_t s);
  // Saturating gain: pair integrals of the time-domain fields (chunk partials), then
  // out += E^-1 Mg E psi for the spectra (Mg built by launch_gain_matrix).
  static hipError_t pair_integrals(const cplx<T>* A, cplx<double>* part, int N, int Nt, int count, const Ctrl* ctrl,
                                   hipStream_t s);
  static hipError_t gain_add(const cplx<T>* psi, long psi_jrows, const cplx<T>* E, int j0, const cplx<double>* Mg,
                             cplx<T>* out, int N, int Nt, int count, const Ctrl* ctrl, hipStream_t s);
  // Element-wise part of one RK4IP stage (1..4) over nn elements.
  static hipError_t rk4ip_stage(int stage, cplx<T>* At, cplx<T>* AI, cplx<T>* k1, const cplx<T>* k2,
                                const cplx<T>* k3, const cplx<T>* k4, cplx<T>* X, const cplx<T>* Eh, T h, long nn,
                                hipStream_t s);
  static hipError_t spec_sums(const cplx<T>* At, int nt, long nn, double domega, double omega0, double* partials,
                              hipStream_t s);
  static hipError_t finish_H(const cplx<double>* H, cplx<T>* Gs, int nt, double fR, hipStream_t s);
  // Batched rounds (several propagations of one plan): R rows listed in `rows`, per-slot buffers at fixed
  // strides (psi0 [S][N][Nt], psi [S][M][N][Nt], E [S][M + 1][N][Nt]); work rows [R][N][Nt].
  static hipError_t phase_to_time_b(int logn, const BatchRow* rows, const cplx<T>* psi0, const cplx<T>* psi,
                                    const cplx<T>* E, cplx<T>* A, int N, int R, int M, const cplx<T>* tw, int lab,
                                    hipStream_t s);
  static hipError_t spectral_out_b(int logn, const BatchRow* rows, cplx<T>* W, const cplx<T>* E, int N, int R, int M,
                                   double domega, double gscale, double inv_omega0, int shock, const cplx<T>* tw,
                                   int lab, hipStream_t s);
  static hipError_t trapz_b(const BatchSlot* slots, int nslots, long nn, hipStream_t s);
  static hipError_t close_b(const BatchSlot* slots, int nslots, long nn, hipStream_t s);
};

// BF16 split contraction path (complex64 fields, Np <= 128).
constexpr int kBf16Kpad = 128;
hipError_t launch_pairs_bf16(int logn, bool raman, const cplx<float>* A, uint32_t* Bhi, uint32_t* Blo,
                             const int2* pairs, int N, int Np, int count, const cplx<float>* Gs,
                             const cplx<float>* tw, const Ctrl* ctrl, hipStream_t s);
hipError_t launch_contract_bf16(int rt, int kpad, const void* Shi, const void* Slo, const uint32_t* Bhi,
                                const uint32_t* Blo, cplx<float>* A_NL, const int* pidx, int N, int Nt, int count,
                                const Ctrl* ctrl, hipStream_t s);
// Column-owner contraction of the rank-r route (complex64 fields, Rpad 64 or 128,
// K = 64): BF16 split (Ua = U hi [Rpad][64] bf16, Ub = its lo and lo2 planes [2][Rpad][64], Ya/Yb = Y' planes of
// 2-row words, kv valid rows) or FP32 (Ua = U^T [64][Rpad], Ya = Y' [count][kv][Nt]).
// col_blocks: tiles of 16 col_blocks columns (4: 64, 3: 48).
hipError_t launch_contract_cols(int rpad, bool bf16, const void* Ua, const void* Ub, const void* Ya, const void* Yb,
                                cplx<float>* A_NL, int N, int kv, int Nt, int count, const Ctrl* ctrl,
                                hipStream_t s, int blocks_per_cu = 0, int col_blocks = 4);
// Column-owner projection Y = V B of the rank-r route (complex64 fields, RQ <= 64,
// KPAD 64 or 128): BF16 split (Va = V hi [RQ][KPAD] bf16, Vb = its lo and lo2 planes [2][RQ][KPAD]) or FP32
// (Va = V^T [KPAD][RQ]).
hipError_t launch_project_cols(int rq, int kpad, bool bf16, const void* Va, const void* Vb, const cplx<float>* A,
                               float* Y, int N, int Nt, int count, const Ctrl* ctrl, hipStream_t s);
// General-route product C = G B with the BF16 split for BF16X3 plans (up to 15 modes; G hi/lo
// [kDenseGRows][KD32] bf16, rows beyond 2 N^2 zero).
constexpr int kDenseGRows = 464;
hipError_t launch_contract_dense_bf16(const void* Ghi, const void* Glo, const float* Bd, cplx<float>* A_NL, int N,
                                      int KD, int KD32, int Nt, int count, const Ctrl* ctrl, hipStream_t s);
// Overlap-save form of the rank-r convolution (complex64 fields): Lh kernel taps, V outputs per segment,
// Gf / twf the segment filter and twiddles (2^11 points); Bhi == nullptr: FP32 output rows in Yout.
hipError_t launch_conv_os(const float* Y, float* Yout, uint32_t* Bhi, uint32_t* Blo, int R, int RQ, int count,
                          int Nt, int Lh, int V, const cplx<float>* Gf, const cplx<float>* twf, const Ctrl* ctrl,
                          hipStream_t s);
// Overlap-save form of the packed routes' pair products and convolution (complex64 fields): Bhi == nullptr
// writes FP32 rows [count][Np][Nt] to Bp, else the BF16 hi/lo planes [count][kBf16Kpad/8][Nt][8].
hipError_t launch_pairs_os(const cplx<float>* A, float* Bp, uint32_t* Bhi, uint32_t* Blo, const int2* pairs, int N,
                           int Np, int count, int Nt, int Lh, int V, const cplx<float>* Gf, const cplx<float>* twf,
                           const Ctrl* ctrl, hipStream_t s);
// Overlap-save form of the general route's pair rows with Raman (complex64 fields), rows [count][KD][Nt].
hipError_t launch_pairs_dense_os(const cplx<float>* A, float* Bd, const int2* pairs, int N, int Np, int count, int KD,
                                 int Nt, int Lh, int V, const cplx<float>* Gf, const cplx<float>* twf,
                                 const Ctrl* ctrl, hipStream_t s);
hipError_t launch_conv_bf16(int logn, const float* Y, uint32_t* Bhi, uint32_t* Blo, int R, int RQ, int count,
                            const cplx<float>* Gs, const cplx<float>* tw, const Ctrl* ctrl, hipStream_t s);

hipError_t launch_norm_final(const double* partials, int nblocks, Ctrl* ctrl, double tol, int fixed_iters,
                             int max_iter, hipStream_t s,
                             Ctrl* host = nullptr);
hipError_t launch_ctrl_reset(Ctrl* ctrl, hipStream_t s);

// Wide rank-r route (complex64 fields, N <= wide_max_modes(); gmm_wide.hip).
int wide_max_modes();
// B_Q(t) = Re(A_m A_n^*) for the Np pairs: BF16 planes [count][2][Np][Nt] bf16, else FP32 [count][Np][Nt].
hipError_t launch_pairs_wide(bool bf16, const cplx<float>* A, void* Bout, int N, int Np, int Nt, int count,
                             const Ctrl* ctrl, hipStream_t s);
// FP32 rows [count][rows][Nt] -> bf16 planes [count][2][rows][Nt] (hi, lo).
hipError_t launch_split_rows(const float* Y, void* planes, int rows, int Nt, int count, const Ctrl* ctrl,
                             hipStream_t s);
// NL_p(t) = sum_l C_(p,l)(t) A_l(t), C [count][Np][Nt] FP32; NL overwrites A in place.
hipError_t launch_fold_wide(const float* C, cplx<float>* A_NL, int N, int Np, int Nt, int count, const Ctrl* ctrl,
                            hipStream_t s);
// Per sub-step, out [n][m] = W X with X [k][m] (BF16: planes [2][k][m], Wst [n][2k] = [W^hi W^hi], Wlo [n][k];
// FP32: X [k][m], Wst [n][k]); rocBLAS on stream s.
hipError_t wide_gemm(void* handle, bool bf16, int m, int n, int k, const void* X, const void* Wst, const void* Wlo,
                     float* out, int count, hipStream_t s);
int wide_blas_create(void** handle);
void wide_blas_destroy(void* handle);
// Norm reduction and stop decision for each slot of a batched round (one block per slot).
hipError_t launch_norm_final_b(const BatchSlot* slots, int nslots, int nblocks, double tol, int fixed_iters,
                               int max_iter, hipStream_t s);
// Zero fill of `bytes` (a multiple of 4) at p, by a kernel.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// Mg_pl = g_p (delta_pl - inv_Isat sum_mn S^R_plmn Phi_mn) (g may be NULL) + K_pl (K may be NULL),
// Phi = dt * sum of the chunk partials.
hipError_t launch_gain_matrix(const cplx<double>* part, int C, const cplx<double>* SR, const double* g,
                              double inv_Isat, double dt, const cplx<double>* K, cplx<double>* Mg, int N, int count,
                              const Ctrl* ctrl, hipStream_t s);

inline int contract_max_rows() { return 256; }
inline int trapz_blocks(long nn) { return (int)((nn + 255) / 256); }

}  // namespace gmm
