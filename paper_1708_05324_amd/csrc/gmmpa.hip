// Host driver and C ABI of the massively parallel GMMNLSE propagator
// (Sec. III.D of Wright et al.).  Everything numerical runs in the kernels of
// gmm_kernels.hpp; this file validates inputs, precomputes per-plan constants
// in FP64, owns device memory, and sequences the kernels of each large step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <vector>

#include "gmmpa.h"
#include "gmm_common.hpp"
#include "gmm_launch.hpp"

using gmm::cplx;
using gmm::Ctrl;
using gmm::Launch;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define GMM_HIP(call)                                                                                \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess) return fail(GMM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Queue a kernel launch; with profiling on, bracket it with two events.
#define GMM_LAUNCH(P, KIND, call)                                                  \
  do {                                                                             \
    hipEvent_t a_ = nullptr, b_ = nullptr;                                         \
    const bool t_ = (P)->prof.on && ((P)->prof.mask >> (KIND) & 1u);               \
    if (t_) {                                                                      \
      a_ = (P)->prof.get();                                                        \
      b_ = (P)->prof.get();                                                        \
      if (!a_ || !b_) return fail(GMM_ERR_HIP, "hipEventCreate failed");           \
      GMM_HIP(hipEventRecord(a_, (P)->stream));                                    \
    }                                                                              \
    GMM_HIP(call);                                                                 \
    if (t_) {                                                                      \
      GMM_HIP(hipEventRecord(b_, (P)->stream));                                    \
      (P)->prof.recs.push_back({a_, b_, (KIND), (P)->prof.cur_step, (P)->prof.cur_iter}); \
    }                                                                              \
  } while (0)

constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

// Host FP64 radix-2 transform, used once per plan for the Raman response:
// X_k = sum_j x_j exp(+2 pi i j k / n).
void host_fft_plus(std::vector<std::complex<double>>& a) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const double ang = 2.0 * kPi * (double)k / (double)len;
        const std::complex<double> w(std::cos(ang), std::sin(ang));
        std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

}  // namespace

// Per-kernel HIP-event timing, off by default.  Every launch is bracketed by
// two events on the plan's stream; launches of speculatively queued
// iterations that exit at once (the step had already converged) are dropped
// when the records are read, so averages cover launches that did work.
struct GmmProfiler {
  struct Rec {
    hipEvent_t a, b;
    int kind, step, iter;
  };
  bool on = false;
  unsigned mask = 0;  // bit k: time kernels of kind k
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::vector<int> step_iters;  // iterations that ran, per large step of the current propagate
  int cur_step = 0, cur_iter = 0;
  double ms[GMM_PROF_KINDS] = {};
  long long n[GMM_PROF_KINDS] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void collect() {  // call after the stream is synchronised
    for (const Rec& r : recs) {
      const bool valid = r.iter == 0 || (r.step < (int)step_iters.size() && r.iter <= step_iters[r.step]);
      float t = 0.f;
      if (valid && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.kind] += t;
        n[r.kind] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
    step_iters.clear();
    cur_step = cur_iter = 0;
  }
  void reset() {
    for (int k = 0; k < GMM_PROF_KINDS; ++k) ms[k] = 0, n[k] = 0;
  }
  // start of a propagate: the per-step bookkeeping covers this call only
  void begin() {
    step_iters.clear();
    cur_step = cur_iter = 0;
  }
  ~GmmProfiler() {
    for (auto& r : recs) pool.push_back(r.a), pool.push_back(r.b);
    for (hipEvent_t e : pool)
      if (e) (void)hipEventDestroy(e);
  }
};

struct gmm_plan_s {
  gmm_params prm{};
  int N = 0, nt = 0, logn = 0, nb = 0, Np = 0, rt = 0, rpad = 0;
  hipStream_t stream = nullptr;
  int device = -1;  // the GPU current when the plan was created (its buffers live there)
  double domega = 0, gamma_hat = 0;
  bool fp64 = true, raman = false, bf16 = false;
  size_t esz = 0;  // bytes per real of the field precision
  // constants
  double* coef = nullptr;  // [N][nb] beta_n / n!
  void* tw = nullptr;      // [nt] exp(-2 pi i m/nt) in field precision
  void* Hs = nullptr;      // [nt] ((1 - fR) + fR H / H0) / nt (blended Raman filter)
  void* ST = nullptr;      // [rpad][rpad] packed coupling matrix, transposed (FP64 / FP32)
  void* Shi = nullptr;     // [rpad][128] bf16 high part of the packed matrix, K contiguous (BF16X3)
  void* Slo = nullptr;     // [2][rpad][128] bf16 lo and lo2 planes
  // rank-r route (Raman on, low-rank packed matrix): S^ = U V
  bool factored = false;
  int rank = 0, rq = 0, kp = 0;  // r, r rounded up to 16, Np rounded up to 64
  // contraction launch chosen by gmm_plan_autotune: kernel (rank-r FP32 route: 0 column-owner, 1 row-register,
  // 2 column-owner on 48-column tiles; rank-r BF16X3 route: 0 column-owner, 1 the same on 48-column tiles)
  // and blocks per CU of the persistent grid (0: as many as fit)
  int tune_kernel = 0, tune_bpc = 0;
  void* VT = nullptr;      // [kp][rq] V transposed, field precision
  void* UT = nullptr;      // [64][rpad] U transposed (contraction operand, K = 64)
  void* Uhi = nullptr;     // [rpad][64] bf16 split of U, K contiguous (BF16X3)
  void* Ulo = nullptr;     // [2][rpad][64]: the lo and lo2 planes
  void* Vhi = nullptr;     // [rq][kp] bf16 split of V, pair index contiguous (BF16X3)
  void* Vlo = nullptr;     // [2][rq][kp]: the lo and lo2 planes
  void* Y = nullptr;       // workspace [cap][rq][nt]: Y = V B
  // wide rank-r route (complex64 fields, N up to 55): both products on rocBLAS, see gmm_wide.hip
  bool wide = false;
  void* blas = nullptr;    // rocblas_handle
  void* Wv = nullptr;      // BF16: [rq][2 Np] = [V^hi V^hi]; FP32: [rq][Np] V
  void* Wv_lo = nullptr;   // BF16: [rq][Np] V^lo
  void* Wu = nullptr;      // BF16: [Np][2 rq] = [U^hi U^hi]; FP32: [Np][rq] U
  void* Wu_lo = nullptr;   // BF16: [Np][rq] U^lo
  // overlap-save form of the Raman convolution (short Raman response)
  int os_lh = 0, os_v = 0;  // kernel taps, outputs per 2^11-point segment (0: full-row transforms)
  void* Gos = nullptr;      // [2^11] segment filter DFT_{+}(g) / 2^11, field precision
  void* twos = nullptr;     // [2^11] exp(-2 pi i m / 2^11), field precision
  // general-tensor route (S^R != S^K, complex S, or S without the packed symmetries)
  bool dense = false;
  int KD = 0, rows_pad = 0;  // real pair rows per sub-step (multiple of 4); output rows 2 N^2 padded to 64
  int KD32 = 0;              // KD rounded up to 32 (BF16 split operand)
  void* G = nullptr;         // [rows_pad][KD] real coupling matrix of the general route, field precision
  void* Ghi = nullptr;       // [rows_pad][KD32] bf16 split of G (BF16X3 plans)
  void* Glo = nullptr;
  // saturating gain (Sec. III.F): G = Mg A per sub-step
  std::vector<std::complex<double>> SRh;  // host copy of S^R (S^K when SR is NULL), [N^4]
  bool gain_on = false;
  bool coupling_on = false;          // linear mode coupling C_p = i sum_n Q_np A_n (in the integrand)
  cplx<double>* Kc = nullptr;        // [N][N] K_pl = i Q_lp
  // linear coupling inside the linear operator: L(w) = i H(w), H = diag(d(w)) + Q^T = U diag(lam) U^H;
  // the iterate psi is then kept in the eigenbasis (psi_eig = U^H psi) and E holds exp(i lam j dz)
  bool cpl_exact = false;
  void* Uc = nullptr;                // [N][N][nt] eigenvectors (column q = eigenvector q), field precision
  double* lam = nullptr;             // [N][nt] eigenvalues (1/m)
  std::vector<double> coefh;         // host copy of coef
  double inv_Isat = 0.0;
  double* gvec = nullptr;               // [N] g_p (1/m)
  cplx<double>* SRd = nullptr;          // [N^4] S^R on the device
  cplx<double>* gpart = nullptr;        // workspace [cap][Nt/256][N][N] pair-integral partials
  cplx<double>* Mg = nullptr;           // workspace [cap][N][N]
  int gain_cap = 0;
  int* pidx = nullptr;     // [N][N]
  int2* pairs = nullptr;   // [Np]
  // workspace
  int cap = 0;  // sub-step capacity
  void *psi0 = nullptr, *I0 = nullptr, *psi = nullptr, *work = nullptr, *Bp = nullptr;
  void* E = nullptr;    // phase table [E_rows][N][nt]: exp(D_w j dz), built per step size
  int E_rows = 0;
  double E_dz = 0.0;
  void* E64 = nullptr;  // single-precision fields: [N][nt] row E64_row of the table in FP64
  int E64_row = -1;
  double* partials = nullptr;
  Ctrl* ctrl = nullptr;
  Ctrl* h_ctrl = nullptr;         // pinned, mapped: the norm kernel stores the control block here
  Ctrl* h_ctrl_dev = nullptr;     // its device-visible address
  hipEvent_t ev = nullptr;        // marks the stop-flag copy the host waits for
  double* h_partials = nullptr;   // pinned
  long long const_bytes = 0, ws_bytes = 0;
  GmmProfiler prof;
};

namespace {

template <typename T>
int dev_alloc(long long* counter, T** ptr, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GMM_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  *ptr = (T*)p;
  *counter += (long long)bytes;
  return GMM_OK;
}

void free_workspace(gmm_plan_s* P) {
  for (void** p : {&P->psi0, &P->I0, &P->psi, &P->work, &P->Bp, &P->Y, &P->E, &P->E64}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  P->E_rows = 0;
  P->E64_row = -1;
  if (P->partials) (void)hipFree(P->partials);
  P->partials = nullptr;
  P->cap = 0;
  P->ws_bytes = 0;
}

size_t field_bytes(const gmm_plan_s* P) { return (size_t)P->N * P->nt * 2 * P->esz; }

// The MPA keeps its sub-step iterates in the lab frame, exp(D_w z_j) psi_j, when the linear operator is the
// diagonal dispersion alone (no gain, no linear coupling): the transforms to and from time then read no phase.
bool lab_frame(const gmm_plan_s* P) { return !P->gain_on && !P->coupling_on && !P->cpl_exact; }

// Pair-integral partials and gain matrices for `cap` sub-steps (only with the gain term on).
int ensure_gain_workspace(gmm_plan_s* P, int cap) {
  if (!(P->gain_on || P->coupling_on) || cap <= P->gain_cap) return GMM_OK;
  for (cplx<double>** q : {&P->gpart, &P->Mg}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  P->gain_cap = 0;
  const size_t nn = (size_t)P->N * P->N;
  void* a = nullptr;
  void* b = nullptr;
  if (hipMalloc(&a, (size_t)cap * gmm::gain_partials(P->nt) * nn * sizeof(cplx<double>)) != hipSuccess ||
      hipMalloc(&b, (size_t)cap * nn * sizeof(cplx<double>)) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    return fail(GMM_ERR_NOMEM, "hipMalloc of the gain workspace failed");
  }
  P->gpart = (cplx<double>*)a;
  P->Mg = (cplx<double>*)b;
  P->gain_cap = cap;
  return GMM_OK;
}

// B' for `cap` sub-steps: [cap][Np][Nt] reals, or two bf16 planes [cap][Kpad/8][Nt][8].
size_t bp_bytes(const gmm_plan_s* P, int cap) {
  if (P->dense) return (size_t)cap * P->KD * P->nt * P->esz;
  // wide route: [cap][Np][Nt] 4-byte words (B: two bf16 planes or FP32 rows, later C), then Y' [cap][RQ][Nt]
  if (P->wide) return (size_t)cap * (P->Np + P->rq) * P->nt * 4;
  if (P->bf16) return 2 * (size_t)cap * gmm::kBf16Kpad * P->nt * 2;
  // packed route: [cap][Np][Nt]; rank-r route: Y' [cap][RQ][Nt] (RQ can exceed Np for small Np)
  const int rows = P->factored ? std::max(P->Np, P->rq) : P->Np;
  return (size_t)cap * rows * P->nt * P->esz;
}
size_t bp_plane_words(const gmm_plan_s* P) { return (size_t)P->cap * gmm::kBf16Kpad * P->nt / 2; }

int ensure_workspace(gmm_plan_s* P, int cap) {
  if (cap <= P->cap) return GMM_OK;
  const size_t fb = field_bytes(P);
  free_workspace(P);
  long long* c = &P->ws_bytes;
  int rc;
  if ((rc = dev_alloc(c, &P->psi0, fb)) || (rc = dev_alloc(c, &P->I0, fb)) || (rc = dev_alloc(c, &P->psi, fb * cap)) ||
      (rc = dev_alloc(c, &P->work, fb * cap)) ||
      (rc = dev_alloc(c, &P->Bp, bp_bytes(P, cap))) ||
      (rc = dev_alloc(c, &P->partials, 2 * sizeof(double) * gmm::trapz_blocks((long)P->N * P->nt))) ||
      (P->factored && (rc = dev_alloc(c, &P->Y, (size_t)cap * P->rq * P->nt * P->esz)))) {
    free_workspace(P);
    return rc;
  }
  // BF16 pair slots beyond Np, and rows R..RQ-1 of the rank-r route, are read
  // by the contraction (with zero coefficients) but never written: keep them 0.
  if (P->bf16 || P->factored || P->dense) {
    if (hipMemset(P->Bp, 0, bp_bytes(P, cap)) != hipSuccess) {
      free_workspace(P);
      return fail(GMM_ERR_HIP, "hipMemset of the pair buffer failed");
    }
  }
  P->cap = cap;
  return GMM_OK;
}

// Device buffers one nonlinear evaluation works in: the plan's own workspace,
// a batch's buffers, or slices of the static scratch of the no-allocation
// entry point.
struct EvalWs {
  void* work = nullptr;             // [cap][N][Nt] field rows
  void* Bp = nullptr;               // pair rows / Y' (layout of bp_bytes)
  void* Y = nullptr;                // rank-r route: [cap][RQ][Nt]
  cplx<double>* gpart = nullptr;    // gain / coupling: pair-integral partials
  cplx<double>* Mg = nullptr;       // gain / coupling: per-sub-step matrices
  int cap = 0, gain_cap = 0;        // sub-steps the buffers hold
  size_t plane_words = 0;           // BF16 planes: words per plane
};

EvalWs plan_ws(const gmm_plan_s* P) {
  EvalWs w;
  w.work = P->work;
  w.Bp = P->Bp;
  w.Y = P->Y;
  w.gpart = P->gpart;
  w.Mg = P->Mg;
  w.cap = P->cap;
  w.gain_cap = P->gain_cap;
  w.plane_words = bp_plane_words(P);
  return w;
}

// Launch candidates of the contraction that gmm_plan_autotune times, in its
// numbering: kernel (rank-r FP32 route: 0 column-owner, 1 row-register, 2
// column-owner on 48-column tiles; rank-r BF16X3 route: 0 column-owner, 1 the
// same on 48-column tiles) and blocks per CU of the persistent grid.
struct ContractCand {
  int kernel, bpc;
};
std::vector<ContractCand> contraction_candidates(const gmm_plan_s* P) {
  std::vector<ContractCand> c;
  if (P->fp64 || P->dense || P->wide) return c;
  if (P->factored && !P->bf16) {
    for (int b : {1, 2}) c.push_back({0, b});
    if (P->rt <= 2)
      for (int b : {1, 2, 3, 4}) c.push_back({1, b});
    for (int b : {1, 2}) c.push_back({2, b});
  } else if (P->factored) {
    for (int b : {1, 2}) c.push_back({0, b});
    for (int b : {1, 2}) c.push_back({1, b});
  } else if (!P->bf16 && P->rt <= 2) {
    for (int b : {1, 2, 3, 4}) c.push_back({0, b});
  }
  return c;
}

// ---------------------------------------------------------------------------
// Typed sequencing of one nonlinear evaluation and one iteration.
template <typename T>
struct Runner {
  gmm_plan_s* P;
  // field at the start of the current large step: psi0, or (lab frame, after the first large step) the previous
  // step's last iterate, a row of psi, which the step's first trapezoid copies to psi0
  const cplx<T>* start = nullptr;
  const cplx<T>* tw() const { return (const cplx<T>*)P->tw; }

  // The route-specific middle of one evaluation over `count` field rows of
  // ws.work (time domain in, NL(t) out in place): pair rows or Y = V B, the Raman
  // convolution, the contraction and the mode projection.  doA / doB: the
  // halves before / from the contraction.
  int mid(int count, const EvalWs& ws, const Ctrl* ctrl, bool doA, bool doB) {
    cplx<T>* W = (cplx<T>*)ws.work;
    if (P->wide) {  // pair rows; Y = V B; Y' = g * Y; C = U Y'; fold (the products on rocBLAS, in the second half)
      if constexpr (std::is_same<T, float>::value) {
        float* BC = (float*)ws.Bp;                                       // B rows, later C
        float* Yp = (float*)ws.Bp + (size_t)ws.cap * P->Np * P->nt;     // Y' [cap][RQ][Nt]
        float* Y = (float*)ws.Y;
        if (doA)
          GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_pairs_wide(P->bf16, W, BC, P->N, P->Np, P->nt, count, ctrl,
                                                               P->stream));
        if (!doB) return GMM_OK;
        GMM_LAUNCH(P, GMM_PROF_PROJECT, gmm::wide_gemm(P->blas, P->bf16, P->nt, P->rq, P->Np, BC, P->Wv, P->Wv_lo, Y,
                                                       count, P->stream));
        const float* Yc = Y;
        if (P->raman) {
          const int R = P->rank + (P->rank & 1);
          if (P->os_lh)
            GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<float>::conv_os(Y, Yp, R, P->rq, count, P->nt, P->os_lh, P->os_v,
                                                                 (const cplx<float>*)P->Gos,
                                                                 (const cplx<float>*)P->twos, ctrl, P->stream));
          else
            GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<float>::conv(P->logn, Y, Yp, R, P->rq, count,
                                                              (const cplx<float>*)P->Hs, tw(), ctrl, P->stream));
          Yc = Yp;
        }
        const void* X = Yc;
        if (P->bf16) {  // Y' -> bf16 planes, into whichever of Y and the Y' region Yc is not
          void* planes = P->raman ? (void*)Y : (void*)Yp;
          GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_split_rows(Yc, planes, P->rq, P->nt, count, ctrl, P->stream));
          X = planes;
        }
        GMM_LAUNCH(P, GMM_PROF_CONTRACT, gmm::wide_gemm(P->blas, P->bf16, P->nt, P->Np, P->rq, X, P->Wu, P->Wu_lo, BC,
                                                        count, P->stream));
        GMM_LAUNCH(P, GMM_PROF_CONTRACT, gmm::launch_fold_wide(BC, W, P->N, P->Np, P->nt, count, ctrl, P->stream));
        return GMM_OK;
      } else {
        return fail(GMM_ERR_UNSUPPORTED, "internal: wide route with complex128 fields");
      }
    }
    if (P->dense) {  // general tensors: real pair rows, then C = G B and the complex projection
      bool os_done = false;
      if constexpr (std::is_same<T, float>::value) {
        if (P->os_lh) {  // Raman on, short h_R: overlap-save segments
          if (doA)
            GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_pairs_dense_os(W, (float*)ws.Bp, P->pairs, P->N, P->Np, count,
                                                                     P->KD, P->nt, P->os_lh, P->os_v,
                                                                     (const cplx<float>*)P->Gos,
                                                                     (const cplx<float>*)P->twos, ctrl, P->stream));
          os_done = true;
        }
      }
      if (doA && !os_done)
        GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<T>::pairs_dense(P->logn, P->raman, W, (T*)ws.Bp, P->pairs, P->N, P->Np,
                                                           count, P->KD, (const cplx<T>*)P->Hs, tw(), ctrl,
                                                           P->stream));
      bool done = false;
      if constexpr (std::is_same<T, float>::value) {
        if (P->bf16 && doB) {
          GMM_LAUNCH(P, GMM_PROF_CONTRACT,
                     gmm::launch_contract_dense_bf16(P->Ghi, P->Glo, (const float*)ws.Bp, W, P->N, P->KD, P->KD32,
                                                     P->nt, count, ctrl, P->stream));
        }
        done = P->bf16;
      }
      if (!done && doB)
        GMM_LAUNCH(P, GMM_PROF_CONTRACT, Launch<T>::contract_dense((const T*)P->G, (const T*)ws.Bp, W, P->N, P->KD,
                                                                   P->rows_pad, P->nt, count, ctrl, P->stream));
    } else if (P->factored) {  // Y = V B; Y' = g * Y (r rows); C = U Y' + projection
      T* Y = (T*)ws.Y;
      if constexpr (std::is_same<T, float>::value) {
        if (doA)
          GMM_LAUNCH(P, GMM_PROF_PROJECT,
                     gmm::launch_project_cols(P->rq, P->kp, P->bf16, P->bf16 ? P->Vhi : P->VT, P->Vlo, W, Y, P->N,
                                            P->nt, count, ctrl, P->stream));
      } else if (doA) {
        GMM_LAUNCH(P, GMM_PROF_PROJECT, Launch<T>::project(P->rq, P->kp, (const T*)P->VT, W, Y, P->pairs, P->N,
                                                         P->Np, P->nt, count, ctrl, P->stream));
      }
      const int R = P->rank + (P->rank & 1);
      if constexpr (std::is_same<T, float>::value) {
        if (P->bf16) {
          uint32_t* bhi = (uint32_t*)ws.Bp;
          uint32_t* blo = bhi + ws.plane_words;
          if (P->os_lh && doA)
            GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_conv_os(Y, nullptr, bhi, blo, R, P->rq, count, P->nt, P->os_lh,
                                                              P->os_v, (const cplx<float>*)P->Gos,
                                                              (const cplx<float>*)P->twos, ctrl, P->stream));
          else if (doA)
            GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_conv_bf16(P->logn, Y, bhi, blo, R, P->rq, count,
                                                                (const cplx<float>*)P->Hs, tw(), ctrl, P->stream));
          if (doB)
            GMM_LAUNCH(P, GMM_PROF_CONTRACT, gmm::launch_contract_cols(P->rpad, true, P->Uhi, P->Ulo, bhi, blo, W,
                                                                     P->N, R, P->nt, count, ctrl, P->stream,
                                                                     P->tune_bpc, P->tune_kernel == 1 ? 3 : 4));
        }
      }
      if (!P->bf16) {
        const bool os_done = P->os_lh != 0;
        if (os_done && doA)
          GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<T>::conv_os(Y, (T*)ws.Bp, R, P->rq, count, P->nt, P->os_lh, P->os_v,
                                                         (const cplx<T>*)P->Gos, (const cplx<T>*)P->twos, ctrl,
                                                         P->stream));
        if (!os_done && doA)
          GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<T>::conv(P->logn, Y, (T*)ws.Bp, R, P->rq, count,
                                                        (const cplx<T>*)P->Hs, tw(), ctrl, P->stream));
        if constexpr (std::is_same<T, float>::value) {
          if (doB && P->tune_kernel == 1)
            GMM_LAUNCH(P, GMM_PROF_CONTRACT, Launch<T>::contract(P->rt, 64, (const T*)P->UT, (const T*)ws.Bp, W,
                                                                 P->pidx, P->N, P->rq, P->nt, count, ctrl, P->stream,
                                                                 P->tune_bpc));
          else if (doB)
            GMM_LAUNCH(P, GMM_PROF_CONTRACT, gmm::launch_contract_cols(P->rpad, false, P->UT, nullptr, ws.Bp, nullptr,
                                                                     W, P->N, P->rq, P->nt, count, ctrl, P->stream,
                                                                     P->tune_bpc, P->tune_kernel == 2 ? 3 : 4));
        } else if (doB) {
          GMM_LAUNCH(P, GMM_PROF_CONTRACT, Launch<T>::contract(P->rt, 64, (const T*)P->UT, (const T*)ws.Bp, W,
                                                               P->pidx, P->N, P->rq, P->nt, count, ctrl, P->stream));
        }
      }
    } else if constexpr (std::is_same<T, float>::value) {
      if (P->bf16) {  // packed route, BF16 split
        uint32_t* bhi = (uint32_t*)ws.Bp;
        uint32_t* blo = bhi + ws.plane_words;
        if (doA && P->os_lh)
          GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_pairs_os(W, nullptr, bhi, blo, P->pairs, P->N, P->Np, count, P->nt,
                                                             P->os_lh, P->os_v, (const cplx<float>*)P->Gos,
                                                             (const cplx<float>*)P->twos, ctrl, P->stream));
        else if (doA)
          GMM_LAUNCH(P, GMM_PROF_PAIRS, gmm::launch_pairs_bf16(P->logn, P->raman, W, bhi, blo, P->pairs, P->N, P->Np,
                                                             count, (const cplx<float>*)P->Hs, tw(), ctrl, P->stream));
        if (doB)
          GMM_LAUNCH(P, GMM_PROF_CONTRACT, gmm::launch_contract_bf16(P->rt, 128, P->Shi, P->Slo, bhi, blo, W, P->pidx,
                                                                   P->N, P->nt, count, ctrl, P->stream));
      }
    }
    if (!P->bf16 && !P->factored && !P->dense) {
      const bool os_done = P->os_lh != 0;
      if (os_done && doA)
        GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<T>::pairs_os(W, (T*)ws.Bp, P->pairs, P->N, P->Np, count, P->nt, P->os_lh,
                                                        P->os_v, (const cplx<T>*)P->Gos, (const cplx<T>*)P->twos, ctrl,
                                                        P->stream));
      if (doA && !os_done)
        GMM_LAUNCH(P, GMM_PROF_PAIRS, Launch<T>::pairs(P->logn, P->raman, W, (T*)ws.Bp, P->pairs, P->N, P->Np, count,
                                                     (const cplx<T>*)P->Hs, tw(), ctrl, P->stream));
      if (doB)
        GMM_LAUNCH(P, GMM_PROF_CONTRACT, Launch<T>::contract(P->rt, 0, (const T*)P->ST, (const T*)ws.Bp, W, P->pidx,
                                                           P->N, P->Np, P->nt, count, ctrl, P->stream,
                                                           P->tune_bpc));
    }
    return GMM_OK;
  }

  // out[c] = N~[ exp(D z_{j0+c}) psi_c ] * exp(-D z_{j0+c}) for c < count.
  // psi_c starts at psi + c * jrows * Nt: jrows = N (one field per sub-step)
  // or 0 (every sub-step reads the same field).  Field rows go through
  // `work`; `out` may be `work` itself.
  // part 0: the whole evaluation; part 1: its first half (transforms to time, gain matrices, pair rows or
  // Y = V B and the Raman convolution); part 2: the rest (contraction, transforms back, gain term).  The MPA
  // driver queues the halves separately so that it can wait for a stop flag in the middle of an iteration.
  int eval(const cplx<T>* psi, long jrows, int count, int j0, double dz, cplx<T>* out, const Ctrl* ctrl,
           int part = 0, const EvalWs* wsp = nullptr) {
    const EvalWs ws = wsp ? *wsp : plan_ws(P);
    const bool doA = part != 2, doB = part != 1;
    if (jrows != 0 && jrows != P->N) return fail(GMM_ERR_ARG, "internal: sub-step stride must be 0 or N rows");
    if (count > ws.cap) return fail(GMM_ERR_ARG, "internal: workspace smaller than the sub-step count");
    cplx<T>* W = (cplx<T>*)ws.work;
    const cplx<T>* E = dz != 0.0 ? (const cplx<T>*)P->E : nullptr;
    // coupled linear operator: psi is in the eigenbasis; the modes are U (exp(i lam z) psi)
    const bool mix = P->cpl_exact && E != nullptr;
    // lab-frame iterates (MPA without gain and coupling terms): stored sub-step fields already carry
    // exp(D z_j), and the outputs keep the frame (the trapezoid applies exp(-D z_j))
    const bool lab = E != nullptr && lab_frame(P);
    if (mix && doA) {
      GMM_LAUNCH(P, GMM_PROF_PHASE, Launch<T>::mode_mix(false, psi, jrows, W, (const cplx<T>*)P->Uc, E, j0, P->N,
                                                      P->nt, count, ctrl, P->stream));
      GMM_LAUNCH(P, GMM_PROF_PHASE, Launch<T>::phase_to_time(P->logn, W, P->N, W, nullptr, P->N, count, j0, tw(),
                                                           ctrl, P->stream));
    } else if (doA) {
      GMM_LAUNCH(P, GMM_PROF_PHASE, Launch<T>::phase_to_time(P->logn, psi, jrows, W, lab && jrows != 0 ? nullptr : E,
                                                           P->N, count, j0, tw(), ctrl, P->stream));
    }
    const bool linear_terms = P->gain_on || P->coupling_on;
    if (linear_terms && doA) {  // pair integrals of the sub-step fields (saturation), then the matrices Mg
      if (count > ws.gain_cap) return fail(GMM_ERR_ARG, "internal: gain workspace smaller than the sub-step count");
      if (P->gain_on && P->inv_Isat != 0.0)
        GMM_LAUNCH(P, GMM_PROF_GAIN, Launch<T>::pair_integrals(W, ws.gpart, P->N, P->nt, count, ctrl, P->stream));
      GMM_LAUNCH(P, GMM_PROF_GAIN,
                 gmm::launch_gain_matrix(ws.gpart, gmm::gain_partials(P->nt), P->SRd,
                                         P->gain_on ? P->gvec : nullptr, P->inv_Isat, P->prm.dt,
                                         P->coupling_on ? P->Kc : nullptr, ws.Mg, P->N, count, ctrl, P->stream));
    }
    {
      const int rc_mid = mid(count, ws, ctrl, doA, doB);
      if (rc_mid) return rc_mid;
    }
    if (!doB) return GMM_OK;
    GMM_LAUNCH(P, GMM_PROF_SPECTRAL, Launch<T>::spectral_out(P->logn, W, out, mix || lab ? nullptr : E, P->N, count, j0,
                                                           P->domega, P->gamma_hat / P->nt, 1.0 / P->prm.omega0,
                                                           P->prm.self_steepening, tw(), ctrl, P->stream));
    if (mix)  // back to the eigenbasis, then exp(-i lam z)
      GMM_LAUNCH(P, GMM_PROF_SPECTRAL, Launch<T>::mode_mix(true, out, P->N, out, (const cplx<T>*)P->Uc, E, j0, P->N,
                                                         P->nt, count, ctrl, P->stream));
    if (linear_terms)
      GMM_LAUNCH(P, GMM_PROF_GAIN, Launch<T>::gain_add(psi, jrows, E, j0, ws.Mg, out, P->N, P->nt, count, ctrl,
                                                       P->stream));
    return GMM_OK;
  }

  // One iteration over the m sub-steps of a large step.  The first iteration
  // also evaluates I_0 = N~[A(z0)] in the same launches (sub-step 0, no phase),
  // since every sub-step then reads psi_0; its trapezoid copies I_0 aside.
  // part 0: the whole iteration; 1: the first half of the evaluation; 2: the rest, the trapezoid and the norm.
  int iteration(int m, double dz, bool first, int part = 0) {
    const long nn = (long)P->N * P->nt;
    cplx<T>* W = (cplx<T>*)P->work;
    const cplx<T>* psi0 = (const cplx<T>*)P->psi0;
    const cplx<T>* src0 = start != nullptr ? start : psi0;
    // The first iteration of a large step that starts from the previous step's last iterate: the control block
    // still says that step is done, so these launches test no stop flag, and the trapezoid clears the block
    // (before the norm reads it) and keeps the start field in psi0 for the later iterations.
    const bool fresh = first && src0 != psi0;
    const Ctrl* c = fresh ? nullptr : P->ctrl;
    int rc = first ? eval(src0, 0, m + 1, 0, dz, W, c, part)
                   : eval((const cplx<T>*)P->psi, P->N, m, 1, dz, W, c, part);
    if (rc || part == 1) return rc;
    const cplx<T>* I0 = first ? W : (const cplx<T>*)P->I0;
    const cplx<T>* I = first ? W + nn : W;
    GMM_LAUNCH(P, GMM_PROF_TRAPZ, Launch<T>::trapz(first ? src0 : psi0, I0, I, (cplx<T>*)P->psi, (cplx<T>*)P->I0,
                                                   first ? 1 : 0, m, nn, (T)dz, P->partials, c, P->stream,
                                                   lab_frame(P) ? (const cplx<T>*)P->E : nullptr,
                                                   lab_frame(P) ? last_factor(m) : nullptr,
                                                   fresh ? (cplx<T>*)P->psi0 : nullptr, fresh ? P->ctrl : nullptr));
    GMM_LAUNCH(P, GMM_PROF_NORM, gmm::launch_norm_final(P->partials, gmm::trapz_blocks(nn), P->ctrl, P->prm.tol,
                                                        P->prm.fixed_iters, P->prm.max_iter, P->stream,
                                                        P->h_ctrl_dev));
    return GMM_OK;
  }

  // exp(D_w m dz) in FP64 for the sub-step that ends a large step of m sub-steps (single-precision fields,
  // full large steps), else nullptr: the table's own row serves.
  const cplx<double>* last_factor(int m) const {
    return P->E64 != nullptr && P->E64_row == m ? (const cplx<double>*)P->E64 : nullptr;
  }

  // Row j of the table in FP64, kept beside it for single-precision fields: the factor that carries the field
  // from one large step to the next is applied once per step, so its rounding would add up step after step.
  int ensure_last_factor(int j, double dz) {
    if (P->E64 == nullptr) {
      const int rc = dev_alloc(&P->ws_bytes, &P->E64, (size_t)P->N * P->nt * sizeof(cplx<double>));
      if (rc) return rc;
    }
    if (P->cpl_exact)
      GMM_HIP(Launch<double>::phase_table_lam((cplx<double>*)P->E64, P->lam, P->N, P->nt, 1, dz, P->stream, j));
    else
      GMM_HIP(Launch<double>::phase_table((cplx<double>*)P->E64, P->coef, P->nb, P->N, P->nt, 1, dz, P->domega,
                                          P->stream, j));
    P->E64_row = j;
    return GMM_OK;
  }

  // Phase factors exp(D_w j dz) for j < rows (FP64 phase, rounded to the field precision); for single-precision
  // fields also row rows - 1 in FP64.
  int ensure_phase_table(int rows, double dz) {
    const bool keep64 = sizeof(T) == 4;
    if (P->E != nullptr && P->E_rows >= rows && P->E_dz == dz)
      return keep64 && P->E64_row != rows - 1 ? ensure_last_factor(rows - 1, dz) : GMM_OK;
    if (P->E != nullptr && P->E_rows < rows) {
      (void)hipFree(P->E);
      P->ws_bytes -= (long long)P->E_rows * field_bytes(P);
      P->E = nullptr;
      P->E_rows = 0;
    }
    if (P->E == nullptr) {
      int rc = dev_alloc(&P->ws_bytes, &P->E, (size_t)rows * field_bytes(P));
      if (rc) return rc;
      P->E_rows = rows;
    }
    if (P->cpl_exact)
      GMM_HIP(Launch<T>::phase_table_lam((cplx<T>*)P->E, P->lam, P->N, P->nt, P->E_rows, dz, P->stream));
    else
      GMM_HIP(Launch<T>::phase_table((cplx<T>*)P->E, P->coef, P->nb, P->N, P->nt, P->E_rows, dz, P->domega,
                                     P->stream));
    P->E_dz = dz;
    return keep64 ? ensure_last_factor(rows - 1, dz) : GMM_OK;
  }

  int spec_sums(const cplx<T>* At, double* energy, double* photons) {
    const long nn = (long)P->N * P->nt;
    const int nblk = gmm::trapz_blocks(nn);
    GMM_HIP(Launch<T>::spec_sums(At, P->nt, nn, P->domega, P->prm.omega0, P->partials, P->stream));
    GMM_HIP(hipMemcpyAsync(P->h_partials, P->partials, 2 * sizeof(double) * nblk, hipMemcpyDeviceToHost,
                           P->stream));
    GMM_HIP(hipStreamSynchronize(P->stream));
    double a = 0, b = 0;
    for (int i = 0; i < nblk; ++i) {
      a += P->h_partials[2 * i];
      b += P->h_partials[2 * i + 1];
    }
    *energy = a * P->nt * P->prm.dt;  // Parseval: sum_t |A|^2 = Nt sum_k |A~|^2
    *photons = b;
    return GMM_OK;
  }

  int propagate(const void* A0, double L, double dz_req, int M, void* Aout, gmm_stats* st) {
    const long nn = (long)P->N * P->nt;
    // small steps: cover L exactly
    const double r = L / dz_req;
    long n_small = (std::fabs(r - std::round(r)) < 1e-9 * std::max(1.0, r)) ? (long)std::llround(r)
                                                                            : (long)std::ceil(r);
    if (n_small < 1) n_small = 1;
    const double dz = L / (double)n_small;
    P->prof.begin();
    int rc = ensure_workspace(P, M + 1);  // the first iteration also evaluates sub-step 0
    if (rc) return rc;
    if ((rc = ensure_gain_workspace(P, M + 1))) return rc;
    if ((rc = ensure_phase_table(M + 1, dz))) return rc;
    gmm_stats s{};
    s.dz_used = dz;
    // A~(0) = (1/Nt) FFT_{+}(A0)
    GMM_HIP(Launch<T>::fft_rows(P->logn, +1, (const cplx<T>*)A0, (cplx<T>*)P->psi0, (T)(1.0 / P->nt), P->N, tw(),
                                P->stream));
    if ((rc = spec_sums((const cplx<T>*)P->psi0, &s.energy_in, &s.photons_in))) return rc;
    if (P->cpl_exact)  // into the eigenbasis of the coupled linear operator (U unitary per frequency)
      GMM_HIP(Launch<T>::mode_mix(true, (const cplx<T>*)P->psi0, P->N, (cplx<T>*)P->psi0, (const cplx<T>*)P->Uc,
                                  nullptr, 0, P->N, P->nt, 1, nullptr, P->stream));
    long done = 0;
    int status = GMM_OK;
    GMM_HIP(gmm::launch_ctrl_reset(P->ctrl, P->stream));  // later large steps: by the close, or (lab frame) by
                                                           // the step's first trapezoid
    start = (const cplx<T>*)P->psi0;
    while (done < n_small) {
      const int m = (int)std::min<long>(M, n_small - done);
      int n_enq = 0;
      if (P->prm.fixed_iters > 0) {
        for (; n_enq < P->prm.fixed_iters; ++n_enq) {
          P->prof.cur_iter = n_enq + 1;
          if ((rc = iteration(m, dz, n_enq == 0))) return rc;
        }
        GMM_HIP(hipStreamSynchronize(P->stream));  // the last norm stored the control block in h_ctrl
      } else {
        // Queue the first iteration and the first half of the second; then, per
        // iteration n: wait for iteration n's norm (which stores the control
        // block in pinned host memory) while the GPU runs the first half of
        // iteration n + 1, and queue its second half and the first half of
        // iteration n + 2 only if not converged.  After convergence only one
        // half-iteration is queued for nothing, and its launches exit at once
        // (device-side guard).
        P->prof.cur_iter = 1;
        if ((rc = iteration(m, dz, true))) return rc;
        n_enq = 1;
        for (;;) {
          GMM_HIP(hipEventRecord(P->ev, P->stream));
          const bool more = n_enq < P->prm.max_iter;
          if (more) {
            P->prof.cur_iter = n_enq + 1;
            if ((rc = iteration(m, dz, false, 1))) return rc;
          }
          GMM_HIP(hipEventSynchronize(P->ev));
          if (P->h_ctrl->done || !more) break;
          if ((rc = iteration(m, dz, false, 2))) return rc;
          ++n_enq;
        }
      }
      const Ctrl c = *P->h_ctrl;
      P->prof.cur_iter = 0;
      if (P->prof.on) P->prof.step_iters.push_back(c.iters);
      if (c.status == 2) return fail(GMM_ERR_DIVERGED, "non-finite relative change in the MPA iteration");
      if (c.status == 1) {
        s.nonconverged_steps++;
        status = GMM_NOT_CONVERGED;
      }
      s.iterations += c.iters;
      s.evaluations += 1 + (long long)c.iters * m;
      if (c.iters > s.max_iters_seen) s.max_iters_seen = c.iters;
      s.last_eps = c.eps;
      // A~(z0 + m dz) = exp(D m dz) psi_m.  Lab-frame iterates already carry the factor: the last one is the
      // next large step's start field as it stands (no close launch; see iteration()).  Otherwise the close
      // applies the factor into psi0 (coupled operator: exp(i lam m dz) psi_m in the eigenbasis, which is also
      // the next large step's psi(z0) there) and resets the control block.
      if (lab_frame(P))
        start = (const cplx<T>*)P->psi + (size_t)(m - 1) * nn;
      else
        GMM_LAUNCH(P, GMM_PROF_CLOSE, Launch<T>::close((const cplx<T>*)P->psi + (size_t)(m - 1) * nn,
                                                     (cplx<T>*)P->psi0, (const cplx<T>*)P->E + (size_t)m * nn, nn,
                                                     P->ctrl, P->stream, last_factor(m)));
      s.large_steps++;
      s.small_steps += m;
      done += m;
      P->prof.cur_step++;
    }
    const cplx<T>* fin = start != nullptr ? start : (const cplx<T>*)P->psi0;  // the field at L
    start = nullptr;
    if (P->cpl_exact)  // back to the modes
      GMM_HIP(Launch<T>::mode_mix(false, (const cplx<T>*)P->psi0, P->N, (cplx<T>*)P->psi0, (const cplx<T>*)P->Uc,
                                  nullptr, 0, P->N, P->nt, 1, nullptr, P->stream));
    if ((rc = spec_sums(fin, &s.energy_out, &s.photons_out))) return rc;
    GMM_HIP(Launch<T>::fft_rows(P->logn, -1, fin, (cplx<T>*)Aout, (T)1, P->N, tw(), P->stream));
    GMM_HIP(hipStreamSynchronize(P->stream));
    if (P->prof.on) P->prof.collect();
    if (st) *st = s;
    return status;
  }

  // Serial RK4IP baseline: n steps of h, four dependent evaluations each.
  int propagate_rk4ip(const void* A0, double L, double dz_req, void* Aout, gmm_stats* st) {
    if (P->cpl_exact)
      return fail(GMM_ERR_UNSUPPORTED, "RK4IP with the coupling in the linear operator is not implemented");
    const long nn = (long)P->N * P->nt;
    const double r = L / dz_req;
    long n_small = (std::fabs(r - std::round(r)) < 1e-9 * std::max(1.0, r)) ? (long)std::llround(r)
                                                                            : (long)std::ceil(r);
    if (n_small < 1) n_small = 1;
    const double h = L / (double)n_small;
    P->prof.begin();
    int rc = ensure_workspace(P, 6);  // AI, k1..k4, X in the sub-step rows
    if (rc) return rc;
    if ((rc = ensure_gain_workspace(P, 1))) return rc;
    if ((rc = ensure_phase_table(2, 0.5 * h))) return rc;  // row 1: exp(D h/2)
    gmm_stats s{};
    s.dz_used = h;
    cplx<T>* At = (cplx<T>*)P->psi0;
    cplx<T>* rows = (cplx<T>*)P->psi;
    cplx<T>*AI = rows, *k1 = rows + nn, *k2 = rows + 2 * nn, *k3 = rows + 3 * nn, *k4 = rows + 4 * nn,
    *X = rows + 5 * nn;
    const cplx<T>* Eh = (const cplx<T>*)P->E + nn;
    GMM_HIP(Launch<T>::fft_rows(P->logn, +1, (const cplx<T>*)A0, At, (T)(1.0 / P->nt), P->N, tw(), P->stream));
    if ((rc = spec_sums(At, &s.energy_in, &s.photons_in))) return rc;
    for (long n = 0; n < n_small; ++n) {
      if ((rc = eval(At, P->N, 1, 0, 0.0, k1, nullptr))) return rc;
      GMM_HIP(Launch<T>::rk4ip_stage(1, At, AI, k1, k2, k3, k4, X, Eh, (T)h, nn, P->stream));
      if ((rc = eval(X, P->N, 1, 0, 0.0, k2, nullptr))) return rc;
      GMM_HIP(Launch<T>::rk4ip_stage(2, At, AI, k1, k2, k3, k4, X, Eh, (T)h, nn, P->stream));
      if ((rc = eval(X, P->N, 1, 0, 0.0, k3, nullptr))) return rc;
      GMM_HIP(Launch<T>::rk4ip_stage(3, At, AI, k1, k2, k3, k4, X, Eh, (T)h, nn, P->stream));
      if ((rc = eval(X, P->N, 1, 0, 0.0, k4, nullptr))) return rc;
      GMM_HIP(Launch<T>::rk4ip_stage(4, At, AI, k1, k2, k3, k4, X, Eh, (T)h, nn, P->stream));
      P->prof.cur_step++;
    }
    s.large_steps = n_small;
    s.small_steps = n_small;
    s.evaluations = 4 * (long long)n_small;
    if ((rc = spec_sums(At, &s.energy_out, &s.photons_out))) return rc;
    GMM_HIP(Launch<T>::fft_rows(P->logn, -1, At, (cplx<T>*)Aout, (T)1, P->N, tw(), P->stream));
    GMM_HIP(hipStreamSynchronize(P->stream));
    if (P->prof.on) P->prof.collect();
    if (st) *st = s;
    return GMM_OK;
  }

  int nonlinear(const void* At, int count, void* out) {
    int rc = ensure_workspace(P, count);
    if (rc) return rc;
    if ((rc = ensure_gain_workspace(P, count))) return rc;
    P->prof.cur_iter = 0;
    rc = eval((const cplx<T>*)At, P->N, count, 0, 0.0, (cplx<T>*)out, nullptr);
    if (rc == GMM_OK && P->prof.on) {
      GMM_HIP(hipStreamSynchronize(P->stream));
      P->prof.collect();
    }
    return rc;
  }

  // Time the candidate launches of the contraction on the plan's own buffers
  // for `count` rows and keep the fastest (see gmm_plan_autotune).
  int autotune(int count, int* n_cand, double* us, int max_cand) {
    const std::vector<ContractCand> cands = contraction_candidates(P);
    if (cands.empty())
      return fail(GMM_ERR_UNSUPPORTED, "the autotuner covers the FP32 packed and rank-r routes and the BF16X3 "
                                       "rank-r route");
    int rc = ensure_workspace(P, count);
    if (rc) return rc;
    GMM_HIP(hipMemsetAsync(P->work, 0, (size_t)count * field_bytes(P), P->stream));
    GMM_HIP(hipMemsetAsync(P->Bp, 0, bp_bytes(P, P->cap), P->stream));
    hipEvent_t e0, e1;
    GMM_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(GMM_ERR_HIP, "hipEventCreate failed");
    }
    const bool prof_on = P->prof.on;
    P->prof.on = false;
    const EvalWs ws = plan_ws(P);
    int best = -1;
    double best_us = 0.0;
    for (size_t c = 0; c < cands.size() && rc == GMM_OK; ++c) {
      P->tune_kernel = cands[c].kernel;
      P->tune_bpc = cands[c].bpc;
      constexpr int kWarm = 2, kRuns = 5;
      for (int i = 0; i < kWarm && rc == GMM_OK; ++i) rc = mid(count, ws, nullptr, false, true);
      if (rc == GMM_OK && hipEventRecord(e0, P->stream) != hipSuccess) rc = fail(GMM_ERR_HIP, "hipEventRecord");
      for (int i = 0; i < kRuns && rc == GMM_OK; ++i) rc = mid(count, ws, nullptr, false, true);
      if (rc == GMM_OK && hipEventRecord(e1, P->stream) != hipSuccess) rc = fail(GMM_ERR_HIP, "hipEventRecord");
      float ms = 0.f;
      if (rc == GMM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(GMM_ERR_HIP, "event timing failed");
      const double t = 1e3 * ms / kRuns;
      if ((int)c < max_cand && us) us[c] = t;
      if (rc == GMM_OK && (best < 0 || t < best_us)) {
        best = (int)c;
        best_us = t;
      }
    }
    P->prof.on = prof_on;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    P->tune_kernel = cands[best].kernel;
    P->tune_bpc = cands[best].bpc;
    if (n_cand) *n_cand = (int)cands.size();
    return best;
  }

  // The same evaluation with its buffers carved from `base` (scratch_bytes
  // long): no allocation, no event, no synchronisation.
  int nonlinear_noalloc(const void* At, int count, void* out, void* base, size_t scratch_bytes) {
    const size_t need = noalloc_bytes(P, count);
    if (need > scratch_bytes)
      return fail(GMM_ERR_UNSUPPORTED, "gmm_nonlinear_noalloc: " + std::to_string(count) + " fields need " +
                                           std::to_string(need) + " bytes of scratch, more than its " +
                                           std::to_string(scratch_bytes));
    EvalWs w;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      void* q = (unsigned char*)base + off;
      off += (bytes + 255) & ~(size_t)255;
      return q;
    };
    w.cap = count;
    w.work = carve((size_t)count * field_bytes(P));
    w.Bp = carve(bp_bytes(P, count));
    w.plane_words = (size_t)count * gmm::kBf16Kpad * P->nt / 2;
    if (P->factored) w.Y = carve((size_t)count * P->rq * P->nt * P->esz);
    if (P->gain_on || P->coupling_on) {
      const size_t nn = (size_t)P->N * P->N;
      w.gpart = (cplx<double>*)carve((size_t)count * gmm::gain_partials(P->nt) * nn * sizeof(cplx<double>));
      w.Mg = (cplx<double>*)carve((size_t)count * nn * sizeof(cplx<double>));
      w.gain_cap = count;
    }
    // rows the contraction reads with zero coefficients must hold zeros, as in the plan's own workspace
    // (a fill kernel, not a memset node, so that the call can be captured in a graph)
    if (P->bf16 || P->factored || P->dense) GMM_HIP(gmm::launch_fill_zero(w.Bp, bp_bytes(P, count), P->stream));
    const bool prof_on = P->prof.on;  // no timing events here (creating one may allocate)
    P->prof.on = false;
    const int rc = eval((const cplx<T>*)At, P->N, count, 0, 0.0, (cplx<T>*)out, nullptr, 0, &w);
    P->prof.on = prof_on;
    return rc;
  }

  // Scratch bytes one no-allocation evaluation of `count` fields takes (each slice 256-byte aligned).
  static size_t noalloc_bytes(const gmm_plan_s* P, int count) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t b = up((size_t)count * field_bytes(P)) + up(bp_bytes(P, count));
    if (P->factored) b += up((size_t)count * P->rq * P->nt * P->esz);
    if (P->gain_on || P->coupling_on) {
      const size_t nn = (size_t)P->N * P->N;
      b += up((size_t)count * gmm::gain_partials(P->nt) * nn * sizeof(cplx<double>)) +
           up((size_t)count * nn * sizeof(cplx<double>));
    }
    return b;
  }
};

template <typename T>
int upload_typed(gmm_plan_s* P, const std::vector<double>& ST, const std::vector<std::complex<double>>& tw) {
  int rc;
  std::vector<T> st(ST.begin(), ST.end());
  if ((rc = dev_alloc(&P->const_bytes, (T**)&P->ST, st.size() * sizeof(T)))) return rc;
  GMM_HIP(hipMemcpy(P->ST, st.data(), st.size() * sizeof(T), hipMemcpyHostToDevice));
  std::vector<cplx<T>> t(tw.size());
  for (size_t i = 0; i < tw.size(); ++i) t[i] = cplx<T>{(T)tw[i].real(), (T)tw[i].imag()};
  if ((rc = dev_alloc(&P->const_bytes, (cplx<T>**)&P->tw, t.size() * sizeof(cplx<T>)))) return rc;
  GMM_HIP(hipMemcpy(P->tw, t.data(), t.size() * sizeof(cplx<T>), hipMemcpyHostToDevice));
  return GMM_OK;
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major,
// destroyed).  Eigenvalues on return in a[i*n+i]; eigenvectors are the columns of v.
void jacobi_eigen(int n, std::vector<double>& a, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  double total = 0.0;
  for (double x : a) total += x * x;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
    if (off <= 1e-32 * total) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) <= 1e-300) continue;
        const double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp - sn * vkq;
          v[(size_t)k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
}

// Host bf16 (round to nearest even) of a float.
// Cyclic Jacobi for a Hermitian n x n matrix a (row-major, overwritten).  Each
// rotation is the real Jacobi rotation of the phase-adjusted 2 x 2 block,
// J = [[c, s e^{i phi}], [-s e^{-i phi}, c]] on columns (p, q), a_pq = |a_pq| e^{i phi}:
// a <- J^H a J, v <- v J.  On return the diagonal of a holds the eigenvalues
// and the columns of v (multiplied from the right) the eigenvectors.
void hermitian_jacobi(int n, std::complex<double>* a, std::complex<double>* v) {
  using C = std::complex<double>;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) (p == q ? diag : off) += std::norm(a[p * n + q]);
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const C apq = a[p * n + q];
        const double b = std::abs(apq);
        if (b == 0.0) continue;
        const C ph = apq / b;
        const double app = a[p * n + p].real(), aqq = a[q * n + q].real();
        const double tau = (aqq - app) / (2.0 * b);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        const C sp = sn * ph, sm = sn * std::conj(ph);
        for (int k = 0; k < n; ++k) {
          const C akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - sm * akq;
          a[k * n + q] = sp * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const C apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - sp * aqk;
          a[q * n + k] = sm * apk + c * aqk;
        }
        a[p * n + q] = a[q * n + p] = 0.0;
        a[p * n + p] = app - t * b;
        a[q * n + q] = aqq + t * b;
        for (int k = 0; k < n; ++k) {
          const C vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - sm * vkq;
          v[k * n + q] = sp * vkp + c * vkq;
        }
      }
  }
}

// Eigen-decomposition of H(w_k) = diag(d(w_k)) + Q^T for every frequency bin
// (d_p = dispersion phase of mode p, Qc[n * N + p] = Q_np): lam [N][nt],
// U [N][N][nt] (U[(p N + q) nt + k] = component p of eigenvector q).  Bins are
// split over host threads; inside a chunk each bin starts from the previous
// bin's eigenvectors (B = V^H H V is then nearly diagonal).
void coupled_eigen(const gmm_plan_s* P, const std::vector<std::complex<double>>& Qc, std::vector<double>& lam,
                   std::vector<std::complex<double>>& U) {
  using C = std::complex<double>;
  const int N = P->N, nt = P->nt, nb = P->nb;
  lam.assign((size_t)N * nt, 0.0);
  U.assign((size_t)N * N * nt, C(0.0));
  auto work = [&](int k_begin, int k_end) {
    std::vector<C> H((size_t)N * N), B((size_t)N * N), T((size_t)N * N), V((size_t)N * N, C(0.0));
    for (int p = 0; p < N; ++p) V[(size_t)p * N + p] = 1.0;
    for (int k = k_begin; k < k_end; ++k) {
      const double w = (double)(k < nt / 2 ? k : k - nt) * P->domega;
      for (int p = 0; p < N; ++p)
        for (int n = 0; n < N; ++n) H[(size_t)p * N + n] = Qc[(size_t)n * N + p];
      for (int p = 0; p < N; ++p) {
        double acc = 0.0;
        for (int n = nb - 1; n >= 0; --n) acc = acc * w + P->coefh[(size_t)p * nb + n];
        H[(size_t)p * N + p] += acc;
      }
      // B = V^H H V
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          C acc = 0.0;
          for (int l = 0; l < N; ++l) acc += H[(size_t)i * N + l] * V[(size_t)l * N + j];
          T[(size_t)i * N + j] = acc;
        }
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          C acc = 0.0;
          for (int l = 0; l < N; ++l) acc += std::conj(V[(size_t)l * N + i]) * T[(size_t)l * N + j];
          B[(size_t)i * N + j] = acc;
        }
      for (int i = 0; i < N; ++i)  // exactly Hermitian before the rotations
        for (int j = i + 1; j < N; ++j) {
          const C m = 0.5 * (B[(size_t)i * N + j] + std::conj(B[(size_t)j * N + i]));
          B[(size_t)i * N + j] = m;
          B[(size_t)j * N + i] = std::conj(m);
        }
      hermitian_jacobi(N, B.data(), V.data());
      for (int q = 0; q < N; ++q) {
        lam[(size_t)q * nt + k] = B[(size_t)q * N + q].real();
        for (int p = 0; p < N; ++p) U[((size_t)p * N + q) * nt + k] = V[(size_t)p * N + q];
      }
    }
  };
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nth = std::max(1, std::min({hw, 16, nt / 64}));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t) pool.emplace_back(work, (int)((long)nt * t / nth), (int)((long)nt * (t + 1) / nth));
  for (auto& th : pool) th.join();
}

uint16_t host_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float host_bf16_value(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}
// A fixed operand in three bf16 planes: v = hi + lo + lo2 to about 2^-26 of v (two planes leave up to 2^-18,
// the same in every evaluation).
void host_bf16_split3(double v, uint16_t* h, uint16_t* l, uint16_t* l2) {
  *h = host_bf16((float)v);
  const double r1 = v - (double)host_bf16_value(*h);
  *l = host_bf16((float)r1);
  *l2 = host_bf16((float)(r1 - (double)host_bf16_value(*l)));
}

// hi/lo split of the packed coupling matrix, rows (p,l) with K = 128 contiguous.
int upload_bf16_split(gmm_plan_s* P, const std::vector<double>& ST) {
  const int K = gmm::kBf16Kpad;
  const size_t n = (size_t)P->rpad * K;
  std::vector<uint16_t> hi(n, 0), lo(2 * n, 0);  // lo: the lo plane, then the lo2 plane
  for (int r = 0; r < P->rpad; ++r)
    for (int k = 0; k < P->Np; ++k) {
      const size_t o = (size_t)r * K + k;
      host_bf16_split3(ST[(size_t)k * P->rpad + r], &hi[o], &lo[o], &lo[n + o]);
    }
  int rc;
  if ((rc = dev_alloc(&P->const_bytes, &P->Shi, hi.size() * 2)) || (rc = dev_alloc(&P->const_bytes, &P->Slo, lo.size() * 2)))
    return rc;
  GMM_HIP(hipMemcpy(P->Shi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice));
  GMM_HIP(hipMemcpy(P->Slo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice));
  return GMM_OK;
}

// Rank-r factor of the packed matrix: S^ = Sbar W with Sbar_{(pl),(mn)} = S_plmn
// symmetric and W = diag(w_mn); Sbar = Q L Q^T gives U = Q_r L_r, V = Q_r^T W.
// Used only when the Raman term is on, r <= min(64, Np/2), rt <= 2, and U V
// reproduces S^ to 1e-12 of its largest entry.
template <typename T>
int try_factor(gmm_plan_s* P, const double* SK, const std::vector<int2>& pairs, const std::vector<double>& ST) {
  const int Np = P->Np, N = P->N;
  if (!P->raman || P->rt > 2) return GMM_OK;
  auto S4 = [&](int a, int b, int c, int d) { return SK[(((size_t)a * N + b) * N + c) * N + d]; };
  std::vector<double> a((size_t)Np * Np), q;
  double smax = 0;
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      a[(size_t)i * Np + j] = S4(pairs[i].x, pairs[i].y, pairs[j].x, pairs[j].y);
      smax = std::max(smax, std::fabs(a[(size_t)i * Np + j]));
    }
  for (int i = 0; i < Np; ++i)  // the factor needs the (pl) <-> (mn) symmetry as well
    for (int j = i + 1; j < Np; ++j)
      if (std::fabs(a[(size_t)i * Np + j] - a[(size_t)j * Np + i]) > 1e-12 * smax) return GMM_OK;
  jacobi_eigen(Np, a, q);
  double lmax = 0;
  for (int i = 0; i < Np; ++i) lmax = std::max(lmax, std::fabs(a[(size_t)i * Np + i]));
  std::vector<int> keep;
  for (int i = 0; i < Np; ++i)
    if (std::fabs(a[(size_t)i * Np + i]) > 1e-12 * lmax) keep.push_back(i);
  const int r = (int)keep.size();
  if (r < 1 || r > 64 || 2 * r > Np) return GMM_OK;
  // U [Np][r], V [r][Np]; check U V against S^ (the transposed ST holds S^)
  std::vector<double> U((size_t)Np * r), V((size_t)r * Np);
  for (int rho = 0; rho < r; ++rho) {
    const int e = keep[rho];
    const double lam = a[(size_t)e * Np + e];
    for (int Q = 0; Q < Np; ++Q) {
      U[(size_t)Q * r + rho] = q[(size_t)Q * Np + e] * lam;
      V[(size_t)rho * Np + Q] = q[(size_t)Q * Np + e] * (pairs[Q].x == pairs[Q].y ? 1.0 : 2.0);
    }
  }
  double err = 0, ref = 0;
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      double x = 0;
      for (int rho = 0; rho < r; ++rho) x += U[(size_t)i * r + rho] * V[(size_t)rho * Np + j];
      const double sh = ST[(size_t)j * P->rpad + i];
      err = std::max(err, std::fabs(x - sh));
      ref = std::max(ref, std::fabs(sh));
    }
  if (!(err <= 1e-12 * ref)) return GMM_OK;
  const int rq = ((r + 15) / 16) * 16, kp = ((Np + 63) / 64) * 64;
  std::vector<T> vt((size_t)kp * rq, T(0)), ut((size_t)64 * P->rpad, T(0));
  for (int k = 0; k < Np; ++k)
    for (int rho = 0; rho < r; ++rho) vt[(size_t)k * rq + rho] = (T)V[(size_t)rho * Np + k];
  for (int rho = 0; rho < r; ++rho)
    for (int row = 0; row < Np; ++row) ut[(size_t)rho * P->rpad + row] = (T)U[(size_t)row * r + rho];
  int rc;
  if ((rc = dev_alloc(&P->const_bytes, &P->VT, vt.size() * sizeof(T))) ||
      (rc = dev_alloc(&P->const_bytes, &P->UT, ut.size() * sizeof(T))))
    return rc;
  GMM_HIP(hipMemcpy(P->VT, vt.data(), vt.size() * sizeof(T), hipMemcpyHostToDevice));
  GMM_HIP(hipMemcpy(P->UT, ut.data(), ut.size() * sizeof(T), hipMemcpyHostToDevice));
  if (P->bf16) {
    // fixed factors in three bf16 planes
    const auto split3 = host_bf16_split3;
    const size_t un = (size_t)P->rpad * 64;
    std::vector<uint16_t> hi(un, 0), lo(2 * un, 0);
    for (int row = 0; row < Np; ++row)
      for (int rho = 0; rho < r; ++rho) {
        const size_t o = (size_t)row * 64 + rho;
        split3(U[(size_t)row * r + rho], &hi[o], &lo[o], &lo[un + o]);
      }
    if ((rc = dev_alloc(&P->const_bytes, &P->Uhi, hi.size() * 2)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Ulo, lo.size() * 2)))
      return rc;
    GMM_HIP(hipMemcpy(P->Uhi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Ulo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice));
    const size_t vn = (size_t)rq * kp;
    std::vector<uint16_t> vh(vn, 0), vl(2 * vn, 0);
    for (int rho = 0; rho < r; ++rho)
      for (int Q = 0; Q < Np; ++Q) {
        const size_t o = (size_t)rho * kp + Q;
        split3(V[(size_t)rho * Np + Q], &vh[o], &vl[o], &vl[vn + o]);
      }
    if ((rc = dev_alloc(&P->const_bytes, &P->Vhi, vh.size() * 2)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Vlo, vl.size() * 2)))
      return rc;
    GMM_HIP(hipMemcpy(P->Vhi, vh.data(), vh.size() * 2, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Vlo, vl.data(), vl.size() * 2, hipMemcpyHostToDevice));
  }
  P->factored = true;
  P->rank = r;
  P->rq = rq;
  P->kp = kp;
  // default contraction launch (gmm_plan_autotune may pick another): BF16X3 the column-owner kernel on
  // 48-column tiles (M + 1 = 11 sub-steps of 2^14 samples fill two rounds of the persistent grid), FP32 the
  // row-register kernel at 3 blocks per CU (the fastest of the candidates on the 15-mode 2^14 workload)
  P->tune_kernel = 1;
  P->tune_bpc = P->bf16 ? 0 : (P->rt <= 2 ? 3 : 0);
  if (!P->bf16 && P->rt > 2) P->tune_kernel = 0;
  return GMM_OK;
}

// Wide rank-r route: S^ = U V from a pivoted Cholesky factorisation of the
// symmetric pair matrix a_ij = S_(pair i)(pair j).  For the overlap tensor of
// Eq. (2) a is the Gram matrix of the pair products F_m F_n, so it is positive
// semi-definite and its Cholesky factor L [Np][r] has the numerical rank r as
// column count.  U = L and V = L^T diag(w) (w = 1 for m = n, 2 otherwise) give
// U V = a diag(w) = S^.  Columns are added while the largest remaining
// diagonal exceeds 1e-13 of the largest initial one; the factor is kept only if
// U V reproduces S^ to 1e-12 of its largest entry (else GMM_ERR_TENSOR).
int factor_wide(gmm_plan_s* P, const double* SK, const std::vector<int2>& pairs) {
  const int Np = P->Np, N = P->N;
  auto S4 = [&](int a, int b, int c, int d) { return SK[(((size_t)a * N + b) * N + c) * N + d]; };
  std::vector<double> a((size_t)Np * Np);
  double smax = 0;
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      a[(size_t)i * Np + j] = S4(pairs[i].x, pairs[i].y, pairs[j].x, pairs[j].y);
      smax = std::max(smax, std::fabs(a[(size_t)i * Np + j]));
    }
  for (int i = 0; i < Np; ++i)
    for (int j = i + 1; j < Np; ++j)
      if (std::fabs(a[(size_t)i * Np + j] - a[(size_t)j * Np + i]) > 1e-12 * smax)
        return fail(GMM_ERR_TENSOR, "the wide rank-r route needs S_plmn = S_mnpl as well");
  std::vector<double> d(Np), L;  // L: column c at L[c * Np .. c * Np + Np)
  std::vector<char> used(Np, 0);
  double dmax0 = 0;
  for (int i = 0; i < Np; ++i) dmax0 = std::max(dmax0, d[i] = a[(size_t)i * Np + i]);
  int r = 0;
  while (r < Np) {
    int piv = -1;
    double best = 0;
    for (int i = 0; i < Np; ++i)
      if (!used[i] && d[i] > best) best = d[piv = i];
    if (piv < 0 || best <= 1e-13 * dmax0) break;
    used[piv] = 1;
    const double sq = std::sqrt(best);
    L.resize((size_t)(r + 1) * Np);
    double* col = &L[(size_t)r * Np];
    for (int i = 0; i < Np; ++i) {
      if (used[i]) {
        col[i] = i == piv ? sq : 0.0;
        continue;
      }
      double x = a[(size_t)i * Np + piv];
      for (int c = 0; c < r; ++c) x -= L[(size_t)c * Np + i] * L[(size_t)c * Np + piv];
      col[i] = x / sq;
      d[i] -= col[i] * col[i];
    }
    ++r;
  }
  if (r < 1 || r > 256) return fail(GMM_ERR_TENSOR, "the wide rank-r route found rank " + std::to_string(r) +
                                                      " (1..256 supported)");
  double err = 0, ref = 0;
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      double x = 0;
      for (int c = 0; c < r; ++c) x += L[(size_t)c * Np + i] * L[(size_t)c * Np + j];
      const double w = pairs[j].x == pairs[j].y ? 1.0 : 2.0;
      err = std::max(err, std::fabs(w * x - w * a[(size_t)i * Np + j]));
      ref = std::max(ref, std::fabs(w * a[(size_t)i * Np + j]));
    }
  if (!(err <= 1e-12 * ref))
    return fail(GMM_ERR_TENSOR, "the pair matrix is not positive semi-definite to rounding (wide rank-r route)");
  const int rq = ((r + 15) / 16) * 16;
  auto Uv = [&](int Q, int rho) { return L[(size_t)rho * Np + Q]; };
  auto Vv = [&](int rho, int Q) { return L[(size_t)rho * Np + Q] * (pairs[Q].x == pairs[Q].y ? 1.0 : 2.0); };
  int rc;
  if (P->bf16) {
    std::vector<uint16_t> wv((size_t)rq * 2 * Np, 0), wvl((size_t)rq * Np, 0), wu((size_t)Np * 2 * rq, 0),
        wul((size_t)Np * rq, 0);
    for (int rho = 0; rho < r; ++rho)
      for (int Q = 0; Q < Np; ++Q) {
        const float v = (float)Vv(rho, Q), u = (float)Uv(Q, rho);
        const uint16_t vh = host_bf16(v), uh = host_bf16(u);
        wv[(size_t)rho * 2 * Np + Q] = wv[(size_t)rho * 2 * Np + Np + Q] = vh;
        wvl[(size_t)rho * Np + Q] = host_bf16(v - host_bf16_value(vh));
        wu[(size_t)Q * 2 * rq + rho] = wu[(size_t)Q * 2 * rq + rq + rho] = uh;
        wul[(size_t)Q * rq + rho] = host_bf16(u - host_bf16_value(uh));
      }
    if ((rc = dev_alloc(&P->const_bytes, &P->Wv, wv.size() * 2)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Wv_lo, wvl.size() * 2)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Wu, wu.size() * 2)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Wu_lo, wul.size() * 2)))
      return rc;
    GMM_HIP(hipMemcpy(P->Wv, wv.data(), wv.size() * 2, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Wv_lo, wvl.data(), wvl.size() * 2, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Wu, wu.data(), wu.size() * 2, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Wu_lo, wul.data(), wul.size() * 2, hipMemcpyHostToDevice));
  } else {
    std::vector<float> wv((size_t)rq * Np, 0.f), wu((size_t)Np * rq, 0.f);
    for (int rho = 0; rho < r; ++rho)
      for (int Q = 0; Q < Np; ++Q) {
        wv[(size_t)rho * Np + Q] = (float)Vv(rho, Q);
        wu[(size_t)Q * rq + rho] = (float)Uv(Q, rho);
      }
    if ((rc = dev_alloc(&P->const_bytes, &P->Wv, wv.size() * 4)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Wu, wu.size() * 4)))
      return rc;
    GMM_HIP(hipMemcpy(P->Wv, wv.data(), wv.size() * 4, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Wu, wu.data(), wu.size() * 4, hipMemcpyHostToDevice));
  }
  if (gmm::wide_blas_create(&P->blas) != 0) return fail(GMM_ERR_HIP, "rocblas_create_handle failed");
  P->wide = true;
  P->factored = true;
  P->rank = r;
  P->rq = rq;
  P->kp = Np;
  return GMM_OK;
}

// Real coupling matrix of the general route, G [rows_pad][KD]: output rows
// 2 (p N + l) + {0: Re C_pl, 1: Im C_pl}; columns Q (x), Np + Q (y), and with
// Raman 2 Np + Q (xr), 3 Np + Q (yr), for the pairs Q = (m <= n):
//   C_pl += (K_plmn + K_plnm) x + i (K_plmn - K_plnm) y   (m < n),  K_plmm x  (m = n)
// with K = (1 - fR) S^K, and the same with R = fR S^R on (xr, yr).
template <typename T, typename FK, typename FR>
int upload_dense(gmm_plan_s* P, FK sk, FR sr) {
  const int N = P->N, Np = P->Np;
  const double fR = P->prm.fR;
  const int kreal = (P->raman ? 4 : 2) * Np;
  P->KD = (kreal + 3) / 4 * 4;
  P->rows_pad = (2 * N * N + 63) / 64 * 64;
  std::vector<T> g((size_t)P->rows_pad * P->KD, T(0));
  auto at = [&](int p, int l, int m, int n) { return (((size_t)p * N + l) * N + m) * N + n; };
  for (int p = 0; p < N; ++p)
    for (int l = 0; l < N; ++l) {
      const size_t ore = (size_t)2 * (p * N + l) * P->KD, oim = ore + P->KD;
      for (int Q = 0; Q < Np; ++Q) {
        int m = 0, n = 0;
        while ((n + 1) * (n + 2) / 2 <= Q) ++n;
        m = Q - n * (n + 1) / 2;
        for (int part = 0; part < (P->raman ? 2 : 1); ++part) {
          const double f = part == 0 ? 1.0 - fR : fR;
          const std::complex<double> a = f * (part == 0 ? sk(at(p, l, m, n)) : sr(at(p, l, m, n)));
          const std::complex<double> b = f * (part == 0 ? sk(at(p, l, n, m)) : sr(at(p, l, n, m)));
          const int cx = 2 * part * Np + Q, cy = cx + Np;
          if (m == n) {
            g[ore + cx] = (T)a.real();
            g[oim + cx] = (T)a.imag();
          } else {
            const std::complex<double> sum = a + b, dif = a - b;
            g[ore + cx] = (T)sum.real();
            g[oim + cx] = (T)sum.imag();
            g[ore + cy] = (T)(-dif.imag());
            g[oim + cy] = (T)dif.real();
          }
        }
      }
    }
  int rc;
  if ((rc = dev_alloc(&P->const_bytes, &P->G, g.size() * sizeof(T)))) return rc;
  GMM_HIP(hipMemcpy(P->G, g.data(), g.size() * sizeof(T), hipMemcpyHostToDevice));
  P->KD32 = (P->KD + 31) / 32 * 32;
  if (P->bf16) {  // hi/lo split of G for the BF16X3 product, K padded to 32 with zeros
    std::vector<uint16_t> hi((size_t)gmm::kDenseGRows * P->KD32, 0), lo((size_t)gmm::kDenseGRows * P->KD32, 0);
    for (int r = 0; r < std::min(P->rows_pad, gmm::kDenseGRows); ++r)
      for (int k = 0; k < P->KD; ++k) {
        const float x = (float)g[(size_t)r * P->KD + k];
        const uint16_t h = host_bf16(x);
        hi[(size_t)r * P->KD32 + k] = h;
        lo[(size_t)r * P->KD32 + k] = host_bf16(x - host_bf16_value(h));
      }
    if ((rc = dev_alloc(&P->const_bytes, &P->Ghi, hi.size() * 2)) ||
        (rc = dev_alloc(&P->const_bytes, &P->Glo, lo.size() * 2)))
      return rc;
    GMM_HIP(hipMemcpy(P->Ghi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice));
    GMM_HIP(hipMemcpy(P->Glo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice));
  }
  return GMM_OK;
}

template <typename T>
int build_raman(gmm_plan_s* P, const double* hR, double blend) {
  // weights h_R(k dt) normalised to unit sum; H = FFT_{+}(w); Hs = ((1 - blend) + blend H / H[0]) / Nt
  const int n = P->nt;
  double sum = 0.0;
  for (int k = 0; k < n; ++k) sum += hR[k];
  if (!(std::fabs(sum) > 0.0) || !std::isfinite(sum)) return fail(GMM_ERR_ARG, "h_R samples sum to zero or non-finite");
  std::vector<std::complex<double>> a(n);
  for (int k = 0; k < n; ++k) a[k] = hR[k] / sum;
  host_fft_plus(a);
  int rc;
  cplx<double>* dH = nullptr;
  if ((rc = dev_alloc(&P->const_bytes, &dH, n * sizeof(cplx<double>)))) return rc;
  std::vector<cplx<double>> h(n);
  for (int k = 0; k < n; ++k) h[k] = cplx<double>{a[k].real(), a[k].imag()};
  GMM_HIP(hipMemcpy(dH, h.data(), n * sizeof(cplx<double>), hipMemcpyHostToDevice));
  if ((rc = dev_alloc(&P->const_bytes, (cplx<T>**)&P->Hs, n * sizeof(cplx<T>)))) return rc;
  GMM_HIP(Launch<T>::finish_H(dH, (cplx<T>*)P->Hs, n, blend, P->stream));
  GMM_HIP(hipStreamSynchronize(P->stream));
  (void)hipFree(dH);
  P->const_bytes -= (long long)(n * sizeof(cplx<double>));
  return GMM_OK;
}

// Overlap-save filter of every route with Raman (the general route filters
// with h_R alone, blend = 1): the normalised weights w_k of h_R are cut after
// the first Lh samples once the absolute sum of everything beyond (the causal
// tail and the wrapped samples near Nt) is at most the precision's tail bound
// of their absolute sum.  Segments of F = 2^11 points then give V = F - Lh + 1
// outputs each.  Used for Nt >= 2^13 and Lh <= F / 2 (at least half of each
// segment is output); otherwise the plan keeps the full-row transforms.
template <typename T>
int build_overlap_save(gmm_plan_s* P, const double* hR, double blend) {
  // tail bound: far below the rounding of the field precision (FP64: below its unit roundoff, so the segmented
  // convolution equals the full-window one to rounding)
  const double tail_bound = sizeof(T) == 4 ? 1e-9 : 1e-17;
  constexpr int F = 1 << gmm::kOsLogF;
  const int n = P->nt;
  if (n < 8192) return GMM_OK;
  double sum = 0.0, asum = 0.0;
  for (int k = 0; k < n; ++k) sum += hR[k];
  for (int k = 0; k < n; ++k) asum += std::fabs(hR[k] / sum);
  int lh = n;
  double tail = 0.0;
  while (lh > 1 && tail + std::fabs(hR[lh - 1] / sum) <= tail_bound * asum) tail += std::fabs(hR[--lh] / sum);
  if (lh > F / 2) return GMM_OK;
  std::vector<std::complex<double>> g(F, 0.0);
  for (int k = 0; k < lh; ++k) g[k] = blend * hR[k] / sum;
  g[0] += 1.0 - blend;
  host_fft_plus(g);
  std::vector<cplx<T>> gf(F), tf(F);
  for (int k = 0; k < F; ++k) {
    gf[k] = cplx<T>{(T)(g[k].real() / F), (T)(g[k].imag() / F)};
    const std::complex<double> t = std::polar(1.0, -2.0 * kPi * (double)k / F);
    tf[k] = cplx<T>{(T)t.real(), (T)t.imag()};
  }
  int rc;
  if ((rc = dev_alloc(&P->const_bytes, &P->Gos, F * sizeof(cplx<T>))) ||
      (rc = dev_alloc(&P->const_bytes, &P->twos, F * sizeof(cplx<T>))))
    return rc;
  GMM_HIP(hipMemcpy(P->Gos, gf.data(), F * sizeof(cplx<T>), hipMemcpyHostToDevice));
  GMM_HIP(hipMemcpy(P->twos, tf.data(), F * sizeof(cplx<T>), hipMemcpyHostToDevice));
  P->os_lh = lh;
  P->os_v = F - lh + 1;
  return GMM_OK;
}

void destroy(gmm_plan_s* P) {
  if (!P) return;
  free_workspace(P);
  for (void* p : {(void*)P->coef, P->tw, P->Hs, P->ST, P->Shi, P->Slo, P->VT, P->UT, P->Uhi, P->Ulo, P->Vhi, P->Vlo,
                  P->G, P->Ghi, P->Glo, (void*)P->gvec, (void*)P->SRd, (void*)P->gpart, (void*)P->Mg, (void*)P->Kc,
                  P->Uc, (void*)P->lam, P->Gos, P->twos, P->Wv, P->Wv_lo, P->Wu, P->Wu_lo,
                  (void*)P->pidx,
                  (void*)P->pairs, (void*)P->ctrl})
    if (p) (void)hipFree(p);
  if (P->h_ctrl) (void)hipHostFree(P->h_ctrl);
  if (P->ev) (void)hipEventDestroy(P->ev);
  gmm::wide_blas_destroy(P->blas);
  if (P->h_partials) (void)hipHostFree(P->h_partials);
  delete P;
}

int create(gmm_plan* out, const gmm_params* p, const double* betas, const double* SK, const double* SR,
           const double* hR, void* stream) {
  if (!out || !p || !betas || !SK) return fail(GMM_ERR_ARG, "null argument");
  *out = nullptr;
  const int N = p->n_modes, nt = p->nt;
  if (N < 1) return fail(GMM_ERR_ARG, "n_modes must be >= 1");
  if (nt < 256 || (nt & (nt - 1))) return fail(GMM_ERR_ARG, "nt must be a power of two >= 256");
  int logn = 0;
  while ((1 << logn) < nt) ++logn;
  if (p->precision != GMM_FP64 && p->precision != GMM_FP32 && p->precision != GMM_BF16X3)
    return fail(GMM_ERR_ARG, "unknown precision");
  const bool fp64 = p->precision == GMM_FP64;
  const bool bf16 = p->precision == GMM_BF16X3;
  if (fp64 ? !Launch<double>::supports_logn(logn) : !Launch<float>::supports_logn(logn))
    return fail(GMM_ERR_UNSUPPORTED, "nt outside 2^8..2^15 (2^14 for FP64)");
  if (p->n_beta < 1) return fail(GMM_ERR_ARG, "n_beta must be >= 1");
  if (!(p->dt > 0) || !(p->omega0 > 0) || !(p->n2 >= 0) || !(p->fR >= 0 && p->fR <= 1))
    return fail(GMM_ERR_ARG, "dt, omega0 must be > 0; n2 >= 0; 0 <= fR <= 1");
  if (p->max_iter < 1 || p->fixed_iters < 0 || !(p->tol >= 0)) return fail(GMM_ERR_ARG, "bad iteration control");
  if (p->factor_policy < 0 || p->factor_policy > 3) return fail(GMM_ERR_ARG, "factor_policy must be 0..3");
  if (p->s_complex != 0 && p->s_complex != 1) return fail(GMM_ERR_ARG, "s_complex must be 0 or 1");
  const double domega = 2.0 * kPi / (nt * p->dt);
  if (p->self_steepening && !(p->omega0 - domega * (nt / 2) > 0))
    return fail(GMM_ERR_ARG, "1 + omega/omega0 <= 0 on the grid: window too fine for the shock term");
  const bool raman = p->fR > 0;
  if (raman && !hR) return fail(GMM_ERR_ARG, "hR required when fR > 0");
  const int Np = N * (N + 1) / 2;
  const int rpad = ((Np + 63) / 64) * 64;
  // the packed, rank-r and general routes hold up to 256 pair rows (22 modes; 15 in BF16X3); beyond, and with
  // factor_policy 3, the wide rank-r route (complex64 fields, up to 55 modes)
  const bool narrow_ok = rpad <= gmm::contract_max_rows() && !(bf16 && Np > gmm::kBf16Kpad);
  const bool want_wide = p->factor_policy == 3 || (p->factor_policy == 0 && !narrow_ok);
  if (!want_wide && rpad > gmm::contract_max_rows())
    return fail(GMM_ERR_UNSUPPORTED, "more than 22 modes: the packed and general routes exceed 256 pair rows");
  if (!want_wide && bf16 && Np > gmm::kBf16Kpad)
    return fail(GMM_ERR_UNSUPPORTED, "the BF16 split packed and general routes support up to 15 modes");
  if (want_wide && fp64)
    return fail(GMM_ERR_UNSUPPORTED, "more than 22 modes (or factor_policy 3) needs complex64 fields: the wide "
                                     "rank-r route runs GMM_FP32 and GMM_BF16X3");
  if (want_wide && N > gmm::wide_max_modes())
    return fail(GMM_ERR_UNSUPPORTED, "more than 55 modes");
  // tensors: real [N^4] or complex [N^4][2] (s_complex); S^R = S^K when SR is NULL
  const size_t n4 = (size_t)N * N * N * N;
  const bool cplxS = p->s_complex == 1;
  auto sk = [&](size_t i) { return cplxS ? std::complex<double>(SK[2 * i], SK[2 * i + 1]) : std::complex<double>(SK[i], 0.0); };
  auto sr = [&](size_t i) {
    if (!SR) return sk(i);
    return cplxS ? std::complex<double>(SR[2 * i], SR[2 * i + 1]) : std::complex<double>(SR[i], 0.0);
  };
  double smax = 0;
  bool has_imag = false;
  for (size_t i = 0; i < n4; ++i) {
    const std::complex<double> a = sk(i), b = sr(i);
    if (!std::isfinite(a.real()) || !std::isfinite(a.imag()) || !std::isfinite(b.real()) || !std::isfinite(b.imag()))
      return fail(GMM_ERR_ARG, "non-finite S^K or S^R");
    smax = std::max(smax, std::max(std::abs(a), std::abs(b)));
    has_imag = has_imag || a.imag() != 0.0 || b.imag() != 0.0;
  }
  const double stol = 1e-12 * smax;
  auto idx4 = [&](int a, int b, int c, int d) { return (((size_t)a * N + b) * N + c) * N + d; };
  // the packed and rank-r routes need a real S^K = S^R with S_plmn = S_plnm = S_lpmn
  bool packable = !has_imag;
  for (size_t i = 0; packable && i < n4; ++i)
    if (std::abs(sk(i) - sr(i)) > stol) packable = false;
  for (int a = 0; packable && a < N; ++a)
    for (int b = 0; packable && b < N; ++b)
      for (int c = 0; packable && c < N; ++c)
        for (int d = 0; d < N; ++d) {
          const double v = sk(idx4(a, b, c, d)).real();
          if (std::fabs(v - sk(idx4(a, b, d, c)).real()) > stol || std::fabs(v - sk(idx4(b, a, c, d)).real()) > stol) {
            packable = false;
            break;
          }
        }
  if ((p->factor_policy == 1 || want_wide) && !packable)
    return fail(GMM_ERR_TENSOR, want_wide ? "the wide rank-r route needs a real S^K = S^R with S_plmn = S_plnm = S_lpmn"
                                          : "the packed contraction needs a real S^K = S^R with S_plmn = S_plnm = S_lpmn");
  const bool dense = !want_wide && (p->factor_policy == 2 || !packable);
  std::vector<double> skr;  // real S^K for the packed routes
  if (!dense) {
    skr.resize(n4);
    for (size_t i = 0; i < n4; ++i) skr[i] = sk(i).real();
  }
  auto S4 = [&](int a, int b, int c, int d) { return skr[idx4(a, b, c, d)]; };

  gmm_plan_s* P = new gmm_plan_s();
  P->prm = *p;
  P->N = N;
  P->nt = nt;
  P->logn = logn;
  P->nb = p->n_beta;
  P->Np = Np;
  P->rpad = rpad;
  P->rt = rpad / 64;
  P->stream = (hipStream_t)stream;
  P->domega = domega;
  P->gamma_hat = p->n2 * p->omega0 / kC;
  P->fp64 = fp64;
  P->bf16 = bf16;
  P->raman = raman;
  P->esz = fp64 ? 8 : 4;
  P->dense = dense;
  P->SRh.resize(n4);
  for (size_t i = 0; i < n4; ++i) P->SRh[i] = sr(i);

  int rc = GMM_OK;
  auto bail = [&](int code) {
    destroy(P);
    return code;
  };
  if (hipGetDevice(&P->device) != hipSuccess) return bail(fail(GMM_ERR_HIP, "hipGetDevice failed"));
  // dispersion coefficients beta_n / n!
  std::vector<double> coef((size_t)N * P->nb);
  for (int q = 0; q < N; ++q) {
    double fact = 1.0;
    for (int n = 0; n < P->nb; ++n) {
      if (n > 0) fact *= n;
      const double b = betas[(size_t)q * P->nb + n];
      if (!std::isfinite(b)) return bail(fail(GMM_ERR_ARG, "non-finite beta"));
      coef[(size_t)q * P->nb + n] = b / fact;
    }
  }
  P->coefh = coef;
  if ((rc = dev_alloc(&P->const_bytes, &P->coef, coef.size() * sizeof(double)))) return bail(rc);
  if (hipMemcpy(P->coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(GMM_ERR_HIP, "copy of dispersion coefficients failed"));
  // mode pairs (m <= n) in triangular order Q = n (n + 1) / 2 + m, and the pair index table
  std::vector<int2> pairs;
  std::vector<int> pidx((size_t)N * N);
  for (int n = 0; n < N; ++n)
    for (int m = 0; m <= n; ++m) {
      pidx[(size_t)m * N + n] = pidx[(size_t)n * N + m] = (int)pairs.size();
      pairs.push_back(make_int2(m, n));
    }
  // packed coupling matrix  S^_{(p,l),(m,n)} = w_mn S_plmn, w = 1 (m = n) or 2; stored transposed
  std::vector<double> ST((size_t)rpad * rpad, 0.0);
  if (!dense)
    for (int r = 0; r < Np; ++r)
      for (int q = 0; q < Np; ++q) {
        const int2 pl = pairs[r], mn = pairs[q];
        const double w = mn.x == mn.y ? 1.0 : 2.0;
        ST[(size_t)q * rpad + r] = w * S4(pl.x, pl.y, mn.x, mn.y);
      }
  // twiddles exp(-2 pi i m / nt)
  std::vector<std::complex<double>> tw(nt);
  for (int m = 0; m < nt; ++m) tw[m] = std::polar(1.0, -2.0 * kPi * (double)m / nt);
  if ((rc = dev_alloc(&P->const_bytes, &P->pidx, pidx.size() * sizeof(int)))) return bail(rc);
  if ((rc = dev_alloc(&P->const_bytes, &P->pairs, pairs.size() * sizeof(int2)))) return bail(rc);
  if (hipMemcpy(P->pidx, pidx.data(), pidx.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(GMM_ERR_HIP, "copy of pair tables failed"));
  rc = fp64 ? upload_typed<double>(P, ST, tw) : upload_typed<float>(P, ST, tw);
  if (rc) return bail(rc);
  if (dense) {
    rc = fp64 ? upload_dense<double>(P, sk, sr) : upload_dense<float>(P, sk, sr);
    if (rc) return bail(rc);
  } else if (bf16 && !want_wide && (rc = upload_bf16_split(P, ST))) {
    return bail(rc);
  }
  if (raman) {  // the general route convolves with H itself; the packed routes with the blend (1 - fR) + fR H
    const double blend = dense ? 1.0 : p->fR;
    rc = fp64 ? build_raman<double>(P, hR, blend) : build_raman<float>(P, hR, blend);
    if (rc) return bail(rc);
    if (!dense && !want_wide && p->factor_policy == 0) {
      rc = fp64 ? try_factor<double>(P, skr.data(), pairs, ST) : try_factor<float>(P, skr.data(), pairs, ST);
      if (rc) return bail(rc);
    }
    if (!(fp64 && dense) &&  // the general route's segmented rows exist for complex64 fields only
        (rc = fp64 ? build_overlap_save<double>(P, hR, blend) : build_overlap_save<float>(P, hR, blend)))
      return bail(rc);
  }
  if (want_wide && (rc = factor_wide(P, skr.data(), pairs))) return bail(rc);
  if (hipEventCreateWithFlags(&P->ev, hipEventDisableTiming) != hipSuccess)
    return bail(fail(GMM_ERR_HIP, "hipEventCreate failed"));
  if ((rc = dev_alloc(&P->const_bytes, &P->ctrl, sizeof(Ctrl)))) return bail(rc);
  if (hipHostMalloc((void**)&P->h_ctrl, sizeof(Ctrl), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&P->h_partials, 2 * sizeof(double) * gmm::trapz_blocks((long)N * nt),
                    hipHostMallocDefault) != hipSuccess)
    return bail(fail(GMM_ERR_NOMEM, "pinned host allocation failed"));
  if (hipHostGetDevicePointer((void**)&P->h_ctrl_dev, P->h_ctrl, 0) != hipSuccess)
    return bail(fail(GMM_ERR_HIP, "hipHostGetDevicePointer of the control block failed"));
  *out = P;
  g_last_error.clear();
  return GMM_OK;
}

// ---------------------------------------------------------------------------
// Batched propagations of one plan (continuous batching): S slots, each an
// independent propagation with its own field, length and step, advance in
// rounds.  A round queues one MPA iteration for every running slot: the
// sub-step rows of all of them go through one launch per kernel kind (their
// field rows packed into one work buffer), then the trapezoid and the norm run
// per slot, and the host reads all control blocks back once.  A slot whose
// large step converged is closed at the start of the next round and starts its
// next large step there; a slot that reached its length gets its final
// transform and frees up, and a new propagation can be admitted into it while
// the others keep running.  Per slot the kernels compute exactly what
// gmm_propagate computes, in the same order.
struct BatchSlotState {
  int state = 0;  // 0 free, 1 running, 2 final transform queued
  long n_small = 0, done = 0;
  double dz = 0.0, E_dz = std::nan("");
  int m = 0;
  bool first = true, need_close = false;
  void* Aout = nullptr;
  long long tag = 0;
  gmm_stats st{};
  int status = GMM_OK;
};

}  // namespace

struct gmm_batch_s {
  gmm_plan_s* P = nullptr;
  int S = 0, M = 0, nblk = 0;
  void *psi0 = nullptr, *I0 = nullptr, *psi = nullptr, *E = nullptr, *work = nullptr, *Bp = nullptr, *Y = nullptr;
  void* E64 = nullptr;         // single-precision fields: [S][N][Nt] exp(D_w M dz) per slot in FP64
  double* partials = nullptr;  // [S][nblk][2]
  double* spec = nullptr;      // [S][2][nblk][2]: spectral sums at admission (0) and at the end (1)
  gmm::Ctrl* ctrl = nullptr;   // [S]
  gmm::BatchRow* rows_d = nullptr;    // [S (M + 1)]
  gmm::BatchSlot* slots_d = nullptr;  // [2 S]: iterating slots, then closing slots
  gmm::BatchRow* rows_h = nullptr;    // pinned mirrors
  gmm::BatchSlot* slots_h = nullptr;
  gmm::Ctrl* ctrl_h = nullptr;        // mapped: the norm kernel stores each slot's control block here
  gmm::Ctrl* ctrl_h_dev = nullptr;    // its device-visible address
  double* spec_h = nullptr;
  std::vector<BatchSlotState> slot;
  std::vector<int> round;       // slots iterating in the queued round
  bool pending = false, spec_dirty = false;
  long long bytes = 0;
};

namespace {

void batch_free(gmm_batch_s* B) {
  if (!B) return;
  for (void* p : {B->psi0, B->I0, B->psi, B->E, B->E64, B->work, B->Bp, B->Y, (void*)B->partials, (void*)B->spec,
                  (void*)B->ctrl, (void*)B->rows_d, (void*)B->slots_d})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)B->rows_h, (void*)B->slots_h, (void*)B->ctrl_h, (void*)B->spec_h})
    if (p) (void)hipHostFree(p);
  delete B;
}

template <typename T>
struct BatchRunner {
  gmm_batch_s* B;
  gmm_plan_s* P;
  size_t nn() const { return (size_t)P->N * P->nt; }
  cplx<T>* at(void* base, size_t row) const { return (cplx<T>*)base + row * nn(); }
  cplx<double>* last_factor(int s) const { return (cplx<double>*)B->E64 + (size_t)s * nn(); }
  const cplx<T>* tw() const { return (const cplx<T>*)P->tw; }

  int spec_sums_into(int s, int which) {
    double* dst = B->spec + ((size_t)s * 2 + which) * 2 * B->nblk;
    GMM_HIP(Launch<T>::spec_sums(at(B->psi0, s), P->nt, (long)nn(), P->domega, P->prm.omega0, dst, P->stream));
    B->spec_dirty = true;
    return GMM_OK;
  }
  void spec_read(int s, int which, double* energy, double* photons) const {
    const double* h = B->spec_h + ((size_t)s * 2 + which) * 2 * B->nblk;
    double a = 0, b = 0;
    for (int i = 0; i < B->nblk; ++i) {
      a += h[2 * i];
      b += h[2 * i + 1];
    }
    *energy = a * P->nt * P->prm.dt;
    *photons = b;
  }

  int submit(const void* A0, double L, double dz_req, void* Aout, long long tag) {
    int s = -1;
    for (int i = 0; i < B->S; ++i)
      if (B->slot[i].state == 0) {
        s = i;
        break;
      }
    if (s < 0) return fail(GMM_ERR_BUSY, "no free slot in the batch");
    const double r = L / dz_req;
    long n_small = (std::fabs(r - std::round(r)) < 1e-9 * std::max(1.0, r)) ? (long)std::llround(r)
                                                                            : (long)std::ceil(r);
    if (n_small < 1) n_small = 1;
    BatchSlotState& q = B->slot[s];
    const double dz = L / (double)n_small;
    GMM_HIP(Launch<T>::fft_rows(P->logn, +1, (const cplx<T>*)A0, at(B->psi0, s), (T)(1.0 / P->nt), P->N, tw(),
                                P->stream));
    int rc = spec_sums_into(s, 0);
    if (rc) return rc;
    if (!(q.E_dz == dz)) {
      GMM_HIP(Launch<T>::phase_table(at(B->E, (size_t)s * (B->M + 1)), P->coef, P->nb, P->N, P->nt, B->M + 1, dz,
                                     P->domega, P->stream));
      if (B->E64 != nullptr)
        GMM_HIP(Launch<double>::phase_table(last_factor(s), P->coef, P->nb, P->N, P->nt, 1, dz, P->domega, P->stream,
                                            B->M));
      q.E_dz = dz;
    }
    GMM_HIP(gmm::launch_ctrl_reset(B->ctrl + s, P->stream));
    q.state = 1;
    q.n_small = n_small;
    q.done = 0;
    q.dz = dz;
    q.m = (int)std::min<long>(B->M, n_small);
    q.first = true;
    q.need_close = false;
    q.Aout = Aout;
    q.tag = tag;
    q.st = gmm_stats{};
    q.st.dz_used = dz;
    q.status = GMM_OK;
    return s;
  }

  int launch() {
    const size_t n = nn();
    const int S = B->S, M = B->M;
    // 1. close the slots whose large step converged in the last round
    int nclose = 0;
    std::vector<int> closing;
    for (int s = 0; s < S; ++s) {
      BatchSlotState& q = B->slot[s];
      if (q.state != 1 || !q.need_close) continue;
      gmm::BatchSlot& d = B->slots_h[S + nclose++];
      d = gmm::BatchSlot{};
      d.psi = at(B->psi, (size_t)s * M);
      d.dst = at(B->psi0, s);
      d.Em = nullptr;  // lab-frame iterates: the last one is the field at the step's end
      d.ctrl = B->ctrl + s;
      d.m = q.m;
      closing.push_back(s);
    }
    // 2. rows of the slots that iterate in this round
    B->round.clear();
    int R = 0, ns = 0;
    for (int s = 0; s < S; ++s) {
      BatchSlotState& q = B->slot[s];
      if (q.state != 1) continue;
      if (q.need_close) {  // the close below finishes this large step
        q.done += q.m;
        q.st.large_steps++;
        q.st.small_steps += q.m;
        q.need_close = false;
        if (q.done >= q.n_small) {
          q.state = 2;  // final transform queued after the close
          continue;
        }
        q.first = true;
        q.m = (int)std::min<long>(M, q.n_small - q.done);
      }
      const int o = R;
      if (q.first)
        for (int j = 0; j <= q.m; ++j) B->rows_h[R++] = gmm::BatchRow{s, -1, j, 0};
      else
        for (int j = 1; j <= q.m; ++j) B->rows_h[R++] = gmm::BatchRow{s, j - 1, j, 0};
      gmm::BatchSlot& d = B->slots_h[ns++];
      d = gmm::BatchSlot{};
      d.psi0 = at(B->psi0, s);
      d.I0 = q.first ? (const void*)at(B->work, o) : (const void*)at(B->I0, s);
      d.I = at(B->work, q.first ? o + 1 : o);
      d.psi = at(B->psi, (size_t)s * M);
      d.I0_keep = at(B->I0, s);
      d.E = at(B->E, (size_t)s * (M + 1));
      d.Em64 = B->E64 != nullptr && q.m == M ? last_factor(s) : nullptr;
      d.partials = B->partials + (size_t)s * 2 * B->nblk;
      d.ctrl = B->ctrl + s;
      d.ctrl_host = B->ctrl_h_dev + s;
      d.dz = q.dz;
      d.first = q.first ? 1 : 0;
      d.m = q.m;
      B->round.push_back(s);
    }
    if (R > 0) GMM_HIP(hipMemcpyAsync(B->rows_d, B->rows_h, (size_t)R * sizeof(gmm::BatchRow),
                                      hipMemcpyHostToDevice, P->stream));
    if (ns + nclose > 0)
      GMM_HIP(hipMemcpyAsync(B->slots_d, B->slots_h, (size_t)2 * S * sizeof(gmm::BatchSlot), hipMemcpyHostToDevice,
                             P->stream));
    GMM_HIP(Launch<T>::close_b(B->slots_d + S, nclose, (long)n, P->stream));
    for (int s : closing) {  // slots at their length: spectral sums and the transform back to time
      BatchSlotState& q = B->slot[s];
      if (q.state != 2) continue;
      int rc = spec_sums_into(s, 1);
      if (rc) return rc;
      GMM_HIP(Launch<T>::fft_rows(P->logn, -1, at(B->psi0, s), (cplx<T>*)q.Aout, (T)1, P->N, tw(), P->stream));
    }
    if (R > 0) {
      EvalWs ws;
      ws.work = B->work;
      ws.Bp = B->Bp;
      ws.Y = B->Y;
      ws.cap = S * (M + 1);
      ws.plane_words = (size_t)ws.cap * gmm::kBf16Kpad * P->nt / 2;
      cplx<T>* W = (cplx<T>*)B->work;
      GMM_HIP(Launch<T>::phase_to_time_b(P->logn, B->rows_d, (const cplx<T>*)B->psi0, (const cplx<T>*)B->psi,
                                         (const cplx<T>*)B->E, W, P->N, R, M, tw(), 1, P->stream));
      const bool prof_on = P->prof.on;  // per-kernel events are for gmm_propagate
      P->prof.on = false;
      const int rc = Runner<T>{P}.mid(R, ws, nullptr, true, true);
      P->prof.on = prof_on;
      if (rc) return rc;
      GMM_HIP(Launch<T>::spectral_out_b(P->logn, B->rows_d, W, (const cplx<T>*)B->E, P->N, R, M, P->domega,
                                        P->gamma_hat / P->nt, 1.0 / P->prm.omega0, P->prm.self_steepening, tw(), 1,
                                        P->stream));
      GMM_HIP(Launch<T>::trapz_b(B->slots_d, ns, (long)n, P->stream));
      GMM_HIP(gmm::launch_norm_final_b(B->slots_d, ns, B->nblk, P->prm.tol, P->prm.fixed_iters, P->prm.max_iter,
                                       P->stream));
    }
    if (B->spec_dirty) {
      GMM_HIP(hipMemcpyAsync(B->spec_h, B->spec, (size_t)S * 4 * B->nblk * sizeof(double), hipMemcpyDeviceToHost,
                             P->stream));
      B->spec_dirty = false;
    }
    B->pending = true;
    return GMM_OK;
  }

  int wait(long long* tags, int* status, gmm_stats* stats, int max_done, int* n_done) {
    *n_done = 0;
    if (!B->pending) return GMM_OK;
    GMM_HIP(hipStreamSynchronize(P->stream));
    B->pending = false;
    for (int s : B->round) {
      BatchSlotState& q = B->slot[s];
      const gmm::Ctrl c = B->ctrl_h[s];
      if (c.status == 2) {  // non-finite relative change: report and free the slot
        q.status = GMM_ERR_DIVERGED;
        q.state = 2;
        q.st.last_eps = c.eps;
        continue;
      }
      if (c.done) {
        if (c.status == 1) {
          q.st.nonconverged_steps++;
          q.status = GMM_NOT_CONVERGED;
        }
        q.st.iterations += c.iters;
        q.st.evaluations += 1 + (long long)c.iters * q.m;
        if (c.iters > q.st.max_iters_seen) q.st.max_iters_seen = c.iters;
        q.st.last_eps = c.eps;
        q.need_close = true;
      } else {
        q.first = false;
      }
    }
    // report the slots whose final transform has run (or that failed), and free them
    for (int s = 0; s < B->S; ++s) {
      BatchSlotState& q = B->slot[s];
      if (q.state != 2) continue;
      const bool in_round = std::find(B->round.begin(), B->round.end(), s) != B->round.end();
      if (in_round && q.status != GMM_ERR_DIVERGED) continue;  // finished transform is queued next round
      if (*n_done >= max_done) break;
      if (q.status != GMM_ERR_DIVERGED) {
        spec_read(s, 0, &q.st.energy_in, &q.st.photons_in);
        spec_read(s, 1, &q.st.energy_out, &q.st.photons_out);
      }
      tags[*n_done] = q.tag;
      if (status) status[*n_done] = q.status;
      if (stats) stats[*n_done] = q.st;
      ++*n_done;
      q.state = 0;
    }
    int running = 0;
    for (const auto& q : B->slot) running += q.state != 0;
    return running;
  }
};

int batch_create(gmm_batch* out, gmm_plan_s* P, int slots, int M) {
  if (P->gain_on || P->coupling_on || P->cpl_exact)
    return fail(GMM_ERR_UNSUPPORTED, "batched propagation without the gain and coupling terms only");
  gmm_batch_s* B = new gmm_batch_s();
  B->P = P;
  B->S = slots;
  B->M = M;
  const size_t nn = (size_t)P->N * P->nt, fb = field_bytes(P);
  B->nblk = gmm::trapz_blocks((long)nn);
  const int cap = slots * (M + 1);
  long long* c = &B->bytes;
  int rc;
  auto bail = [&](int code) {
    batch_free(B);
    return code;
  };
  if ((rc = dev_alloc(c, &B->psi0, fb * slots)) || (rc = dev_alloc(c, &B->I0, fb * slots)) ||
      (rc = dev_alloc(c, &B->psi, fb * slots * M)) || (rc = dev_alloc(c, &B->E, fb * slots * (M + 1))) ||
      (P->esz == 4 && (rc = dev_alloc(c, &B->E64, nn * sizeof(gmm::cplx<double>) * slots))) ||
      (rc = dev_alloc(c, &B->work, fb * cap)) || (rc = dev_alloc(c, &B->Bp, bp_bytes(P, cap))) ||
      (P->factored && (rc = dev_alloc(c, &B->Y, (size_t)cap * P->rq * P->nt * P->esz))) ||
      (rc = dev_alloc(c, &B->partials, (size_t)slots * 2 * B->nblk * sizeof(double))) ||
      (rc = dev_alloc(c, &B->spec, (size_t)slots * 4 * B->nblk * sizeof(double))) ||
      (rc = dev_alloc(c, &B->ctrl, (size_t)slots * sizeof(gmm::Ctrl))) ||
      (rc = dev_alloc(c, &B->rows_d, (size_t)cap * sizeof(gmm::BatchRow))) ||
      (rc = dev_alloc(c, &B->slots_d, (size_t)2 * slots * sizeof(gmm::BatchSlot))))
    return bail(rc);
  if (hipMemset(B->Bp, 0, bp_bytes(P, cap)) != hipSuccess ||
      hipMemset(B->ctrl, 0, (size_t)slots * sizeof(gmm::Ctrl)) != hipSuccess)
    return bail(fail(GMM_ERR_HIP, "hipMemset of the batch buffers failed"));
  if (hipHostMalloc((void**)&B->rows_h, (size_t)cap * sizeof(gmm::BatchRow), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&B->slots_h, (size_t)2 * slots * sizeof(gmm::BatchSlot), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&B->ctrl_h, (size_t)slots * sizeof(gmm::Ctrl),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&B->spec_h, (size_t)slots * 4 * B->nblk * sizeof(double), hipHostMallocDefault) !=
          hipSuccess)
    return bail(fail(GMM_ERR_NOMEM, "pinned host allocation failed"));
  if (hipHostGetDevicePointer((void**)&B->ctrl_h_dev, B->ctrl_h, 0) != hipSuccess)
    return bail(fail(GMM_ERR_HIP, "hipHostGetDevicePointer of the control blocks failed"));
  B->slot.assign(slots, BatchSlotState{});
  *out = B;
  return GMM_OK;
}

// Static device scratch of gmm_nonlinear_noalloc: one copy per GPU, held
// until the process ends.  In host code `scratch` names a host-side stand-in,
// never the device memory: host code uses only the address that
// hipGetSymbolAddress returns for the current device (scratch_address below).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on GPU `dev`, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GMM_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    int cur = -1;
    GMM_HIP(hipGetDevice(&cur));
    if (cur != dev) GMM_HIP(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || ptr == nullptr)
      return fail(GMM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GMM_OK;
}

}  // namespace

extern "C" {

int gmm_plan_create(gmm_plan* out, const gmm_params* p, const double* betas, const double* SK, const double* SR,
                    const double* hR, void* stream) {
  try {
    return create(out, p, betas, SK, SR, hR, stream);
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_propagate(gmm_plan plan, const void* A0, double L, double dz, int M, void* Aout, gmm_stats* st) {
  if (!plan || !A0 || !Aout) return fail(GMM_ERR_ARG, "null argument");
  if (!(L > 0) || !(dz > 0) || !std::isfinite(L) || !std::isfinite(dz)) return fail(GMM_ERR_ARG, "L and dz must be > 0");
  if (M < 1) return fail(GMM_ERR_ARG, "M must be >= 1");
  if (L / dz > 1e12) return fail(GMM_ERR_ARG, "too many small steps");
  try {
    int rc = plan->fp64 ? Runner<double>{plan}.propagate(A0, L, dz, M, Aout, st)
                        : Runner<float>{plan}.propagate(A0, L, dz, M, Aout, st);
    if (rc >= 0) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_propagate_rk4ip(gmm_plan plan, const void* A0, double L, double dz, void* Aout, gmm_stats* st) {
  if (!plan || !A0 || !Aout) return fail(GMM_ERR_ARG, "null argument");
  if (!(L > 0) || !(dz > 0) || !std::isfinite(L) || !std::isfinite(dz)) return fail(GMM_ERR_ARG, "L and dz must be > 0");
  if (L / dz > 1e12) return fail(GMM_ERR_ARG, "too many small steps");
  try {
    int rc = plan->fp64 ? Runner<double>{plan}.propagate_rk4ip(A0, L, dz, Aout, st)
                        : Runner<float>{plan}.propagate_rk4ip(A0, L, dz, Aout, st);
    if (rc >= 0) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_plan_set_gain(gmm_plan plan, const double* g, double I_sat) {
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  if (!g) {
    plan->gain_on = false;
    return GMM_OK;
  }
  if (!(I_sat > 0)) return fail(GMM_ERR_ARG, "I_sat must be > 0 (infinity: no saturation)");
  if (plan->cpl_exact)
    return fail(GMM_ERR_UNSUPPORTED, "the gain term with the coupling in the linear operator is not implemented");
  if (plan->N > gmm::kGainNmax) return fail(GMM_ERR_UNSUPPORTED, "the gain term supports up to 22 modes");
  for (int p = 0; p < plan->N; ++p)
    if (!std::isfinite(g[p])) return fail(GMM_ERR_ARG, "non-finite gain coefficient");
  const size_t n4 = plan->SRh.size();
  if (!plan->gvec && (dev_alloc(&plan->const_bytes, &plan->gvec, plan->N * sizeof(double)) ||
                      dev_alloc(&plan->const_bytes, &plan->SRd, n4 * sizeof(cplx<double>))))
    return GMM_ERR_NOMEM;
  std::vector<cplx<double>> sr(n4);
  for (size_t i = 0; i < n4; ++i) sr[i] = cplx<double>{plan->SRh[i].real(), plan->SRh[i].imag()};
  if (hipMemcpy(plan->gvec, g, plan->N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(plan->SRd, sr.data(), n4 * sizeof(cplx<double>), hipMemcpyHostToDevice) != hipSuccess)
    return fail(GMM_ERR_HIP, "copy of the gain constants failed");
  plan->inv_Isat = std::isinf(I_sat) ? 0.0 : 1.0 / I_sat;
  plan->gain_on = true;
  g_last_error.clear();
  return GMM_OK;
}

int gmm_plan_set_coupling(gmm_plan plan, const double* Q, int q_complex) {
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  if (!Q) {
    plan->coupling_on = false;
    return GMM_OK;
  }
  if (q_complex != 0 && q_complex != 1) return fail(GMM_ERR_ARG, "q_complex must be 0 or 1");
  const int N = plan->N;
  if (N > gmm::kGainNmax) return fail(GMM_ERR_UNSUPPORTED, "linear coupling supports up to 22 modes");
  std::vector<cplx<double>> K((size_t)N * N);
  for (int n = 0; n < N; ++n)
    for (int p = 0; p < N; ++p) {
      const size_t i = (size_t)n * N + p;  // Q_np: coefficient of A_n in the equation of mode p
      const double re = q_complex ? Q[2 * i] : Q[i], im = q_complex ? Q[2 * i + 1] : 0.0;
      if (!std::isfinite(re) || !std::isfinite(im)) return fail(GMM_ERR_ARG, "non-finite coupling coefficient");
      K[(size_t)p * N + n] = cplx<double>{-im, re};  // K_pn = i Q_np
    }
  if (!plan->Kc && dev_alloc(&plan->const_bytes, &plan->Kc, K.size() * sizeof(cplx<double>))) return GMM_ERR_NOMEM;
  if (hipMemcpy(plan->Kc, K.data(), K.size() * sizeof(cplx<double>), hipMemcpyHostToDevice) != hipSuccess)
    return fail(GMM_ERR_HIP, "copy of the coupling matrix failed");
  if (plan->cpl_exact) {  // one placement of the coupling at a time
    plan->cpl_exact = false;
    plan->E_dz = std::nan("");
  }
  plan->coupling_on = true;
  g_last_error.clear();
  return GMM_OK;
}

int gmm_plan_set_coupling_exact(gmm_plan plan, const double* Q, int q_complex) {
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  if (!Q) {
    if (plan->cpl_exact) {
      plan->cpl_exact = false;
      plan->E_dz = std::nan("");
    }
    return GMM_OK;
  }
  if (q_complex != 0 && q_complex != 1) return fail(GMM_ERR_ARG, "q_complex must be 0 or 1");
  const int N = plan->N;
  if (N > gmm::kGainNmax) return fail(GMM_ERR_UNSUPPORTED, "linear coupling supports up to 22 modes");
  if (plan->gain_on)
    return fail(GMM_ERR_UNSUPPORTED, "the gain term with the coupling in the linear operator is not implemented");
  try {
    std::vector<std::complex<double>> Qc((size_t)N * N);
    double qmax = 0.0;
    for (size_t i = 0; i < Qc.size(); ++i) {
      const double re = q_complex ? Q[2 * i] : Q[i], im = q_complex ? Q[2 * i + 1] : 0.0;
      if (!std::isfinite(re) || !std::isfinite(im)) return fail(GMM_ERR_ARG, "non-finite coupling coefficient");
      Qc[i] = {re, im};
      qmax = std::max(qmax, std::abs(Qc[i]));
    }
    for (int n = 0; n < N; ++n)
      for (int p = 0; p < N; ++p)
        if (std::abs(Qc[(size_t)n * N + p] - std::conj(Qc[(size_t)p * N + n])) > 1e-12 * qmax)
          return fail(GMM_ERR_ARG, "the coupling in the linear operator needs a Hermitian Q (Q_np = conj(Q_pn))");
    std::vector<double> lam;
    std::vector<std::complex<double>> U;
    coupled_eigen(plan, Qc, lam, U);
    const size_t nU = (size_t)N * N * plan->nt;
    if (!plan->Uc && (dev_alloc(&plan->const_bytes, &plan->Uc, nU * 2 * plan->esz) ||
                      dev_alloc(&plan->const_bytes, &plan->lam, lam.size() * sizeof(double))))
      return GMM_ERR_NOMEM;
    hipError_t e;
    if (plan->fp64) {
      std::vector<cplx<double>> u(nU);
      for (size_t i = 0; i < nU; ++i) u[i] = {U[i].real(), U[i].imag()};
      e = hipMemcpy(plan->Uc, u.data(), nU * sizeof(cplx<double>), hipMemcpyHostToDevice);
    } else {
      std::vector<cplx<float>> u(nU);
      for (size_t i = 0; i < nU; ++i) u[i] = {(float)U[i].real(), (float)U[i].imag()};
      e = hipMemcpy(plan->Uc, u.data(), nU * sizeof(cplx<float>), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess || hipMemcpy(plan->lam, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice) !=
                               hipSuccess)
      return fail(GMM_ERR_HIP, "copy of the coupled-operator eigenvectors failed");
  } catch (const std::bad_alloc&) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
  plan->coupling_on = false;  // one placement of the coupling at a time
  plan->cpl_exact = true;
  plan->E_dz = std::nan("");
  g_last_error.clear();
  return GMM_OK;
}

int gmm_nonlinear(gmm_plan plan, const void* At, int count, void* out) {
  if (!plan || !At || !out) return fail(GMM_ERR_ARG, "null argument");
  if (count < 1) return fail(GMM_ERR_ARG, "count must be >= 1");
  if (At == out) return fail(GMM_ERR_ARG, "out must not alias At");
  return plan->fp64 ? Runner<double>{plan}.nonlinear(At, count, out) : Runner<float>{plan}.nonlinear(At, count, out);
}

int gmm_nonlinear_noalloc(gmm_plan plan, const void* At, int count, void* out) {
  if (!plan || !At || !out) return fail(GMM_ERR_ARG, "null argument");
  if (count < 1) return fail(GMM_ERR_ARG, "count must be >= 1");
  if (At == out) return fail(GMM_ERR_ARG, "out must not alias At");
  try {
    void* base = nullptr;
    int rc = scratch_address(plan->device, &base);
    if (rc) return rc;
    rc = plan->fp64 ? Runner<double>{plan}.nonlinear_noalloc(At, count, out, base, kScratchBytes)
                    : Runner<float>{plan}.nonlinear_noalloc(At, count, out, base, kScratchBytes);
    if (rc == GMM_OK) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_plan_autotune(gmm_plan plan, int count, int* n_candidates, double* us, int max_candidates) {
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  if (count < 1 || count > 4096) return fail(GMM_ERR_ARG, "count must be 1..4096");
  try {
    const int rc = plan->fp64 ? Runner<double>{plan}.autotune(count, n_candidates, us, max_candidates)
                              : Runner<float>{plan}.autotune(count, n_candidates, us, max_candidates);
    if (rc >= 0) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_plan_set_contraction(gmm_plan plan, int candidate) {
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  const std::vector<ContractCand> c = contraction_candidates(plan);
  if (candidate < 0 || candidate >= (int)c.size()) return fail(GMM_ERR_ARG, "no such contraction candidate");
  plan->tune_kernel = c[candidate].kernel;
  plan->tune_bpc = c[candidate].bpc;
  return GMM_OK;
}

int gmm_batch_create(gmm_batch* out, gmm_plan plan, int slots, int M) {
  if (!out) return fail(GMM_ERR_ARG, "null argument");
  *out = nullptr;
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  if (slots < 1 || slots > 4096) return fail(GMM_ERR_ARG, "slots must be 1..4096");
  if (M < 1 || M > 1024) return fail(GMM_ERR_ARG, "M must be 1..1024");
  try {
    const int rc = batch_create(out, plan, slots, M);
    if (rc == GMM_OK) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_batch_submit(gmm_batch b, const void* A0, double L, double dz, void* Aout, long long tag) {
  if (!b || !A0 || !Aout) return fail(GMM_ERR_ARG, "null argument");
  if (!(L > 0) || !(dz > 0) || !std::isfinite(L) || !std::isfinite(dz)) return fail(GMM_ERR_ARG, "L and dz must be > 0");
  if (L / dz > 1e12) return fail(GMM_ERR_ARG, "too many small steps");
  gmm_plan_s* P = b->P;
  if (P->gain_on || P->coupling_on || P->cpl_exact)
    return fail(GMM_ERR_UNSUPPORTED, "batched propagation without the gain and coupling terms only");
  try {
    const int rc = P->fp64 ? BatchRunner<double>{b, P}.submit(A0, L, dz, Aout, tag)
                           : BatchRunner<float>{b, P}.submit(A0, L, dz, Aout, tag);
    if (rc >= 0) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_batch_launch(gmm_batch b) {
  if (!b) return fail(GMM_ERR_ARG, "null batch");
  if (b->pending) return fail(GMM_ERR_ARG, "a round is already queued: call gmm_batch_wait first");
  gmm_plan_s* P = b->P;
  if (P->gain_on || P->coupling_on || P->cpl_exact)
    return fail(GMM_ERR_UNSUPPORTED, "batched propagation without the gain and coupling terms only");
  try {
    const int rc = P->fp64 ? BatchRunner<double>{b, P}.launch() : BatchRunner<float>{b, P}.launch();
    if (rc == GMM_OK) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_batch_wait(gmm_batch b, long long* tags, int* status, gmm_stats* stats, int max_done, int* n_done) {
  if (!b || !n_done || (max_done > 0 && !tags)) return fail(GMM_ERR_ARG, "null argument");
  if (max_done < b->S) return fail(GMM_ERR_ARG, "max_done must be at least the slot count");
  try {
    const int rc = b->P->fp64 ? BatchRunner<double>{b, b->P}.wait(tags, status, stats, max_done, n_done)
                              : BatchRunner<float>{b, b->P}.wait(tags, status, stats, max_done, n_done);
    if (rc >= 0) g_last_error.clear();
    return rc;
  } catch (...) {
    return fail(GMM_ERR_NOMEM, "host allocation failed");
  }
}

int gmm_batch_destroy(gmm_batch b) {
  if (b && b->pending) (void)hipStreamSynchronize(b->P->stream);
  batch_free(b);
  return GMM_OK;
}

long long gmm_batch_device_bytes(gmm_batch b) { return b ? b->bytes : 0; }

int gmm_plan_destroy(gmm_plan plan) {
  destroy(plan);
  return GMM_OK;
}

const char* gmm_last_error(void) { return g_last_error.c_str(); }

long long gmm_plan_device_bytes(gmm_plan plan) { return plan ? plan->const_bytes + plan->ws_bytes : 0; }

int gmm_plan_rank(gmm_plan plan) { return plan && plan->factored ? plan->rank : 0; }

int gmm_profile_enable(gmm_plan plan, int kinds) {
  if (!plan) return fail(GMM_ERR_ARG, "null plan");
  plan->prof.mask = (unsigned)kinds & ((1u << GMM_PROF_KINDS) - 1u);
  plan->prof.on = plan->prof.mask != 0;
  plan->prof.reset();
  return GMM_OK;
}

int gmm_profile_read(gmm_plan plan, double* total_ms, long long* launches, int n_kinds) {
  if (!plan || !total_ms || !launches || n_kinds < 1) return fail(GMM_ERR_ARG, "bad profile_read arguments");
  for (int k = 0; k < n_kinds; ++k) {
    total_ms[k] = k < GMM_PROF_KINDS ? plan->prof.ms[k] : 0.0;
    launches[k] = k < GMM_PROF_KINDS ? plan->prof.n[k] : 0;
  }
  return GMM_OK;
}

}  // extern "C"
