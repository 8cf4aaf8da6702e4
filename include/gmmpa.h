/*
 * gmmpa.h - C ABI of the MI355X (gfx950) massively parallel GMMNLSE propagator.
 *
 * The library integrates the generalized multimode nonlinear Schroedinger
 * equation, Eq. (1) of Wright et al., "Multimode Nonlinear Fiber Optics:
 * Massively Parallel Numerical Solver, Tutorial and Outlook", with the
 * massively parallel algorithm (MPA) of its Sec. III.D: change of variables
 * Eq. (cov), integral form Eq. (MPA_eq), M small steps dz per large step
 * L = M dz, integrands evaluated in parallel, trapezoid rule, fixed-point
 * iteration until the relative change falls below a threshold.
 *
 * Conventions (all SI units):
 *   t_k = (k - Nt/2) dt;  omega_k = 2 pi fftfreq(Nt, dt)[k];
 *   a field is A(t) = sum_k A~(omega_k) exp(-i omega_k t), i.e. d/dt <-> -i omega;
 *   D_omega = i (db0 + db1 omega + sum_{n>=2} beta_n omega^n / n!)   (Sec. III.D);
 *   self-steepening factor (1 + omega/omega0)                      (Eq. (MPA_eq));
 *   Raman convolution: circular over the window with weights h_R(k dt),
 *   normalised to unit sum (zero-frequency gain 1).
 *
 * Fields cross the boundary as device buffers of interleaved complex numbers,
 * mode-major: element (p, k) at index p*Nt + k.  The element type is complex
 * double for GMM_FP64 plans and complex float for GMM_FP32 and GMM_BF16X3 plans.
 *
 * Return codes: 0 success; GMM_NOT_CONVERGED (+1) the propagation completed
 * but at least one large step stopped at max_iter without reaching tol (the
 * output is valid, the statistics say which); negative values are errors and
 * leave the output unspecified.  No call throws; gmm_last_error() gives a
 * message for the last failure on the calling thread.
 */
#ifndef GMMPA_H
#define GMMPA_H

#ifdef __cplusplus
extern "C" {
#endif

#define GMM_OK 0
#define GMM_NOT_CONVERGED 1
#define GMM_ERR_ARG (-1)         /* invalid argument (size, step, grid, null pointer) */
#define GMM_ERR_NOMEM (-2)       /* device allocation failed */
#define GMM_ERR_TENSOR (-3)      /* coupling tensor lacks the symmetry the packed path needs */
#define GMM_ERR_HIP (-4)         /* a HIP runtime call failed */
#define GMM_ERR_UNSUPPORTED (-5) /* valid input outside what the library implements */
#define GMM_ERR_DIVERGED (-6)    /* the iteration produced non-finite values */
#define GMM_ERR_BUSY (-7)        /* a batch has no free slot */

typedef struct gmm_plan_s* gmm_plan;
typedef struct gmm_batch_s* gmm_batch;

typedef enum {
  GMM_FP64 = 0,   /* complex128 fields, FP64 transforms, FP64 MFMA contraction */
  GMM_FP32 = 1,   /* complex64 fields, FP32 transforms, FP32 MFMA contraction */
  GMM_BF16X3 = 2  /* complex64 fields, FP32 transforms; contraction as S^hi B^hi + S^hi B^lo + S^lo B^hi
                     with bf16 hi/lo splits on MFMA, FP32 accumulation (packed, rank-r and general routes up
                     to 15 modes; the wide rank-r route up to 55).  On the packed and rank-r routes the
                     fixed matrices (S^, or its factors U and V) carry a third plane lo2 and a fourth
                     product S^lo2 B^hi, so that no fixed rounding of the coupling repeats in every
                     evaluation.  Single-precision plans keep
                     the phase factor that ends each large step in FP64. */
} gmm_precision;
/* With Raman and Nt >= 2^13, the Raman convolution drops the samples of h_R
 * beyond the first Lh <= 1024 once their absolute sum is at most 1e-9 (GMM_FP32,
 * GMM_BF16X3) or 1e-17 (GMM_FP64) of the whole, and then runs on 2^11-point
 * overlap-save segments; otherwise it convolves over the full window. */

typedef struct {
  int n_modes;          /* N >= 1 spatial modes */
  int nt;               /* Nt time samples: a power of two, 2^8..2^15 (2^14 max for GMM_FP64) */
  int n_beta;           /* columns of betas, >= 1 */
  double dt;            /* time step (s) */
  double omega0;        /* carrier angular frequency (rad/s) */
  double n2;            /* nonlinear index (m^2/W) */
  double fR;            /* Raman fraction, 0 <= fR <= 1 */
  int self_steepening;  /* 1: keep (1 + (i/omega0) d/dt); 0: replace it by 1 */
  int precision;        /* gmm_precision */
  double tol;           /* threshold on ||psi^(n+1) - psi^(n)|| / ||psi^(n+1)|| (FP64).  The error a stopped
                           iteration leaves keeps its sign from one large step to the next, so it adds up
                           along the fibre: over 1 m of the 15-mode GRIN workload (11 000 large steps) the
                           field is within 9.6e-4 of FP64 at tol 1e-5, 1.5e-4 at 1e-6 and 2.5e-5 at 1e-7
                           (FP32 and GMM_BF16X3 alike) */
  int max_iter;         /* iteration cap per large step (>= 1) */
  int fixed_iters;      /* > 0: run exactly this many iterations per large step, ignore tol */
  int factor_policy;    /* contraction route.  0 (auto): a real S^K = S^R with S_plmn = S_plnm = S_lpmn
                           uses the packed matrix S^ (Np = N(N+1)/2 real rows), and, when the Raman term
                           is on and S^ has numerical rank r <= min(64, Np/2), its factor S^ = U V so
                           only r rows are convolved (same result to rounding); any other tensor uses
                           the general route.  1: the packed matrix S^ itself (GMM_ERR_TENSOR if the
                           tensor does not allow it).  2: the general route for any tensor: complex
                           C_pl from 2 N^2 x 4 Np real coefficients (S^K != S^R, complex S, polarised
                           modes), NL_p = sum_l C_pl A_l.  These three hold up to 256 pair rows (22
                           modes; 15 in GMM_BF16X3).  3, and 0 beyond those limits: the wide rank-r
                           route, N <= 55, complex64 fields only (GMM_FP32, GMM_BF16X3): S^ = U V from
                           a pivoted Cholesky factor of the pair matrix, which must be positive
                           semi-definite to rounding (the overlap tensor of Eq. (2) is: it is a Gram
                           matrix), else GMM_ERR_TENSOR; both products run as library GEMMs
                           (rocBLAS), the pair products and the fold as kernels */
  int s_complex;        /* 0: SK and SR hold N^4 real values; 1: N^4 complex values, interleaved
                           (re, im) doubles */
} gmm_params;

typedef struct {
  int large_steps;       /* large steps taken */
  int small_steps;       /* small steps dz covered (sum of M per large step) */
  long long iterations;  /* total iterations over all large steps */
  long long evaluations; /* nonlinear-operator evaluations (sub-step integrands) */
  int max_iters_seen;    /* largest iteration count of one large step */
  int nonconverged_steps;/* large steps that stopped at max_iter */
  double last_eps;       /* relative change of the last iteration of the last large step */
  double dz_used;        /* small step actually used (L is covered exactly) */
  double energy_in, energy_out;   /* sum_p int |A_p|^2 dt at z = 0 and z = L (J), FP64 */
  double photons_in, photons_out; /* sum_{p,k} |A~_p(w_k)|^2 / (w0 + w_k), FP64 (arbitrary units) */
} gmm_stats;

/*
 * gmm_plan_create - validate and copy the inputs of Eq. (1), precompute what
 * does not change along the fibre, and bind a HIP stream.
 *   out    : receives the plan (owned by the caller until gmm_plan_destroy).
 *   p      : parameters (copied).
 *   betas  : host [N][n_beta] Taylor coefficients about omega0 (rad/m, s/m,
 *            s^2/m, ...); columns 0 and 1 relative to the first mode
 *            (paragraph after Eq. (1)).  Copied.
 *   SK     : host [N^4] coupling tensor S^K_plmn of Eq. (1), index
 *            ((p*N+l)*N+m)*N+n, in m^-2 (Eq. (2) for real scalar modes); real,
 *            or complex when p->s_complex = 1 ([N^4][2] doubles).  Any tensor is
 *            accepted; factor_policy says which contraction route it takes.
 *            Copied.
 *   SR     : host Raman tensor S^R_plmn in the same layout, or NULL for
 *            S^R = S^K (Eq. (2) with real scalar modes).  Copied.
 *   hR     : host [Nt] samples h_R(k dt), k = 0..Nt-1 (1/s); required when
 *            fR > 0, ignored otherwise.  Copied.
 *   stream : hipStream_t on which all work of this plan is queued (NULL =
 *            the null stream).  Borrowed, not owned.
 * Allocates device memory for the constants; workspace is allocated by the
 * first propagate and grown as needed.
 */
int gmm_plan_create(gmm_plan* out, const gmm_params* p, const double* betas, const double* SK,
                    const double* SR, const double* hR, void* stream);

/*
 * gmm_propagate - propagate A0 over a fibre of length L with the MPA.
 *   A0   : device [N][Nt] field at z = 0, time domain, sqrt(W).  Read only.
 *   L    : fibre length (m) > 0.
 *   dz   : requested small step (m) > 0; the step used is L/n with
 *          n = round(L/dz) when L/dz is an integer to 1e-9, else ceil(L/dz).
 *   M    : small steps per large step (>= 1); a last, shorter large step takes
 *          the remaining n mod M small steps.
 *   Aout : device [N][Nt] field at z = L (may alias A0).
 *   st   : statistics (may be NULL).
 * Work is queued on the plan's stream; the call returns after the result is
 * complete (it reads the per-step convergence flag from the device).
 * One propagate at a time per plan.
 */
int gmm_propagate(gmm_plan plan, const void* A0, double L, double dz, int M, void* Aout, gmm_stats* st);

/*
 * gmm_propagate_rk4ip - serial baseline of Sec. III.D: propagate A0 over L
 * with 4th-order Runge-Kutta in the interaction picture (Hult, J. Lightwave
 * Technol. 25, 2007), the kind of serial integrator the MPA is compared with
 * in Fig. 3.  Each step of h evaluates the nonlinear operator four times in
 * sequence (no sub-step parallelism).  Same plan, arguments and step rule as
 * gmm_propagate (no M); st->evaluations = 4 n, st->iterations = 0.
 * Returns after the result is complete.
 */
int gmm_propagate_rk4ip(gmm_plan plan, const void* A0, double L, double dz, void* Aout, gmm_stats* st);

/*
 * gmm_plan_set_gain - turn on the saturating-gain term of Sec. III.F,
 *   G_p = g_p [A_p - sum_lmn S^R_plmn A_l int A_m A_n^* dtau / I_sat],
 * which every later propagate (MPA and RK4IP) and gmm_nonlinear add to the
 * right-hand side beside the nonlinear term (without its factor
 * i (n2 w0/c)(1 + (i/w0) d/dt)).  S^R is the plan's Raman tensor (S^K when it
 * was created with SR = NULL).
 *   g     : host [N] small-signal field gain per mode (1/m), copied; NULL turns
 *           the term off.
 *   I_sat : saturation fluence (J/m^2) > 0; INFINITY for unsaturated gain.
 * Returns GMM_ERR_ARG for bad values, GMM_ERR_UNSUPPORTED above 22 modes.
 */
int gmm_plan_set_gain(gmm_plan plan, const double* g, double I_sat);

/*
 * gmm_plan_set_coupling - turn on linear mode coupling (Sec. III.F), the term
 *   C_p = i sum_n Q_np A_n
 * with a z-independent coupling matrix, added like the gain term beside the
 * nonlinear term (the MPA then needs L = M dz << 1/|Q| to converge quickly).
 *   Q         : host [N][N] coupling coefficients (1/m), Q[n*N + p] = Q_np;
 *               real, or complex when q_complex = 1 ([N][N][2] doubles).
 *               Copied.  NULL turns the term off.
 * Returns GMM_ERR_ARG for bad values, GMM_ERR_UNSUPPORTED above 22 modes.
 * Turns off the form of gmm_plan_set_coupling_exact (one placement at a time).
 */
int gmm_plan_set_coupling(gmm_plan plan, const double* Q, int q_complex);

/*
 * gmm_plan_set_coupling_exact - the same coupling term (Sec. III.F) placed in
 * the linear operator instead of the integrand: per frequency
 *   L(w) = diag(D_w) + i Q^T  = i H(w),  H = diag(d(w)) + Q^T Hermitian,
 * and the change of variables of Sec. III.D (Eq. (cov), Eq. (MPA_eq)) uses
 * exp(L(w) z) = U(w) exp(i lam(w) z) U(w)^H.  The coupling is then exact for any
 * step; only the nonlinear term stays in the integrand.  The plan computes the
 * eigen-decomposition of H at every frequency bin (FP64, host threads) and
 * keeps U (field precision, N^2 Nt complex) and lam (FP64) on the device;
 * gmm_propagate iterates in the eigenbasis (two per-frequency mode mixings per
 * evaluation, one at each end of the propagation).
 *   Q         : as for gmm_plan_set_coupling; must be Hermitian,
 *               Q_np = conj(Q_pn) to 1e-12 of its largest entry (real: symmetric).
 *               Copied.  NULL turns the term off.
 * Returns GMM_ERR_ARG for bad values or a non-Hermitian Q, GMM_ERR_UNSUPPORTED
 * above 22 modes or with the gain term on.  gmm_propagate_rk4ip returns
 * GMM_ERR_UNSUPPORTED while it is on; gmm_nonlinear is unaffected (it has no
 * linear part).  Turns off the form of gmm_plan_set_coupling.
 */
int gmm_plan_set_coupling_exact(gmm_plan plan, const double* Q, int q_complex);

/*
 * gmm_nonlinear - the integrand factor of Eq. (MPA_eq) for `count` fields:
 *   out_c(w) = i (n2 w0/c) (1 + s w/w0) F{ sum_lmn [(1-fR) S_plmn A_l A_m A_n^*
 *                                            + fR S_plmn A_l (h_R * A_m A_n^*)] }
 *   At   : device [count][N][Nt] spectra A~ (FFT order).  Read only.
 *   out  : device [count][N][Nt] (must not alias At).
 * Queued on the plan's stream; returns without synchronising.
 */
int gmm_nonlinear(gmm_plan plan, const void* At, int count, void* out);

/*
 * gmm_nonlinear_noalloc - gmm_nonlinear for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, kernels and result as gmm_nonlinear
 * (bit for bit), but the workspace of the evaluation comes from a static
 * device array of GMM_NOALLOC_SCRATCH_BYTES that the library holds on each GPU
 * it runs on until the process ends; the call itself allocates nothing,
 * creates no event and does not synchronise (queued on the plan's stream).
 * The plan's constants must exist (gmm_plan_create allocates them).
 * Workspace bytes for `count` fields (each of the parts rounded up to 256):
 *   field rows        count N Nt c          (c = 16 for GMM_FP64, 8 otherwise)
 *   pair rows         GMM_BF16X3 packed and rank-r routes: 512 count Nt;
 *                     packed route: count Np Nt e; rank-r route: count max(Np, RQ) Nt e;
 *                     general route: count KD Nt e
 *                     (e = 8 for GMM_FP64, 4 otherwise; Np = N(N+1)/2; KD = 4 Np with
 *                     Raman, 2 Np without, rounded up to 4)
 *   rank-r route      count RQ Nt e         (RQ = rank rounded up to 16)
 *   gain or coupling  count N^2 (C + 1) 16  (C = min(64, Nt/128))
 * The 15-mode 2^14-sample BF16X3 plan takes about 13 MB per field, so up to 4
 * fields a call.
 * Returns GMM_ERR_UNSUPPORTED when count fields need more than the scratch
 * (nothing is queued then).  Every call on one GPU shares that GPU's scratch
 * and leaves its contents behind: calls that overlap on one GPU (different
 * streams or host threads) race and must be ordered by the caller.
 */
#define GMM_NOALLOC_SCRATCH_BYTES (64LL << 20)
int gmm_nonlinear_noalloc(gmm_plan plan, const void* At, int count, void* out);

/*
 * gmm_plan_autotune - choose the launch of the contraction (a4 + a5 of the
 * iteration, the MFMA product and the mode projection) for this plan by
 * timing the candidates on the plan's own buffers, `count` sub-step rows per
 * launch (M + 1 for gmm_propagate, slots (M + 1) for a batch); the fastest is
 * kept for every later call on the plan (propagate, batches, gmm_nonlinear).
 *   FP32 rank-r route: column-owner kernel on 64-column tiles at 1 or 2
 *   blocks per CU, the row-register kernel at 1 to 4 blocks per CU, or the
 *   column-owner kernel on 48-column tiles at 1 or 2 blocks per CU (the two
 *   kernels sum in a different order, so their results differ by rounding);
 *   FP32 packed route: the row-register kernel at 1 to 4 blocks per CU;
 *   BF16X3 rank-r route: the column-owner kernel on 64- or 48-column tiles at
 *   1 or 2 blocks per CU.
 * Until then a plan uses, on the rank-r route, the 48-column column-owner
 * kernel in BF16X3 and the row-register kernel at 3 blocks per CU in FP32.
 * Other routes: GMM_ERR_UNSUPPORTED.  Allocates the plan's workspace for
 * `count` rows, overwrites it and synchronises the plan's stream.
 *   n_candidates : receives the number of candidates (may be NULL).
 *   us           : receives the mean microseconds per launch of candidate i,
 *                  for i < max_candidates (may be NULL).
 * Returns the index of the chosen candidate (>= 0) or an error.
 */
int gmm_plan_autotune(gmm_plan plan, int count, int* n_candidates, double* us, int max_candidates);

/* Use contraction candidate `candidate` (numbered as by gmm_plan_autotune,
 * e.g. a tuning result kept from an earlier run) for every later call on the
 * plan.  GMM_ERR_ARG if the plan's route has no such candidate. */
int gmm_plan_set_contraction(gmm_plan plan, int candidate);

/*
 * Batched propagations of one plan with continuous admission: the MPA of
 * Sec. III.D for up to `slots` independent propagations at once, each with its
 * own launch field, length and step (same plan: modes, tensors, grid,
 * precision, M).  Work advances in rounds: a round is one MPA iteration of
 * every running propagation, queued as one launch per kernel kind over the
 * sub-step rows of all of them; then the trapezoid rule and the FP64
 * convergence norm per propagation, and one read-back of all stop flags.  A
 * propagation whose large step converged closes it and starts the next in the
 * following round; one that reached its length is transformed back, reported
 * and its slot freed, and gmm_batch_submit can admit a new one there while the
 * others run.  Per propagation the result, statistics and iteration counts are
 * bit for bit those of gmm_propagate on the same plan.  The plan must outlive
 * the batch and have the gain and coupling terms off (GMM_ERR_UNSUPPORTED).
 *
 * gmm_batch_create  - allocate the device buffers of `slots` propagations with
 *                     M small steps per large step (all queued on the plan's
 *                     stream).
 * gmm_batch_submit  - admit one propagation into a free slot: A0 device [N][Nt]
 *                     (read before the call's queued work ends: keep it alive
 *                     until the next gmm_batch_wait), length L, requested step
 *                     dz (same rule as gmm_propagate), Aout device [N][Nt]
 *                     written when it completes, `tag` returned with it.
 *                     Returns the slot index (>= 0), or GMM_ERR_BUSY when every
 *                     slot is taken.  Allowed while a round is queued.
 * gmm_batch_launch  - queue one round (no host wait).  GMM_ERR_ARG if a round
 *                     is queued and not yet waited for.
 * gmm_batch_wait    - wait for the queued round (nothing to do if none) and
 *                     report the propagations that completed in it: their tags,
 *                     return codes (GMM_OK, GMM_NOT_CONVERGED, GMM_ERR_DIVERGED)
 *                     and statistics into tags / status / stats (status and stats
 *                     may be NULL; arrays of max_done >= slots entries);
 *                     *n_done is their count.  Returns the number of
 *                     propagations still in the batch (0: idle), or an error.
 * gmm_batch_destroy - release the batch (waits for a queued round).
 * gmm_batch_device_bytes - device bytes the batch holds.
 */
int gmm_batch_create(gmm_batch* out, gmm_plan plan, int slots, int M);
int gmm_batch_submit(gmm_batch b, const void* A0, double L, double dz, void* Aout, long long tag);
int gmm_batch_launch(gmm_batch b);
int gmm_batch_wait(gmm_batch b, long long* tags, int* status, gmm_stats* stats, int max_done, int* n_done);
int gmm_batch_destroy(gmm_batch b);
long long gmm_batch_device_bytes(gmm_batch b);

/* Release every device buffer of the plan.  NULL is accepted. */
int gmm_plan_destroy(gmm_plan plan);

/* Message describing the last error on the calling thread ("" if none). */
const char* gmm_last_error(void);

/* Device bytes currently held by the plan (constants + workspace). */
long long gmm_plan_device_bytes(gmm_plan plan);

/* Rank r of the factor S^ = U V the plan contracts through (the rank-r route:
 * factor_policy 0, Raman on, r small enough; the wide rank-r route), or 0 when
 * it uses the packed matrix itself or the general route. */
int gmm_plan_rank(gmm_plan plan);

/*
 * Per-kernel timing with HIP events on the plan's stream (for benchmarks).
 * gmm_profile_enable(plan, kinds) clears the totals and brackets every later
 * launch of the kernel kinds whose bit (1 << GMM_PROF_*) is set in `kinds`
 * with two events (0 turns timing off; GMM_PROF_ALL times every kind).
 * Launches of queued iterations that exit at once (the large step had
 * already converged) are not counted.
 * gmm_profile_read copies, for the first n_kinds kernel kinds below, the
 * summed duration in ms and the number of counted launches.
 */
#define GMM_PROF_PHASE 0    /* phase factors + inverse transform (sub-step fields) */
#define GMM_PROF_PAIRS 1    /* pair products + Raman convolution (rank-r route: convolution of Y) */
#define GMM_PROF_CONTRACT 2 /* coupling contraction (MFMA) + mode projection */
#define GMM_PROF_SPECTRAL 3 /* forward transform + shock + back-phase */
#define GMM_PROF_TRAPZ 4    /* cumulative trapezoid + FP64 partial norms */
#define GMM_PROF_NORM 5     /* norm reduction + stop decision */
#define GMM_PROF_CLOSE 6    /* large-step close */
#define GMM_PROF_PROJECT 7  /* rank-r route: Y = V B on MFMA (pair products formed on the fly) */
#define GMM_PROF_GAIN 8     /* saturating gain and linear coupling: pair integrals, matrices, spectral update */
#define GMM_PROF_KINDS 9
#define GMM_PROF_ALL ((1 << GMM_PROF_KINDS) - 1)
int gmm_profile_enable(gmm_plan plan, int kinds);
int gmm_profile_read(gmm_plan plan, double* total_ms, long long* launches, int n_kinds);

#ifdef __cplusplus
}
#endif
#endif /* GMMPA_H */
