/*
 * chase.h - C interface of an MI355X (gfx950) implementation of Chebyshev
 * filtered subspace iteration with a condition-number-driven choice of the
 * QR variant (Di Napoli & Wu, "Estimating the condition number of Chebyshev
 * filtered vectors with application to the ChASE library", arXiv 2603.10514).
 *
 * Problem statement (Sec. 1.2, Alg. 1): given a Hermitian (complex) or
 * symmetric (real) matrix H of order N, find the nev lowest eigenpairs
 * (Lambda, Y), ascending, using a search space of l = nev + nex vectors, a
 * Chebyshev filter whose per-vector degrees are optimised (Sec. 2.2), the
 * estimate of kappa_2 of the filtered block (estimate (1.1), estimate (1.2)) to
 * pick CholeskyQR / CholeskyQR2 / shifted CholeskyQR2 / Householder QR
 * (Alg. 3), Rayleigh-Ritz, and residual-based locking (the residual of Sec. 2.3.1).
 *
 * Conventions for every entry point:
 *  - Matrices are column-major.  Complex matrices are interleaved
 *    (re, im) pairs of double (or float for FP32 buffers).
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns its own workspace.
 *  - H must be exactly Hermitian: the kernels read it through H^H = H (the
 *    reduction index runs along a column, which is contiguous).
 *  - stream: a hipStream_t (NULL = the library's own stream of the calling
 *    thread).  Work is ordered on that stream; entry points that return host
 *    results synchronise it before returning.
 *  - Errors: a negative chase_status; nothing the caller owns has been
 *    written when CHASE_EINVAL is returned.  chase_last_error() gives a
 *    thread-local message.
 *  - All entry points are thread-safe for distinct handles / streams.
 */
#ifndef CHASE_MI355X_H
#define CHASE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum chase_status {
  CHASE_OK = 0,
  CHASE_NOT_CONVERGED = 1, /* fewer than nev pairs locked within max_iter      */
  CHASE_EINVAL = -1,       /* an argument is invalid (see chase_last_error)   */
  CHASE_ENOMEM = -2,       /* device workspace could not be allocated          */
  CHASE_EDEVICE = -3,      /* a HIP / rocSOLVER call failed                    */
  CHASE_EINTERNAL = -4,
  CHASE_EBUSY = -5         /* asynchronous solve still running                 */
} chase_status;

typedef enum chase_dtype { CHASE_REAL64 = 0, CHASE_COMPLEX128 = 1 } chase_dtype;

/* Precision of the filter.  MIXED: filter in FP32 (complex64 for complex H)
 * on MFMA with FP32 accumulation while the lowest unconverged residual is
 * above the switch threshold, FP64 afterwards; Gram matrix, Cholesky, shift,
 * Rayleigh-Ritz and residuals always in FP64. */
typedef enum chase_precision { CHASE_PREC_FP64 = 0, CHASE_PREC_MIXED = 1 } chase_precision;

/* QR variants of Alg. 3 (AUTO = chosen from the estimate each iteration). */
typedef enum chase_qr {
  CHASE_QR_AUTO = 0,
  CHASE_QR_CHOL1 = 1,       /* CholeskyQR, one pass (Alg. 2, cholDeg = 1)     */
  CHASE_QR_CHOL2 = 2,       /* CholeskyQR2 (Alg. 2, cholDeg = 2)              */
  CHASE_QR_SHIFTED = 3,     /* shifted pass then CholeskyQR2 (Alg. 3)         */
  CHASE_QR_HOUSEHOLDER = 4  /* Householder QR                                 */
} chase_qr;

/* One record per iteration of Alg. 1 (the quantities of Sec. 4.3 / 4.4). */
typedef struct chase_iter_log {
  int32_t iter;          /* 1-based                                            */
  int32_t locked;        /* k: pairs locked before this iteration              */
  int32_t newly_locked;
  int32_t qr_variant;    /* chase_qr actually run (HOUSEHOLDER after fallback) */
  int32_t chol_failed;   /* 1 if a Cholesky failed and Householder QR ran       */
  int32_t filter_prec;   /* CHASE_PREC_MIXED if any column of this iteration was
                            filtered in FP32, else CHASE_PREC_FP64             */
  int32_t deg_min, deg_max;
  int64_t matvecs;       /* sum of this iteration's degrees                    */
  double cond_est;       /* estimate (1.2) with eta = 1 (may be +inf)             */
  double cond_exact;     /* value returned by opts->block_cb, else NaN          */
  double c, e, gamma, lam1; /* filter centre, half-width, normalisation point,
                               lowest Ritz value (the rho_1 point)              */
  double t_filter, t_qr, t_rr, t_resid; /* seconds, device events               */
  double qr_fro2;        /* shifted branch of Alg. 3: ||X||_F^2 = trace(X^H X) of
                            the block [Y | filtered]; NaN on the other branches */
  double qr_shift;       /* the shift s = 11 (N l + l (l + 1)) u ||X||_F^2 added
                            to the Gram matrix (u = 2^-53); NaN otherwise        */
  int32_t ncols;         /* active (filtered) columns of this iteration        */
  const int32_t *degrees; /* their degrees (valid during log_cb): ascending over
                             the first ncols - ncols_fp32 (FP64 filter) and over
                             the last ncols_fp32 (FP32 filter)                  */
  int32_t ncols_fp32;    /* columns of this iteration filtered in FP32          */
} chase_iter_log;

typedef struct chase_opts {
  int32_t struct_size;       /* sizeof(chase_opts); set by chase_opts_default  */
  chase_dtype dtype;
  chase_precision precision;
  int32_t deg_opt;           /* 1: per-vector optimised degrees (Sec. 2.2)      */
  int32_t min_deg, max_deg;  /* clamp of the optimised degrees (default 1, 36)  */
  int32_t deg_margin;        /* degrees added to the predicted one (default 2)  */
  int32_t max_iter;          /* default 25                                      */
  chase_qr qr_policy;        /* default AUTO (Alg. 3)                           */
  double est_hi, est_lo;     /* Alg. 3 thresholds, default 1e8 and 20           */
  int32_t have_bounds;       /* 1: use lambda_1, lambda_l, lambda_max below     */
  double lambda_1, lambda_l, lambda_max; /* lambda_max must bound the spectrum
                                            (Sec. 1.2); a Ritz value above it
                                            raises it by that value + twice its
                                            residual + 1e-3 of the Ritz span  */
  int32_t warm_start;        /* 1: evecs holds the start block V0 on entry      */
  uint64_t seed;             /* random start block / Lanczos vector otherwise   */
  int32_t lanczos_steps;     /* steps per Lanczos run, default 40               */
  int32_t lanczos_nvec;      /* independent Lanczos runs, 1..8, default 4       */
  const void *lanczos_v0;    /* optional device start vectors: N x lanczos_nvec,
                                column-major, leading dimension N               */
  int32_t inject_chol_fail_iter; /* test hook: the Cholesky of this iteration
                                    reports failure (-1 = off)                  */
  double mixed_switch;       /* MIXED: switch the filter to FP64 once the lowest
                                unconverged residual <= mixed_switch *
                                max(|lambda_1|, |lambda_max|) (default 6e-5), or
                                once an FP32 iteration fails to halve it         */
  int32_t mixed_buffer32;    /* MIXED, after that switch: 1 (default) keeps the
                                nex buffer columns (Ritz index >= nev among the
                                search space) in the FP32 filter, 0 moves the
                                whole block to FP64                              */
  void *stream;              /* hipStream_t or NULL                              */
  void (*log_cb)(const chase_iter_log *rec, void *user);
  void *log_user;
  /* Diagnostic hook (Sec. 4.3 compares the estimate with the exact kappa_2):
   * called once per iteration, after the filter and before the QR, with the
   * device block [Y | filtered] (N x ncols, column-major, leading dimension
   * ld, complex interleaved for COMPLEX128) after the stream has been
   * synchronised.  The block must not be modified.  The value returned is
   * stored as cond_exact in that iteration's log record (NaN if none). */
  double (*block_cb)(const void *X, int64_t N, int64_t ld, int32_t ncols, int32_t iter,
                     void *user);
  void *block_user;
} chase_opts;

typedef struct chase_info {
  int32_t iters;
  int32_t converged;         /* locked pairs (== nev on success)               */
  int64_t matvecs;           /* sum of all degrees over all iterations         */
  int32_t filter_launches;   /* filter GEMM kernel dispatches (one per degree
                                step, two when the step's last partial wave is
                                split along K)                                 */
  int32_t filter_fp32_iters; /* iterations whose whole filter ran in FP32      */
  double t_total, t_filter, t_qr, t_rr, t_resid, t_lanczos; /* seconds          */
  double lambda_1, lambda_l, lambda_max; /* bounds used by the first filter;
                              lambda_max is the upper bound at the end: raised
                              when a Ritz value exceeded it (then it was no
                              bound: Ritz values never exceed the spectrum)  */
  int64_t matvecs_fp32;      /* part of matvecs filtered in FP32 (all columns,
                                or the buffer columns after the switch)       */
  double t_filter_fp32;      /* part of t_filter spent in FP32 filter steps     */
  double ritz_max;           /* largest Ritz value of the last Rayleigh-Ritz
                                (the lambda_l estimate for a warm restart)      */
  int32_t filter_launches_fp32; /* part of filter_launches in FP32             */
} chase_info;

/* Defaults: dtype REAL64, FP64, deg_opt 1, degrees [1, 36], margin 2,
 * max_iter 25, AUTO, thresholds 1e8 / 20, no bounds, no warm start, seed 1,
 * 40 Lanczos steps, no injection, mixed_switch 6e-5, NULL stream/log. */
void chase_opts_default(chase_opts *opts);

/* ---------------------------------------------------------------- solve --
 * chase_solve: Alg. 1 end to end, synchronous.
 *   H      device, N x N, leading dimension ldh >= N, read only.
 *   nev, nex: 1 <= nev, 1 <= nex (Alg. 1 needs a search space larger than
 *          nev), nev + nex <= N.
 *   degree: initial filter degree (Sec. 4.3 uses 20), >= 1.
 *   tol:   residual tolerance of the residual of Sec. 2.3.1 (> 0).
 *   evals  host [nev]: ascending eigenvalues (locked ones first).
 *   evecs  device, N x (nev + nex), ldv >= N: on exit columns 0..nev-1 are the
 *          eigenvectors, the rest the remaining Ritz vectors (a warm start for
 *          the next problem of a sequence).  With opts->warm_start it holds
 *          the start block on entry.
 *   resid  host [nev] or NULL: residual norms of the returned pairs.
 *   info   host or NULL.
 * Returns CHASE_OK, CHASE_NOT_CONVERGED (evals/resid then hold the current
 * Ritz values for the unconverged part) or an error. */
chase_status chase_solve(const void *H, int64_t N, int64_t ldh, int32_t nev, int32_t nex,
                         int32_t degree, double tol, const chase_opts *opts, double *evals,
                         void *evecs, int64_t ldv, double *resid, chase_info *info);

/* Bytes of device workspace one solve of this shape needs (admission). */
size_t chase_workspace_bytes(int64_t N, int32_t nev, int32_t nex, chase_dtype dtype,
                             chase_precision precision);

/* ---------------------------------------------------- asynchronous solves --
 * A handle owns a stream, a rocBLAS handle, a workspace sized for
 * (N_max, nev_max + nex_max) and a host worker thread.  chase_solve_async
 * returns at once; the solve runs on the handle's stream; results land in
 * the caller's buffers, which must stay valid until chase_handle_wait (or a
 * query returning CHASE_OK / an error).  One solve at a time per handle. */
typedef struct chase_handle chase_handle;
chase_status chase_handle_create(int64_t N_max, int32_t nev_max, int32_t nex_max,
                                 const chase_opts *opts, chase_handle **out);
chase_status chase_solve_async(chase_handle *h, const void *H, int64_t N, int64_t ldh,
                               int32_t nev, int32_t nex, int32_t degree, double tol,
                               const chase_opts *opts, double *evals, void *evecs,
                               int64_t ldv, double *resid, chase_info *info);
/* CHASE_EBUSY while running; otherwise the solve's status (non-blocking). */
chase_status chase_handle_query(chase_handle *h);
/* Blocks until the current solve ends; returns its status. */
chase_status chase_handle_wait(chase_handle *h);
void chase_handle_destroy(chase_handle *h);

/* ------------------------------------------------------ step entry points --
 * Each runs one step of the hot path on device buffers, for testing the
 * steps one by one against a reference.  Workspace is allocated per call.
 * The calls that take a dtype (and chase_filter its precision) return
 * CHASE_EINVAL for a value outside the enum before touching any buffer. */

/* Chebyshev filter with per-vector degrees (Alg. 4, Sec. 2.2): column a of
 * out = p_{m_a}(H) V[:, a], p_m(x) = C_m((x-c)/e) / C_m((gamma-c)/e).
 * degrees: host int32[ncols], ascending, each >= 1 (ncols == 0: no-op, the
 * pointers are not used).  prec MIXED runs the
 * recurrence in FP32 (H and V rounded to FP32) and writes FP64 results. */
chase_status chase_filter(chase_dtype dtype, chase_precision prec, const void *H, int64_t N,
                          int64_t ldh, const void *V, int64_t ldv, int32_t ncols,
                          const int32_t *degrees, double c, double e, double gamma,
                          void *out, int64_t ldo, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as chase_filter in FP64 (dtype REAL64 or COMPLEX128), with every
 * buffer beyond the inputs and outputs in a static device array of
 * CHASE_FILTER_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it
 * runs on until the process ends: the three step buffers (N x ncols each)
 * and the partial tiles of the GEMM's remainder split.  The call allocates
 * nothing, does not synchronise and returns once the work is enqueued on
 * `stream` (NULL: the default stream); `out` is valid when the stream has
 * reached that point.  H, V, out and degrees as for chase_filter (degrees
 * on the host, read during the call).
 * Limits and errors: EINVAL when 3 N ncols times the element size (8 or 16
 * bytes) exceeds CHASE_FILTER_NOALLOC_SCRATCH_BYTES (each buffer rounded up
 * to 256 bytes), and for the argument errors of chase_filter; EDEVICE if a
 * launch fails.  Every call on one GPU uses that GPU's one array, so calls
 * that overlap in time on the same GPU (on different streams or host
 * threads) race and must be serialised by the caller. */
#define CHASE_FILTER_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
chase_status chase_filter_noalloc(chase_dtype dtype, const void *H, int64_t N, int64_t ldh,
                                  const void *V, int64_t ldv, int32_t ncols,
                                  const int32_t *degrees, double c, double e, double gamma,
                                  void *out, int64_t ldo, void *stream);

/* ln of estimate (1.2): m_next ln|rho(theta_next)| + (m_max - m_next) ln|rho(lam1)|
 * (eta = 1); |rho(x)| = |t| + sqrt(t^2 - 1) for |t| = |x - c|/e > 1, else 1. */
double chase_log_cond_estimate(double theta_next, int32_t m_next, int32_t m_max, double lam1,
                               double c, double e);
/* Alg. 3 choice: SHIFTED if est > hi, CHOL1 if est < lo, CHOL2 otherwise. */
chase_qr chase_select_qr(double est, double hi, double lo);

/* Per-vector degrees from Ritz values and residuals (host, ncols entries):
 * m = ceil(ln(r/tol) / ln|rho(theta)|) + margin clamped to [min_deg, max_deg];
 * |rho| = 1 -> max_deg; r <= tol -> min_deg. */
void chase_degrees(const double *theta, const double *resid, int32_t ncols, double tol,
                   double c, double e, int32_t min_deg, int32_t max_deg, int32_t margin,
                   int32_t *degrees_out);

/* Orthonormalise X (device, N x ncols, in place) with one QR variant
 * (Alg. 2 for CHOL1 / CHOL2, Alg. 3's shifted pass followed by CholeskyQR2
 * for SHIFTED, Householder QR).
 * chol_failed (host, may be NULL) is set to 1 when a Cholesky failed and the
 * Householder QR was applied to the block as it stood before that pass.
 * shift (host [2], may be NULL): for SHIFTED, shift[0] = ||X||_F^2 (the trace
 * of the Gram matrix the library formed) and shift[1] = the shift
 * 11 (N ncols + ncols (ncols + 1)) 2^-53 shift[0] that it added to that Gram
 * matrix's diagonal (Alg. 3); NaN for the other variants. */
chase_status chase_qr_factor(chase_dtype dtype, void *X, int64_t N, int64_t ldx, int32_t ncols,
                             chase_qr variant, int32_t *chol_failed, double *shift,
                             void *stream);

/* Rayleigh-Ritz on an orthonormal Q (device, N x ncols): ritz (host, ascending),
 * V = Q Z and HV = H Q Z (device, N x ncols).  CHASE_EDEVICE if the
 * eigensolver of the projected ncols x ncols matrix reports no convergence. */
chase_status chase_rayleigh_ritz(chase_dtype dtype, const void *H, int64_t N, int64_t ldh,
                                 const void *Q, int64_t ldq, int32_t ncols, double *ritz,
                                 void *V, int64_t ldv, void *HV, int64_t ldhv, void *stream);

/* the residual of Sec. 2.3.1: resid[a] = ||HV[:,a] - ritz[a] V[:,a]||_2 / ||V[:,a]||_2 (host out). */
chase_status chase_residuals(chase_dtype dtype, const void *HV, int64_t ldhv, const void *V,
                             int64_t ldv, int64_t N, int32_t ncols, const double *ritz,
                             double *resid, void *stream);

/* Spectral bounds for the filter interval (Alg. 1 and Sec. 1.2: only the
 * estimate of lambda_n has to bound the spectrum from above).  nvec
 * independent Lanczos runs of min(steps, N) steps, each with full
 * reorthogonalisation, from the columns of the device block V0 (N x nvec,
 * column-major, leading dimension N, 1 <= nvec <= 8; the runs normalise
 * their start vectors).  H is the device matrix (N x N, column-major, ldh).
 * Host outputs: alpha, beta [nvec * steps], run r's T_k coefficients at
 * [r * steps, r * steps + k) (beta_j couples steps j and j + 1; the last one
 * is the final residual norm), zero past k; bounds [3] = (lambda_1 estimate,
 * lambda_l estimate for l = nsearch, upper bound):
 *   upper    = max over runs of theta_max + 2 |beta_k| |e_k^T s_max| (the
 *              largest Ritz value of T_k plus twice its Ritz pair's residual)
 *   lambda_1 = smallest Ritz value over the runs
 *   lambda_l = the Ritz value where the run-averaged spectral-density count
 *              sum over Ritz values <= x of N |e_1^T s_j|^2 first reaches l,
 *              clamped to [lambda_1 + 1e-3 w, upper - 1e-3 w], w = upper - lambda_1.
 * Work is enqueued on `stream` (NULL: the library's) and the call returns
 * after it has finished.  Orders up to 4096 run every step in one
 * cooperative launch whose blocks meet at grid barriers (waits limited in
 * time: see chase_set_panel_wait_limit).  Errors: EINVAL for NULL pointers
 * or invalid sizes; EDEVICE when a barrier wait timed out; EDEVICE / ENOMEM
 * as for the other calls. */
chase_status chase_lanczos(chase_dtype dtype, const void *H, int64_t N, int64_t ldh,
                           const void *V0, int32_t nvec, int32_t steps, int32_t nsearch,
                           double *alpha, double *beta, double *bounds, void *stream);

/* The bounds of chase_lanczos from coefficients computed elsewhere (host
 * only, no device work): alpha, beta [nvec * steps] hold run r's T_k at
 * [r * steps, r * steps + steps) in the layout chase_lanczos returns (a run
 * whose beta_j is zero ends at step j); N is the matrix order, bounds [3] as
 * for chase_lanczos.  Errors: EINVAL for NULL pointers, nvec or steps < 1,
 * or nsearch outside 1..N. */
chase_status chase_lanczos_bounds(const double *alpha, const double *beta, int32_t nvec,
                                  int32_t steps, int64_t N, int32_t nsearch, double *bounds);

/* Bounds for the next problem of a sequence H_{j+1} = H_j + D (host only):
 * a warm start (Alg. 1 takes an optional start block and optional spectral
 * bounds) reuses the previous problem's subspace and bounds, and by Weyl's
 * inequality every eigenvalue moves by at most ||D||_2.  prev [3] = (lowest
 * Ritz value, largest Ritz value of the search space, upper bound) of the
 * previous solve (evals[0], info.ritz_max, info.lambda_max); delta >= ||D||_2
 * (a bound the caller knows).  out [3] = (prev[0] - delta, prev[1],
 * prev[2] + delta), ready for opts.lambda_1 / lambda_l / lambda_max.
 * Errors: EINVAL for NULL pointers, delta < 0 or non-finite values, or
 * prev not ordered (prev[0] <= prev[1] < prev[2]). */
chase_status chase_sequence_bounds(const double *prev, double delta, double *out);

/* Test hook for the failure path of the library's grid barriers: the
 * blocks of the Householder QR's panel factorisation (the fallback of
 * Alg. 3) and of the one-launch Lanczos of small orders (the spectral
 * bounds of Alg. 1) meet at grid barriers whose waits give up after a
 * wall-clock limit (two seconds; the cooperative launch keeps every block
 * resident, so a correct run never reaches it), after which the call
 * (chase_qr_factor, chase_lanczos, chase_solve) reports EDEVICE.
 * ticks > 0 sets that limit in ticks of
 * the device's wall clock (hipDeviceAttributeWallClockRate), ticks <= 0
 * restores the default; process-wide, takes effect at the next launch.
 * Always CHASE_OK. */
chase_status chase_set_panel_wait_limit(int64_t ticks);

const char *chase_strerror(chase_status s);
const char *chase_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHASE_MI355X_H */
