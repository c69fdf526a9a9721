// Internal interface of the host driver (not part of the C ABI).
#pragma once
#include <vector>

#include "../../include/chase.h"
#include "common.hpp"
#include "kernels.hpp"

namespace chase {

// Device workspace of one solve shape, carved out of a single allocation.
struct Work {
  int64_t N = 0;
  int L = 0;
  bool cplx = false, mixed = false;
  int nsplit = 1, lz_steps = 0, lz_nvec = 1, lz_split = 1;
  char *base = nullptr;
  size_t bytes = 0;
  void *X0 = nullptr, *B1 = nullptr, *B2 = nullptr, *Xq = nullptr;  // N x L
  void *P = nullptr;                                                  // nsplit x L x L
  void *G = nullptr, *R = nullptr, *Ri = nullptr, *T = nullptr, *A = nullptr;  // L x L
  double *theta = nullptr, *resid = nullptr, *E = nullptr, *trace = nullptr;
  int *flag = nullptr, *perm = nullptr, *rinfo = nullptr;
  void *tau = nullptr;
  void *H32 = nullptr;                                  // N x N in FP32 (mixed)
  void *LV = nullptr, *LW = nullptr, *Lh = nullptr, *LhP = nullptr;  // Lanczos runs
  double *lz_ab = nullptr;
  void *SK = nullptr;                                   // remainder-split partials
  void *hh = nullptr;                                   // Householder QR state
  // eigensolver of the Rayleigh-Ritz matrix: tridiagonal (d, e), the two
  // p vectors of the reduction, the divide and conquer arrays, the T of one
  // block reflector of the back-transform
  double *eg_d = nullptr, *eg_e = nullptr;
  void *eg_p[2] = {nullptr, nullptr};
  void *eg_T = nullptr;
  DcPtrs dc = {};
  size_t sk_bytes = 0;
  // pinned host mirrors
  double *h_theta = nullptr, *h_resid = nullptr, *h_ab = nullptr;
  double *h_aux = nullptr;  // [0] ||X||_F^2, [1] shift of the last shifted pass
  int *h_flag = nullptr;    // [0..1] QR failure flag, [2] eigensolver info,
                            // [3] Householder panel barrier time-out
  int *h_perm = nullptr;
};

size_t work_bytes(int64_t N, int L, bool cplx, bool mixed, int lz_steps, int lz_nvec);

// Per-thread (or per-handle) execution context.
struct Ctx {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Work w;
  hipEvent_t ev[8] = {};
  bool init = false;
  int h_cap_L = 0, h_cap_lz = 0;
  void ensure_init();
  void free_pinned();
  void ensure_work(int64_t N, int L, bool cplx, bool mixed, int lz_steps, int lz_nvec = 1);
  void release();
};

Ctx &thread_ctx();

// Host logic shared with the C ABI (pure functions).
double rho_abs(double x, double c, double e);
double log_cond_estimate(double theta_next, int m_next, int m_max, double lam1, double c,
                         double e);
chase_qr select_qr(double est, double hi, double lo);
void degrees(const double *theta, const double *resid, int n, double tol, double c, double e,
             int min_deg, int max_deg, int margin, int *out);
// Bounds from nvec Lanczos runs; alpha and beta hold run r's k coefficients
// at [r * k, (r + 1) * k).
void lanczos_bounds_from_runs(const std::vector<double> &alpha, const std::vector<double> &beta,
                              int nvec, int64_t N, int nsearch, double bounds[3]);

// Steps (device buffers; enqueue on ctx.stream).
// Alg. 4 on explicit buffers (no context): V is the input block, bufs the
// three rotating step buffers (V may be bufs[2]), tail_ws the remainder
// split's scratch (may be null: no split).  Returns the GEMM dispatches.
int filter_enqueue(hipStream_t st, void *tail_ws, size_t tail_bytes, bool cplx, bool f32,
                   const void *H, int64_t ldh, int64_t N, const void *V, int64_t ldv,
                   void *const bufs[3], int64_t ldb, int ncols, const int *deg_sorted, double cc,
                   double e, double gamma, void *out, int64_t ldo);
// The same on the context's buffers: bufs[0] holds the input, bufs[1..2] and
// bufs[0] rotate.
int filter(Ctx &c, bool cplx, bool f32, const void *H, int64_t ldh, int64_t N, void *bufs[3],
           int64_t ldb, int ncols, const std::vector<int> &deg_sorted, double cc, double e,
           double gamma, void *out, int64_t ldo);
struct QrOut {
  void *Q;          // buffer that holds Q
  bool failed;      // a Cholesky failed and the Householder QR ran instead
  chase_qr ran;
  double fro2, shift;  // shifted branch: ||X||_F^2 = trace(X^H X) and the shift; NaN otherwise
};
// A QR whose Cholesky passes are enqueued but whose failure flag has not been
// read yet (it is copied to the pinned mirror h_flag on the stream).
struct QrPending {
  void *X, *Xalt;
  void *inputs[3];
  int npass;
  chase_qr variant;
  void *out;  // where Q lands when no Cholesky fails
};
QrPending qr_enqueue(Ctx &c, bool cplx, void *X, void *Xalt, int64_t ld, int64_t N, int L,
                     chase_qr variant, int inject);
// After the stream has been synchronised: read the flag; on a failure enqueue
// the Householder QR of the failing pass's input (not synchronised).
QrOut qr_finish(Ctx &c, bool cplx, const QrPending &p, int64_t ld, int64_t N, int L);
// qr_enqueue, synchronise, qr_finish.
QrOut qr(Ctx &c, bool cplx, void *X, void *Xalt, int64_t ld, int64_t N, int L, chase_qr variant,
         int inject);
void rayleigh_ritz(Ctx &c, bool cplx, const void *H, int64_t ldh, int64_t N, const void *Q,
                   int64_t ldq, int Lp, void *W, void *Vout, int64_t ldv, void *HV, int64_t ldhv);
void lanczos(Ctx &c, bool cplx, const void *H, int64_t ldh, int64_t N, const void *V0, int nvec,
             int steps, uint64_t seed, std::vector<double> &alpha, std::vector<double> &beta);

chase_status solve(Ctx &c, const chase_opts &o, const void *H, int64_t N, int64_t ldh, int nev,
                   int nex, int degree, double tol, double *evals, void *evecs, int64_t ldv,
                   double *resid, chase_info *info);

}  // namespace chase
