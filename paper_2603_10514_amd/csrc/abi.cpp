// extern "C" entry points declared in include/chase.h: argument checks,
// error mapping, asynchronous handles and the per-step entry points.
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "solver.hpp"

namespace chase {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *get_error() { return g_err.c_str(); }
}  // namespace chase

using namespace chase;

struct chase_handle {
  Ctx ctx;
  std::thread th;
  std::atomic<int> running{0};
  chase_status result = CHASE_OK;
  int64_t N_max = 0;
  int L_max = 0;
  int device = 0;
  chase_opts opts;
};

namespace {

chase_status fail(chase_status s, const std::string &msg) {
  set_error(msg);
  return s;
}

template <class F> chase_status guarded(F &&f) {
  try {
    return f();
  } catch (const InvalidArg &) {
    return CHASE_EINVAL;
  } catch (const OutOfMemory &) {
    return CHASE_ENOMEM;
  } catch (const DeviceError &) {
    return CHASE_EDEVICE;
  } catch (const std::exception &e) {
    set_error(e.what());
    return CHASE_EINTERNAL;
  } catch (...) {
    set_error("unknown internal error");
    return CHASE_EINTERNAL;
  }
}

chase_status check_opts(const chase_opts *o) {
  if (o == nullptr) return fail(CHASE_EINVAL, "opts is NULL");
  if (o->struct_size != (int32_t)sizeof(chase_opts))
    return fail(CHASE_EINVAL, "opts->struct_size mismatch (use chase_opts_default)");
  if (o->dtype != CHASE_REAL64 && o->dtype != CHASE_COMPLEX128)
    return fail(CHASE_EINVAL, "unknown dtype");
  if (o->precision != CHASE_PREC_FP64 && o->precision != CHASE_PREC_MIXED)
    return fail(CHASE_EINVAL, "unknown precision");
  if (o->min_deg < 1 || o->max_deg < o->min_deg || o->deg_margin < 0)
    return fail(CHASE_EINVAL, "need 1 <= min_deg <= max_deg and deg_margin >= 0");
  if (o->max_iter < 1) return fail(CHASE_EINVAL, "max_iter must be >= 1");
  if (o->qr_policy < CHASE_QR_AUTO || o->qr_policy > CHASE_QR_HOUSEHOLDER)
    return fail(CHASE_EINVAL, "unknown qr_policy");
  if (!(o->est_hi >= o->est_lo)) return fail(CHASE_EINVAL, "need est_hi >= est_lo");
  if (o->have_bounds &&
      !(o->lambda_1 <= o->lambda_l && o->lambda_l < o->lambda_max))
    return fail(CHASE_EINVAL, "need lambda_1 <= lambda_l < lambda_max");
  if (!o->have_bounds && o->lanczos_steps < 1)
    return fail(CHASE_EINVAL, "lanczos_steps must be >= 1");
  if (!o->have_bounds && (o->lanczos_nvec < 1 || o->lanczos_nvec > 8))
    return fail(CHASE_EINVAL, "lanczos_nvec must be in 1..8");
  return CHASE_OK;
}

chase_status check_solve(const void *H, int64_t N, int64_t ldh, int32_t nev, int32_t nex,
                         int32_t degree, double tol, const chase_opts *o, const double *evals,
                         const void *evecs, int64_t ldv) {
  chase_status s = check_opts(o);
  if (s != CHASE_OK) return s;
  if (H == nullptr || evals == nullptr || evecs == nullptr)
    return fail(CHASE_EINVAL, "H, evals and evecs must not be NULL");
  if (N < 1 || N > 2147483647LL) return fail(CHASE_EINVAL, "need 1 <= N < 2^31");
  if (nev < 1 || nex < 1 || (int64_t)nev + nex > N)
    return fail(CHASE_EINVAL,
                "need 1 <= nev, 1 <= nex (the search space exceeds nev, Alg. 1), nev + nex <= N");
  if (ldh < N || ldv < N) return fail(CHASE_EINVAL, "need ldh >= N and ldv >= N");
  if (degree < 1) return fail(CHASE_EINVAL, "degree must be >= 1");
  if (!(tol > 0.0)) return fail(CHASE_EINVAL, "tol must be > 0");
  return CHASE_OK;
}

}  // namespace

extern "C" {

void chase_opts_default(chase_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(chase_opts);
  o->dtype = CHASE_REAL64;
  o->precision = CHASE_PREC_FP64;
  o->deg_opt = 1;
  o->min_deg = 1;
  o->max_deg = 36;
  o->deg_margin = 2;
  o->max_iter = 25;
  o->qr_policy = CHASE_QR_AUTO;
  o->est_hi = 1e8;
  o->est_lo = 20.0;
  o->seed = 1;
  o->lanczos_steps = 40;
  o->lanczos_nvec = 4;
  o->inject_chol_fail_iter = -1;
  o->mixed_switch = 6e-5;
  o->mixed_buffer32 = 1;
}

chase_status chase_solve(const void *H, int64_t N, int64_t ldh, int32_t nev, int32_t nex,
                         int32_t degree, double tol, const chase_opts *opts, double *evals,
                         void *evecs, int64_t ldv, double *resid, chase_info *info) {
  chase_status s = check_solve(H, N, ldh, nev, nex, degree, tol, opts, evals, evecs, ldv);
  if (s != CHASE_OK) return s;
  return guarded([&] {
    Ctx &c = thread_ctx();
    c.ensure_init();
    hipStream_t own = c.stream;
    if (opts->stream) c.stream = (hipStream_t)opts->stream;
    chase_status r;
    try {
      r = solve(c, *opts, H, N, ldh, nev, nex, degree, tol, evals, evecs, ldv, resid, info);
    } catch (...) {
      c.stream = own;
      throw;
    }
    c.stream = own;
    return r;
  });
}

size_t chase_workspace_bytes(int64_t N, int32_t nev, int32_t nex, chase_dtype dtype,
                             chase_precision precision) {
  if (N < 2 || nev < 1 || nex < 1 || (int64_t)nev + nex > N) return 0;
  return work_bytes(N, nev + nex, dtype == CHASE_COMPLEX128, precision == CHASE_PREC_MIXED, 40, 4);
}

chase_status chase_handle_create(int64_t N_max, int32_t nev_max, int32_t nex_max,
                                 const chase_opts *opts, chase_handle **out) {
  chase_status s = check_opts(opts);
  if (s != CHASE_OK) return s;
  if (out == nullptr) return fail(CHASE_EINVAL, "out is NULL");
  if (N_max < 2 || nev_max < 1 || nex_max < 1 || (int64_t)nev_max + nex_max > N_max)
    return fail(CHASE_EINVAL, "invalid maximum shape");
  return guarded([&] {
    chase_handle *h = new chase_handle();
    h->N_max = N_max;
    h->L_max = nev_max + nex_max;
    h->opts = *opts;
    CHASE_HIP(hipGetDevice(&h->device));
    try {
      h->ctx.stream = nullptr;  // the handle's own stream
      h->ctx.ensure_init();
      h->ctx.ensure_work(N_max, h->L_max, opts->dtype == CHASE_COMPLEX128,
                         opts->precision == CHASE_PREC_MIXED,
                         opts->have_bounds ? 0 : std::max(1, opts->lanczos_steps),
                         std::max(1, opts->lanczos_nvec));
    } catch (...) {
      h->ctx.release();
      delete h;
      throw;
    }
    *out = h;
    return CHASE_OK;
  });
}

chase_status chase_solve_async(chase_handle *h, const void *H, int64_t N, int64_t ldh,
                               int32_t nev, int32_t nex, int32_t degree, double tol,
                               const chase_opts *opts, double *evals, void *evecs, int64_t ldv,
                               double *resid, chase_info *info) {
  if (h == nullptr) return fail(CHASE_EINVAL, "handle is NULL");
  if (h->running.load()) return fail(CHASE_EBUSY, "handle busy");
  const chase_opts *o = opts ? opts : &h->opts;
  chase_status s = check_solve(H, N, ldh, nev, nex, degree, tol, o, evals, evecs, ldv);
  if (s != CHASE_OK) return s;
  if (N > h->N_max || nev + nex > h->L_max)
    return fail(CHASE_EINVAL, "problem larger than the handle's maximum shape");
  if (h->th.joinable()) h->th.join();
  h->opts = *o;
  h->opts.stream = nullptr;  // always the handle's stream
  h->running.store(1);
  h->result = CHASE_EBUSY;
  h->th = std::thread([=] {
    chase_status r = guarded([&] {
      CHASE_HIP(hipSetDevice(h->device));
      return solve(h->ctx, h->opts, H, N, ldh, nev, nex, degree, tol, evals, evecs, ldv, resid,
                   info);
    });
    h->result = r;
    h->running.store(0);
  });
  return CHASE_OK;
}

chase_status chase_handle_query(chase_handle *h) {
  if (h == nullptr) return fail(CHASE_EINVAL, "handle is NULL");
  if (h->running.load()) return CHASE_EBUSY;
  return h->result;
}

chase_status chase_handle_wait(chase_handle *h) {
  if (h == nullptr) return fail(CHASE_EINVAL, "handle is NULL");
  if (h->th.joinable()) h->th.join();
  return h->result;
}

void chase_handle_destroy(chase_handle *h) {
  if (h == nullptr) return;
  if (h->th.joinable()) h->th.join();
  h->ctx.release();
  delete h;
}

// ------------------------------------------------------------ step calls --
static bool dtype_ok(chase_dtype d) { return d == CHASE_REAL64 || d == CHASE_COMPLEX128; }

chase_status chase_filter(chase_dtype dtype, chase_precision prec, const void *H, int64_t N,
                          int64_t ldh, const void *V, int64_t ldv, int32_t ncols,
                          const int32_t *deg, double c, double e, double gamma, void *out,
                          int64_t ldo, void *stream) {
  if (!dtype_ok(dtype)) return fail(CHASE_EINVAL, "unknown dtype");
  if (prec != CHASE_PREC_FP64 && prec != CHASE_PREC_MIXED)
    return fail(CHASE_EINVAL, "unknown precision");
  if (N < 1 || ncols < 0 || ncols > N || ldh < N || ldv < N || ldo < N)
    return fail(CHASE_EINVAL, "invalid sizes");
  if (ncols == 0) return CHASE_OK;  // nothing is read or written
  if (!H || !V || !out || !deg) return fail(CHASE_EINVAL, "NULL argument");
  if (!(e > 0.0)) return fail(CHASE_EINVAL, "half-width e must be > 0");
  for (int a = 0; a < ncols; ++a)
    if (deg[a] < 1 || (a > 0 && deg[a] < deg[a - 1]))
      return fail(CHASE_EINVAL, "degrees must be >= 1 and ascending");
  return guarded([&] {
    const bool cplx = dtype == CHASE_COMPLEX128, f32 = prec == CHASE_PREC_MIXED;
    Ctx &cx = thread_ctx();
    cx.ensure_work(N, ncols, cplx, f32, 0);
    hipStream_t own = cx.stream;
    cx.stream = stream ? (hipStream_t)stream : own;
    Work &w = cx.w;
    std::vector<int> d(deg, deg + ncols);
    gather_cols(cplx, f32, V, ldv, w.X0, N, (int)N, ncols, nullptr, cx.stream);
    if (f32) convert_to32(cplx, H, ldh, w.H32, N, (int)N, (int)N, cx.stream);
    void *bufs[3] = {w.X0, w.B1, w.B2};
    filter(cx, cplx, f32, f32 ? w.H32 : H, f32 ? N : ldh, N, bufs, N, ncols, d, c, e, gamma, out,
           ldo);
    hipError_t err = hipStreamSynchronize(cx.stream);
    cx.stream = own;
    if (err != hipSuccess) {
      set_error(std::string("filter: ") + hipGetErrorString(err));
      throw DeviceError();
    }
    return CHASE_OK;
  });
}

double chase_log_cond_estimate(double theta_next, int32_t m_next, int32_t m_max, double lam1,
                               double c, double e) {
  return log_cond_estimate(theta_next, m_next, m_max, lam1, c, e);
}

chase_qr chase_select_qr(double est, double hi, double lo) { return select_qr(est, hi, lo); }

void chase_degrees(const double *theta, const double *resid, int32_t ncols, double tol, double c,
                   double e, int32_t min_deg, int32_t max_deg, int32_t margin,
                   int32_t *degrees_out) {
  if (!theta || !resid || !degrees_out || ncols <= 0) return;
  degrees(theta, resid, ncols, tol, c, e, min_deg, max_deg, margin, degrees_out);
}

chase_status chase_qr_factor(chase_dtype dtype, void *X, int64_t N, int64_t ldx, int32_t ncols,
                             chase_qr variant, int32_t *chol_failed, double *shift,
                             void *stream) {
  if (!dtype_ok(dtype)) return fail(CHASE_EINVAL, "unknown dtype");
  if (!X) return fail(CHASE_EINVAL, "X is NULL");
  if (N < 1 || ncols < 1 || ncols > N || ldx < N) return fail(CHASE_EINVAL, "invalid sizes");
  if (variant < CHASE_QR_CHOL1 || variant > CHASE_QR_HOUSEHOLDER)
    return fail(CHASE_EINVAL, "variant must be CHOL1, CHOL2, SHIFTED or HOUSEHOLDER");
  return guarded([&] {
    const bool cplx = dtype == CHASE_COMPLEX128;
    Ctx &cx = thread_ctx();
    cx.ensure_work(N, ncols, cplx, false, 0);
    hipStream_t own = cx.stream;
    cx.stream = stream ? (hipStream_t)stream : own;
    Work &w = cx.w;
    w.h_flag[3] = 0;
    hh_panel_clear_error(w.hh, cx.stream);
    copy_cols(cplx, X, ldx, w.Xq, N, (int)N, ncols, cx.stream);
    QrOut q = qr(cx, cplx, w.Xq, w.B1, N, N, ncols, variant, 0);
    copy_cols(cplx, q.Q, N, X, ldx, (int)N, ncols, cx.stream);
    hipError_t err = hipStreamSynchronize(cx.stream);
    cx.stream = own;
    if (err != hipSuccess) {
      set_error(std::string("qr: ") + hipGetErrorString(err));
      throw DeviceError();
    }
    if (w.h_flag[3] != 0) {
      set_error("qr: a Householder panel launch's grid barrier timed out");
      throw DeviceError();
    }
    if (chol_failed) *chol_failed = q.failed ? 1 : 0;
    if (shift) {
      shift[0] = q.fro2;
      shift[1] = q.shift;
    }
    return CHASE_OK;
  });
}

chase_status chase_rayleigh_ritz(chase_dtype dtype, const void *H, int64_t N, int64_t ldh,
                                 const void *Q, int64_t ldq, int32_t ncols, double *ritz, void *V,
                                 int64_t ldv, void *HV, int64_t ldhv, void *stream) {
  if (!dtype_ok(dtype)) return fail(CHASE_EINVAL, "unknown dtype");
  if (!H || !Q || !ritz || !V || !HV) return fail(CHASE_EINVAL, "NULL argument");
  if (N < 1 || ncols < 1 || ncols > N || ldh < N || ldq < N || ldv < N || ldhv < N)
    return fail(CHASE_EINVAL, "invalid sizes");
  return guarded([&] {
    const bool cplx = dtype == CHASE_COMPLEX128;
    Ctx &cx = thread_ctx();
    cx.ensure_work(N, ncols, cplx, false, 0);
    hipStream_t own = cx.stream;
    cx.stream = stream ? (hipStream_t)stream : own;
    rayleigh_ritz(cx, cplx, H, ldh, N, Q, ldq, ncols, cx.w.B2, V, ldv, HV, ldhv);
    CHASE_HIP(hipMemcpyAsync(ritz, cx.w.theta, 8 * (size_t)ncols, hipMemcpyDeviceToHost,
                             cx.stream));
    CHASE_HIP(hipMemcpyAsync(cx.w.h_flag + 2, cx.w.rinfo, 4, hipMemcpyDeviceToHost, cx.stream));
    hipError_t err = hipStreamSynchronize(cx.stream);
    cx.stream = own;
    if (err != hipSuccess) {
      set_error(std::string("rayleigh_ritz: ") + hipGetErrorString(err));
      throw DeviceError();
    }
    if (cx.w.h_flag[2] != 0) {
      set_error("rayleigh_ritz: the projected eigenproblem did not converge (info " +
                std::to_string(cx.w.h_flag[2]) + ")");
      throw DeviceError();
    }
    return CHASE_OK;
  });
}

chase_status chase_residuals(chase_dtype dtype, const void *HV, int64_t ldhv, const void *V,
                             int64_t ldv, int64_t N, int32_t ncols, const double *ritz,
                             double *resid, void *stream) {
  if (!dtype_ok(dtype)) return fail(CHASE_EINVAL, "unknown dtype");
  if (!HV || !V || !ritz || !resid) return fail(CHASE_EINVAL, "NULL argument");
  if (N < 1 || ncols < 1 || ldhv < N || ldv < N) return fail(CHASE_EINVAL, "invalid sizes");
  return guarded([&] {
    const bool cplx = dtype == CHASE_COMPLEX128;
    Ctx &cx = thread_ctx();
    cx.ensure_work(N, ncols, cplx, false, 0);
    hipStream_t st = stream ? (hipStream_t)stream : cx.stream;
    CHASE_HIP(hipMemcpyAsync(cx.w.theta, ritz, 8 * (size_t)ncols, hipMemcpyHostToDevice, st));
    residuals(cplx, HV, ldhv, V, ldv, (int)N, ncols, cx.w.theta, cx.w.resid, st);
    CHASE_HIP(hipMemcpyAsync(resid, cx.w.resid, 8 * (size_t)ncols, hipMemcpyDeviceToHost, st));
    CHASE_HIP(hipStreamSynchronize(st));
    return CHASE_OK;
  });
}

chase_status chase_lanczos(chase_dtype dtype, const void *H, int64_t N, int64_t ldh,
                           const void *V0, int32_t nvec, int32_t steps, int32_t nsearch,
                           double *alpha, double *beta, double *bounds, void *stream) {
  if (!dtype_ok(dtype)) return fail(CHASE_EINVAL, "unknown dtype");
  if (!H || !V0 || !alpha || !beta || !bounds) return fail(CHASE_EINVAL, "NULL argument");
  if (N < 1 || ldh < N || steps < 1 || nsearch < 1 || nsearch > N)
    return fail(CHASE_EINVAL, "invalid sizes");
  if (nvec < 1 || nvec > 8) return fail(CHASE_EINVAL, "nvec must be in 1..8");
  return guarded([&] {
    const bool cplx = dtype == CHASE_COMPLEX128;
    Ctx &cx = thread_ctx();
    cx.ensure_work(N, std::max(1, nsearch), cplx, false, steps, nvec);
    hipStream_t own = cx.stream;
    cx.stream = stream ? (hipStream_t)stream : own;
    std::vector<double> a, b;
    try {
      lanczos(cx, cplx, H, ldh, N, V0, nvec, steps, 0, a, b);
    } catch (...) {
      cx.stream = own;
      throw;
    }
    cx.stream = own;
    const int k = (int)a.size() / nvec;
    for (int r = 0; r < nvec; ++r)
      for (int j = 0; j < steps; ++j) {
        alpha[(size_t)r * steps + j] = j < k ? a[(size_t)r * k + j] : 0.0;
        beta[(size_t)r * steps + j] = j < k ? b[(size_t)r * k + j] : 0.0;
      }
    lanczos_bounds_from_runs(a, b, nvec, N, nsearch, bounds);
    return CHASE_OK;
  });
}

chase_status chase_lanczos_bounds(const double *alpha, const double *beta, int32_t nvec,
                                  int32_t steps, int64_t N, int32_t nsearch, double *bounds) {
  if (!alpha || !beta || !bounds) return fail(CHASE_EINVAL, "NULL argument");
  if (nvec < 1 || steps < 1 || N < 1 || nsearch < 1 || nsearch > N)
    return fail(CHASE_EINVAL, "invalid sizes");
  return guarded([&] {
    std::vector<double> a(alpha, alpha + (size_t)nvec * steps);
    std::vector<double> b(beta, beta + (size_t)nvec * steps);
    lanczos_bounds_from_runs(a, b, nvec, N, nsearch, bounds);
    return CHASE_OK;
  });
}

chase_status chase_sequence_bounds(const double *prev, double delta, double *out) {
  if (!prev || !out) return fail(CHASE_EINVAL, "NULL argument");
  if (!(delta >= 0.0) || !std::isfinite(delta) || !std::isfinite(prev[0]) ||
      !std::isfinite(prev[1]) || !std::isfinite(prev[2]))
    return fail(CHASE_EINVAL, "delta must be >= 0 and the bounds finite");
  if (!(prev[0] <= prev[1] && prev[1] < prev[2]))
    return fail(CHASE_EINVAL, "need prev[0] <= prev[1] < prev[2]");
  const double lo = prev[0] - delta, mid = prev[1], hi = prev[2] + delta;
  out[0] = lo;
  out[1] = mid;
  out[2] = hi;
  return CHASE_OK;
}

chase_status chase_set_panel_wait_limit(int64_t ticks) {
  hh_panel_set_wait_limit((long long)ticks);
  return CHASE_OK;
}

const char *chase_strerror(chase_status s) {
  switch (s) {
    case CHASE_OK: return "ok";
    case CHASE_NOT_CONVERGED: return "not converged within max_iter";
    case CHASE_EINVAL: return "invalid argument";
    case CHASE_ENOMEM: return "out of device memory";
    case CHASE_EDEVICE: return "device or library error";
    case CHASE_EINTERNAL: return "internal error";
    case CHASE_EBUSY: return "handle busy";
  }
  return "unknown status";
}

const char *chase_last_error(void) { return get_error(); }

}  // extern "C"
