// Host driver of Chebyshev filtered subspace iteration (Alg. 1 of the paper)
// on one gfx950 GPU: workspace, the filter loop, the CholeskyQR variants of
// Alg. 2 / Alg. 3 with a device-side failure flag, Rayleigh-Ritz, residuals,
// locking, the degree policy and the condition-number estimate.
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>

#include "gemm.hpp"
#include "kernels.hpp"

namespace chase {

static const double kUnitRoundoff = 1.1102230246251565e-16;  // 2^-53

// ------------------------------------------------------------ host logic --
// |rho| of x for the interval [c - e, c + e] (the interval map of Sec. 2.1, convergence ratio of
// Sec. 2.2): |t| + sqrt(t^2 - 1) outside, 1 inside.
double rho_abs(double x, double c, double e) {
  const double t = (x - c) / e;
  if (std::fabs(t) <= 1.0) return 1.0;
  return std::fabs(t) + std::sqrt(t * t - 1.0);
}

// estimate (1.2) with eta = 1, in log space.
double log_cond_estimate(double theta_next, int m_next, int m_max, double lam1, double c,
                         double e) {
  return m_next * std::log(rho_abs(theta_next, c, e)) +
         (double)(m_max - m_next) * std::log(rho_abs(lam1, c, e));
}

// Alg. 3 branch choice.
chase_qr select_qr(double est, double hi, double lo) {
  if (est > hi) return CHASE_QR_SHIFTED;
  if (est < lo) return CHASE_QR_CHOL1;
  return CHASE_QR_CHOL2;
}

// Per-vector degree: enough steps for the residual to fall from r to tol at
// the rate 1/|rho(theta)| per step (Sec. 2.2), plus a margin.
void degrees(const double *theta, const double *resid, int n, double tol, double c, double e,
             int min_deg, int max_deg, int margin, int *out) {
  for (int a = 0; a < n; ++a) {
    if (resid[a] <= tol) { out[a] = min_deg; continue; }
    const double rho = rho_abs(theta[a], c, e);
    if (rho <= 1.0) { out[a] = max_deg; continue; }
    const double d = std::ceil(std::log(resid[a] / tol) / std::log(rho)) + margin;
    out[a] = (int)std::min<double>(std::max<double>(d, min_deg), max_deg);
  }
}

// Eigenvalues of the symmetric tridiagonal T (diagonal d[0..n), off-diagonal
// e[0..n-1)) by implicit QR steps with the Wilkinson shift (Golub & Van Loan,
// Matrix Computations, Sec. 8.3), in band storage: each step chases a bulge
// down the active block with Givens rotations.  Only rows 0 and n-1 of the
// eigenvector matrix are accumulated (first[j], last[j]: first and last
// component of the unit eigenvector of w[j]); O(n) work per step.  Output in
// ascending order of w.
static void tridiag_eig(int n, std::vector<double> d, std::vector<double> e,
                        std::vector<double> &w, std::vector<double> &first,
                        std::vector<double> &last) {
  std::vector<double> z0(n, 0.0), z1(n, 0.0);  // rows 0 and n-1 of Q
  z0[0] = 1.0;
  z1[n - 1] = 1.0;
  e.resize(std::max(n - 1, 0));
  const double eps = std::numeric_limits<double>::epsilon();
  const int max_steps = 30 * std::max(n, 1);
  for (int step = 0; step < max_steps; ++step) {
    for (int i = 0; i + 1 < n; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    int m = n - 1;
    while (m > 0 && e[m - 1] == 0.0) --m;
    if (m == 0) break;
    int l = m - 1;
    while (l > 0 && e[l - 1] != 0.0) --l;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 nearer d[m]
    const double del = 0.5 * (d[m - 1] - d[m]);
    const double em = e[m - 1];
    const double mu = d[m] - em * em / (del + (del >= 0.0 ? 1.0 : -1.0) * std::hypot(del, em));
    double x = d[l] - mu, zb = e[l];
    for (int k = l; k < m; ++k) {
      // rotation G = [c s; -s c] with G^T (x, zb)^T = (r, 0)^T
      const double r = std::hypot(x, zb);
      const double c = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? -zb / r : 0.0;
      if (k > l) e[k - 1] = r;  // row k-1 loses its bulge
      const double p = d[k], q = e[k], t = d[k + 1];
      d[k] = c * c * p - 2.0 * c * sn * q + sn * sn * t;
      d[k + 1] = sn * sn * p + 2.0 * c * sn * q + c * c * t;
      e[k] = c * sn * (p - t) + (c * c - sn * sn) * q;
      if (k + 1 < m) {  // new bulge at (k, k + 2)
        zb = -sn * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      const double a0 = z0[k], b0 = z0[k + 1], a1 = z1[k], b1 = z1[k + 1];
      z0[k] = c * a0 - sn * b0; z0[k + 1] = sn * a0 + c * b0;
      z1[k] = c * a1 - sn * b1; z1[k + 1] = sn * a1 + c * b1;
    }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  w.resize(n);
  first.resize(n);
  last.resize(n);
  for (int j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    first[j] = z0[idx[j]];
    last[j] = z1[idx[j]];
  }
}

// Bounds from nvec Lanczos runs (Sec. 1.2 needs only the upper end to bound
// the spectrum): upper = max over runs of the largest Ritz value of T_k plus
// twice the residual norm |beta_k| |e_k^T s_max| of its Ritz pair; lambda_1
// estimate = smallest Ritz value over the runs; lambda_l estimate = the Ritz
// value where the spectral-density count, (1/nvec) sum over runs and Ritz
// values <= x of N |e_1^T s_j|^2, first reaches l, clamped into the
// interval.  A run whose Krylov space became invariant (a zero beta) ends
// there.
void lanczos_bounds_from_runs(const std::vector<double> &alpha, const std::vector<double> &beta,
                              int nvec, int64_t N, int nsearch, double bounds[3]) {
  const int kmax = (int)alpha.size() / nvec;
  std::vector<std::pair<double, double>> dos;  // (Ritz value, weight)
  double low = INFINITY, up = -INFINITY;
  for (int r = 0; r < nvec; ++r) {
    const double *a = alpha.data() + (size_t)r * kmax;
    const double *b = beta.data() + (size_t)r * kmax;
    int k = kmax;
    for (int j = 0; j < kmax; ++j)
      if (b[j] == 0.0) { k = j + 1; break; }
    std::vector<double> w, first, last;
    tridiag_eig(k, std::vector<double>(a, a + k), std::vector<double>(b, b + k - 1), w, first,
                last);
    const double top_resid = std::fabs(b[k - 1]) * std::fabs(last[k - 1]);
    up = std::max(up, w[k - 1] + 2.0 * top_resid);
    low = std::min(low, w[0]);
    for (int j = 0; j < k; ++j) dos.push_back({w[j], (double)N * first[j] * first[j] / nvec});
  }
  std::stable_sort(dos.begin(), dos.end(),
                   [](const std::pair<double, double> &x, const std::pair<double, double> &y) {
                     return x.first < y.first;
                   });
  double cum = 0.0;
  double mid = dos.back().first;
  for (const auto &d : dos) {
    cum += d.second;
    if (cum >= (double)nsearch) { mid = d.first; break; }
  }
  const double span = up - low;
  mid = std::min(std::max(mid, low + 1e-3 * span), up - 1e-3 * span);
  bounds[0] = low;
  bounds[1] = mid;
  bounds[2] = up;
}

// --------------------------------------------------------------- workspace --
static inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }
// Scratch of the big GEMMs' remainder split: at most one wave of resident
// blocks (<= 1024) x one 128 x 64 complex (or 128 x 128 real) FP64 tile.
static const size_t kTailScratch = (size_t)80 << 20;

// K splits of the products with few output tiles: about 1024 work-groups,
// at least kSplitRows rows each, at most kMaxSplits splits (a product with
// one output tile, such as the Gram of a 32-column panel, then spreads over
// the whole chip instead of 32 work-groups).
constexpr int kSplitRows = 128, kMaxSplits = 256;
static int gram_splits(int64_t N, int L) {
  const int t = (L + 63) / 64;
  const int tiles = t * (t + 1) / 2;
  int s = (1024 + tiles - 1) / tiles;
  const int smax = (int)std::max<int64_t>(1, N / kSplitRows);
  s = std::min(std::min(s, smax), kMaxSplits);
  return std::max(s, 1);
}
static int lz_splits(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(128, N / 512)); }

struct Layout {
  size_t off[32];
  size_t total;
};

static Layout layout(int64_t N, int L, bool cplx, bool mixed, int lz_steps, int nv) {
  const size_t es = cplx ? 16 : 8;
  const int ns = gram_splits(N, L);
  const int lzs = lz_splits(N);
  const int k = lz_steps > 0 ? (int)std::min<int64_t>(lz_steps, N) : 0;
  const size_t sz[] = {
      al(es * N * L), al(es * N * L), al(es * N * L), al(es * N * L),  // X0 B1 B2 Xq
      al(es * (size_t)ns * L * L),                                     // P
      al(es * L * L), al(es * L * L), al(es * L * L), al(es * L * L), al(es * L * L),  // G R Ri T A
      al(8 * (size_t)L), al(8 * (size_t)L), al(8 * (size_t)L), al(64),  // theta resid E trace
      al(16), al(4 * (size_t)L), al(16),                                 // flag perm rinfo
      al(es * L),                                                         // tau
      mixed ? al(es / 2 * (size_t)N * N) : 0,                             // H32
      k ? al(es * (size_t)N * (k + 1) * nv) : 0,                          // LV
      k ? al(es * (size_t)N * nv) : 0,                                    // LW
      k ? al(es * (size_t)k * nv * nv) : 0,                               // Lh
      k ? al(es * (size_t)lzs * k * nv * nv) : 0,                         // LhP
      k ? al(16 * (size_t)k * nv) : 0,                                    // lz_ab
      al(kTailScratch),                                                   // SK
      al(kHhStateBytes),                                                  // hh
      al(8 * (size_t)L), al(8 * (size_t)L),                              // eg_d eg_e
      al(es * L), al(es * L),                                             // eg_p
      al(es * (size_t)kHhMaxOuter * kHhMaxOuter),                         // eg_T
      al(8 * (size_t)L * 5) + al(4 * (size_t)L * 5),                     // dc arrays
  };
  Layout lo{};
  size_t o = 0;
  const int n = sizeof(sz) / sizeof(sz[0]);
  for (int i = 0; i < n; ++i) {
    lo.off[i] = o;
    o += sz[i];
  }
  lo.total = o;
  return lo;
}

size_t work_bytes(int64_t N, int L, bool cplx, bool mixed, int lz_steps, int lz_nvec) {
  return layout(N, L, cplx, mixed, lz_steps, lz_nvec).total;
}

void Ctx::ensure_init() {
  if (init) return;
  if (stream == nullptr) {
    CHASE_HIP(hipStreamCreate(&stream));
    own_stream = true;
  }
  for (auto &e : ev) CHASE_HIP(hipEventCreate(&e));
  init = true;
}

void Ctx::ensure_work(int64_t N, int L, bool cplx, bool mixed, int lz_steps, int lz_nvec) {
  ensure_init();
  if (w.base && w.N == N && w.L == L && w.cplx == cplx && w.mixed == mixed &&
      w.lz_steps == lz_steps && w.lz_nvec == lz_nvec)
    return;
  Layout lo = layout(N, L, cplx, mixed, lz_steps, lz_nvec);
  if (w.base == nullptr || w.bytes < lo.total) {
    if (w.base) {
      CHASE_HIP(hipStreamSynchronize(stream));
      CHASE_HIP(hipFree(w.base));
      w.base = nullptr;
      w.bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, lo.total) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of " + std::to_string(lo.total) + " bytes of workspace failed");
      throw OutOfMemory();
    }
    w.base = (char *)p;
    w.bytes = lo.total;
  }
  w.N = N;
  w.L = L;
  w.cplx = cplx;
  w.mixed = mixed;
  w.lz_steps = lz_steps;
  w.lz_nvec = lz_nvec;
  w.nsplit = gram_splits(N, L);
  w.lz_split = lz_splits(N);
  char *b = w.base;
  int i = 0;
  w.X0 = b + lo.off[i++]; w.B1 = b + lo.off[i++]; w.B2 = b + lo.off[i++]; w.Xq = b + lo.off[i++];
  w.P = b + lo.off[i++];
  w.G = b + lo.off[i++]; w.R = b + lo.off[i++]; w.Ri = b + lo.off[i++]; w.T = b + lo.off[i++];
  w.A = b + lo.off[i++];
  w.theta = (double *)(b + lo.off[i++]); w.resid = (double *)(b + lo.off[i++]);
  w.E = (double *)(b + lo.off[i++]); w.trace = (double *)(b + lo.off[i++]);
  w.flag = (int *)(b + lo.off[i++]);
  w.perm = (int *)(b + lo.off[i++]); w.rinfo = (int *)(b + lo.off[i++]);
  w.tau = b + lo.off[i++];
  w.H32 = mixed ? (void *)(b + lo.off[i]) : nullptr; i++;
  w.LV = b + lo.off[i++]; w.LW = b + lo.off[i++]; w.Lh = b + lo.off[i++]; w.LhP = b + lo.off[i++];
  w.lz_ab = (double *)(b + lo.off[i++]);
  w.SK = b + lo.off[i++];
  w.sk_bytes = kTailScratch;
  w.hh = b + lo.off[i++];
  w.eg_d = (double *)(b + lo.off[i++]);
  w.eg_e = (double *)(b + lo.off[i++]);
  w.eg_p[0] = b + lo.off[i++];
  w.eg_p[1] = b + lo.off[i++];
  w.eg_T = b + lo.off[i++];
  {
    double *dd = (double *)(b + lo.off[i]);
    int *ii = (int *)(b + lo.off[i] + al(8 * (size_t)L * 5));
    w.dc.dl = dd; w.dc.zl = dd + L; w.dc.tsec = dd + 2 * (size_t)L;
    w.dc.zh = dd + 3 * (size_t)L; w.dc.dval = dd + 4 * (size_t)L;
    w.dc.org = ii; w.dc.src_nd = ii + L; w.dc.src_df = ii + 2 * (size_t)L;
    w.dc.srcbuf = ii + 3 * (size_t)L; w.dc.kcnt = ii + 4 * (size_t)L;
    ++i;
  }
  // pinned host mirrors, grown on demand
  const int lz_cols = std::max(lz_steps, 1) * std::max(lz_nvec, 1);
  if (L > h_cap_L || lz_cols > h_cap_lz) {
    CHASE_HIP(hipStreamSynchronize(stream));
    free_pinned();
    h_cap_L = std::max(L, h_cap_L);
    h_cap_lz = std::max(lz_cols, h_cap_lz);
    CHASE_HIP(hipHostMalloc((void **)&w.h_theta, 8 * (size_t)h_cap_L));
    CHASE_HIP(hipHostMalloc((void **)&w.h_resid, 8 * (size_t)h_cap_L));
    CHASE_HIP(hipHostMalloc((void **)&w.h_ab, 16 * (size_t)h_cap_lz));
    CHASE_HIP(hipHostMalloc((void **)&w.h_flag, 16));
    CHASE_HIP(hipHostMalloc((void **)&w.h_aux, 32));
    CHASE_HIP(hipHostMalloc((void **)&w.h_perm, 4 * (size_t)h_cap_L));
  }
}

void Ctx::free_pinned() {
  if (w.h_theta) (void)hipHostFree(w.h_theta);
  if (w.h_resid) (void)hipHostFree(w.h_resid);
  if (w.h_ab) (void)hipHostFree(w.h_ab);
  if (w.h_flag) (void)hipHostFree(w.h_flag);
  if (w.h_aux) (void)hipHostFree(w.h_aux);
  if (w.h_perm) (void)hipHostFree(w.h_perm);
  w.h_theta = w.h_resid = w.h_ab = w.h_aux = nullptr;
  w.h_flag = w.h_perm = nullptr;
  h_cap_L = h_cap_lz = 0;
}

void Ctx::release() {
  if (w.base) (void)hipFree(w.base);
  free_pinned();
  w = Work();
  if (init) {
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (own_stream) (void)hipStreamDestroy(stream);
  }
  init = false;
  stream = nullptr;
  own_stream = false;
}

Ctx &thread_ctx() {
  static thread_local Ctx *c = new Ctx();  // lives until the process ends
  return *c;
}

// ------------------------------------------------------------------ steps --
static GemmArgs gargs() {
  GemmArgs a;
  std::memset(&a, 0, sizeof(a));
  a.alpha = 1.0;
  return a;
}

// Arguments of a big-tile GEMM, with the remainder-split scratch attached.
static GemmArgs bigargs(Ctx &c) {
  GemmArgs a = gargs();
  a.tail_ws = c.w.SK;
  a.tail_ws_bytes = c.w.sk_bytes;
  return a;
}

// Alg. 4 with per-vector degrees: one filter-GEMM launch per degree step,
// each on the active suffix of the degree-sorted block.  V (read only
// unless it is one of bufs) holds the input columns; the steps' outputs
// rotate through the three buffers: step 1 reads V and writes bufs[0],
// step 2 reads bufs[0] (previous V) and writes bufs[1], step i >= 3 reads
// bufs[(i - 2) % 3] (previous bufs[(i - 3) % 3]) and writes
// bufs[(i - 1) % 3].  Passing V == bufs[2] makes it a ring of three buffers.
// Column a's last step (degree m_a) writes out[:, a] instead.
int filter_enqueue(hipStream_t st, void *tail_ws, size_t tail_bytes, bool cplx, bool f32,
                   const void *H, int64_t ldh, int64_t N, const void *V, int64_t ldv,
                   void *const bufs[3], int64_t ldb, int ncols, const int *deg_sorted, double cc,
                   double e, double gamma, void *out, int64_t ldo) {
  if (ncols <= 0) return 0;
  const double sigma1 = e / (gamma - cc);
  double s = sigma1, sprev = 0.0;
  const int mmax = deg_sorted[ncols - 1];
  int launches = 0;
  auto first_at_least = [&](int d) {
    return (int)(std::lower_bound(deg_sorted, deg_sorted + ncols, d) - deg_sorted);
  };
  for (int step = 1; step <= mmax; ++step) {
    const int start = first_at_least(step);
    GemmArgs a = gargs();
    a.tail_ws = tail_ws;
    a.tail_ws_bytes = tail_bytes;
    a.A = H; a.lda = ldh;
    if (step == 1) {
      a.B = V; a.ldb = ldv;
    } else {
      a.B = bufs[(step - 2) % 3]; a.ldb = ldb;
    }
    a.M = (int)N; a.N = ncols - start; a.K = (int)N;
    a.col0 = start;
    a.alpha = (step == 1 ? 1.0 : 2.0) * s / e;
    a.beta = step == 1 ? 0.0 : -sprev * s;
    a.shift = cc;
    if (step == 2) {
      a.Xprev = V; a.ldp = ldv;
    } else if (step > 2) {
      a.Xprev = bufs[(step - 3) % 3]; a.ldp = ldb;
    }
    a.Onext = bufs[(step - 1) % 3]; a.ldn = ldb;
    a.Ofinal = out; a.ldf = ldo;
    a.final_end = first_at_least(step + 1);
    launches += gemm(cplx, f32, true, true, true, GEMM_BIG, a, 1, st);
    sprev = s;
    s = 1.0 / (2.0 / sigma1 - s);
  }
  CHASE_HIP(hipGetLastError());
  return launches;
}

int filter(Ctx &c, bool cplx, bool f32, const void *H, int64_t ldh, int64_t N, void *bufs[3],
           int64_t ldb, int ncols, const std::vector<int> &deg_sorted, double cc, double e,
           double gamma, void *out, int64_t ldo) {
  // bufs[0] holds the input; it is the ring's third buffer
  void *const ring[3] = {bufs[1], bufs[2], bufs[0]};
  return filter_enqueue(c.stream, c.w.SK, c.w.sk_bytes, cplx, f32, H, ldh, N, bufs[0], ldb, ring,
                        ldb, ncols, deg_sorted.data(), cc, e, gamma, out, ldo);
}

// Tile shape of the K-split products X^H Y (Gram matrices, V^H C).
#ifndef CHASE_GRAM_SHAPE
#define CHASE_GRAM_SHAPE GEMM_BIG
#endif

// G = X^H X (upper triangle by tiles, deterministic split-K) -> Hermitian G.
static void gram(Ctx &c, bool cplx, const void *X, int64_t ldx, int64_t N, int L, void *G,
                 int average_with_B, const void *B = nullptr, int64_t ldB = 0,
                 bool qr_flag = true) {
  Work &w = c.w;
  // partials buffer holds w.nsplit * w.L^2 elements: never use more splits
  const int64_t cap = (int64_t)w.nsplit * w.L * w.L / ((int64_t)L * L);
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(gram_splits(N, L), cap));
  const int bk = gemm_bk();
  GemmArgs a = gargs();
  a.A = X; a.lda = ldx;
  a.B = B ? B : X; a.ldb = B ? ldB : ldx;
  a.M = L; a.N = L; a.K = (int)N;
  a.tri = average_with_B ? 0 : 1;
  a.k_per_split = (int)(((N + ns - 1) / ns + bk - 1) / bk * bk);
  a.C = w.P; a.ldc = L; a.split_stride = (int64_t)L * L;
  a.flag = (average_with_B || !qr_flag) ? nullptr : w.flag;
  gemm(cplx, false, true, false, false, CHASE_GRAM_SHAPE, a, ns, c.stream);
  reduce_hermitian(cplx, w.P, ns, (int64_t)L * L, L, L, G, L, average_with_B, c.stream);
}

// Blocked right-looking Cholesky G = R^H R (upper), R^{-1} alongside.
static void potrf(Ctx &c, bool cplx, int L, int pass, int inject) {
  Work &w = c.w;
  const int nb = 64;
  const int nbk = (L + nb - 1) / nb;
  fill_zero(cplx, w.Ri, L, L, L, c.stream);
  for (int p = 0; p < nbk; ++p) {
    const int p0 = p * nb, b = std::min(nb, L - p0);
    chol_diag(cplx, w.G, L, w.R, L, w.Ri, L, p0, b, w.flag, pass, inject && p == 0, c.stream);
    const int rest = L - p0 - b;
    if (rest <= 0) continue;
    const size_t es = cplx ? 16 : 8;
    {  // R[p-block, right] = Ri_pp^H G[p-block, right]
      GemmArgs a = gargs();
      a.A = (char *)w.Ri + es * ((size_t)p0 + (size_t)p0 * L); a.lda = L;
      a.B = (char *)w.G + es * p0; a.ldb = L; a.col0 = p0 + b;
      a.M = b; a.N = rest; a.K = b;
      a.C = (char *)w.R + es * p0; a.ldc = L; a.ccol0 = p0 + b;
      a.flag = w.flag;
      gemm(cplx, false, true, false, false, GEMM_SMALL, a, 1, c.stream);
    }
    {  // G[right, right] -= R[p-block, right]^H R[p-block, right]
      GemmArgs a = gargs();
      a.A = (char *)w.R + es * ((size_t)p0 + (size_t)(p0 + b) * L); a.lda = L;
      a.B = (char *)w.R + es * p0; a.ldb = L; a.col0 = p0 + b;
      a.M = rest; a.N = rest; a.K = b;
      a.C = (char *)w.G + es * (p0 + b); a.ldc = L; a.ccol0 = p0 + b;
      a.alpha = -1.0; a.beta = 1.0; a.tri = 1;
      a.flag = w.flag;
      gemm(cplx, false, true, false, false, GEMM_SMALL, a, 1, c.stream);
    }
  }
  // off-diagonal blocks of R^{-1}, left to right:
  // Ri[0:J, J-block] = -(Ri[0:J, 0:J] R[0:J, J-block]) Ri_JJ
  const size_t es = cplx ? 16 : 8;
  for (int jb = 1; jb < nbk; ++jb) {
    const int J = jb * nb, b = std::min(nb, L - J);
    {
      GemmArgs a = gargs();
      a.A = w.Ri; a.lda = L;
      a.B = w.R; a.ldb = L; a.col0 = J;
      a.M = J; a.N = b; a.K = J;
      a.C = w.T; a.ldc = J; a.ccol0 = 0;
      a.flag = w.flag;
      gemm(cplx, false, false, false, false, GEMM_SMALL, a, 1, c.stream);
    }
    {
      GemmArgs a = gargs();
      a.A = w.T; a.lda = J;
      a.B = (char *)w.Ri + es * J; a.ldb = L; a.col0 = J;
      a.M = J; a.N = b; a.K = b;
      a.C = w.Ri; a.ldc = L; a.ccol0 = J;
      a.alpha = -1.0;
      a.flag = w.flag;
      gemm(cplx, false, false, false, false, GEMM_SMALL, a, 1, c.stream);
    }
  }
}

// Xout = Xin R^{-1} (R^{-1} upper triangular: K range capped per column block).
static void trsm(Ctx &c, bool cplx, const void *Xin, void *Xout, int64_t ld, int64_t N, int L) {
  GemmArgs a = bigargs(c);
  a.A = Xin; a.lda = ld;
  a.B = c.w.Ri; a.ldb = L;
  a.M = (int)N; a.N = L; a.K = L;
  a.kcap = 1;
  a.C = Xout; a.ldc = ld;
  a.flag = c.w.flag;
  gemm(cplx, false, false, false, false, GEMM_BIG, a, 1, c.stream);
}

// Split count of a K-split product with `tiles` output tiles over K rows.
static int ksplits(int64_t K, int tiles) {
  int s = (1024 + tiles - 1) / tiles;
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / kSplitRows));
  return std::max(1, std::min(s, kMaxSplits));
}

// C (Mp x n) <- (I - V op(T) V^H) C with op(T) = T^H (trans) or T: the block
// reflector of one panel (V: Mp x nbp with explicit unit diagonal; T: nbp x
// nbp, leading dimension nbp).  W = V^H C goes through K-split partials in P
// and lands in Ri, op(T) W in A.
static void apply_block_reflector(Ctx &c, bool cplx, const void *V, int64_t ldv, int64_t Mp,
                                  int nbp, const void *T, bool trans, void *C, int64_t ldc,
                                  int n) {
  Work &w = c.w;
  const int64_t cap = (int64_t)w.nsplit * w.L * w.L / ((int64_t)nbp * n);
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(ksplits(Mp, (n + 63) / 64), cap));
  const int bk = gemm_bk();
  {
    GemmArgs a = gargs();
    a.A = V; a.lda = ldv;
    a.B = C; a.ldb = ldc;
    a.M = nbp; a.N = n; a.K = (int)Mp;
    a.k_per_split = (int)(((Mp + ns - 1) / ns + bk - 1) / bk * bk);
    a.C = w.P; a.ldc = nbp; a.split_stride = (int64_t)nbp * n;
    gemm(cplx, false, true, false, false, CHASE_GRAM_SHAPE, a, ns, c.stream);
    sum_splits(cplx, w.P, ns, (int64_t)nbp * n, nbp, nbp, n, w.Ri, nbp, c.stream);
  }
  {
    GemmArgs a = gargs();
    a.A = T; a.lda = nbp;
    a.B = w.Ri; a.ldb = nbp;
    a.M = nbp; a.N = n; a.K = nbp;
    a.C = w.A; a.ldc = nbp;
    gemm(cplx, false, trans, false, false, GEMM_SMALL, a, 1, c.stream);
  }
  {
    GemmArgs a = bigargs(c);
    a.A = V; a.lda = ldv;
    a.B = w.A; a.ldb = nbp;
    a.M = (int)Mp; a.N = n; a.K = nbp;
    a.C = C; a.ldc = ldc;
    a.alpha = -1.0; a.beta = 1.0;
    gemm(cplx, false, false, false, false, GEMM_BIG, a, 1, c.stream);
  }
}

// Width of the block reflectors of the Householder QR (a multiple of the
// column-step panel width, at most kHhMaxOuter).
#ifndef CHASE_HH_OUTER
#define CHASE_HH_OUTER 128
#endif
// 1: a panel's column steps in one cooperative launch when its rows fit
#ifndef CHASE_HH_PANEL
#define CHASE_HH_PANEL 1
#endif

// Blocked Householder QR of X (N x L) in the geqrf convention, then the
// explicit Q (the first L columns of H_0 ... H_{L-1}) in X, as orgqr/ungqr
// form it.  Two levels of blocking: column steps (hh_column) factor panels
// of nbi columns, whose block reflectors update the rest of their outer
// panel of nbo columns; the outer panel's block reflector (its compact WY
// factor T from V^H V) then updates the trailing columns, where the
// products are wide enough for the MFMA tiles.  Q is accumulated from the
// identity with the outer block reflectors, last panel first.  V (N x L,
// leading dimension ld) receives the reflector vectors; the outer T of
// panel p sits at G + p nbo^2; tau in w.tau.
static void householder(Ctx &c, bool cplx, void *X, void *V, int64_t ld, int64_t N, int L) {
  if (L <= 0) return;
  Work &w = c.w;
  const size_t es = cplx ? 16 : 8;
  // widths <= L / 2 keep the T store (ceil(L / nbo) nbo^2) and W (nbo x L)
  // within the L x L buffers
  const int nbi = std::max(1, std::min(kHhNB, L / 2));
  const int nbo = std::max(nbi, std::min(CHASE_HH_OUTER, L / 2) / nbi * nbi);
  const int np = (L + nbo - 1) / nbo;
  auto at = [&](void *B, int64_t r, int64_t col) { return (char *)B + es * (r + col * ld); };
  auto tstore = [&](int p) { return (char *)w.G + es * (size_t)p * nbo * nbo; };
  fill_zero(cplx, V, ld, (int)N, L, c.stream);
  fill_zero(false, w.flag, 1, 1, 1, c.stream);  // the Gram's skip flag
  hh_panel_reset(w.hh, c.stream);
  unsigned hp_base = 0;
  for (int p = 0; p < np; ++p) {
    const int j0 = p * nbo, nbop = std::min(nbo, L - j0);
    for (int jq = j0; jq < j0 + nbop; jq += nbi) {
      const int nbq = std::min(nbi, j0 + nbop - jq);
      const int64_t Mq = N - jq;
      void *Vq = at(V, jq, jq);
      void *tq = (char *)w.tau + es * jq;
      // the panel's column steps in one launch, or one launch per step when
      // its rows do not fit the blocks' LDS
      if (!CHASE_HH_PANEL ||
          !hh_panel(cplx, at(X, jq, jq), ld, (int)Mq, nbq, Vq, ld, tq, w.hh, &hp_base, c.stream))
        for (int jj = 0; jj <= nbq; ++jj)
          hh_column(cplx, at(X, jq, jq), ld, (int)Mq, nbq, jj, Vq, ld, tq, w.hh, c.stream);
      const int rest = j0 + nbop - jq - nbq;
      if (rest > 0) {
        gram(c, cplx, Vq, ld, Mq, nbq, w.T, 0);  // S = V^H V
        hh_larft(cplx, w.T, nbq, tq, w.R, nbq, nbq, c.stream);
        apply_block_reflector(c, cplx, Vq, ld, Mq, nbq, w.R, true, at(X, jq, jq + nbq), ld, rest);
      }
    }
    const int nt = L - j0 - nbop;
    gram(c, cplx, at(V, j0, j0), ld, N - j0, nbop, w.T, 0);
    hh_larft(cplx, w.T, nbop, (char *)w.tau + es * j0, tstore(p), nbop, nbop, c.stream);
    if (nt > 0)
      apply_block_reflector(c, cplx, at(V, j0, j0), ld, N - j0, nbop, tstore(p), true,
                            at(X, j0, j0 + nbop), ld, nt);
  }
  set_identity(cplx, X, ld, (int)N, L, c.stream);
  for (int p = np - 1; p >= 0; --p) {
    const int j0 = p * nbo, nbop = std::min(nbo, L - j0);
    apply_block_reflector(c, cplx, at(V, j0, j0), ld, N - j0, nbop, tstore(p), false,
                          at(X, j0, j0), ld, L - j0);
  }
  // the panel launches' time-out flag (sticky on the device since the
  // caller's hh_panel_clear_error), read after the caller's synchronisation
  CHASE_HIP(hipMemcpyAsync(w.h_flag + 3, hh_panel_error(w.hh), 4, hipMemcpyDeviceToHost,
                           c.stream));
  CHASE_HIP(hipGetLastError());
}

// Alg. 3 for one variant.  The passes of CholeskyQR (Alg. 2) alternate
// between X and Xalt; after a failed Cholesky every later kernel of the QR
// sees the flag and does nothing, so the input of the failing pass is intact
// and the Householder QR is applied to it.  The flag (and, on the shifted
// branch, ||X||_F^2 and the shift) are copied to pinned host memory on the
// stream; qr_finish reads them once the caller has synchronised.
QrPending qr_enqueue(Ctx &c, bool cplx, void *X, void *Xalt, int64_t ld, int64_t N, int L,
                     chase_qr variant, int inject) {
  Work &w = c.w;
  QrPending p;
  std::memset(&p, 0, sizeof(p));
  p.X = X;
  p.Xalt = Xalt;
  p.variant = variant;
  w.h_flag[0] = w.h_flag[1] = 0;
  w.h_aux[0] = w.h_aux[1] = NAN;
  if (variant == CHASE_QR_HOUSEHOLDER) {
    householder(c, cplx, X, Xalt, ld, N, L);
    p.npass = 0;
    p.out = X;
    return p;
  }
  p.npass = variant == CHASE_QR_CHOL1 ? 1 : variant == CHASE_QR_CHOL2 ? 2 : 3;
  const bool shifted = variant == CHASE_QR_SHIFTED;
  fill_zero(false, w.flag, 1, 1, 1, c.stream);  // two ints
  void *in = X;
  // shift s = 11 (N L + L (L + 1)) u ||X||_F^2 with ||X||_F^2 = trace(X^H X)
  const double coef = 11.0 * ((double)N * L + (double)L * (L + 1)) * kUnitRoundoff;
  for (int q = 0; q < p.npass; ++q) {
    void *out = (in == X) ? Xalt : X;
    p.inputs[q] = in;
    gram(c, cplx, in, ld, N, L, w.G, 0);
    if (shifted && q == 0) trace_shift(cplx, w.G, L, L, coef, 1, w.trace, w.flag, c.stream);
    potrf(c, cplx, L, q, inject && q == 0);
    trsm(c, cplx, in, out, ld, N, L);
    in = out;
  }
  p.out = in;
  CHASE_HIP(hipGetLastError());
  CHASE_HIP(hipMemcpyAsync(w.h_flag, w.flag, 8, hipMemcpyDeviceToHost, c.stream));
  if (shifted)
    CHASE_HIP(hipMemcpyAsync(w.h_aux, w.trace, 16, hipMemcpyDeviceToHost, c.stream));
  return p;
}

QrOut qr_finish(Ctx &c, bool cplx, const QrPending &p, int64_t ld, int64_t N, int L) {
  Work &w = c.w;
  const double fro2 = p.variant == CHASE_QR_SHIFTED ? w.h_aux[0] : NAN;
  const double shift = p.variant == CHASE_QR_SHIFTED ? w.h_aux[1] : NAN;
  if (p.npass > 0 && w.h_flag[0] != 0) {
    const int fp = std::min(std::max(w.h_flag[1], 0), p.npass - 1);
    void *in = p.inputs[fp];
    householder(c, cplx, in, in == p.X ? p.Xalt : p.X, ld, N, L);
    return {in, true, CHASE_QR_HOUSEHOLDER, fro2, shift};
  }
  return {p.out, false, p.variant, fro2, shift};
}

QrOut qr(Ctx &c, bool cplx, void *X, void *Xalt, int64_t ld, int64_t N, int L, chase_qr variant,
         int inject) {
  QrPending p = qr_enqueue(c, cplx, X, Xalt, ld, N, L, variant, inject);
  CHASE_HIP(hipStreamSynchronize(c.stream));
  return qr_finish(c, cplx, p, ld, N, L);
}

// Eigenvalues (ascending, into w.theta) and eigenvectors of the Hermitian
// n x n matrix A (ld n, destroyed) on the device; returns the eigenvector
// matrix (n x n, ld n): A itself for n <= kEigQrMax, else w.R.  w.rinfo is
// set to 1 if a tridiagonal QR (small orders, leaves) did not converge.
// Above kEigQrMax: Householder reduction T = Q^H A Q (one launch per column
// down to kEigSmallMax remaining columns, the rest in one work-group),
// divide and conquer on T (the leaves by tridiagonal QR, each level's
// rank-one merges batched, their products Z = Q_hat U batched for small
// merges and on the MFMA GEMM core for large ones), then X = Q Z (one
// work-group up to kEigSmallMax, else block reflectors of kHhMaxOuter
// columns, last first).
// Buffers: V = w.G; the divide and conquer's Z ping-pong in w.Ri / w.T, the
// gathered columns in w.P, U in w.R, the products in w.A; X in w.R.
static const void *heevd(Ctx &c, bool cplx, void *A, int n) {
  Work &w = c.w;
  hipStream_t st = c.stream;
  const size_t es = cplx ? 16 : 8;
  fill_zero(false, w.rinfo, 1, 1, 1, st);
  if (n <= kEigQrMax) {
    heev_small(cplx, A, n, n, w.theta, w.rinfo, st);
    return A;
  }
  if (n > kEigMaxN) {
    set_error("Rayleigh-Ritz: " + std::to_string(n) + " columns exceed the eigensolver's " +
              std::to_string(kEigMaxN));
    throw InvalidArg();
  }
  // 1. reduction to tridiagonal form: one launch per column while more than
  // kEigSmallMax columns remain, the rest in one work-group
  fill_zero(cplx, w.G, n, n, n, st);
  const int j0 = std::max(0, n - kEigSmallMax);
  for (int j = 0; j < j0; ++j)
    hetrd_step(cplx, A, n, n, j, w.G, n, w.tau, w.eg_d, w.eg_e, w.eg_p[(j + 1) & 1],
               w.eg_p[j & 1], st);
  hetrd_tail(cplx, A, n, n, j0, w.G, n, w.tau, w.eg_d, w.eg_e, w.eg_p[(j0 + 1) & 1], st);
  // 2. divide and conquer
  const int D = dc_depth(n);
  double *Zc = (double *)w.Ri, *Zn = (double *)w.T;
  double *Qg = (double *)w.P, *U = (double *)w.R, *Zk = (double *)A;
  fill_zero(false, Zc, n, n, n, st);
  fill_zero(false, Zn, n, n, n, st);
  dc_leaves(w.eg_d, w.eg_e, n, D, w.theta, Zc, w.rinfo, st);
  for (int t = D - 1; t >= 0; --t) {
    dc_merge_pre(w.eg_e, n, t, w.theta, Zc, Qg, U, w.dc, st);
    if (((n + (1 << t) - 1) >> t) <= kDcGemmSmall) {
      dc_gemm_small(Qg, U, Zk, n, t, st);
    } else for (int i = 0; i < (1 << t); ++i) {
      const int s0 = (int)(((int64_t)i * n) >> t);
      const int nn = (int)(((int64_t)(i + 1) * n) >> t) - s0;
      GemmArgs a = gargs();
      a.A = Qg + s0 + (size_t)s0 * n; a.lda = n;
      a.B = U + (size_t)s0 * n; a.ldb = n;
      a.M = nn; a.N = nn; a.K = nn;
      a.C = Zk + s0 + (size_t)s0 * n; a.ldc = n;
      gemm(false, false, false, false, false, nn >= 256 ? GEMM_BIG : GEMM_SMALL, a, 1, st);
    }
    dc_merge_post(n, t, w.theta, Zk, Zc, Zn, w.dc, st);
    std::swap(Zc, Zn);
  }
  // 3. X = H_0 ... H_{n-2} Z
  void *X = w.R;
  if (n <= kEigSmallMax) {
    ormtr_small(cplx, w.G, n, w.tau, Zc, n, n, X, n, st);
    CHASE_HIP(hipGetLastError());
    return X;
  }
  real_to_elem(cplx, Zc, n, X, n, st);
  const int nb = kHhMaxOuter;
  for (int j0 = (n - 2) / nb * nb; j0 >= 0; j0 -= nb) {
    const int nbp = std::min(nb, n - 1 - j0);
    const int64_t Mp = n - 1 - j0;
    const void *Vp = (const char *)w.G + es * ((size_t)(j0 + 1) + (size_t)j0 * n);
    gram(c, cplx, Vp, n, Mp, nbp, w.T, 0, nullptr, 0, false);  // V^H V
    hh_larft(cplx, w.T, nbp, (const char *)w.tau + es * j0, w.eg_T, nbp, nbp, st);
    apply_block_reflector(c, cplx, Vp, n, Mp, nbp, w.eg_T, false, (char *)X + es * (j0 + 1), n,
                          n);
  }
  CHASE_HIP(hipGetLastError());
  return X;
}

// Rayleigh-Ritz on the orthonormal Q (N x Lp): W = H Q, A~ = Q^H W
// symmetrised, (theta, Z) = eigh(A~), V = Q Z, HV = W Z.
void rayleigh_ritz(Ctx &c, bool cplx, const void *H, int64_t ldh, int64_t N, const void *Q,
                   int64_t ldq, int Lp, void *W, void *Vout, int64_t ldv, void *HV, int64_t ldhv) {
  Work &w = c.w;
  {
    GemmArgs a = bigargs(c);
    a.A = H; a.lda = ldh;
    a.B = Q; a.ldb = ldq;
    a.M = (int)N; a.N = Lp; a.K = (int)N;
    a.C = W; a.ldc = N;
    gemm(cplx, false, true, false, false, GEMM_BIG, a, 1, c.stream);
  }
  gram(c, cplx, Q, ldq, N, Lp, w.A, 1, W, N);
  const void *Z = heevd(c, cplx, w.A, Lp);
  {
    GemmArgs a = bigargs(c);
    a.A = Q; a.lda = ldq;
    a.B = Z; a.ldb = Lp;
    a.M = (int)N; a.N = Lp; a.K = Lp;
    a.C = Vout; a.ldc = ldv;
    gemm(cplx, false, false, false, false, GEMM_BIG, a, 1, c.stream);
  }
  {
    GemmArgs a = bigargs(c);
    a.A = W; a.lda = N;
    a.B = Z; a.ldb = Lp;
    a.M = (int)N; a.N = Lp; a.K = Lp;
    a.C = HV; a.ldc = ldhv;
    gemm(cplx, false, false, false, false, GEMM_BIG, a, 1, c.stream);
  }
  CHASE_HIP(hipGetLastError());
}

// Small orders take the one-launch Lanczos (lanczos_coop) unless this is 0.
#ifndef CHASE_LZ_COOP
#define CHASE_LZ_COOP 1
#endif

// nvec independent Lanczos runs of k steps, each with full
// reorthogonalisation against its own basis (classical Gram-Schmidt, twice),
// advanced together so that every step streams H once for all of them.  The
// runs' basis vectors are interleaved step by step: column j * nvec + r of LV
// is run r's j-th vector, so the first (j + 1) nvec columns are every run's
// basis so far.  Run r's coefficients come back on the host at
// alpha/beta[r * k + j].
void lanczos(Ctx &c, bool cplx, const void *H, int64_t ldh, int64_t N, const void *V0, int nvec,
             int steps, uint64_t seed, std::vector<double> &alpha, std::vector<double> &beta) {
  Work &w = c.w;
  const int k = (int)std::min<int64_t>(steps, N);
  const int nv = nvec;
  const size_t es = cplx ? 16 : 8;
  const int nsl = lz_splits(N);
  const int bk = gemm_bk();
  const int64_t ldh_ = k * nv;  // leading dimension of the coefficient blocks
  if (V0)
    CHASE_HIP(hipMemcpyAsync(w.LW, V0, es * N * nv, hipMemcpyDeviceToDevice, c.stream));
  else
    randn(cplx, w.LW, N, (int)N, nv, seed, c.stream);
  norm_scale_cols(cplx, w.LW, N, (int)N, nv, w.LV, N, w.lz_ab + (size_t)k * nv, c.stream);
  // small orders: every step in one cooperative launch, else the steps
  // after the product in one launch each (one work-group per run); larger
  // orders: several wide launches per step
  const bool small = N <= kLzSmallMaxN && k + 1 <= kLzSmallMaxBasis;
  bool coop = false;
  if (small && CHASE_LZ_COOP) {
    hh_panel_clear_error(w.hh, c.stream);
    coop = lanczos_coop(cplx, H, ldh, (int)N, k, nv, w.LV, w.LW, w.lz_ab, w.SK, w.sk_bytes, w.hh,
                        c.stream);
    if (coop)
      CHASE_HIP(hipMemcpyAsync(w.h_flag + 3, hh_panel_error(w.hh), 4, hipMemcpyDeviceToHost,
                               c.stream));
  }
  for (int j = 0; j < k && !coop; ++j) {
    const int nb = (j + 1) * nv;  // basis vectors so far, all runs
    void *Vj = (char *)w.LV + es * (size_t)N * j * nv;
    gemv_block(cplx, H, ldh, (int)N, (int)N, Vj, N, nv, w.LW, N, w.SK, w.sk_bytes, c.stream);
    if (small) {
      lz_step_small(cplx, w.LV, N, (int)N, j, nv, w.LW, N, w.lz_ab, k, c.stream);
      continue;
    }
    dot_re_cols(cplx, Vj, w.LW, N, (int)N, nv, w.lz_ab + (size_t)j * nv, c.stream);
    for (int rep = 0; rep < 2; ++rep) {
      GemmArgs a = gargs();
      a.A = w.LV; a.lda = N;
      a.B = w.LW; a.ldb = N;
      a.M = nb; a.N = nv; a.K = (int)N;
      a.k_per_split = (int)(((N + nsl - 1) / nsl + bk - 1) / bk * bk);
      a.C = w.LhP; a.ldc = ldh_; a.split_stride = ldh_ * nv;
      gemm(cplx, false, true, false, false, GEMM_SMALL, a, nsl, c.stream);
      sum_splits_diag(cplx, w.LhP, nsl, ldh_ * nv, ldh_, nb, nv, w.Lh, ldh_, c.stream);
      GemmArgs b = gargs();
      b.A = w.LV; b.lda = N;
      b.B = w.Lh; b.ldb = ldh_;
      b.M = (int)N; b.N = nv; b.K = nb;
      b.C = w.LW; b.ldc = N;
      b.alpha = -1.0; b.beta = 1.0;
      gemm(cplx, false, false, false, false, GEMM_BIG, b, 1, c.stream);
    }
    // beta_j of every run; v_{j+1} = w / beta_j
    norm_scale_cols(cplx, w.LW, N, (int)N, nv, (char *)w.LV + es * (size_t)N * nb, N,
                    w.lz_ab + (size_t)k * nv + (size_t)j * nv, c.stream);
  }
  CHASE_HIP(hipGetLastError());
  CHASE_HIP(hipMemcpyAsync(w.h_ab, w.lz_ab, 16 * (size_t)k * nv, hipMemcpyDeviceToHost,
                           c.stream));
  CHASE_HIP(hipStreamSynchronize(c.stream));
  if (coop && w.h_flag[3] != 0) {
    set_error("Lanczos: a grid barrier of the one-launch run timed out");
    throw DeviceError();
  }
  alpha.assign((size_t)k * nv, 0.0);
  beta.assign((size_t)k * nv, 0.0);
  for (int r = 0; r < nv; ++r)
    for (int j = 0; j < k; ++j) {
      alpha[(size_t)r * k + j] = w.h_ab[(size_t)j * nv + r];
      beta[(size_t)r * k + j] = w.h_ab[(size_t)k * nv + (size_t)j * nv + r];
    }
}

// -------------------------------------------------------------- the solve --
static double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.0;
  }
  return ms * 1e-3;
}

chase_status solve(Ctx &c, const chase_opts &o, const void *H, int64_t N, int64_t ldh, int nev,
                   int nex, int degree, double tol, double *evals, void *evecs, int64_t ldv,
                   double *resid, chase_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  const bool cplx = o.dtype == CHASE_COMPLEX128;
  const bool mixed = o.precision == CHASE_PREC_MIXED;
  const int L = nev + nex;
  const size_t es = cplx ? 16 : 8;
  const int lz = o.have_bounds ? 0 : std::max(1, o.lanczos_steps);
  const int lzv = std::max(1, o.lanczos_nvec);
  c.ensure_work(N, L, cplx, mixed, lz, lzv);
  Work &w = c.w;
  hipStream_t s = c.stream;
  chase_info inf;
  std::memset(&inf, 0, sizeof(inf));
  w.h_flag[3] = 0;
  hh_panel_clear_error(w.hh, s);

  // spectral bounds (Alg. 1: lambda_1, lambda_l, upper bound of lambda_n)
  double gamma, alpha, beta;
  if (o.have_bounds) {
    gamma = o.lambda_1; alpha = o.lambda_l; beta = o.lambda_max;
  } else {
    CHASE_HIP(hipEventRecord(c.ev[6], s));
    std::vector<double> la, lb;
    lanczos(c, cplx, H, ldh, N, o.lanczos_v0, lzv, lz, o.seed + 0x9E3779B97F4A7C15ull, la, lb);
    CHASE_HIP(hipEventRecord(c.ev[7], s));
    double bd[3];
    lanczos_bounds_from_runs(la, lb, lzv, N, L, bd);
    gamma = bd[0]; alpha = bd[1]; beta = bd[2];
    CHASE_HIP(hipEventSynchronize(c.ev[7]));
    inf.t_lanczos = elapsed(c.ev[6], c.ev[7]);
  }
  inf.lambda_1 = gamma; inf.lambda_l = alpha; inf.lambda_max = beta;

  // start block and step 0 (CholeskyQR2 of the start block)
  if (!o.warm_start) randn(cplx, evecs, ldv, (int)N, L, o.seed, s);
  copy_cols(cplx, evecs, ldv, w.Xq, N, (int)N, L, s);
  {
    QrOut q0 = qr(c, cplx, w.Xq, w.B1, N, N, L, CHASE_QR_CHOL2, 0);
    copy_cols(cplx, q0.Q, N, evecs, ldv, (int)N, L, s);
  }
  if (mixed) convert_to32(cplx, H, ldh, w.H32, N, (int)N, (int)N, s);

  int k = 0;
  std::vector<int> m(L, degree);
  std::vector<double> theta_act, r_act, lam, res_locked;
  double lam1 = gamma;
  int it = 0;
  const double sw = o.mixed_switch * std::max(std::fabs(gamma), std::fabs(beta));
  bool filter32 = mixed;
  double rmin_prev = -1.0;
  for (it = 1; it <= o.max_iter; ++it) {
    const double cc = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
    const int Lp = L - k;
    if (mixed && !theta_act.empty()) {
      // FP32 while the residuals are above the switch point and still fall:
      // an FP32 pass that does not halve the lowest unconverged residual has
      // reached the FP32 floor (about 1e2 u32 ||H||), so FP64 takes over
      const double rmin = *std::min_element(r_act.begin(), r_act.end());
      filter32 = filter32 && rmin > sw && !(rmin_prev > 0.0 && rmin > 0.5 * rmin_prev);
      rmin_prev = rmin;
    }
    const bool f32 = mixed && filter32;
    // after the switch, MIXED keeps the buffer columns (Ritz index >= nev - k
    // among the active ones) in FP32: they need not converge, and the
    // Rayleigh-Ritz step on the whole block only gains from them
    const int nW = (mixed && !filter32 && o.mixed_buffer32) ? nev - k : Lp;
    // degree-sorted order of the active columns (stable), within each group
    std::vector<int> order(Lp);
    std::iota(order.begin(), order.end(), 0);
    auto by_degree = [&](int a, int b) { return m[a] < m[b]; };
    std::stable_sort(order.begin(), order.begin() + nW, by_degree);
    std::stable_sort(order.begin() + nW, order.end(), by_degree);
    // the permutation goes up from its own pinned mirror, which the host
    // rewrites only after the next end-of-iteration synchronisation
    std::vector<int> msorted(Lp);
    for (int a = 0; a < Lp; ++a) {
      msorted[a] = m[order[a]];
      w.h_perm[a] = order[a] + k;
    }
    CHASE_HIP(hipMemcpyAsync(w.perm, w.h_perm, 4 * (size_t)Lp, hipMemcpyHostToDevice, s));
    void *bufs[3] = {w.X0, w.B1, w.B2};
    gather_cols(cplx, f32, evecs, ldv, w.X0, N, (int)N, nW, w.perm, s);
    CHASE_HIP(hipEventRecord(c.ev[0], s));
    const std::vector<int> msW(msorted.begin(), msorted.begin() + nW);
    int nl = filter(c, cplx, f32, f32 ? w.H32 : H, f32 ? N : ldh, N, bufs, N, nW, msW, cc,
                    e, gamma, (char *)w.Xq + es * (size_t)k * N, N);
    CHASE_HIP(hipEventRecord(c.ev[5], s));
    int64_t mv32 = 0;
    int nl32 = f32 ? nl : 0;
    if (nW < Lp) {  // the buffer columns through the FP32 filter
      const std::vector<int> msB(msorted.begin() + nW, msorted.end());
      gather_cols(cplx, true, evecs, ldv, w.X0, N, (int)N, Lp - nW, w.perm + nW, s);
      const int nb = filter(c, cplx, true, w.H32, N, N, bufs, N, Lp - nW, msB, cc, e, gamma,
                            (char *)w.Xq + es * (size_t)(k + nW) * N, N);
      nl += nb;
      nl32 += nb;
      for (int v : msB) mv32 += v;
    }
    CHASE_HIP(hipEventRecord(c.ev[1], s));
    inf.filter_launches += nl;
    inf.filter_launches_fp32 += nl32;
    if (f32) inf.filter_fp32_iters++;
    int64_t mv = 0;
    int mmax = 0, mmin = 1 << 30;
    for (int a = 0; a < Lp; ++a) { mv += m[a]; mmax = std::max(mmax, m[a]); mmin = std::min(mmin, m[a]); }
    inf.matvecs += mv;
    // estimate (1.2): theta_{k+1} = lowest unconverged Ritz value, m[0] its degree
    const double th_next = theta_act.empty() ? gamma : theta_act[0];
    const double lest = log_cond_estimate(th_next, m[0], mmax, lam1, cc, e);
    const double est = lest < 709.0 ? std::exp(lest) : INFINITY;
    chase_qr variant = o.qr_policy == CHASE_QR_AUTO ? select_qr(est, o.est_hi, o.est_lo)
                                                     : o.qr_policy;
    // [Y | filtered]
    if (k > 0) copy_cols(cplx, evecs, ldv, w.Xq, N, (int)N, k, s);
    double kappa = NAN;
    if (o.block_cb) {
      CHASE_HIP(hipStreamSynchronize(s));
      kappa = o.block_cb(w.Xq, N, N, L, it, o.block_user);
    }
    // QR, Rayleigh-Ritz and residuals are enqueued back to back; the QR's
    // failure flag, the eigensolver's info and the Ritz values and residuals
    // come back with one synchronisation.  After a Cholesky failure (rare)
    // the Householder QR runs on the failing pass's input and Rayleigh-Ritz
    // and the residuals are redone on its Q.
    QrPending qp = qr_enqueue(c, cplx, w.Xq, w.B1, N, N, L, variant, o.inject_chol_fail_iter == it);
    CHASE_HIP(hipEventRecord(c.ev[2], s));
    void *Vout = (char *)evecs + es * (size_t)k * ldv;
    auto rr_resid = [&](const void *Qbuf) {
      const void *Q2 = (const char *)Qbuf + es * (size_t)k * N;
      rayleigh_ritz(c, cplx, H, ldh, N, Q2, N, Lp, w.B2, Vout, ldv, w.X0, N);
      CHASE_HIP(hipEventRecord(c.ev[3], s));
      residuals(cplx, w.X0, N, Vout, ldv, (int)N, Lp, w.theta, w.resid, s);
      CHASE_HIP(hipEventRecord(c.ev[4], s));
      CHASE_HIP(hipMemcpyAsync(w.h_theta, w.theta, 8 * (size_t)Lp, hipMemcpyDeviceToHost, s));
      CHASE_HIP(hipMemcpyAsync(w.h_resid, w.resid, 8 * (size_t)Lp, hipMemcpyDeviceToHost, s));
      CHASE_HIP(hipMemcpyAsync(w.h_flag + 2, w.rinfo, 4, hipMemcpyDeviceToHost, s));
      CHASE_HIP(hipStreamSynchronize(s));
    };
    rr_resid(qp.out);
    double t_qr = elapsed(c.ev[1], c.ev[2]), t_rr = elapsed(c.ev[2], c.ev[3]);
    double t_res = elapsed(c.ev[3], c.ev[4]);
    QrOut q = qr_finish(c, cplx, qp, N, N, L);
    if (q.failed) {
      CHASE_HIP(hipEventRecord(c.ev[2], s));  // after the Householder QR of qr_finish
      rr_resid(q.Q);
      t_qr += elapsed(c.ev[4], c.ev[2]);  // approximate: the redo's QR span
      t_rr += elapsed(c.ev[2], c.ev[3]);
      t_res += elapsed(c.ev[3], c.ev[4]);
    }
    if (w.h_flag[3] != 0) {
      set_error("Householder QR: a panel launch's grid barrier timed out");
      throw DeviceError();
    }
    if (w.h_flag[2] != 0) {
      set_error("Rayleigh-Ritz: the projected eigenproblem did not converge (info " +
                std::to_string(w.h_flag[2]) + ")");
      throw DeviceError();
    }
    chase_iter_log rec;
    std::memset(&rec, 0, sizeof(rec));
    rec.t_filter = elapsed(c.ev[0], c.ev[1]);
    rec.t_qr = t_qr;
    rec.t_rr = t_rr;
    rec.t_resid = t_res;
    rec.qr_fro2 = q.fro2;
    rec.qr_shift = q.shift;
    inf.t_filter += rec.t_filter; inf.t_qr += rec.t_qr; inf.t_rr += rec.t_rr;
    if (f32) {
      inf.t_filter_fp32 += rec.t_filter;
      inf.matvecs_fp32 += mv;
    } else if (mv32 > 0) {
      inf.t_filter_fp32 += elapsed(c.ev[5], c.ev[1]);
      inf.matvecs_fp32 += mv32;
    }
    inf.t_resid += rec.t_resid;
    std::vector<double> th(w.h_theta, w.h_theta + Lp), rr(w.h_resid, w.h_resid + Lp);
    int j = k;
    while (j < nev && rr[j - k] < tol) ++j;
    const int newly = j - k;
    for (int a = 0; a < newly; ++a) { lam.push_back(th[a]); res_locked.push_back(rr[a]); }
    rec.iter = it; rec.locked = k; rec.newly_locked = newly; rec.qr_variant = q.ran;
    rec.chol_failed = q.failed;
    rec.filter_prec = (f32 || mv32 > 0) ? CHASE_PREC_MIXED : CHASE_PREC_FP64;
    rec.deg_min = mmin; rec.deg_max = mmax; rec.matvecs = mv; rec.cond_est = est;
    rec.cond_exact = kappa;
    rec.ncols = Lp;
    rec.degrees = msorted.data();
    rec.ncols_fp32 = f32 ? Lp : Lp - nW;
    rec.c = cc; rec.e = e; rec.gamma = gamma; rec.lam1 = lam1;
    if (o.log_cb) o.log_cb(&rec, o.log_user);
    k = j;
    inf.ritz_max = th.back();
    theta_act.assign(th.begin() + newly, th.end());
    r_act.assign(rr.begin() + newly, rr.end());
    if (k >= nev) break;
    lam1 = k > 0 ? lam[0] : th[0];
    gamma = theta_act[0];
    alpha = th.back();
    // beta must bound the spectrum (Sec. 1.2).  A Ritz value never exceeds
    // lambda_n, so one above beta proves the bound wrong: move beta past it
    // by twice its residual (an eigenvalue lies within one residual of it)
    // plus a margin that keeps the damped interval open.  Inert whenever
    // beta is a true bound.
    if (th.back() > beta) {
      beta = th.back() + 2.0 * rr.back() + 1e-3 * (th.back() - th.front());
      inf.lambda_max = beta;
    }
    const double c2 = 0.5 * (alpha + beta), e2 = 0.5 * (beta - alpha);
    m.assign(L - k, degree);
    if (o.deg_opt)
      degrees(theta_act.data(), r_act.data(), L - k, tol, c2, e2, o.min_deg, o.max_deg,
              o.deg_margin, m.data());
  }
  if (it > o.max_iter) it = o.max_iter;
  // outputs
  for (int a = 0; a < nev; ++a) {
    if (a < k) {
      evals[a] = lam[a];
      if (resid) resid[a] = res_locked[a];
    } else {
      evals[a] = theta_act[a - k];
      if (resid) resid[a] = r_act[a - k];
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  inf.iters = it;
  inf.converged = k;
  inf.t_total = std::chrono::duration<double>(t1 - t0).count();
  if (info) *info = inf;
  return k >= nev ? CHASE_OK : CHASE_NOT_CONVERGED;
}

}  // namespace chase
