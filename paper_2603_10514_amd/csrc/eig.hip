// Hermitian eigensolver of the projected Rayleigh-Ritz matrix (Alg. 1 solves
// the l' x l' problem A~ W = W Lambda every iteration): Householder
// reduction to a real symmetric tridiagonal T = Q^H A Q, divide and conquer
// on T (Cuppen's splitting with deflation, the secular equation solved root
// by root, Loewner's formula for the eigenvector components), and the
// back-transform X = Q Z.  Orders up to kEigSmallMax run in one work-group
// with the matrix in LDS; above, one launch per Householder column, the
// divide and conquer levels batched over their merges, and the
// back-transform as block reflectors on the GEMM core (host side in
// solver.cpp).
#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "num.hpp"

namespace chase {

constexpr double kEps = 2.220446049250313e-16;  // 2^-52
constexpr double kRsqMin = 1e-290;  // rsqrt_refined's inputs stay above this

__device__ __forceinline__ double2 make_e(double r, double i, double2 *) { return make_double2(r, i); }
__device__ __forceinline__ double make_e(double r, double, double *) { return r; }
template <typename E> __device__ __forceinline__ E mk(double r, double i) {
  return make_e(r, i, (E *)nullptr);
}

// Sums over the 256 threads of a block in a fixed order (lanes of a wave by
// xor steps, then the four wave sums in order); every thread gets the value.
__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return __shfl(v, 0);
}
__device__ __forceinline__ double wave_max(double v) {
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  return __shfl(v, 0);
}
__device__ __forceinline__ double wave_prod(double v) {
  for (int m = 32; m >= 1; m >>= 1) v *= __shfl_xor(v, m);
  return __shfl(v, 0);
}
__device__ __forceinline__ void wg_sum2(double &a, double &b, double *sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[4 + w] = b;
  }
  __syncthreads();
  a = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  b = (sh[4] + sh[5]) + (sh[6] + sh[7]);
}
__device__ __forceinline__ double wg_max(double a, double *sh) {
  a = wave_max(a);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = a;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// Householder reflector H = I - tau v v^H with H^H (alpha, x)^T = (beta, 0)^T,
// beta real, v = (1, x / (alpha - beta)) (the geqrf convention): from alpha
// and ||x||^2.  tau = 0 and beta = alpha when x = 0 and alpha is real.
template <typename E>
__device__ __forceinline__ void reflector(E alpha, double xn2, E &tau, double &beta, E &scale) {
  typedef Num<E> X;
  const double ar = X::re(alpha), ai = X::im(alpha);
  if (xn2 == 0.0 && ai == 0.0) {
    tau = X::zero();
    beta = ar;
    scale = X::zero();
    return;
  }
  beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
  tau = mk<E>((beta - ar) / beta, -ai / beta);
  // 1 / (alpha - beta)
  const double dr = ar - beta, di = ai, den = dr * dr + di * di;
  scale = mk<E>(dr / den, -di / den);
}

// ------------------------------------------ tridiagonal QR (small orders) --
// v of lane k (k uniform across the wave).
__device__ __forceinline__ double lane_val(double v, int k) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Eigenvalues and eigenvectors of the symmetric tridiagonal (d, e) of order
// m <= 64 held in LDS, by implicit QR steps with the Wilkinson shift (Golub
// & Van Loan, Sec. 8.3), in the first wave of the block: lane i keeps d[i]
// and e[i] in registers, every lane runs the sweep's rotation chain (the
// entries it needs come by lane reads with a uniform index), and lane t < m
// applies each rotation to row t of Z (ldz, initialised by the caller) as
// it is generated, carrying the rotated column in a register.  The
// negligible off-diagonals and the active block come from a wave vote.  On
// return d holds the (unsorted) eigenvalues; ctl[3] = 1 if the sweep limit
// was reached.  Every thread of the block calls it (one barrier at the end).
__device__ void ql_tridiag(double *d, double *e, double *Z, int ldz, int m, int *ctl) {
  const int t = threadIdx.x;
  if (t < 64) {
    const int lane = t;
    const bool row = lane < m;
    double dl = row ? d[lane] : 0.0;
    double el = lane + 1 < m ? e[lane] : 0.0;
    const int max_sweeps = 30 * m + 30;
    int failed = 0;
    for (int sweep = 0;; ++sweep) {
      const double dn = __shfl_down(dl, 1);
      if (lane + 1 < m && fabs(el) <= kEps * (fabs(dl) + fabs(dn))) el = 0.0;
      const unsigned long long nz = __ballot(lane + 1 < m && el != 0.0);
      // the trailing unreduced block is rows lo..hi
      const int hi = nz ? 64 - __clzll((long long)nz) : 0;
      if (hi == 0 || sweep >= max_sweeps) {
        failed = hi != 0;
        break;
      }
      const unsigned long long split = ~nz & ((1ull << (hi - 1)) - 1);
      const int lo = split ? 64 - __clzll((long long)split) : 0;
      const double del = 0.5 * (lane_val(dl, hi - 1) - lane_val(dl, hi));
      const double em = lane_val(el, hi - 1);
      const double mu = lane_val(dl, hi) - em * em / (del + copysign(hypot(del, em), del));
      // p, q: the current d[k], e[k] (already rotated by step k - 1)
      double p = lane_val(dl, lo), q = lane_val(el, lo);
      double x = p - mu, zb = q;
      double zc = row ? Z[lane + lo * ldz] : 0.0;
      for (int k = lo; k < hi; ++k) {
        const double u = lane_val(dl, k + 1);
        const double en = k + 1 < hi ? lane_val(el, k + 1) : 0.0;
        const double zn = row ? Z[lane + (k + 1) * ldz] : 0.0;
        // the entries are of the order of the matrix norm: no scaling
        // against overflow is needed, and one reciprocal square root serves
        // r, c and s (the refined hardware one on the chain; the correctly
        // rounded pair near the bottom of the exponent range)
        const double r2 = x * x + zb * zb;
        double ri = 0.0, r = 0.0;
        if (r2 > kRsqMin) {
          ri = rsqrt_refined(r2);
          r = r2 * ri;
        } else if (r2 > 0.0) {
          r = sqrt(r2);
          ri = 1.0 / r;
        }
        const double c = r2 > 0.0 ? x * ri : 1.0, s = -zb * ri;
        if (k > lo && lane == k - 1) el = r;
        const double dk = c * c * p - 2.0 * c * s * q + s * s * u;
        const double dk1 = s * s * p + 2.0 * c * s * q + c * c * u;
        const double ek = c * s * (p - u) + (c * c - s * s) * q;
        if (lane == k) {
          dl = dk;
          el = ek;
        }
        if (k + 1 < hi) {
          zb = -s * en;
          q = c * en;
          x = ek;
        }
        p = dk1;
        if (row) {
          Z[lane + k * ldz] = c * zc - s * zn;
          zc = s * zc + c * zn;
        }
      }
      if (lane == hi) dl = p;
      if (row) Z[lane + hi * ldz] = zc;
    }
    if (row) {
      d[lane] = dl;
      e[lane] = el;
    }
    if (lane == 0) ctl[3] = failed;
  }
  __syncthreads();
}

// rank[i] = position of d[i] in ascending order (ties by index), i < m.
__device__ __forceinline__ void rank_ascending(const double *d, int m, int *rank) {
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double v = d[i];
    int r = 0;
    for (int j = 0; j < m; ++j) r += (d[j] < v || (d[j] == v && j < i)) ? 1 : 0;
    rank[i] = r;
  }
}

// ------------------------------------------- one work-group (LDS) pieces --
// Householder reduction of the m x m Hermitian matrix in LDS (sA[c][r] =
// A(r, c), m <= MX <= 64) to the tridiagonal (sd, se): step j forms the
// reflector of column j below the diagonal (wave 0, lane = row, the unit
// entry stored with it), p = tau B v with four threads per row, then every
// wave forms kappa = -tau (p^H v) / 2 itself (m <= 64: lane = row, the same
// sum in every wave) and the update B - v w^H - w v^H takes w = p + kappa v
// entry by entry: three barriers per step.  The reflectors stay below the
// subdiagonal of sA (unit entry stored), their tau in stau.  256 threads.
template <typename E, int MX>
__device__ void tridiag_lds(E (*sA)[MX + 1], int m, double *sd, double *se, E *stau, E *sp) {
  typedef Num<E> X;
  static_assert(MX <= 64, "one wave holds a column");
  const int t = threadIdx.x, lane = t & 63;
  for (int j = 0; j + 1 < m; ++j) {
    if (t < 64) {
      const int r = lane;
      const E x = (r >= j + 2 && r < m) ? sA[j][r] : X::zero();
      const double xn2 = wave_sum(X::abs2(x));
      E tau, scale;
      double beta;
      reflector<E>(sA[j][j + 1], xn2, tau, beta, scale);
      if (r >= j + 2 && r < m) sA[j][r] = X::mul(x, scale);
      if (r == j + 1) sA[j][j + 1] = X::real(1.0);
      if (r == 0) {
        stau[j] = tau;
        se[j] = beta;
        sd[j] = X::re(sA[j][j]);
      }
    }
    __syncthreads();
    const E tj = stau[j];
    {
      const int r = t >> 2, q = t & 3;
      E acc = X::zero();
      if (r >= j + 1 && r < m)
        for (int c = j + 1 + q; c < m; c += 4) acc = acc + X::mul(sA[c][r], sA[j][c]);
      acc = X::add_xor(acc, 1);
      acc = X::add_xor(acc, 2);
      if (q == 0 && r < MX) sp[r] = (r >= j + 1 && r < m) ? X::mul(tj, acc) : X::zero();
    }
    __syncthreads();
    E kap;
    {
      const bool in = lane >= j + 1 && lane < m;
      const E pv = in ? X::mul(X::cj(sp[lane]), sA[j][lane]) : X::zero();
      const double sr = wave_sum(X::re(pv)), si = wave_sum(X::im(pv));
      kap = X::scale(X::mul(tj, mk<E>(sr, si)), -0.5);
    }
    const int mm = m - j - 1;
    for (int idx = t; idx < mm * mm; idx += 256) {
      const int r = j + 1 + idx % mm, c = j + 1 + idx / mm;
      const E wr = sp[r] + X::mul(kap, sA[j][r]), wc = sp[c] + X::mul(kap, sA[j][c]);
      sA[c][r] = sA[c][r] - X::mul(sA[j][r], X::cj(wc)) - X::mul(wr, X::cj(sA[j][c]));
    }
    __syncthreads();
  }
  if (t == 0) sd[m - 1] = X::re(sA[m - 1][m - 1]);
  __syncthreads();
}

// X = H_0 ... H_{m-2} Z for the reflectors held in sV (as tridiag_lds leaves
// them) with column c of Z (zload(r, c)) held by the four threads 4c .. 4c+3
// (rows sub, sub + 4, ...); xstore(r, c, value) receives the result.
template <typename E, int MX, typename ZL, typename XS>
__device__ __forceinline__ void backtransform_lds(const E (*sV)[MX + 1], const E *stau, int m,
                                                  ZL zload, XS xstore) {
  typedef Num<E> X;
  const int t = threadIdx.x;
  const int c = t >> 2, sub = t & 3;
  E xr[MX / 4];
#pragma unroll
  for (int k = 0; k < MX / 4; ++k) {
    const int r = sub + 4 * k;
    xr[k] = (c < m && r < m) ? X::real(zload(r, c)) : X::zero();
  }
  for (int j = m - 2; j >= 0; --j) {
    E dot = X::zero();
#pragma unroll
    for (int k = 0; k < MX / 4; ++k) {
      const int r = sub + 4 * k;
      if (r >= j + 1 && r < m) dot = dot + X::mul(X::cj(sV[j][r]), xr[k]);
    }
    dot = X::add_xor(dot, 1);
    dot = X::add_xor(dot, 2);
    const E f = X::mul(stau[j], dot);
#pragma unroll
    for (int k = 0; k < MX / 4; ++k) {
      const int r = sub + 4 * k;
      if (r >= j + 1 && r < m) xr[k] = xr[k] - X::mul(f, sV[j][r]);
    }
  }
  if (c < m) {
#pragma unroll
    for (int k = 0; k < MX / 4; ++k) {
      const int r = sub + 4 * k;
      if (r < m) xstore(r, c, xr[k]);
    }
  }
}

// A (n x n, n <= kEigSmallMax, Hermitian) -> eigenvalues ascending in theta,
// eigenvectors in A's columns: reduction in LDS, tridiagonal QR, back
// transform (for small orders, where the QR's sequential sweeps are short).
template <typename E>
__global__ __launch_bounds__(256) void k_heev_small(E *A, int64_t lda, int n, double *theta,
                                                    int *info) {
  constexpr int MX = kEigSmallMax;
  __shared__ E sA[MX][MX + 1];  // sA[c][r] = A(r, c)
  __shared__ double sZ[MX * (MX + 1)];
  __shared__ double sd[MX], se[MX];
  __shared__ E stau[MX], sp[MX];
  __shared__ int srank[MX], ctl[4];
  const int t = threadIdx.x;
  for (int idx = t; idx < n * n; idx += 256) {
    const int r = idx % n, c = idx / n;
    sA[c][r] = A[r + (int64_t)c * lda];
  }
  __syncthreads();
  tridiag_lds<E, MX>(sA, n, sd, se, stau, sp);
  for (int idx = t; idx < n * (MX + 1); idx += 256) sZ[idx] = 0.0;
  __syncthreads();
  if (t < n) sZ[t + t * (MX + 1)] = 1.0;
  __syncthreads();
  ql_tridiag(sd, se, sZ, MX + 1, n, ctl);
  rank_ascending(sd, n, srank);
  __syncthreads();
  backtransform_lds<E, MX>(
      sA, stau, n, [&](int r, int c) { return sZ[r + c * (MX + 1)]; },
      [&](int r, int c, E v) { A[r + (int64_t)srank[c] * lda] = v; });
  for (int c = t; c < n; c += 256) theta[srank[c]] = sd[c];
  if (t == 0) info[0] = ctl[3];
}

// The last m = n - j0 <= kEigSmallMax columns of the reduction in one
// work-group: the trailing block (with launch j0 - 1's update B - v w^H -
// w v^H applied while it is loaded) is reduced in LDS; its reflectors go to
// V (column j0 + c, rows j0 + c + 1 ..), tau, d and e as the per-column
// launches would have written them.
template <typename E>
__global__ __launch_bounds__(256) void k_hetrd_tail(const E *A, int64_t lda, int n, int j0, E *V,
                                                    int64_t ldv, E *tau, double *d, double *e,
                                                    const E *pin) {
  typedef Num<E> X;
  constexpr int MX = kEigSmallMax;
  __shared__ E sA[MX][MX + 1];
  __shared__ double sd[MX], se[MX];
  __shared__ E stau[MX], sp[MX], svp[MX], swp[MX];
  const int t = threadIdx.x, m = n - j0;
  if (j0 > 0 && t < 64) {  // w of the previous step (rows j0 .. n-1)
    const int r = t;
    const E v = r < m ? V[j0 + r + (int64_t)(j0 - 1) * ldv] : X::zero();
    const E p = r < m ? pin[j0 + r] : X::zero();
    const E pv = X::mul(X::cj(p), v);
    const double sr = wave_sum(X::re(pv)), si = wave_sum(X::im(pv));
    const E kap = X::scale(X::mul(tau[j0 - 1], mk<E>(sr, si)), -0.5);
    if (r < m) {
      svp[r] = v;
      swp[r] = p + X::mul(kap, v);
    }
  }
  __syncthreads();
  for (int idx = t; idx < m * m; idx += 256) {
    const int r = idx % m, c = idx / m;
    E a = A[(j0 + r) + (int64_t)(j0 + c) * lda];
    if (j0 > 0) a = a - X::mul(svp[r], X::cj(swp[c])) - X::mul(swp[r], X::cj(svp[c]));
    sA[c][r] = a;
  }
  __syncthreads();
  tridiag_lds<E, MX>(sA, m, sd, se, stau, sp);
  for (int i = t; i < m; i += 256) {
    d[j0 + i] = sd[i];
    if (i + 1 < m) {
      e[j0 + i] = se[i];
      tau[j0 + i] = stau[i];
    }
  }
  for (int idx = t; idx < m * m; idx += 256) {
    const int r = idx % m, c = idx / m;
    if (r >= c + 1 && c + 1 < m) V[(j0 + r) + (int64_t)(j0 + c) * ldv] = sA[c][r];
  }
}

// X = H_0 ... H_{n-2} Z (n <= kEigSmallMax) from the reflectors in V
// (column j, rows j + 1 ..) and tau, Z real (ld ldz).
template <typename E>
__global__ __launch_bounds__(256) void k_ormtr_small(const E *V, int64_t ldv, const E *tau,
                                                     const double *Z, int64_t ldz, int n, E *Xo,
                                                     int64_t ldx) {
  constexpr int MX = kEigSmallMax;
  __shared__ E sV[MX][MX + 1];
  __shared__ E stau[MX];
  const int t = threadIdx.x;
  for (int idx = t; idx < n * n; idx += 256) {
    const int r = idx % n, c = idx / n;
    sV[c][r] = V[r + (int64_t)c * ldv];
  }
  for (int i = t; i + 1 < n; i += 256) stau[i] = tau[i];
  __syncthreads();
  backtransform_lds<E, MX>(
      sV, stau, n, [&](int r, int c) { return Z[r + (int64_t)c * ldz]; },
      [&](int r, int c, E v) { Xo[r + (int64_t)c * ldx] = v; });
}

// ------------------------------------------------ Householder reduction --
// Launch j (0 <= j < n) of the reduction to tridiagonal form.  Every block
// first rebuilds, from what launch j - 1 left (v_{j-1} in V, p_{j-1} =
// tau B v_{j-1} in pin), the vector w = p + kappa v with kappa = -tau
// (p^H v) / 2, so that the step's two-sided update is B - v w^H - w v^H;
// it applies that update to column j on the fly, forms the reflector v_j of
// the column below the diagonal (block 0 stores it, tau_j, d_j and
// e_j = beta), then applies the update to its RB rows of the trailing block
// and computes those rows of p_j = tau_j B' v_j.
template <typename E, int RB>
__global__ __launch_bounds__(256) void k_hetrd_step(E *__restrict__ A, int64_t lda, int n, int j,
                                                    E *__restrict__ V, int64_t ldv,
                                                    E *__restrict__ tau, double *__restrict__ d,
                                                    double *__restrict__ e,
                                                    const E *__restrict__ pin,
                                                    E *__restrict__ pout) {
  typedef Num<E> X;
  extern __shared__ __align__(16) char eig_dyn[];
  const int m = n - j;  // rows and columns j .. n-1 (local index r - j)
  // blocks whose rows all precede the trailing block have nothing to do
  // (block 0 always stays: it stores the reflector)
  if (blockIdx.x > 0 && (int)(blockIdx.x + 1) * RB <= j + 1) return;
  E *s_vp = (E *)eig_dyn, *s_w = s_vp + m, *s_v = s_w + m;  // 3 m elements
  __shared__ E s_part[256];
  __shared__ double s_red[8];
  const int t = threadIdx.x;
  constexpr int U = 8;  // loads in flight per thread
  if (j > 0) {
    const E *vcol = V + (int64_t)(j - 1) * ldv;
    double sr = 0.0, si = 0.0;
    for (int i0 = t; i0 < m; i0 += 256 * U) {
      E v[U], p[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + 256 * u;
        v[u] = i < m ? vcol[j + i] : X::zero();
        p[u] = i < m ? pin[j + i] : X::zero();
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + 256 * u;
        if (i < m) {
          s_vp[i] = v[u];
          s_w[i] = p[u];
          const E pv = X::mul(X::cj(p[u]), v[u]);
          sr += X::re(pv);
          si += X::im(pv);
        }
      }
    }
    wg_sum2(sr, si, s_red);
    const E kap = X::scale(X::mul(tau[j - 1], mk<E>(sr, si)), -0.5);
    for (int i = t; i < m; i += 256) s_w[i] = s_w[i] + X::mul(kap, s_vp[i]);
    __syncthreads();
  }
  // column j with the previous step's update
  double xr2 = 0.0;
  {
    const E w0 = j > 0 ? s_w[0] : X::zero(), v0 = j > 0 ? s_vp[0] : X::zero();
    const E *acol = A + (int64_t)j * lda;
    for (int i0 = t; i0 < m; i0 += 256 * U) {
      E c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + 256 * u;
        c[u] = i < m ? acol[j + i] : X::zero();
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + 256 * u;
        if (i < m) {
          E cc = c[u];
          if (j > 0) cc = cc - X::mul(s_vp[i], X::cj(w0)) - X::mul(s_w[i], X::cj(v0));
          s_v[i] = cc;
          if (i >= 2) xr2 += X::abs2(cc);
        }
      }
    }
  }
  double dummy = 0.0;
  wg_sum2(xr2, dummy, s_red);
  if (j == n - 1) {
    if (blockIdx.x == 0 && t == 0) d[j] = X::re(s_v[0]);
    return;
  }
  E tj, scale;
  double beta;
  reflector<E>(s_v[1], xr2, tj, beta, scale);
  __syncthreads();  // every thread has read s_v[1]
  for (int i = t; i < m; i += 256)
    if (i >= 2) s_v[i] = X::mul(s_v[i], scale);
  if (t == 0) s_v[1] = X::real(1.0);
  __syncthreads();
  if (blockIdx.x == 0) {
    E *vout = V + (int64_t)j * ldv;
    for (int i = 1 + t; i < m; i += 256) vout[j + i] = s_v[i];
    if (t == 0) {
      tau[j] = tj;
      d[j] = X::re(s_v[0]);
      e[j] = beta;
    }
  }
  // rows blockIdx.x RB + (0 .. RB-1) of the trailing block (columns j+1 ..
  // n-1): a block owns the same rows in every launch, so that it finds them
  // in its XCD's L2 (blocks go to the XCDs round-robin by index)
  constexpr int QL = 256 / RB;
  const int rr = t % RB, q = t / RB;
  const int r = blockIdx.x * RB + rr;
  E acc = X::zero();
  if (r > j && r < n) {
    const int ir = r - j;
    const E vpr = j > 0 ? s_vp[ir] : X::zero(), wr = j > 0 ? s_w[ir] : X::zero();
    for (int c0 = j + 1 + q; c0 < n; c0 += QL * U) {
      E a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + QL * u;
        a[u] = c < n ? A[r + (int64_t)c * lda] : X::zero();
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + QL * u;
        if (c < n) {
          const int ic = c - j;
          E x = a[u];
          if (j > 0) x = x - X::mul(vpr, X::cj(s_w[ic])) - X::mul(wr, X::cj(s_vp[ic]));
          A[r + (int64_t)c * lda] = x;
          acc = acc + X::mul(x, s_v[ic]);
        }
      }
    }
  }
  s_part[t] = acc;
  __syncthreads();
  if (q == 0 && r > j && r < n) {
    E sum = X::zero();
    for (int k = 0; k < QL; ++k) sum = sum + s_part[rr + k * RB];
    pout[r] = X::mul(tj, sum);
  }
}

// ------------------------------------------------ divide and conquer --
// The tree: depth D, block i of depth t covers [i n / 2^t, (i + 1) n / 2^t);
// the leaves (depth D) have at most kDcLeaf rows; an internal block splits
// at the boundary of its two children, where the coupling rho = e[mid - 1]
// is removed from the two diagonal entries next to it (T = diag(T1, T2) +
// |rho| u u^T with u = (e_last, sign(rho) e_first)).
__device__ __forceinline__ int dc_bound(int i, int n, int t) {
  return (int)(((int64_t)i * n) >> t);
}

// One leaf per block: QR iteration on the leaf's tridiagonal, eigenvalues
// ascending to w[a..b), eigenvectors to the diagonal block of Z (ld n).
__global__ __launch_bounds__(64) void k_dc_leaf(const double *d, const double *e, int n, int D,
                                                double *w, double *Z, int *info) {
  __shared__ double sZ[kDcLeaf * (kDcLeaf + 1)];
  __shared__ double sd[kDcLeaf], se[kDcLeaf];
  __shared__ int srank[kDcLeaf], ctl[4];
  const int t = threadIdx.x;
  const int a = dc_bound(blockIdx.x, n, D), b = dc_bound(blockIdx.x + 1, n, D), m = b - a;
  constexpr int LZ = kDcLeaf + 1;
  for (int i = t; i < m; i += 64) {
    double v = d[a + i];
    if (i == 0 && a > 0) v -= fabs(e[a - 1]);
    if (i == m - 1 && b < n) v -= fabs(e[b - 1]);
    sd[i] = v;
    se[i] = i + 1 < m ? e[a + i] : 0.0;
  }
  for (int idx = t; idx < m * LZ; idx += 64) sZ[idx] = (idx % LZ == idx / LZ) ? 1.0 : 0.0;
  __syncthreads();
  ql_tridiag(sd, se, sZ, LZ, m, ctl);
  rank_ascending(sd, m, srank);
  __syncthreads();
  for (int idx = t; idx < m * m; idx += 64) {
    const int r = idx % m, c = idx / m;
    Z[(a + r) + (int64_t)(a + srank[c]) * n] = sZ[r + c * LZ];
  }
  for (int i = t; i < m; i += 64) w[a + srank[i]] = sd[i];
  if (t == 0 && ctl[3]) info[0] = 1;
}

// Merge of the two children of block i at depth t: the rank-one problem
// D + rho z z^T (z = the last row of Q1 and sign(rho) times the first row of
// Q2, scaled by 1/sqrt(2), rho = 2 |e[mid - 1]|), sorted; deflation of tiny
// z components and of close pairs (a Givens rotation of two columns of Q
// zeroes one component); the rotations are applied to the columns of Zc.
// Outputs (DcPtrs at s + .): the k non-deflated (dl, zl, source column),
// the deflated eigenvalues and their source columns, and k in kcnt[s].
__global__ __launch_bounds__(256) void k_dc_deflate(const double *w, const double *e, int n, int t,
                                                    double *Zc, DcPtrs a) {
  __shared__ double sD[kEigMaxN], sz[kEigMaxN];
  __shared__ int sperm[kEigMaxN], snd[kEigMaxN], sdf[kEigMaxN];
  __shared__ int rp[kEigMaxN], rn[kEigMaxN];
  __shared__ double rc[kEigMaxN], rs[kEigMaxN];
  __shared__ double sred[8];
  __shared__ int scnt[3];
  const int th = threadIdx.x;
  const int i = blockIdx.x;
  const int s = dc_bound(i, n, t), mid = dc_bound(2 * i + 1, n, t + 1), end = dc_bound(i + 1, n, t);
  const int n1 = mid - s, nn = end - s;
  const double rho_off = e[mid - 1];
  const double sgn = rho_off >= 0.0 ? 1.0 : -1.0;
  const double rho = 2.0 * fabs(rho_off);
  const double r2 = 0.70710678118654752440;
  // stable merge of the two sorted halves of w[s..end) (slots start as the
  // identity, so that every index stays in range even for non-finite input)
  for (int k = th; k < nn; k += 256) {
    sD[k] = 0.0;
    sz[k] = 0.0;
    sperm[k] = k;
  }
  __syncthreads();
  double mx = 0.0;
  for (int k = th; k < nn; k += 256) {
    const double v = w[s + k];
    double z;
    int pos;
    if (k < n1) {
      z = Zc[(mid - 1) + (int64_t)(s + k) * n] * r2;
      int lo = 0, hi = nn - n1;  // count of second-half values < v
      while (lo < hi) {
        const int h = (lo + hi) >> 1;
        if (w[mid + h] < v) lo = h + 1; else hi = h;
      }
      pos = k + lo;
    } else {
      z = sgn * Zc[mid + (int64_t)(s + k) * n] * r2;
      int lo = 0, hi = n1;  // count of first-half values <= v
      while (lo < hi) {
        const int h = (lo + hi) >> 1;
        if (w[s + h] <= v) lo = h + 1; else hi = h;
      }
      pos = (k - n1) + lo;
    }
    sD[pos] = v;
    sz[pos] = z;
    sperm[pos] = k;
    mx = fmax(mx, fmax(fabs(v), fabs(z)));
  }
  const double tol = 8.0 * kEps * wg_max(mx, sred);
  __syncthreads();
  if (th == 0) {
    int k = 0, nd = 0, nr = 0;
    int pj = -1;
    for (int nj = 0; nj < nn; ++nj) {
      if (rho * fabs(sz[nj]) <= tol) {
        sdf[nd++] = nj;
        continue;
      }
      if (pj < 0) {
        pj = nj;
        continue;
      }
      double sv = sz[pj], cv = sz[nj];
      const double tau = hypot(cv, sv);
      const double tdiff = sD[nj] - sD[pj];
      cv /= tau;
      sv = -sv / tau;
      if (fabs(tdiff * cv * sv) <= tol) {
        // rotate columns pj, nj: z[pj] -> 0, z[nj] -> tau
        sz[nj] = tau;
        sz[pj] = 0.0;
        rp[nr] = pj;
        rn[nr] = nj;
        rc[nr] = cv;
        rs[nr] = sv;
        ++nr;
        const double tt = sD[pj] * cv * cv + sD[nj] * sv * sv;
        sD[nj] = sD[pj] * sv * sv + sD[nj] * cv * cv;
        sD[pj] = tt;
        sdf[nd++] = pj;
        pj = nj;
      } else {
        snd[k++] = pj;
        pj = nj;
      }
    }
    if (pj >= 0) snd[k++] = pj;
    scnt[0] = k;
    scnt[1] = nd;
    scnt[2] = nr;
  }
  __syncthreads();
  const int k = scnt[0], nd = scnt[1], nr = scnt[2];
  // the rotations on the columns of Zc (rows s .. end), in order
  if (nr > 0)
    for (int r = s + th; r < end; r += 256)
      for (int q = 0; q < nr; ++q) {
        const int64_t cp = (int64_t)(s + sperm[rp[q]]) * n, cn = (int64_t)(s + sperm[rn[q]]) * n;
        const double x = Zc[r + cp], y = Zc[r + cn];
        Zc[r + cp] = rc[q] * x + rs[q] * y;
        Zc[r + cn] = -rs[q] * x + rc[q] * y;
      }
  for (int q = th; q < k; q += 256) {
    a.dl[s + q] = sD[snd[q]];
    a.zl[s + q] = sz[snd[q]];
    a.src_nd[s + q] = s + sperm[snd[q]];
  }
  for (int q = th; q < nd; q += 256) {
    a.dval[s + q] = sD[sdf[q]];
    a.src_df[s + q] = s + sperm[sdf[q]];
  }
  if (th == 0) a.kcnt[s] = k;
}

// Root j of 1 / rho + sum_i zl_i^2 / (dl_i - lambda) = 0 in the shifted
// variable tau = lambda - dl_o, o the nearer pole (so that the differences
// dl_i - lambda = (dl_i - dl_o) - tau keep their relative accuracy), by
// Newton steps safeguarded by bisection (a step that leaves the bracket is
// replaced by its midpoint; the bracket shrinks with every evaluation):
// one wave per root, four roots per block.
__global__ __launch_bounds__(256) void k_dc_secular(const double *e, int n, int t, DcPtrs a) {
  __shared__ double sdl[kEigMaxN], szz[kEigMaxN];
  const int i = blockIdx.x;
  const int s = dc_bound(i, n, t), mid = dc_bound(2 * i + 1, n, t + 1);
  const int k = a.kcnt[s];
  const int j0 = blockIdx.y * 4;
  if (j0 >= k) return;
  const double rho = 2.0 * fabs(e[mid - 1]);
  for (int q = threadIdx.x; q < k; q += 256) {
    sdl[q] = a.dl[s + q];
    const double z = a.zl[s + q];
    szz[q] = z * z;
  }
  __syncthreads();
  const int j = j0 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= k) return;
  const double ir = 1.0 / rho;
  int o;
  double lo, hi;
  if (j < k - 1) {
    const double h = 0.5 * (sdl[j + 1] - sdl[j]);
    double f = 0.0;
    for (int q = lane; q < k; q += 64) f += szz[q] / ((sdl[q] - sdl[j]) - h);
    f = ir + wave_sum(f);
    if (f > 0.0) {
      o = j; lo = 0.0; hi = h;
    } else {
      o = j + 1; lo = -h; hi = 0.0;
    }
  } else {
    double zz = 0.0;
    for (int q = lane; q < k; q += 64) zz += szz[q];
    o = k - 1; lo = 0.0; hi = rho * wave_sum(zz);
  }
  // f increases from -inf to +inf on the bracket: Newton steps that stay
  // strictly inside the shrinking bracket, else the midpoint, until a step
  // (or the bracket) is below 2 u of the iterate
  const double dlo = sdl[o];
  double mdl = 0.5 * (lo + hi), tau = mdl;
  for (int it = 0; it < 200; ++it) {
    double f = 0.0, fp = 0.0;
    for (int q = lane; q < k; q += 64) {
      const double r = szz[q] / ((sdl[q] - dlo) - mdl);
      f += r;
      fp += r / ((sdl[q] - dlo) - mdl);
    }
    f = ir + wave_sum(f);
    fp = wave_sum(fp);
    tau = mdl;
    if (f == 0.0) break;
    if (f > 0.0) hi = mdl; else lo = mdl;
    double nx = mdl - f / fp;
    if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
    const double tol = 2.0 * kEps * fmax(fabs(lo), fabs(hi));
    if (fabs(nx - mdl) <= 2.0 * kEps * fabs(nx) || hi - lo <= tol || nx == lo || nx == hi) {
      tau = nx;
      break;
    }
    mdl = nx;
  }
  if (tau == 0.0) tau = (o == j) ? hi : lo;
  if (lane == 0) {
    a.org[s + j] = o;
    a.tsec[s + j] = tau;
  }
}

// Loewner's formula: the z of which the computed roots are the exact
// eigenvalues, zh_i^2 = prod_j (lambda_j - dl_i) / (rho prod_{j != i}
// (dl_j - dl_i)), with the sign of zl_i (Gu & Eisenstat); one wave per i.
__global__ __launch_bounds__(256) void k_dc_lowner(const double *e, int n, int t, DcPtrs a) {
  __shared__ double sdl[kEigMaxN], st[kEigMaxN];
  __shared__ int so[kEigMaxN];
  const int bi = blockIdx.x;
  const int s = dc_bound(bi, n, t), mid = dc_bound(2 * bi + 1, n, t + 1);
  const int k = a.kcnt[s];
  const int i0 = blockIdx.y * 4;
  if (i0 >= k) return;
  const double rho = 2.0 * fabs(e[mid - 1]);
  for (int q = threadIdx.x; q < k; q += 256) {
    sdl[q] = a.dl[s + q];
    st[q] = a.tsec[s + q];
    so[q] = a.org[s + q];
  }
  __syncthreads();
  const int i = i0 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= k) return;
  const double di = sdl[i];
  double p = 1.0;
  for (int j = lane; j < k; j += 64) {
    const double lmd = (sdl[so[j]] - di) + st[j];  // lambda_j - dl_i
    p *= (j == i) ? lmd / rho : lmd / (sdl[j] - di);
  }
  p = wave_prod(p);
  if (lane == 0) a.zh[s + i] = copysign(sqrt(fabs(p)), a.zl[s + i]);
}

// Eigenvector j of D + rho zh zh^T: u_i = zh_i / (dl_i - lambda_j),
// normalised, in column s + j of U (rows 0 .. nn-1, zero from k on); columns
// j >= k are zero.  One wave per column.
__global__ __launch_bounds__(256) void k_dc_vectors(int n, int t, DcPtrs a, double *U) {
  __shared__ double sdl[kEigMaxN], szh[kEigMaxN];
  const int bi = blockIdx.x;
  const int s = dc_bound(bi, n, t), end = dc_bound(bi + 1, n, t), nn = end - s;
  const int j0 = blockIdx.y * 4;
  if (j0 >= nn) return;
  const int k = a.kcnt[s];
  for (int q = threadIdx.x; q < k; q += 256) {
    sdl[q] = a.dl[s + q];
    szh[q] = a.zh[s + q];
  }
  __syncthreads();
  const int j = j0 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= nn) return;
  double *col = U + (int64_t)(s + j) * n;
  if (j >= k) {
    for (int q = lane; q < nn; q += 64) col[q] = 0.0;
    return;
  }
  const int o = a.org[s + j];
  const double tau = a.tsec[s + j], dlo = sdl[o];
  double ss = 0.0;
  for (int q = lane; q < k; q += 64) {
    const double u = szh[q] / ((sdl[q] - dlo) - tau);
    ss += u * u;
  }
  const double inv = 1.0 / sqrt(wave_sum(ss));
  for (int q = lane; q < nn; q += 64)
    col[q] = q < k ? szh[q] / ((sdl[q] - dlo) - tau) * inv : 0.0;
}

// Qg[s.., s + j] = Zc[s.., src_nd[s + j]] for j < k, zero for k <= j < nn.
__global__ __launch_bounds__(256) void k_dc_gather(const double *Zc, int n, int t, DcPtrs a,
                                                   double *Qg) {
  const int bi = blockIdx.x, j = blockIdx.y;
  const int s = dc_bound(bi, n, t), end = dc_bound(bi + 1, n, t), nn = end - s;
  if (j >= nn) return;
  const int k = a.kcnt[s];
  double *dst = Qg + (int64_t)(s + j) * n;
  if (j < k) {
    const double *src = Zc + (int64_t)a.src_nd[s + j] * n;
    for (int r = s + threadIdx.x; r < end; r += 256) dst[r] = src[r];
  } else {
    for (int r = s + threadIdx.x; r < end; r += 256) dst[r] = 0.0;
  }
}

// The merged eigenvalues, sorted: entries q < k are the secular roots
// (dl_o + tau), the others the deflated values; w[s + rank] and the source
// of that column (srcbuf: s + q for column q of Zk, -1 - c for column c of
// Zc).  One thread per entry.
__global__ __launch_bounds__(256) void k_dc_rank(int n, int t, DcPtrs a, double *w) {
  __shared__ double sv[kEigMaxN];
  const int bi = blockIdx.x;
  const int s = dc_bound(bi, n, t), end = dc_bound(bi + 1, n, t), nn = end - s;
  const int k = a.kcnt[s];
  for (int q = threadIdx.x; q < nn; q += 256)
    sv[q] = q < k ? a.dl[s + a.org[s + q]] + a.tsec[s + q] : a.dval[s + q - k];
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += 256) {
    const double v = sv[q];
    int r = 0;
    for (int p = 0; p < nn; ++p) r += (sv[p] < v || (sv[p] == v && p < q)) ? 1 : 0;
    w[s + r] = v;
    a.srcbuf[s + r] = q < k ? s + q : -1 - a.src_df[s + q - k];
  }
}

// Zn[s.., g] = (column srcbuf[g] of Zk or Zc)[s..end) for every column g.
__global__ __launch_bounds__(256) void k_dc_place(const double *Zk, const double *Zc, int n, int t,
                                                  const int *srcbuf, double *Zn) {
  const int g = blockIdx.x;
  int b = min((int)(((int64_t)g << t) / n), (1 << t) - 1);  // block of depth t holding g
  while (b > 0 && dc_bound(b, n, t) > g) --b;
  while (b + 1 < (1 << t) && dc_bound(b + 1, n, t) <= g) ++b;
  const int s = dc_bound(b, n, t), end = dc_bound(b + 1, n, t);
  const int src = min(max(srcbuf[g], -n), n - 1);  // in range even after non-finite input
  const double *col = src >= 0 ? Zk + (int64_t)src * n : Zc + (int64_t)(-1 - src) * n;
  double *dst = Zn + (int64_t)g * n;
  for (int r = s + threadIdx.x; r < end; r += 256) dst[r] = col[r];
}

// Zk[s.., s..] = Qg[s.., s..] U[0.., s..] for every merge of depth t whose
// order is at most kDcGemmSmall (ld n each): 32 x 32 output tiles, FP64
// fused multiply-adds through LDS, one block per (merge, tile).
__global__ __launch_bounds__(256) void k_dc_gemm(const double *Qg, const double *U, double *Zk,
                                                 int n, int t) {
  __shared__ double sa[32][33], sb[32][33];
  const int bi = blockIdx.x;
  const int s = dc_bound(bi, n, t), nn = dc_bound(bi + 1, n, t) - s;
  const int tpd = (nn + 31) / 32;
  if ((int)blockIdx.y >= tpd * tpd) return;
  const int i0 = (blockIdx.y % tpd) * 32, j0 = (blockIdx.y / tpd) * 32;
  const int th = threadIdx.x, r = th & 31, cq = th >> 5;  // rows r, columns cq + 8 k
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < nn; k0 += 32) {
    for (int idx = th; idx < 32 * 32; idx += 256) {
      const int a = idx & 31, b = idx >> 5;  // row a, k index b
      sa[b][a] = (i0 + a < nn && k0 + b < nn) ? Qg[(s + i0 + a) + (int64_t)(s + k0 + b) * n] : 0.0;
      sb[a][b] = (k0 + a < nn && j0 + b < nn) ? U[(k0 + a) + (int64_t)(s + j0 + b) * n] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const double av = sa[kk][r];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += av * sb[kk][cq + 8 * q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = j0 + cq + 8 * q;
    if (i0 + r < nn && c < nn) Zk[(s + i0 + r) + (int64_t)(s + c) * n] = acc[q];
  }
}

// X (n x n, ld ldx) = Z (real, ld n) as elements of type E.
template <typename E>
__global__ void k_real_to_elem(const double *Z, int n, E *X, int64_t ldx) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256)
    X[r + (int64_t)c * ldx] = Num<E>::real(Z[r + (int64_t)c * n]);
}

// -------------------------------------------------------------- launchers --
void heev_small(bool cplx, void *A, int64_t lda, int n, double *theta, int *info, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(k_heev_small<double2>, dim3(1), dim3(256), 0, s, (double2 *)A, lda, n, theta,
                       info);
  else
    hipLaunchKernelGGL(k_heev_small<double>, dim3(1), dim3(256), 0, s, (double *)A, lda, n, theta,
                       info);
}

template <typename E, int RB>
static void hetrd_step_t(E *A, int64_t lda, int n, int j, E *V, int64_t ldv, E *tau, double *d,
                         double *e, const E *pin, E *pout, hipStream_t s) {
  static const bool attr = [] {
    // dynamic LDS above the default limit: the three vectors of the largest order
    return hipFuncSetAttribute((const void *)k_hetrd_step<E, RB>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(3 * kEigMaxN * sizeof(E))) == hipSuccess;
  }();
  if (!attr) {
    (void)hipGetLastError();
    set_error("hipFuncSetAttribute of the tridiagonal reduction failed");
    throw DeviceError();
  }
  const size_t lds = 3 * (size_t)(n - j) * sizeof(E);
  hipLaunchKernelGGL((k_hetrd_step<E, RB>), dim3((n + RB - 1) / RB), dim3(256), lds, s, A, lda, n,
                     j, V, ldv, tau, d, e, pin, pout);
}

void hetrd_step(bool cplx, void *A, int64_t lda, int n, int j, void *V, int64_t ldv, void *tau,
                double *d, double *e, const void *pin, void *pout, hipStream_t s) {
  if (cplx)
    hetrd_step_t<double2, 8>((double2 *)A, lda, n, j, (double2 *)V, ldv, (double2 *)tau, d, e,
                             (const double2 *)pin, (double2 *)pout, s);
  else
    hetrd_step_t<double, 16>((double *)A, lda, n, j, (double *)V, ldv, (double *)tau, d, e,
                             (const double *)pin, (double *)pout, s);
}

void hetrd_tail(bool cplx, const void *A, int64_t lda, int n, int j0, void *V, int64_t ldv,
                void *tau, double *d, double *e, const void *pin, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(k_hetrd_tail<double2>, dim3(1), dim3(256), 0, s, (const double2 *)A, lda, n,
                       j0, (double2 *)V, ldv, (double2 *)tau, d, e, (const double2 *)pin);
  else
    hipLaunchKernelGGL(k_hetrd_tail<double>, dim3(1), dim3(256), 0, s, (const double *)A, lda, n,
                       j0, (double *)V, ldv, (double *)tau, d, e, (const double *)pin);
}

void ormtr_small(bool cplx, const void *V, int64_t ldv, const void *tau, const double *Z,
                 int64_t ldz, int n, void *X, int64_t ldx, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(k_ormtr_small<double2>, dim3(1), dim3(256), 0, s, (const double2 *)V, ldv,
                       (const double2 *)tau, Z, ldz, n, (double2 *)X, ldx);
  else
    hipLaunchKernelGGL(k_ormtr_small<double>, dim3(1), dim3(256), 0, s, (const double *)V, ldv,
                       (const double *)tau, Z, ldz, n, (double *)X, ldx);
}

void dc_gemm_small(const double *Qg, const double *U, double *Zk, int n, int t, hipStream_t s) {
  const int nmax = (n + (1 << t) - 1) >> t;
  const int tpd = (nmax + 31) / 32;
  hipLaunchKernelGGL(k_dc_gemm, dim3(1u << t, (unsigned)(tpd * tpd)), dim3(256), 0, s, Qg, U, Zk,
                     n, t);
}

int dc_depth(int n) {
  int D = 0;
  while ((n + (1 << D) - 1) >> D > kDcLeaf) ++D;
  return D;
}

void dc_leaves(const double *d, const double *e, int n, int D, double *w, double *Z, int *info,
               hipStream_t s) {
  hipLaunchKernelGGL(k_dc_leaf, dim3(1u << D), dim3(64), 0, s, d, e, n, D, w, Z, info);
}

void dc_merge_pre(const double *e, int n, int t, const double *w, double *Zc, double *Qg,
                  double *U, const DcPtrs &a, hipStream_t s) {
  const unsigned nb = 1u << t;
  const int nmax = (n + (1 << t) - 1) >> t;
  const unsigned g4 = (unsigned)((nmax + 3) / 4);
  hipLaunchKernelGGL(k_dc_deflate, dim3(nb), dim3(256), 0, s, w, e, n, t, Zc, a);
  hipLaunchKernelGGL(k_dc_secular, dim3(nb, g4), dim3(256), 0, s, e, n, t, a);
  hipLaunchKernelGGL(k_dc_lowner, dim3(nb, g4), dim3(256), 0, s, e, n, t, a);
  hipLaunchKernelGGL(k_dc_vectors, dim3(nb, g4), dim3(256), 0, s, n, t, a, U);
  hipLaunchKernelGGL(k_dc_gather, dim3(nb, (unsigned)nmax), dim3(256), 0, s, Zc, n, t, a, Qg);
}

void dc_merge_post(int n, int t, double *w, const double *Zk, const double *Zc, double *Zn,
                   const DcPtrs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_dc_rank, dim3(1u << t), dim3(256), 0, s, n, t, a, w);
  hipLaunchKernelGGL(k_dc_place, dim3((unsigned)n), dim3(256), 0, s, Zk, Zc, n, t, a.srcbuf, Zn);
}

void real_to_elem(bool cplx, const double *Z, int n, void *X, int64_t ldx, hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  if (cplx)
    hipLaunchKernelGGL(k_real_to_elem<double2>, grid, dim3(256), 0, s, Z, n, (double2 *)X, ldx);
  else
    hipLaunchKernelGGL(k_real_to_elem<double>, grid, dim3(256), 0, s, Z, n, (double *)X, ldx);
}

}  // namespace chase
