// gfx950 kernels of the solver other than the GEMM core, the GEMM
// instantiations, and their launchers.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "gemm.hpp"
#include "kernels.hpp"
#include "num.hpp"

namespace chase {

// Deterministic block reduction of one double over 256 threads.
__device__ __forceinline__ double block_sum256(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// P[0] + P[stride] + ... + P[(n - 1) stride] added in this order, the loads
// issued sixteen at a time (the split partial sums of a K-split product;
// there can be a few hundred of them)
template <typename E>
__device__ __forceinline__ E sum_strided(const E *P, int n, int64_t stride) {
  E s = Num<E>::zero();
  for (int q = 0; q < n; q += 16) {
    E x[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) x[u] = q + u < n ? P[(int64_t)(q + u) * stride] : Num<E>::zero();
#pragma unroll
    for (int u = 0; u < 16; ++u) s = s + x[u];
  }
  return s;
}

// -------------------------------------------------- Hermitian reduction --
template <typename E>
__global__ void k_reduce_herm(const E *P, int nsplit, int64_t sstride, int64_t ldp, int n, E *G,
                              int64_t ldg, int average) {
  const int i = blockIdx.x * 16 + threadIdx.x;
  const int j = blockIdx.y * 16 + threadIdx.y;
  if (i >= n || j >= n || i > j) return;
  E s = sum_strided(P + (int64_t)j * ldp + i, nsplit, sstride);
  if (average) {
    const E t = sum_strided(P + (int64_t)i * ldp + j, nsplit, sstride);
    s = Num<E>::scale(s + Num<E>::cj(t), 0.5);
  }
  if (i == j) s = Num<E>::real(Num<E>::re(s));
  G[(int64_t)j * ldg + i] = s;
  G[(int64_t)i * ldg + j] = Num<E>::cj(s);
}

template <typename E>
__global__ __launch_bounds__(256) void k_trace_shift(E *G, int64_t ldg, int n, double coef,
                                                     int add_shift, double *out, const int *flag) {
  __shared__ double sh[256];
  if (flag != nullptr && flag[0] != 0) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += Num<E>::re(G[(int64_t)i * ldg + i]);
  const double tr = block_sum256(v, sh);
  const double s = coef * tr;
  if (add_shift)
    for (int i = threadIdx.x; i < n; i += 256) {
      E g = G[(int64_t)i * ldg + i];
      G[(int64_t)i * ldg + i] = g + Num<E>::real(s);
    }
  if (threadIdx.x == 0) {
    out[0] = tr;
    out[1] = add_shift ? s : 0.0;
  }
}

// ------------------------------------------- Cholesky of a diagonal block --
// One work-group factors the b x b (b <= 64) diagonal block of G at (p0, p0)
// from its upper triangle (G = R^H R), writes R and R^{-1} (upper, zero
// below the diagonal) and reports a non-positive or non-finite pivot
// through flag.  The block sits in LDS, padded past b with a unit diagonal
// (so the padded block's factor is diag(R, I)), and is factored by panels
// of eight columns, right-looking: wave 0 factors the 8 x 8 diagonal block
// in registers (lane 8 i + j holds entry (i, j); pivots and rows move by
// lane shuffles, no barrier) together with its inverse T_pp; then
// R_p,right = T_pp^H G_p,right for the panel's rows, and the trailing
// block takes the rank-8 update.  Three barriers per panel.  R^{-1} is then
// formed by block rows from the bottom, X_pr = -T_p sum_{p<s<=r} R_ps X_sr,
// two barriers per block row, its diagonal blocks being the T_pp.
constexpr int kCholThreads = 512;

template <typename E> __device__ __forceinline__ E shfl_e(E v, int src);
template <> __device__ __forceinline__ double shfl_e(double v, int src) { return __shfl(v, src); }
template <> __device__ __forceinline__ double2 shfl_e(double2 v, int src) {
  return make_double2(__shfl(v.x, src), __shfl(v.y, src));
}

template <typename E>
__global__ __launch_bounds__(kCholThreads) void k_chol_diag(const E *G, int64_t ldg, E *R, int64_t ldr,
                                                   E *Ri, int64_t ldi, int p0, int b, int *flag,
                                                   int pass, int inject) {
  typedef Num<E> X;
  __shared__ E sR[64][65];  // sR[i][c] = entry (i, c): the block, then R, then R^{-1}
  __shared__ E sT[8][8][8], sW[8][64];
  __shared__ int s_fail;
  if (flag[0] != 0) return;
  const int t = threadIdx.x;
  if (inject) {
    if (t == 0) { flag[0] = p0 + 1; flag[1] = pass; }
    return;
  }
  for (int idx = t; idx < 64 * 64; idx += kCholThreads) {
    const int i = idx & 63, c = idx >> 6;
    E v = X::zero();
    if (c < b) {
      if (i <= c) v = G[(int64_t)(p0 + c) * ldg + p0 + i];
    } else if (i == c) {
      v = X::real(1.0);
    }
    sR[i][c] = v;
  }
  if (t == 0) s_fail = 0;
  __syncthreads();
  const int nblk = (b + 7) / 8;
#pragma unroll 1
  for (int p = 0; p < nblk; ++p) {
    const int g0 = 8 * p, g1 = g0 + 8, ncol = 8 * nblk - g1;
    if (t < 64) {  // wave 0: R_pp and T_pp = R_pp^{-1}, lane 8 i + j
      const int i = t >> 3, j = t & 7;
      E a = j >= i ? sR[g0 + i][g0 + j] : X::zero();
      double dinv_i = 0.0;
      int fail = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double piv = X::re(shfl_e(a, 9 * q));
        const E aqj = shfl_e(a, 8 * q + j), aqi = shfl_e(a, 8 * q + i);
        if (fail == 0 && (!(piv > 0.0) || !isfinite(piv))) fail = q + 1;
        if (fail == 0) {
          // the refined reciprocal square root unless the pivot is near
          // underflow (uniform across the wave)
          double inv, rq;
          if (piv > 1e-290) {
            inv = rsqrt_refined(piv);
            rq = piv * inv;
          } else {
            rq = sqrt(piv);
            inv = 1.0 / rq;
          }
          if (i == q) dinv_i = inv;
          const E rqj = X::scale(aqj, inv), rqi = X::scale(aqi, inv);
          if (i == q)
            a = j == q ? X::real(rq) : (j > q ? rqj : X::zero());
          else if (i > q && j >= i)
            a = a - X::mul(X::cj(rqi), rqj);
        }
      }
      if (fail != 0) {
        if (t == 0) s_fail = g0 + fail;
      } else {
        // column j of T_pp by back substitution: T(q, j) = (delta_qj -
        // sum_{m > q} R(q, m) T(m, j)) / R(q, q), the sums accumulated row
        // by row as the T(q, j) become known
        E acc = X::zero(), tv = X::zero();
#pragma unroll
        for (int q = 7; q >= 0; --q) {
          const E cand = X::scale(X::sel(i == j, X::real(1.0), X::zero()) - acc, dinv_i);
          const E tqj = shfl_e(cand, 8 * q + j);
          const E riq = shfl_e(a, 8 * i + q);
          if (i == q) tv = j >= q ? tqj : X::zero();
          if (i < q) acc = acc + X::mul(riq, tqj);
        }
        sR[g0 + i][g0 + j] = j >= i ? a : X::zero();
        sT[p][i][j] = tv;
      }
    }
    __syncthreads();
    if (s_fail != 0) {
      if (t == 0) { flag[0] = p0 + s_fail; flag[1] = pass; }
      return;
    }
    // R_p,right = T_pp^H G_p,right: rows g0 .. g0 + 7, columns g1 .. 8 nblk
    {
      const int wi = t & 7, wc = t >> 3;
      if (wc < ncol) {
        E s = X::zero();
        for (int m = 0; m <= wi; ++m) s = s + X::mul(X::cj(sT[p][m][wi]), sR[g0 + m][g1 + wc]);
        sW[wi][wc] = s;
      }
    }
    __syncthreads();
    // trailing update G_right,right -= R_p,right^H R_p,right (upper), and
    // R_p,right into R's rows
    for (int idx = t; idx < ncol * ncol; idx += kCholThreads) {
      const int r = idx % ncol, cc = idx / ncol;
      if (r <= cc) {
        E s = sR[g1 + r][g1 + cc];
#pragma unroll
        for (int m = 0; m < 8; ++m) s = s - X::mul(X::cj(sW[m][r]), sW[m][cc]);
        sR[g1 + r][g1 + cc] = s;
      }
    }
    for (int idx = t; idx < 8 * ncol; idx += kCholThreads) sR[g0 + (idx & 7)][g1 + (idx >> 3)] = sW[idx & 7][idx >> 3];
    __syncthreads();
  }
  // R out; X's diagonal blocks are the T_pp
  for (int idx = t; idx < 64 * 64; idx += kCholThreads) {
    const int i = idx & 63, c = idx >> 6;
    if (i < b && c < b) R[(int64_t)(p0 + c) * ldr + p0 + i] = i <= c ? sR[i][c] : X::zero();
  }
  __syncthreads();
  for (int idx = t; idx < 64 * nblk; idx += kCholThreads) {
    const int q = idx >> 6, i = (idx & 63) >> 3, j = idx & 7;
    sR[8 * q + i][8 * q + j] = j >= i ? sT[q][i][j] : X::zero();
  }
  __syncthreads();
  // block rows p from the bottom: X_pr = -T_p sum_{p < s <= r} R_ps X_sr,
  // i.e. W(i, c) = sum over k in [8 (p + 1), c] of R(8 p + i, k) X(k, c) (X
  // is upper triangular) and X(8 p + i, c) = -sum_{m >= i} T_p(i, m) W(m, c);
  // X overwrites R's block row p, which no later block row reads.
  {
    const int wi = t & 7, wc = t >> 3;  // 8 rows x 64 columns
#pragma unroll 1
    for (int p = nblk - 2; p >= 0; --p) {
      const int r0 = 8 * p, c0 = r0 + 8, cx = c0 + wc;
      const bool act = cx < 8 * nblk;
      E w = X::zero();
      if (act)
        for (int k = c0; k <= cx; ++k) w = w + X::mul(sR[r0 + wi][k], sR[k][cx]);
      sW[wi][wc] = w;
      __syncthreads();
      if (act) {
        E x = X::zero();
        for (int m = wi; m < 8; ++m) x = x + X::mul(sT[p][wi][m], sW[m][wc]);
        sR[r0 + wi][cx] = -x;
      }
      __syncthreads();
    }
  }
  for (int idx = t; idx < 64 * 64; idx += kCholThreads) {
    const int i = idx & 63, c = idx >> 6;
    if (i < b && c < b) Ri[(int64_t)(p0 + c) * ldi + p0 + i] = i <= c ? sR[i][c] : X::zero();
  }
}

template <typename E>
__global__ void k_fill_zero(E *A, int64_t lda, int rows, int cols) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i < rows && j < cols) A[(int64_t)j * lda + i] = Num<E>::zero();
}

// ------------------------------------------------------------ residuals --
template <typename E>
__global__ __launch_bounds__(256) void k_resid(const E *HV, int64_t ldhv, const E *V, int64_t ldv,
                                               int n, const double *theta, double *out) {
  __shared__ double sh[256];
  const int a = blockIdx.x;
  const double th = theta[a];
  const E *h = HV + (int64_t)a * ldhv;
  const E *v = V + (int64_t)a * ldv;
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const E hv = h[i], vv = v[i];
    const double dr = Num<E>::re(hv) - th * Num<E>::re(vv);
    const double di = Num<E>::im(hv) - th * Num<E>::im(vv);
    s1 += dr * dr + di * di;
    s2 += Num<E>::abs2(vv);
  }
  s1 = block_sum256(s1, sh);
  s2 = block_sum256(s2, sh);
  if (threadIdx.x == 0) out[a] = sqrt(s1) / sqrt(s2);
}

// ------------------------------------------------------- column movement --
template <typename Ein, typename Eout>
__global__ void k_gather(const Ein *src, int64_t lds, Eout *dst, int64_t ldd, int n,
                         const int *perm) {
  const int i = blockIdx.x * 256 + threadIdx.x, a = blockIdx.y;
  if (i >= n) return;
  const int c = perm ? perm[a] : a;
  const Ein v = src[(int64_t)c * lds + i];
  dst[(int64_t)a * ldd + i] = make_elem<Eout>((double)re_of(v), (double)im_of(v));
}

// -------------------------------------------------------- random blocks --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed and
// counted by (row, column); Box-Muller turns two 32-bit words into two
// standard normal numbers.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0; c[1] = (uint32_t)p1; c[2] = n2; c[3] = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

template <typename E>
__global__ void k_randn(E *V, int64_t ldv, int n, uint64_t seed) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)j, 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
  const double u2 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
  const double rad = sqrt(-2.0 * log(u1));
  const double z0 = rad * cos(6.283185307179586 * u2), z1 = rad * sin(6.283185307179586 * u2);
  if (sizeof(E) == sizeof(double))
    V[(int64_t)j * ldv + i] = make_elem<E>(z0, 0.0);
  else
    V[(int64_t)j * ldv + i] = make_elem<E>(z0 * 0.7071067811865476, z1 * 0.7071067811865476);
}

// ----------------------------------------------------- Lanczos helpers --
// ------------------------------------------------- block matrix-vector --
// Partial sums of y = A X for a column-major A (M x K, lda) and a block X of
// NV right-hand sides (K x NV, ldx).  The work is HBM-bound: every element
// of A is loaded once.  A work-group of 256 threads owns RPT * 256 rows (row
// r0 + t + 256 q for thread t) and the column range [c0, c0 + kchunk) of
// split blockIdx.y; each column's slice of A is one coalesced load per wave,
// X's rows are staged in LDS and broadcast.  The split's sums go to
// P + blockIdx.y * sstride (M x NV, leading dimension ldp).
template <typename E, int NV, int RPT>
__global__ __launch_bounds__(256) void k_gemv_cm(const E *__restrict__ A, int64_t lda, int M,
                                                 int K, const E *__restrict__ X, int64_t ldx,
                                                 int kchunk, E *__restrict__ P, int64_t ldp,
                                                 int64_t sstride) {
  constexpr int CB = 64, U = 8;
  __shared__ E xs[CB][NV];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 256 * RPT + t;
  const int c0 = blockIdx.y * kchunk;
  const int c1 = min(K, c0 + kchunk);
  E acc[RPT][NV];
#pragma unroll
  for (int q = 0; q < RPT; ++q)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[q][v] = Num<E>::zero();
  bool ok[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) ok[q] = r0 + 256 * q < M;
  for (int cb = c0; cb < c1; cb += CB) {
    const int nc = min(CB, c1 - cb);
    __syncthreads();
    for (int e = t; e < nc * NV; e += 256) {
      const int j = e / NV, v = e % NV;
      xs[j][v] = X[(int64_t)(cb + j) + v * ldx];
    }
    __syncthreads();
    int j0 = 0;
    for (; j0 + U <= nc; j0 += U) {
      E a[U][RPT];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const E *col = A + (int64_t)(cb + j0 + u) * lda + r0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) a[u][q] = ok[q] ? col[256 * q] : Num<E>::zero();
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[q][v] = acc[q][v] + Num<E>::mul(a[u][q], xs[j0 + u][v]);
    }
    for (; j0 < nc; ++j0) {
      const E *col = A + (int64_t)(cb + j0) * lda + r0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const E a = ok[q] ? col[256 * q] : Num<E>::zero();
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[q][v] = acc[q][v] + Num<E>::mul(a, xs[j0][v]);
      }
    }
  }
  E *out = P + blockIdx.y * sstride;
#pragma unroll
  for (int q = 0; q < RPT; ++q)
    if (ok[q])
#pragma unroll
      for (int v = 0; v < NV; ++v) out[r0 + 256 * q + v * ldp] = acc[q][v];
}

// y[:, v] = sum over nsplit partials (each M x nv, leading dimension M).
template <typename E>
__global__ void k_gemv_reduce(const E *P, int nsplit, int64_t sstride, int M, E *Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int v = blockIdx.y;
  E s = Num<E>::zero();
  for (int q = 0; q < nsplit; ++q) s = s + P[q * sstride + (int64_t)v * M + i];
  Y[i + v * ldy] = s;
}

// out[c] = Re(v_c^H w_c) for the ncols columns (one work-group per column).
template <typename E>
__global__ __launch_bounds__(256) void k_dot_re_cols(const E *v, const E *w, int64_t ld, int n,
                                                     double *out) {
  __shared__ double sh[256];
  const E *a = v + blockIdx.x * ld;
  const E *b = w + blockIdx.x * ld;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256)
    s += Num<E>::re(a[i]) * Num<E>::re(b[i]) + Num<E>::im(a[i]) * Num<E>::im(b[i]);
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// beta[c] = ||w_c||, vout_c = w_c / beta[c] (zero when beta[c] = 0).
template <typename E>
__global__ __launch_bounds__(256) void k_norm_scale_cols(const E *w, int64_t ldw, int n, E *vout,
                                                         int64_t ldo, double *beta) {
  __shared__ double sh[256];
  const E *a = w + blockIdx.x * ldw;
  E *o = vout + blockIdx.x * ldo;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += Num<E>::abs2(a[i]);
  s = sqrt(block_sum256(s, sh));
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  for (int i = threadIdx.x; i < n; i += 256) o[i] = Num<E>::scale(a[i], inv);
  if (threadIdx.x == 0) beta[blockIdx.x] = s;
}

// One Lanczos step after the product w = H v_j, for orders small enough that
// one work-group per run can stream the run's whole basis (there the
// solver's form with several wide launches per step is latency-bound):
// two passes of classical Gram-Schmidt against the run's basis v_0..v_j
// (h = V^H w, then w -= V h; alpha_j = Re h_j of the first pass, i.e.
// Re(v_j^H w) before any update), beta_j = ||w||, v_{j+1} = w / beta_j.
// Sixteen waves: wave q forms the inner products with v_q, v_{q+16}, ...
// over all N entries and reduces them by shuffles, so a pass needs one
// work-group barrier; the update and the norm use every thread.  The same
// layout as the wide form: run r's basis vector i is column i nv + r of LV;
// alpha at ab[j nv + r], beta at ab[(k + j) nv + r].
constexpr int kLzSmallThreads = 1024;
template <typename E>
__device__ __forceinline__ E wave_sum64(E v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = Num<E>::add_xor(v, m);
  return v;
}

template <typename E>
__global__ __launch_bounds__(kLzSmallThreads) void k_lz_step_small(E *LV, int64_t ldv, int N, int j,
                                                                   int nv, E *W, int64_t ldw,
                                                                   double *ab, int k) {
  constexpr int NW = kLzSmallThreads / 64;
  __shared__ E s_h[kLzSmallMaxBasis];
  __shared__ double s_n[NW];
  const int r = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nb = j + 1;
  E *w = W + (int64_t)r * ldw;
  auto vcol = [&](int i) { return LV + ((int64_t)i * nv + r) * ldv; };
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = wave; i < nb; i += NW) {
      const E *vi = vcol(i);
      E a0 = Num<E>::zero(), a1 = Num<E>::zero();
      int n = lane;
      for (; n + 64 < N; n += 128) {
        a0 = a0 + Num<E>::mul(Num<E>::cj(vi[n]), w[n]);
        a1 = a1 + Num<E>::mul(Num<E>::cj(vi[n + 64]), w[n + 64]);
      }
      if (n < N) a0 = a0 + Num<E>::mul(Num<E>::cj(vi[n]), w[n]);
      const E sum = wave_sum64(a0 + a1);
      if (lane == 0) s_h[i] = sum;
    }
    __syncthreads();
    if (pass == 0 && t == 0) ab[(int64_t)j * nv + r] = Num<E>::re(s_h[j]);
    for (int n = t; n < N; n += kLzSmallThreads) {
      E x = w[n];
      for (int i = 0; i < nb; ++i) x = x - Num<E>::mul(vcol(i)[n], s_h[i]);
      w[n] = x;
    }
    __syncthreads();
  }
  double sq = 0.0;
  for (int n = t; n < N; n += kLzSmallThreads) sq += Num<E>::abs2(w[n]);
  sq = wave_sum64(sq);
  if (lane == 0) s_n[wave] = sq;
  __syncthreads();
  double tot = 0.0;
  for (int q = 0; q < NW; ++q) tot += s_n[q];
  const double beta = sqrt(tot);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  E *vn = vcol(j + 1);
  for (int n = t; n < N; n += kLzSmallThreads) vn[n] = Num<E>::scale(w[n], inv);
  if (t == 0) ab[(int64_t)(k + j) * nv + r] = beta;
}

// out (rows x nv, leading dimension ldo) = sum over nsplit partials (each
// rows x nv, leading dimension ldp), keeping only the entries of row q in
// column q % nv and zeroing the others: the coefficients of each Lanczos run
// against its own basis vectors when the runs' bases are interleaved.
template <typename E>
__global__ void k_sum_splits_diag(const E *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                                  int nv, E *out, int64_t ldo) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= rows) return;
  const int c = blockIdx.y;
  out[(int64_t)c * ldo + q] =
      q % nv == c ? sum_strided(P + (int64_t)c * ldp + q, nsplit, sstride) : Num<E>::zero();
}

// ------------------------------------------------- Householder QR (HHQR) --
// Blocked Householder QR in the geqrf convention: reflector j is
// H_j = I - tau_j v_j v_j^H with v_j(j) = 1, chosen so that
// H_j^H (alpha, x) = (beta, 0) with beta real (beta = -sign(Re alpha) *
// ||(alpha, x)||; tau = 0 when x = 0 and alpha is real).  The hh_state
// buffer holds, twice (alternating column steps), the row of the pivot and
// the per-block partial sums of a column step (offsets below).
constexpr int kHhMaxBlocks = 256;  // row blocks of one column launch
constexpr size_t kHhRow = 0, kHhPart = 2 * 16 * kHhNB,
                 kHhPartBytes = 8 * (size_t)kHhMaxBlocks * 2 * kHhNB;
static_assert(kHhPart + 2 * kHhPartBytes <= kHhStateBytes, "hh_state size");

template <typename E> __device__ __forceinline__ E recip(E a);
template <> __device__ __forceinline__ double recip(double a) { return 1.0 / a; }
template <> __device__ __forceinline__ double2 recip(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// One column step of the panel factorisation.  P is the panel (Mp x nbp,
// column-major, leading dimension ld) from the diagonal element of its first
// column down; Vb the same block of the explicit reflector store (zero on
// entry above the diagonal); tau the panel's tau entries.  Launch jj
// (0 <= jj <= nbp):
//  * jj >= 1 forms reflector jj-1 from the previous launch's block sums
//    (nprev blocks, added in block order by every block, so all agree):
//    beta (written to P[jj-1, jj-1]), tau, the scale 1 / (alpha - beta) and
//    w_c = v^H P[:, c]; scales the vector below the unit diagonal, stores it
//    in P and Vb, and applies H^H to columns jj..nbp-1;
//  * jj < nbp writes this block's sums s_c = sum_{r > jj} conj(P[r, jj])
//    P[r, c] (c = jj..nbp-1) and, from the block holding row jj, that row.
// Nothing waits on another block: the launch boundary orders the steps.
// Each wave reduces its NB accumulators by a halving exchange that leaves
// accumulator `lane` in lane `lane`: 63 exchanges in all for 64 values,
// against 6 per value for a butterfly sum of each.
template <typename E, int NB>
__global__ __launch_bounds__(256) void k_hh_column(E *__restrict__ P, int64_t ld, int Mp, int nbp,
                                                   int jj, int nprev, E *__restrict__ Vb,
                                                   int64_t ldv, E *__restrict__ tau, char *hs) {
  constexpr int ES = sizeof(E) / sizeof(double);
  constexpr int D = NB * ES;  // doubles summed per row
  static_assert(D <= 64 && (D & (D - 1)) == 0, "one wave reduces the sums");
  const E *rowp = (const E *)(hs + kHhRow) + ((jj + 1) & 1) * NB;
  E *rowc = (E *)(hs + kHhRow) + (jj & 1) * NB;
  const double *partp = (const double *)(hs + kHhPart + ((jj + 1) & 1) * kHhPartBytes);
  double *partc = (double *)(hs + kHhPart + (jj & 1) * kHhPartBytes);
  __shared__ E s_w[NB];
  __shared__ E s_ct, s_sc;
  __shared__ double s_red[4][64];
  __shared__ double s_sum[64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool upd = jj >= 1, fact = jj < nbp;
  if (upd) {
    const int p = jj - 1;  // the reflector formed here
    {  // thread (g, q) adds the sums of blocks g, g + G, ... for entry q, eight loads at a time
      constexpr int G = 256 / D;
      const int q = t % D, g = t / D;
      double v = 0.0;
      for (int b0 = g; b0 < nprev; b0 += 8 * G) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int b = b0 + u * G;
          x[u] = b < nprev ? partp[(int64_t)b * D + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
      }
      s_red[g * D / 64][(g * D) % 64 + q] = v;
    }
    __syncthreads();
    if (t < D) {
      constexpr int G = 256 / D;
      double v = 0.0;
      for (int g = 0; g < G; ++g) v += s_red[g * D / 64][(g * D) % 64 + t];
      s_sum[t] = v;
    }
    __syncthreads();
    if (t == 0) {
      const E alpha = rowp[p];
      const double xn2 = s_sum[ES * p];
      E tv = Num<E>::zero(), sc = Num<E>::zero();
      double beta = Num<E>::re(alpha);
      if (xn2 != 0.0 || Num<E>::im(alpha) != 0.0) {
        beta = -copysign(sqrt(Num<E>::abs2(alpha) + xn2), Num<E>::re(alpha));
        tv = Num<E>::scale(Num<E>::real(beta) - alpha, 1.0 / beta);
        sc = recip(alpha - Num<E>::real(beta));
      }
      s_ct = Num<E>::cj(tv);
      s_sc = sc;
      if (blockIdx.x == 0) {
        tau[p] = tv;
        P[p + p * ld] = Num<E>::real(beta);
      }
    }
    __syncthreads();
    if (t > p && t < nbp) {
      E sv;
      if constexpr (ES == 2) sv = make_double2(s_sum[2 * t], s_sum[2 * t + 1]);
      else sv = s_sum[t];
      s_w[t] = rowp[t] + Num<E>::mul(Num<E>::cj(s_sc), sv);
    }
    __syncthreads();
  }
  double acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = 0.0;
  const int rbeg = upd ? jj - 1 : 0;
  for (int64_t r = rbeg + (int64_t)blockIdx.x * 256 + t; r < Mp; r += (int64_t)gridDim.x * 256) {
    // all loads of the row first and without branches, so that they are in
    // flight together: columns outside jj..nbp-1 load a valid column and are
    // ignored; row jj-1 of column jj-1 (beta, being written by block 0) is
    // replaced by Vb's zero
    const E xprev = upd ? *(r > jj - 1 ? &P[r + (jj - 1) * ld] : &Vb[r + (jj - 1) * ldv])
                        : Num<E>::zero();
    E pv[NB];
    if (fact) {
#pragma unroll
      for (int c = 0; c < NB; ++c) pv[c] = P[r + min(max(c, jj), nbp - 1) * ld];
    }
    E cv = Num<E>::zero();  // conj(tau) v_r of reflector jj-1
    if (upd) {
      const E v = r > jj - 1 ? Num<E>::mul(xprev, s_sc) : Num<E>::real(1.0);
      if (r > jj - 1) P[r + (jj - 1) * ld] = v;
      Vb[r + (jj - 1) * ldv] = v;
      cv = Num<E>::mul(s_ct, v);
    }
    if (!fact) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (upd && c >= jj && c < nbp) {
        pv[c] = pv[c] - Num<E>::mul(cv, s_w[c]);
        P[r + c * ld] = pv[c];
      }
    const bool lead = r == jj;
    E x = Num<E>::zero();
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c == jj && r > jj) x = Num<E>::cj(pv[c]);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c >= jj && c < nbp) {
        if (lead) rowc[c] = pv[c];
        const E y = Num<E>::mul(x, pv[c]);
        acc[ES * c] += Num<E>::re(y);
        if (ES == 2) acc[ES * c + ES - 1] += Num<E>::im(y);
      }
    }
  }
  if (!fact) return;
  // wave reduction: fold to D lanes' worth, then halve the set per exchange
#pragma unroll
  for (int m = 32; m >= D; m >>= 1)
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] += __shfl_xor(acc[i], m);
#pragma unroll
  for (int h = D / 2; h >= 1; h >>= 1) {
    const bool up = (lane & h) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double send = up ? acc[i] : acc[i + h];
      const double keep = up ? acc[i + h] : acc[i];
      acc[i] = keep + __shfl_xor(send, h);
    }
  }
  __syncthreads();           // s_red is reused
  s_red[wave][lane] = acc[0];  // lane holds accumulator lane % D
  __syncthreads();
  if (t < D) partc[(int64_t)blockIdx.x * D + t] = s_red[0][t] + s_red[1][t] + s_red[2][t] + s_red[3][t];
}

// The same panel factorisation in one cooperative launch: block b holds
// rows [b R, (b + 1) R) of the panel (all nbp columns) in LDS from start to
// end, so a column step reads and writes only LDS; the steps are separated
// by a grid barrier instead of kernel boundaries.  Column step j:
//  * every block applies reflector j - 1 to its rows (v_r = P[r, j-1] sc for
//    r > j - 1, v = 1 at the pivot row; P[r, c] -= conj(tau) v_r w_c for
//    c > j - 1) and, in the same pass, sums s_c = sum_{r > j} conj(P[r, j])
//    P[r, c] (c >= j) over its rows into its slot of the partial sums; the
//    block holding row j publishes that row;
//  * grid barrier;
//  * every block adds the partial sums of all blocks in block order (all
//    agree bit for bit) and forms beta, tau, the scale 1 / (alpha - beta)
//    and w_c = v^H P[:, c] exactly as k_hh_column does.
// After the last reflector the rows go back to P (R on and above the
// diagonal, the vectors below) and to Vb (explicit vectors, unit diagonal).
// The barrier is a counter of arrivals that starts the launch at `base`;
// a wait longer than `limit` wall-clock ticks sets *err and stops waiting
// (the cooperative launch makes every block resident, so a correct run
// never gets near it).
constexpr size_t kHpBase = kHhStateBytes - kHpStateBytes;  // panel-kernel state
constexpr size_t kHpRow = 0, kHpCtr = 2 * 16 * kHhNB, kHpPart = kHpCtr + 256;
static_assert(kHpPart + 2 * (size_t)kHpMaxBlocks * kHhNB * 16 <= kHpStateBytes, "hp state");
static_assert(kHpBase >= kHhPart + 2 * kHhPartBytes, "panel state overlaps the column state");

// Cross-block data (partial sums, pivot row) moves by agent-coherent loads
// and stores (relaxed atomics at agent scope: no cache of one XCD keeps a
// stale copy), so the barrier needs no cache write-back or invalidation:
// the writers wait for their stores to complete, then thread 0 counts the
// block in and waits for the others.
__device__ __forceinline__ void hp_put(void *dst, double2 v) {
  __hip_atomic_store((double *)dst, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store((double *)dst + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void hp_put(void *dst, double v) {
  __hip_atomic_store((double *)dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename E> __device__ __forceinline__ E hp_get(const void *src);
template <> __device__ __forceinline__ double2 hp_get(const void *src) {
  double2 v;
  v.x = __hip_atomic_load((const double *)src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load((const double *)src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}
template <> __device__ __forceinline__ double hp_get(const void *src) {
  return __hip_atomic_load((const double *)src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void hp_barrier(unsigned *ctr, unsigned target, int *err,
                                           long long limit) {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    unsigned polls = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      // now and then: another block's time-out
      if ((++polls & 63) == 0 &&
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        break;
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  asm volatile("" ::: "memory");
}

constexpr int kHpGroups = 32;                 // row groups: 32 x 32 = 1024 threads
constexpr int kHpThreads = kHpGroups * kHhNB;
constexpr int kHpLoads = 256 / kHpGroups;    // partial-sum loads in flight per thread
constexpr int kHpUnroll = 2;                 // rows per LDS round trip of a column step

template <typename E, int NB, int NG>
__global__ __launch_bounds__(NB * NG) void k_hh_panel(E *__restrict__ P, int64_t ld, int Mp, int nbp,
                                                  int R, E *__restrict__ Vb, int64_t ldv,
                                                  E *__restrict__ tau, char *hs, unsigned base,
                                                  long long limit) {
  static_assert(NB == 32 && NG * kHpLoads >= 256, "thread (g, c): NG row groups x 32 columns");
  constexpr int NT = NB * NG;
  extern __shared__ __align__(16) char hp_lds[];
  E *Pl = (E *)hp_lds;  // R x NB, row-major
  __shared__ E s_red[NG][NB];
  __shared__ E s_w[NB], s_row[NB];
  __shared__ E s_ct, s_sc;
  unsigned *ctr = (unsigned *)(hs + kHpCtr);
  int *err = (int *)(hs + kHpCtr + 64);
  const int t = threadIdx.x, c = t % NB, g = t / NB;
  const int G = gridDim.x;
  const int r0 = blockIdx.x * R;
  const int nr = max(0, min(R, Mp - r0));  // rows of this block
  for (int idx = t; idx < nr * nbp; idx += NT) {
    const int rl = idx % nr, cc = idx / nr;
    Pl[rl * NB + cc] = P[(int64_t)r0 + rl + (int64_t)cc * ld];
  }
  __syncthreads();
  for (int j = 0; j <= nbp; ++j) {
    const int p = j - 1;
    const bool upd = j >= 1, fact = j < nbp;
    const E ct = upd ? s_ct : Num<E>::zero(), sc = upd ? s_sc : Num<E>::zero();
    const E wc = (upd && c > p && c < nbp) ? s_w[c] : Num<E>::zero();
    const E wj = (upd && fact) ? s_w[j] : Num<E>::zero();
    E acc = Num<E>::zero();
    const int jc = fact ? j : nbp - 1;  // a valid column to read when there is no next one
    // rows g, g + NG, ... of the block, kHpUnroll at a time: all their old
    // values are read first (the compiler barrier keeps these reads ahead of
    // the writes of other lanes of this wave to the same rows)
    for (int rb = g; rb < nr; rb += NG * kHpUnroll) {
      E op[kHpUnroll], oj[kHpUnroll], oc[kHpUnroll];
#pragma unroll
      for (int u = 0; u < kHpUnroll; ++u) {
        const E *row = Pl + min(rb + NG * u, nr - 1) * NB;
        op[u] = upd ? row[p] : Num<E>::zero();
        oj[u] = row[jc];
        oc[u] = row[c < nbp ? c : 0];
      }
      asm volatile("" ::: "memory");
#pragma unroll
      for (int u = 0; u < kHpUnroll; ++u) {
        const int rl = rb + NG * u;
        if (rl >= nr) break;
        const int r = r0 + rl;
        E *row = Pl + rl * NB;
        E nc = oc[u], xj = oj[u];
        if (upd && r >= p) {
          const E v = r > p ? Num<E>::mul(op[u], sc) : Num<E>::real(1.0);
          const E cv = Num<E>::mul(ct, v);
          if (fact) xj = oj[u] - Num<E>::mul(cv, wj);
          nc = (fact && c == j) ? xj : oc[u] - Num<E>::mul(cv, wc);
          if (c == p && r > p) row[p] = v;
          if (c > p && c < nbp) row[c] = nc;
        }
        if (fact && c >= j && c < nbp) {
          if (r > j) acc = acc + Num<E>::mul(Num<E>::cj(xj), nc);
          if (r == j) s_row[c] = nc;
        }
      }
    }
    if (!fact) break;
    s_red[g][c] = acc;
    __syncthreads();
    E *partc = (E *)(hs + kHpPart) + (size_t)(j & 1) * kHpMaxBlocks * NB;
    E *rowj = (E *)(hs + kHpRow) + (j & 1) * NB;
    if (t < NB) {
      E v = s_red[0][t];
      for (int q = 1; q < NG; ++q) v = v + s_red[q][t];
      hp_put(&partc[(size_t)blockIdx.x * NB + t], v);
      if (j >= r0 && j < r0 + nr && t >= j && t < nbp) hp_put(&rowj[t], s_row[t]);
    }
    hp_barrier(ctr, base + (unsigned)(G * (j + 1)), err, limit);
    {  // all blocks' sums, block order (thread (g, c) takes blocks g, g + NG, ...),
       // every load in flight at once
      E x[kHpLoads];
      const bool col = c >= j && c < nbp;
#pragma unroll
      for (int u = 0; u < kHpLoads; ++u) {
        const int b = g + NG * u;
        x[u] = (col && b < G) ? hp_get<E>(&partc[(size_t)b * NB + c]) : Num<E>::zero();
      }
      const E rv = (g == 0 && col) ? hp_get<E>(&rowj[c]) : Num<E>::zero();
      E v = x[0];
#pragma unroll
      for (int u = 1; u < kHpLoads; ++u) v = v + x[u];
      s_red[g][c] = v;
      if (g == 0) s_row[c] = rv;
    }
    __syncthreads();
    if (t == j) {  // the reflector's scalars
      const E alpha = s_row[j];
      E sj = s_red[0][j];
      for (int q = 1; q < NG; ++q) sj = sj + s_red[q][j];
      const double xn2 = Num<E>::re(sj);
      E tv = Num<E>::zero(), scn = Num<E>::zero();
      double beta = Num<E>::re(alpha);
      if (xn2 != 0.0 || Num<E>::im(alpha) != 0.0) {
        beta = -copysign(sqrt(Num<E>::abs2(alpha) + xn2), Num<E>::re(alpha));
        tv = Num<E>::scale(Num<E>::real(beta) - alpha, 1.0 / beta);
        scn = recip(alpha - Num<E>::real(beta));
      }
      s_ct = Num<E>::cj(tv);
      s_sc = scn;
      if (blockIdx.x == 0) tau[j] = tv;
      if (j >= r0 && j < r0 + nr) Pl[(j - r0) * NB + j] = Num<E>::real(beta);
    }
    __syncthreads();
    if (t > j && t < nbp) {
      E sv = s_red[0][t];
      for (int q = 1; q < NG; ++q) sv = sv + s_red[q][t];
      s_w[t] = s_row[t] + Num<E>::mul(Num<E>::cj(s_sc), sv);
    }
    __syncthreads();
  }
  __syncthreads();
  for (int idx = t; idx < nr * nbp; idx += NT) {
    const int rl = idx % nr, cc = idx / nr;
    const int64_t r = (int64_t)r0 + rl;
    const E x = Pl[rl * NB + cc];
    P[r + (int64_t)cc * ld] = x;
    if (r >= cc) Vb[r + (int64_t)cc * ldv] = r > cc ? x : Num<E>::real(1.0);
  }
}

// T (nb x nb, upper triangular) of the compact WY form H_0 ... H_{nb-1} =
// I - V T V^H from S = V^H V and tau: T[i][i] = tau_i and
// T[0:i, i] = -tau_i T[0:i, 0:i] S[0:i, i] for blocks of eight columns (side
// by side, eight steps), then pairs of neighbouring blocks joined level by
// level: for the columns L = [a, a + h) and R = [a + h, a + 2h),
// T[L, R] = -T[L, L] S[L, R] T[R, R] (the product of the two compact WY
// forms), W = S[L, R] T[R, R] first (held where T[L, R] goes), then
// -T[L, L] W.  T is a packed upper triangle in LDS, S is read from global
// memory; 8 + 3 log2(nb / 8) barriers instead of one or two per column.
constexpr int kLarftThreads = 8 * kHhMaxOuter;
constexpr int kLarftLeaf = 8;
template <typename E>
__global__ __launch_bounds__(kLarftThreads) void k_hh_larft(const E *S, int64_t lds, const E *tau,
                                                            E *T, int64_t ldt, int nb) {
  typedef Num<E> X;
  __shared__ E sh[kHhMaxOuter * (kHhMaxOuter + 1) / 2];  // (k, i), k <= i, at i (i + 1) / 2 + k
  const int tid = threadIdx.x;
  auto at = [](int k, int i) { return i * (i + 1) / 2 + k; };
  // blocks of eight columns: thread (q, t) of wave q forms T[8q + t, 8q + i]
  {
    const int q = tid >> 6, t = tid & 63, c0 = kLarftLeaf * q;
    const bool act = t < kLarftLeaf && c0 < nb;
    const int gt = c0 + t;
#pragma unroll 1
    for (int i = 0; i < kLarftLeaf; ++i) {
      const int gi = c0 + i;
      if (act && gi < nb && t <= i) {
        E v;
        if (t == i) {
          v = tau[gi];
        } else {
          E acc = X::zero();
          for (int k = t; k < i; ++k)
            acc = acc + X::mul(sh[at(gt, c0 + k)], S[(c0 + k) + (int64_t)gi * lds]);
          v = -X::mul(tau[gi], acc);
        }
        sh[at(gt, gi)] = v;
      }
      __syncthreads();
    }
  }
  for (int h = kLarftLeaf; h < nb; h *= 2) {
    // pair p: L = [2hp, 2hp + h), R = [2hp + h, min(2hp + 2h, nb)); entry
    // (r, c) of the h x h block T[L, R] (c within R's columns)
    const int npairs = (nb + 2 * h - 1) / (2 * h);
    const int per = h * h;
    // W = S[L, R] T[R, R]
    for (int idx = tid; idx < npairs * per; idx += kLarftThreads) {
      const int p = idx / per, r = (idx % per) % h, c = (idx % per) / h;
      const int a = 2 * h * p, gr = a + r, gc = a + h + c;
      if (gc >= nb) continue;
      E acc = X::zero();
      for (int k0 = 0; k0 <= c; k0 += 8) {  // S's loads eight at a time
        E sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          sv[u] = k0 + u <= c ? S[gr + (int64_t)(a + h + k0 + u) * lds] : X::zero();
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (k0 + u <= c) acc = acc + X::mul(sv[u], sh[at(a + h + k0 + u, gc)]);
      }
      sh[at(gr, gc)] = acc;
    }
    __syncthreads();
    // T[L, R] = -T[L, L] W, formed in registers, then stored
    constexpr int kMaxOut = kHhMaxOuter * kHhMaxOuter / 4 / kLarftThreads;  // h <= nb / 2
    E out[kMaxOut > 0 ? kMaxOut : 1];
#pragma unroll
    for (int u = 0; u < (kMaxOut > 0 ? kMaxOut : 1); ++u) {
      const int idx = tid + u * kLarftThreads;
      out[u] = X::zero();
      if (idx < npairs * per) {
        const int p = idx / per, r = (idx % per) % h, c = (idx % per) / h;
        const int a = 2 * h * p, gr = a + r, gc = a + h + c;
        if (gc < nb) {
          E acc = X::zero();
          for (int k = r; k < h; ++k) acc = acc + X::mul(sh[at(gr, a + k)], sh[at(a + k, gc)]);
          out[u] = -acc;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (kMaxOut > 0 ? kMaxOut : 1); ++u) {
      const int idx = tid + u * kLarftThreads;
      if (idx < npairs * per) {
        const int p = idx / per, r = (idx % per) % h, c = (idx % per) / h;
        const int a = 2 * h * p, gr = a + r, gc = a + h + c;
        if (gc < nb) sh[at(gr, gc)] = out[u];
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += kLarftThreads) {
    const int r = idx % nb, c = idx / nb;
    T[r + (int64_t)c * ldt] = r <= c ? sh[at(r, c)] : X::zero();
  }
}

// out (rows x cols) = sum over nsplit partials (fixed order).
template <typename E>
__global__ void k_sum_splits(const E *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                             E *out, int64_t ldo) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= rows) return;
  const int64_t c = blockIdx.y;
  out[c * ldo + q] = sum_strided(P + c * ldp + q, nsplit, sstride);
}

// A (rows x cols) = the first cols columns of the identity.
template <typename E> __global__ void k_set_identity(E *A, int64_t lda, int rows) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  const int64_t j = blockIdx.y;
  A[i + j * lda] = Num<E>::real(i == j ? 1.0 : 0.0);
}

// ========================================================== launchers ==
static inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

#define DISPATCH_E(cplx, KERNEL, grid, block, s, ...)                                   \
  do {                                                                                  \
    if (cplx)                                                                           \
      hipLaunchKernelGGL(KERNEL<double2>, grid, block, 0, s, __VA_ARGS__);              \
    else                                                                                \
      hipLaunchKernelGGL(KERNEL<double>, grid, block, 0, s, __VA_ARGS__);               \
  } while (0)

void reduce_hermitian(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int n,
                      void *G, int64_t ldg, int average, hipStream_t s) {
  if (n <= 0) return;
  dim3 grid(blocks(n, 16), blocks(n, 16)), block(16, 16);
  if (cplx)
    hipLaunchKernelGGL(k_reduce_herm<double2>, grid, block, 0, s, (const double2 *)P, nsplit,
                       sstride, ldp, n, (double2 *)G, ldg, average);
  else
    hipLaunchKernelGGL(k_reduce_herm<double>, grid, block, 0, s, (const double *)P, nsplit,
                       sstride, ldp, n, (double *)G, ldg, average);
}

void trace_shift(bool cplx, void *G, int64_t ldg, int n, double coef, int add_shift,
                 double *trace_out, const int *flag, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(k_trace_shift<double2>, dim3(1), dim3(256), 0, s, (double2 *)G, ldg, n,
                       coef, add_shift, trace_out, flag);
  else
    hipLaunchKernelGGL(k_trace_shift<double>, dim3(1), dim3(256), 0, s, (double *)G, ldg, n,
                       coef, add_shift, trace_out, flag);
}

void chol_diag(bool cplx, void *G, int64_t ldg, void *R, int64_t ldr, void *Ri, int64_t ldi,
               int p0, int b, int *flag, int pass, int inject, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(k_chol_diag<double2>, dim3(1), dim3(kCholThreads), 0, s, (const double2 *)G,
                       ldg, (double2 *)R, ldr, (double2 *)Ri, ldi, p0, b, flag, pass, inject);
  else
    hipLaunchKernelGGL(k_chol_diag<double>, dim3(1), dim3(kCholThreads), 0, s, (const double *)G,
                       ldg, (double *)R, ldr, (double *)Ri, ldi, p0, b, flag, pass, inject);
}

void fill_zero(bool cplx, void *A, int64_t lda, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid(blocks(rows, 256), cols);
  if (cplx)
    hipLaunchKernelGGL(k_fill_zero<double2>, grid, dim3(256), 0, s, (double2 *)A, lda, rows, cols);
  else
    hipLaunchKernelGGL(k_fill_zero<double>, grid, dim3(256), 0, s, (double *)A, lda, rows, cols);
}

void residuals(bool cplx, const void *HV, int64_t ldhv, const void *V, int64_t ldv, int n,
               int ncols, const double *theta, double *resid, hipStream_t s) {
  if (ncols <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(k_resid<double2>, dim3(ncols), dim3(256), 0, s, (const double2 *)HV, ldhv,
                       (const double2 *)V, ldv, n, theta, resid);
  else
    hipLaunchKernelGGL(k_resid<double>, dim3(ncols), dim3(256), 0, s, (const double *)HV, ldhv,
                       (const double *)V, ldv, n, theta, resid);
}

void gather_cols(bool cplx, bool to32, const void *src, int64_t lds, void *dst, int64_t ldd,
                 int n, int ncols, const int *perm, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 grid(blocks(n, 256), ncols);
  if (cplx) {
    if (to32)
      hipLaunchKernelGGL((k_gather<double2, float2>), grid, dim3(256), 0, s, (const double2 *)src,
                         lds, (float2 *)dst, ldd, n, perm);
    else
      hipLaunchKernelGGL((k_gather<double2, double2>), grid, dim3(256), 0, s,
                         (const double2 *)src, lds, (double2 *)dst, ldd, n, perm);
  } else {
    if (to32)
      hipLaunchKernelGGL((k_gather<double, float>), grid, dim3(256), 0, s, (const double *)src,
                         lds, (float *)dst, ldd, n, perm);
    else
      hipLaunchKernelGGL((k_gather<double, double>), grid, dim3(256), 0, s, (const double *)src,
                         lds, (double *)dst, ldd, n, perm);
  }
}

void copy_cols(bool cplx, const void *src, int64_t lds, void *dst, int64_t ldd, int n, int ncols,
               hipStream_t s) {
  gather_cols(cplx, false, src, lds, dst, ldd, n, ncols, nullptr, s);
}

void convert_to32(bool cplx, const void *src, int64_t lds, void *dst, int64_t ldd, int rows,
                  int cols, hipStream_t s) {
  gather_cols(cplx, true, src, lds, dst, ldd, rows, cols, nullptr, s);
}

void randn(bool cplx, void *V, int64_t ldv, int n, int ncols, uint64_t seed, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 grid(blocks(n, 256), ncols);
  if (cplx)
    hipLaunchKernelGGL(k_randn<double2>, grid, dim3(256), 0, s, (double2 *)V, ldv, n, seed);
  else
    hipLaunchKernelGGL(k_randn<double>, grid, dim3(256), 0, s, (double *)V, ldv, n, seed);
}

template <typename E, int NV>
static void gemv_launch(const E *A, int64_t lda, int M, int K, const E *X, int64_t ldx, E *Y,
                        int64_t ldy, void *scratch, size_t scratch_bytes, hipStream_t s) {
  constexpr int RPT = sizeof(E) == 16 ? 2 : 4;
  const int rb = (M + 256 * RPT - 1) / (256 * RPT);
  // enough work-groups to keep every CU streaming, limited by the scratch
  // that holds one M x NV partial per split and by 64 columns per split
  const size_t per = sizeof(E) * (size_t)M * NV;
  int S = (2048 + rb - 1) / rb;
  S = (int)std::min<int64_t>(S, (K + 63) / 64);
  S = (int)std::min<size_t>((size_t)S, scratch_bytes / per);
  if (S <= 1) {
    hipLaunchKernelGGL((k_gemv_cm<E, NV, RPT>), dim3(rb, 1), dim3(256), 0, s, A, lda, M, K, X, ldx,
                       K, Y, ldy, (int64_t)0);
    return;
  }
  int kchunk = (K + S - 1) / S;
  kchunk = (kchunk + 7) / 8 * 8;
  S = (K + kchunk - 1) / kchunk;
  E *P = (E *)scratch;
  hipLaunchKernelGGL((k_gemv_cm<E, NV, RPT>), dim3(rb, S), dim3(256), 0, s, A, lda, M, K, X, ldx,
                     kchunk, P, (int64_t)M, (int64_t)M * NV);
  hipLaunchKernelGGL(k_gemv_reduce<E>, dim3(blocks(M, 256), NV), dim3(256), 0, s, (const E *)P, S,
                     (int64_t)M * NV, M, Y, ldy);
}

template <typename E>
static void gemv_nv(const E *A, int64_t lda, int M, int K, const E *X, int64_t ldx, int nv, E *Y,
                    int64_t ldy, void *scratch, size_t scratch_bytes, hipStream_t s) {
  switch (nv) {
    case 1: gemv_launch<E, 1>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 2: gemv_launch<E, 2>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 3: gemv_launch<E, 3>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 4: gemv_launch<E, 4>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 5: gemv_launch<E, 5>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 6: gemv_launch<E, 6>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 7: gemv_launch<E, 7>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    case 8: gemv_launch<E, 8>(A, lda, M, K, X, ldx, Y, ldy, scratch, scratch_bytes, s); break;
    default: throw InvalidArg();
  }
}

void gemv_block(bool cplx, const void *A, int64_t lda, int M, int K, const void *X, int64_t ldx,
                int nv, void *Y, int64_t ldy, void *scratch, size_t scratch_bytes,
                hipStream_t s) {
  if (M <= 0 || nv <= 0) return;
  if (K <= 0) {
    fill_zero(cplx, Y, ldy, M, nv, s);
    return;
  }
  if (cplx)
    gemv_nv<double2>((const double2 *)A, lda, M, K, (const double2 *)X, ldx, nv, (double2 *)Y,
                     ldy, scratch, scratch_bytes, s);
  else
    gemv_nv<double>((const double *)A, lda, M, K, (const double *)X, ldx, nv, (double *)Y, ldy,
                    scratch, scratch_bytes, s);
}

void dot_re_cols(bool cplx, const void *v, const void *w, int64_t ld, int n, int ncols,
                 double *out, hipStream_t s) {
  if (ncols <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(k_dot_re_cols<double2>, dim3(ncols), dim3(256), 0, s, (const double2 *)v,
                       (const double2 *)w, ld, n, out);
  else
    hipLaunchKernelGGL(k_dot_re_cols<double>, dim3(ncols), dim3(256), 0, s, (const double *)v,
                       (const double *)w, ld, n, out);
}

void norm_scale_cols(bool cplx, const void *w, int64_t ldw, int n, int ncols, void *vout,
                     int64_t ldo, double *beta, hipStream_t s) {
  if (ncols <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(k_norm_scale_cols<double2>, dim3(ncols), dim3(256), 0, s,
                       (const double2 *)w, ldw, n, (double2 *)vout, ldo, beta);
  else
    hipLaunchKernelGGL(k_norm_scale_cols<double>, dim3(ncols), dim3(256), 0, s, (const double *)w,
                       ldw, n, (double *)vout, ldo, beta);
}

void sum_splits_diag(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                     int nv, void *out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || nv <= 0) return;
  dim3 grid(blocks(rows, 256), nv);
  if (cplx)
    hipLaunchKernelGGL(k_sum_splits_diag<double2>, grid, dim3(256), 0, s, (const double2 *)P,
                       nsplit, sstride, ldp, rows, nv, (double2 *)out, ldo);
  else
    hipLaunchKernelGGL(k_sum_splits_diag<double>, grid, dim3(256), 0, s, (const double *)P, nsplit,
                       sstride, ldp, rows, nv, (double *)out, ldo);
}

void lz_step_small(bool cplx, void *LV, int64_t ldv, int N, int j, int nv, void *W, int64_t ldw,
                   double *ab, int k, hipStream_t s) {
  if (N < 1 || N > kLzSmallMaxN || j < 0 || j >= k || k + 1 > kLzSmallMaxBasis || nv < 1)
    throw InvalidArg();
  if (cplx)
    hipLaunchKernelGGL(k_lz_step_small<double2>, dim3(nv), dim3(kLzSmallThreads), 0, s,
                       (double2 *)LV, ldv, N, j, nv, (double2 *)W, ldw, ab, k);
  else
    hipLaunchKernelGGL(k_lz_step_small<double>, dim3(nv), dim3(kLzSmallThreads), 0, s,
                       (double *)LV, ldv, N, j, nv, (double *)W, ldw, ab, k);
}

static unsigned hh_blocks(int Mp, int jj) {
  const int rbeg = jj >= 1 ? jj - 1 : 0;
  return std::min<unsigned>(kHhMaxBlocks, blocks(Mp - rbeg, 256));
}

void hh_column(bool cplx, void *P, int64_t ld, int Mp, int nbp, int jj, void *Vb, int64_t ldv,
               void *tau, void *hh_state, hipStream_t s) {
  if (nbp < 1 || nbp > kHhNB || jj < 0 || jj > nbp || Mp < nbp) throw InvalidArg();
  const unsigned nblk = hh_blocks(Mp, jj);
  const int nprev = jj >= 1 ? (int)hh_blocks(Mp, jj - 1) : 0;
  if (cplx)
    hipLaunchKernelGGL((k_hh_column<double2, kHhNB>), dim3(nblk), dim3(256), 0, s, (double2 *)P,
                       ld, Mp, nbp, jj, nprev, (double2 *)Vb, ldv, (double2 *)tau,
                       (char *)hh_state);
  else
    hipLaunchKernelGGL((k_hh_column<double, kHhNB>), dim3(nblk), dim3(256), 0, s, (double *)P, ld,
                       Mp, nbp, jj, nprev, (double *)Vb, ldv, (double *)tau, (char *)hh_state);
}

// Wall-clock ticks a grid-barrier wait (panel and Lanczos launches) may take before it gives
// up; <= 0: two seconds.
static std::atomic<long long> g_hp_wait_ticks{0};
void hh_panel_set_wait_limit(long long ticks) { g_hp_wait_ticks.store(ticks); }

template <typename E>
static bool hh_panel_launch(E *P, int64_t ld, int Mp, int nbp, E *Vb, int64_t ldv, E *tau,
                            char *hs, unsigned *base, hipStream_t s) {
  struct Info { int ncu, per; long long ticks; };
  auto kern = k_hh_panel<E, kHhNB, kHpGroups>;
  // once per process (thread-safe static initialisation)
  static const Info info = [&] {
    const size_t lds_max = (size_t)kHpMaxRows * kHhNB * sizeof(E);
    Info f{0, 0, 0};
    int dev = 0, khz = 0;
    CHASE_HIP(hipGetDevice(&dev));
    CHASE_HIP(hipDeviceGetAttribute(&f.ncu, hipDeviceAttributeMultiprocessorCount, dev));
    CHASE_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    CHASE_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_max));
    CHASE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.per, kern, kHpThreads, lds_max));
    f.ticks = (long long)khz * 1000LL * 2;  // two seconds
    return f;
  }();
  // about kHpRows rows per block, one block per compute unit at most
  int G = std::max(1, std::min(info.ncu, (Mp + kHpRows - 1) / kHpRows));
  int R = (Mp + G - 1) / G;
  if (R > kHpMaxRows || G > kHpGroups * kHpLoads || info.per < 1) return false;
  G = (Mp + R - 1) / R;
  const size_t lds = (size_t)R * kHhNB * sizeof(E);
  unsigned b0 = *base;
  const long long set = g_hp_wait_ticks.load();
  long long ticks = set > 0 ? set : info.ticks;
  void *args[] = {&P, &ld, &Mp, &nbp, &R, &Vb, &ldv, &tau, &hs, &b0, &ticks};
  CHASE_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(G), dim3(kHpThreads), args, lds, s));
  *base += (unsigned)(G * nbp);
  return true;
}

bool hh_panel(bool cplx, void *P, int64_t ld, int Mp, int nbp, void *Vb, int64_t ldv, void *tau,
              void *hh_state, unsigned *base, hipStream_t s) {
  if (nbp < 1 || nbp > kHhNB || Mp < nbp) throw InvalidArg();
  char *hs = (char *)hh_state + kHpBase;
  if (cplx)
    return hh_panel_launch<double2>((double2 *)P, ld, Mp, nbp, (double2 *)Vb, ldv, (double2 *)tau,
                                    hs, base, s);
  return hh_panel_launch<double>((double *)P, ld, Mp, nbp, (double *)Vb, ldv, (double *)tau, hs,
                                 base, s);
}

void hh_panel_reset(void *hh_state, hipStream_t s) {
  fill_zero(false, (char *)hh_state + kHpBase + kHpCtr, 1, 8, 1, s);  // the counter's 64 bytes
}

void hh_panel_clear_error(void *hh_state, hipStream_t s) {
  fill_zero(false, (char *)hh_state + kHpBase + kHpCtr + 64, 1, 8, 1, s);
}

const void *hh_panel_error(const void *hh_state) {
  return (const char *)hh_state + kHpBase + kHpCtr + 64;
}

// ------------------------------------------ Lanczos in one launch (small N) --
// The solver's nv Lanczos runs (full reorthogonalisation: classical
// Gram-Schmidt twice against the run's own basis) for small orders, all k
// steps in one cooperative launch.  Block b owns rows [b R, b R + R) of
// every vector and keeps its rows of the basis in LDS.  Step j:
//  * w = H v_j on the block's rows, v_j staged in LDS chunk by chunk (V0 for
//    j = 0; else the other blocks' rows of w_j from the exchange buffer XV,
//    scaled by 1 / beta_{j-1} exactly as each block scales its own rows);
//  * two Gram-Schmidt passes h = V^H w, w -= V h, the inner products as
//    block partial sums, a grid barrier, and every block adding all blocks'
//    partials in block order (all blocks agree bit for bit);
//  * the block's rows of w (unnormalised) go to XV with its partial sum of
//    |w|^2; after the barrier every block forms beta_j and v_{j+1} = w /
//    beta_j.
// Three grid barriers per step.  Cross-block data moves by agent-coherent
// stores and loads (as in the Householder panel kernel); the partial sums
// use two areas of `part`, alternating barrier by barrier.  Output as the
// per-step launches write it: alpha_j of run r at ab[j nv + r], beta_j at
// ab[(k + j) nv + r].
constexpr int kLzcRows = 16;  // least rows per block (32 and 64 measured slower)
constexpr int kLzcThreads = 256;
constexpr size_t kLzcMaxLds = 144 * 1024;
constexpr size_t kLzcStageBytes = 32 * 1024;  // staged chunk of v_j

// out[e] = sum_{g < G} pr[g slot + e] for e < nE, every block in the same
// order: the blocks split into Q consecutive ranges per value (Q from nE
// alone), each range added in block order by one thread with its loads
// issued sixteen at a time, then the ranges in order.  sQ: max(kLzcThreads,
// nE) elements.  Ends with a barrier of the block.
template <typename E>
__device__ void lzc_sum_partials(const E *pr, int nE, int G, size_t slot, E *sQ, E *out) {
  const int t = threadIdx.x;
  const int Q = max(1, min(G, kLzcThreads / nE));
  for (int idx = t; idx < nE * Q; idx += kLzcThreads) {
    const int e = idx % nE, q = idx / nE;
    const int g0 = q * G / Q, g1 = (q + 1) * G / Q;
    E s = Num<E>::zero();
    for (int g = g0; g < g1; g += 16) {
      E x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        x[u] = g + u < g1 ? hp_get<E>(pr + (size_t)(g + u) * slot + e) : Num<E>::zero();
#pragma unroll
      for (int u = 0; u < 16; ++u) s = s + x[u];
    }
    sQ[idx] = s;
  }
  __syncthreads();
  for (int e = t; e < nE; e += kLzcThreads) {
    E s = Num<E>::zero();
    for (int q = 0; q < Q; ++q) s = s + sQ[q * nE + e];
    out[e] = s;
  }
  __syncthreads();
}

template <typename E, int NV>
__global__ __launch_bounds__(kLzcThreads) void k_lanczos_coop(
    const E *__restrict__ H, int64_t ldh, int N, int k, int R, const E *__restrict__ V0, E *XV,
    double *ab, E *part, char *hs, unsigned base, long long limit) {
  typedef Num<E> X;
  constexpr int CH = (int)(kLzcStageBytes / (NV * sizeof(E)));  // columns per staged chunk
  extern __shared__ __align__(16) char lzc_lds[];
  const int nQ = max(kLzcThreads, (k + 1) * NV);
  E *sB = (E *)lzc_lds;                    // (k + 1) x NV x R: this block's rows of the basis
  E *sW = sB + (size_t)(k + 1) * NV * R;   // NV x R: its rows of w
  E *sRed = sW + (size_t)NV * R;           // kLzcThreads x NV: product partials
  E *sH = sRed + (size_t)kLzcThreads * NV; // (k + 1) x NV: Gram-Schmidt coefficients
  E *sQ = sH + (size_t)(k + 1) * NV;       // nQ: range sums of lzc_sum_partials
  E *sV = sQ + nQ;                         // CH x NV: staged chunk of v_j
  __shared__ double sInv[NV];
  unsigned *ctr = (unsigned *)(hs + kHpCtr);
  int *err = (int *)(hs + kHpCtr + 64);
  const int t = threadIdx.x, G = gridDim.x, b = blockIdx.x;
  const int r0 = b * R, nr = min(R, N - r0);
  const int CG = kLzcThreads / R, row = t % R, cg = t / R;
  const size_t slot = (size_t)(k + 1) * NV;  // one block's partial sums
  unsigned nbar = 0;
  auto put_area = [&]() { return part + (size_t)((nbar + 1) & 1) * G * slot + (size_t)b * slot; };
  auto get_area = [&]() { return (const E *)(part + (size_t)(nbar & 1) * G * slot); };
  auto sync_grid = [&]() {
    ++nbar;
    hp_barrier(ctr, base + nbar * (unsigned)G, err, limit);
  };
  for (int e = t; e < NV * R; e += kLzcThreads) {
    const int rr = e % R, r = e / R;
    sB[(size_t)r * R + rr] = rr < nr ? V0[(int64_t)r * N + r0 + rr] : X::zero();
  }
  for (int j = 0; j < k; ++j) {
    const int nb = j + 1;
    // w = H v_j on this block's rows: thread (row, cg) takes the columns cg,
    // cg + CG, ... of each chunk, sixteen loads of H in flight; the column
    // groups' sums are then added in order
    E acc[NV];
#pragma unroll
    for (int r = 0; r < NV; ++r) acc[r] = X::zero();
    const E *vj = j == 0 ? V0 : XV;
    for (int c0 = 0; c0 < N; c0 += CH) {
      const int nc = min(CH, N - c0);
      __syncthreads();  // the previous chunk is consumed
      for (int e0 = t; e0 < nc * NV; e0 += 16 * kLzcThreads) {
        E x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = e0 + u * kLzcThreads;  // column c0 + e % nc of run e / nc
          x[u] = e < nc * NV ? hp_get<E>(vj + (int64_t)(e / nc) * N + c0 + e % nc) : X::zero();
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = e0 + u * kLzcThreads;
          if (e < nc * NV)
            sV[(e % nc) * NV + e / nc] = j == 0 ? x[u] : X::scale(x[u], sInv[e / nc]);
        }
      }
      __syncthreads();
      if (row < nr) {
        const E *hr = H + r0 + row + (int64_t)c0 * ldh;
        for (int c = cg; c < nc; c += 16 * CG) {
          E h[16];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            h[u] = c + u * CG < nc ? hr[(int64_t)(c + u * CG) * ldh] : X::zero();
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (c + u * CG < nc)
#pragma unroll
              for (int r = 0; r < NV; ++r)
                acc[r] = acc[r] + X::mul(h[u], sV[(c + u * CG) * NV + r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NV; ++r) sRed[(size_t)t * NV + r] = acc[r];
    __syncthreads();
    for (int e = t; e < NV * R; e += kLzcThreads) {
      const int rr = e % R, r = e / R;
      E s = X::zero();
      for (int q = 0; q < CG; ++q) s = s + sRed[(size_t)(q * R + rr) * NV + r];
      sW[(size_t)r * R + rr] = s;
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      // h_i = v_i^H w (i <= j): this block's rows, then every block's
      E *pw = put_area();
      for (int e = t; e < nb * NV; e += kLzcThreads) {
        const E *bi = sB + (size_t)e * R;  // entry e = i NV + r: basis vector i of run r
        const E *wr = sW + (size_t)(e % NV) * R;
        E s = X::zero();
        for (int rr = 0; rr < nr; ++rr) s = s + X::mul(X::cj(bi[rr]), wr[rr]);
        hp_put(pw + e, s);
      }
      sync_grid();
      lzc_sum_partials(get_area(), nb * NV, G, slot, sQ, sH);
      if (pass == 0 && b == 0 && t < NV) ab[(int64_t)j * NV + t] = X::re(sH[(size_t)j * NV + t]);
      // w -= sum_i v_i h_i
      for (int e = t; e < NV * R; e += kLzcThreads) {
        const int rr = e % R, r = e / R;
        if (rr < nr) {
          E x = sW[(size_t)r * R + rr];
          for (int i = 0; i < nb; ++i)
            x = x - X::mul(sB[((size_t)i * NV + r) * R + rr], sH[(size_t)i * NV + r]);
          sW[(size_t)r * R + rr] = x;
        }
      }
      __syncthreads();
    }
    // beta_j = ||w||: the rows of w and the partial |w|^2 go out together;
    // every block forms beta_j and v_{j+1} = w / beta_j from them
    E *pw = put_area();
    if (t < NV) {
      double sq = 0.0;
      for (int rr = 0; rr < nr; ++rr) sq += X::abs2(sW[(size_t)t * R + rr]);
      hp_put(pw + t, X::real(sq));
    }
    if (j + 1 < k)
      for (int e = t; e < NV * R; e += kLzcThreads) {
        const int rr = e % R, r = e / R;
        if (rr < nr) hp_put(XV + (int64_t)r * N + r0 + rr, sW[(size_t)r * R + rr]);
      }
    sync_grid();
    lzc_sum_partials(get_area(), NV, G, slot, sQ, sH);
    if (t < NV) {
      const double beta = sqrt(X::re(sH[t]));
      sInv[t] = beta > 0.0 ? 1.0 / beta : 0.0;
      if (b == 0) ab[(int64_t)(k + j) * NV + t] = beta;
    }
    __syncthreads();
    for (int e = t; e < NV * R; e += kLzcThreads) {
      const int rr = e % R, r = e / R;
      sB[((size_t)(j + 1) * NV + r) * R + rr] =
          rr < nr ? X::scale(sW[(size_t)r * R + rr], sInv[r]) : X::zero();
    }
  }
}

template <typename E, int NV>
static bool lzc_launch(const E *H, int64_t ldh, int N, int k, const E *V0, E *XV, double *ab,
                       E *part, size_t part_bytes, char *hs, hipStream_t s) {
  struct Info { int ncu, per; long long ticks; };
  auto kern = k_lanczos_coop<E, NV>;
  static const Info info = [&] {
    Info f{0, 0, 0};
    int dev = 0, khz = 0;
    CHASE_HIP(hipGetDevice(&dev));
    CHASE_HIP(hipDeviceGetAttribute(&f.ncu, hipDeviceAttributeMultiprocessorCount, dev));
    CHASE_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    CHASE_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kLzcMaxLds));
    CHASE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.per, kern, kLzcThreads, kLzcMaxLds));
    f.ticks = (long long)khz * 1000LL * 2;  // two seconds
    return f;
  }();
  // rows per block: a power of two from kLzcRows, one block per compute
  // unit at most
  int R = kLzcRows;
  while ((int64_t)R * info.ncu < N) R *= 2;
  if (R > kLzcThreads || info.per < 1) return false;
  const int G = (N + R - 1) / R;
  const size_t nq = std::max<size_t>(kLzcThreads, (size_t)(k + 1) * NV);
  const size_t lds = sizeof(E) * ((size_t)(k + 1) * NV * R + (size_t)NV * R +
                                  (size_t)kLzcThreads * NV + (size_t)(k + 1) * NV + nq) +
                     kLzcStageBytes;
  if (lds > kLzcMaxLds || 2 * sizeof(E) * (size_t)G * (k + 1) * NV > part_bytes) return false;
  const long long set = g_hp_wait_ticks.load();
  long long ticks = set > 0 ? set : info.ticks;
  unsigned b0 = 0;
  int R_ = R;
  void *args[] = {&H, &ldh, &N, &k, &R_, &V0, &XV, &ab, &part, &hs, &b0, &ticks};
  CHASE_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(G), dim3(kLzcThreads), args, lds,
                                       s));
  return true;
}

template <typename E>
static bool lzc_nv(const E *H, int64_t ldh, int N, int k, int nv, const E *V0, E *XV, double *ab,
                   E *part, size_t part_bytes, char *hs, hipStream_t s) {
  switch (nv) {
#define LZC(n) \
  case n: return lzc_launch<E, n>(H, ldh, N, k, V0, XV, ab, part, part_bytes, hs, s);
    LZC(1) LZC(2) LZC(3) LZC(4) LZC(5) LZC(6) LZC(7) LZC(8)
#undef LZC
    default: return false;
  }
}

bool lanczos_coop(bool cplx, const void *H, int64_t ldh, int N, int k, int nv, const void *V0,
                  void *XV, double *ab, void *part, size_t part_bytes, void *hh_state,
                  hipStream_t s) {
  if (N < 1 || k < 1 || nv < 1) throw InvalidArg();
  char *hs = (char *)hh_state + kHpBase;
  hh_panel_reset(hh_state, s);
  if (cplx)
    return lzc_nv<double2>((const double2 *)H, ldh, N, k, nv, (const double2 *)V0, (double2 *)XV,
                           ab, (double2 *)part, part_bytes, hs, s);
  return lzc_nv<double>((const double *)H, ldh, N, k, nv, (const double *)V0, (double *)XV, ab,
                        (double *)part, part_bytes, hs, s);
}

void hh_larft(bool cplx, const void *S, int64_t lds, const void *tau, void *T, int64_t ldt,
              int nb, hipStream_t s) {
  if (nb < 1 || nb > kHhMaxOuter) throw InvalidArg();
  if (cplx)
    hipLaunchKernelGGL(k_hh_larft<double2>, dim3(1), dim3(kLarftThreads), 0, s, (const double2 *)S,
                       lds, (const double2 *)tau, (double2 *)T, ldt, nb);
  else
    hipLaunchKernelGGL(k_hh_larft<double>, dim3(1), dim3(kLarftThreads), 0, s, (const double *)S,
                       lds, (const double *)tau, (double *)T, ldt, nb);
}

void sum_splits(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                int cols, void *out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid(blocks(rows, 256), cols);
  if (cplx)
    hipLaunchKernelGGL(k_sum_splits<double2>, grid, dim3(256), 0, s, (const double2 *)P, nsplit,
                       sstride, ldp, rows, (double2 *)out, ldo);
  else
    hipLaunchKernelGGL(k_sum_splits<double>, grid, dim3(256), 0, s, (const double *)P, nsplit,
                       sstride, ldp, rows, (double *)out, ldo);
}

void set_identity(bool cplx, void *A, int64_t lda, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid(blocks(rows, 256), cols);
  if (cplx)
    hipLaunchKernelGGL(k_set_identity<double2>, grid, dim3(256), 0, s, (double2 *)A, lda, rows);
  else
    hipLaunchKernelGGL(k_set_identity<double>, grid, dim3(256), 0, s, (double *)A, lda, rows);
}

// ------------------------------------------------------------- GEMM ------
// K chunk of every tile (also the split granularity) and the K chunk of the
// big tiles.  Measured on MI355X at N = 20000 x 1300 columns: complex FP64
// 63 TFLOP/s with BK = 8 (50 KB LDS, 2 blocks / CU) against 57 with BK = 16
// (99 KB, 1 block / CU); real FP64 53 with BK = 16 against 52 with BK = 8.
#ifndef CHASE_BIG_BK_CPLX
#define CHASE_BIG_BK_CPLX 8
#endif
#ifndef CHASE_BIG_BK_REAL
#define CHASE_BIG_BK_REAL 16
#endif
// Complex big tiles: three-product form (M3) on waves of 32 x 32.  Measured
// at N = 20000 x 1300 columns (filter, algorithmic 8 flops per complex MAC):
// FP64 four-product 128x64 62.8 TFLOP/s, M3 128x64 (8 waves) 73.1, M3 64x64
// (4 waves, 3 blocks / CU) 78.5; FP32 122.3 / 146.6 / 145.2.
#ifndef CHASE_CPLX_3M
#define CHASE_CPLX_3M 1
#endif
#ifndef CHASE_CPLX_3M_BM
#define CHASE_CPLX_3M_BM 64
#endif
// Real big tiles (waves of BM/2 x BN/2).
#ifndef CHASE_REAL_BM
#define CHASE_REAL_BM 128
#endif
#ifndef CHASE_REAL_BN
#define CHASE_REAL_BN 128
#endif
constexpr int kBK = 16;
int gemm_bk() { return kBK; }

// Blocks of one launch that run at once (occupancy x compute units).
template <typename K> static int resident_blocks(K kernel, int nthreads) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, nthreads, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return ncu * per;
}

// Launch of one GEMM kernel over the tiles of C, with the remainder split:
// the tiles beyond the last full wave of resident blocks are split along K
// across the idle slots of that wave; their partial sums go to the scratch
// and a reduce kernel applies the epilogue.
template <auto KERNEL, typename T, bool CPLX, int EPI, typename FT, int SHAPE, int BM, int BN,
          int NT>
static int launch_tiles(GemmArgs &a, int splits, hipStream_t s) {
  const int nbm = (a.M + BM - 1) / BM, nbn = (a.N + BN - 1) / BN;
  if (nbm <= 0 || nbn <= 0) return 0;
  if (splits < 1) splits = 1;
  if (a.k_per_split <= 0) a.k_per_split = ((a.K + kBK - 1) / kBK) * kBK;
  const int T_ = nbm * nbn;
  a.tile0 = 0;
  a.ntiles = 0;
  a.Pk = nullptr;
  if (SHAPE == GEMM_BIG && splits == 1 && !a.tri && a.tail_ws != nullptr) {
    static const int C = resident_blocks(KERNEL, NT);
    const size_t es = sizeof(T) * (CPLX ? 2 : 1);
    const int full = C > 0 ? (T_ / C) * C : T_;
    const int R = T_ - full;
    int S = R > 0 ? std::min(C / R, 8) : 0;
    S = std::min(S, a.K / (2 * kBK));
    if (R > 0 && S >= 2 && (size_t)R * S * BM * BN * es <= a.tail_ws_bytes) {
      if (full > 0) {
        GemmArgs b = a;
        b.ntiles = full;
        hipLaunchKernelGGL(KERNEL, dim3((unsigned)full, 1), dim3(NT), 0, s, b);
      }
      GemmArgs b = a;
      b.tile0 = full;
      b.ntiles = R;
      b.Pk = a.tail_ws;
      b.k_per_split = ((a.K + S - 1) / S + kBK - 1) / kBK * kBK;
      hipLaunchKernelGGL(KERNEL, dim3((unsigned)R, (unsigned)S), dim3(NT), 0, s, b);
      const int64_t elems = (int64_t)R * BM * BN;
      hipLaunchKernelGGL((gemm_reduce_kernel<T, CPLX, BM, BN, EPI, FT>),
                         dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s, b, S);
      return full > 0 ? 2 : 1;
    }
  }
  dim3 grid((unsigned)T_, (unsigned)splits);
  hipLaunchKernelGGL(KERNEL, grid, dim3(NT), 0, s, a);
  return 1;
}

template <typename T, bool CPLX, bool AT, int EPI, typename FT, int SHAPE>
static int gemm_launch(GemmArgs &a, int splits, hipStream_t s) {
  constexpr bool M3 = CPLX && SHAPE == GEMM_BIG && CHASE_CPLX_3M;
  constexpr int BM = SHAPE == GEMM_BIG ? (M3 ? CHASE_CPLX_3M_BM : (CPLX ? 128 : CHASE_REAL_BM)) : 64;
  constexpr int BN = SHAPE == GEMM_BIG ? (CPLX ? 64 : CHASE_REAL_BN) : 64;
  constexpr int WM = M3 ? 32 : BM / 2, WN = M3 ? 32 : BN / 2;
  constexpr int NT = 64 * (BM / WM) * (BN / WN);
  constexpr int BK = SHAPE == GEMM_BIG ? (CPLX ? CHASE_BIG_BK_CPLX : CHASE_BIG_BK_REAL) : kBK;
  constexpr int MINB = 1;
  static_assert(kBK % BK == 0, "split granularity");
  // direct global -> LDS loads: complex 64 x 64 three-product tiles with
  // both operands K-contiguous and 16-byte aligned rows
  constexpr bool DMA = CHASE_GEMM_DMA && M3 && AT && BM == 64 && BN == 64 && WM == 32 && WN == 32;
  constexpr bool DMAR = CHASE_GEMM_DMA && !CPLX && AT && sizeof(T) == 8 && SHAPE == GEMM_BIG &&
                        ((BM == 128 && BN == 128 && WM == 64 && WN == 64) ||
                         (BM == 64 && BN == 64 && WM == 32 && WN == 32)) && BK == 16;
  if constexpr (DMAR) {
    const bool aligned = (uintptr_t)a.A % 16 == 0 && (uintptr_t)a.B % 16 == 0 &&
                         a.lda % 2 == 0 && a.ldb % 2 == 0;
    if (aligned) {
      if constexpr (BM == 128 && BN == 128) {
        // 64 x 64 tiles instead when the 128-column padding of the output
        // costs more than the larger tile gains (about 11% measured: real
        // N = 20000 x 1300 runs at 60.7 against 57.2 TFLOP/s; 10000 x 300
        // at 48.2 against 57.2) or when the matrix is small
        const double w128 = ((a.N + 127) / 128 * 128) / (double)a.N;
        const double w64 = ((a.N + 63) / 64 * 64) / (double)a.N;
        if (w128 > 1.11 * w64 || a.M < 4096)
          return launch_tiles<gemm_kernel<T, CPLX, AT, false, 64, 64, BK, 32, 32, EPI, FT, MINB,
                                          M3, true>,
                              T, CPLX, EPI, FT, SHAPE, 64, 64, 256>(a, splits, s);
      }
      return launch_tiles<gemm_kernel<T, CPLX, AT, false, BM, BN, BK, WM, WN, EPI, FT, MINB, M3,
                                      true>,
                          T, CPLX, EPI, FT, SHAPE, BM, BN, NT>(a, splits, s);
    }
  }
  if constexpr (DMA) {
    constexpr int BKD = 128 / (2 * (int)sizeof(T));
    static_assert(kBK % BKD == 0, "split granularity");
    const size_t es = 2 * sizeof(T);
    const bool aligned = (uintptr_t)a.A % 16 == 0 && (uintptr_t)a.B % 16 == 0 &&
                         ((size_t)a.lda * es) % 16 == 0 && ((size_t)a.ldb * es) % 16 == 0;
    if (aligned)
      return launch_tiles<gemm_kernel<T, CPLX, AT, CPLX && AT, BM, BN, BKD, WM, WN, EPI, FT, MINB,
                                      M3, true>,
                          T, CPLX, EPI, FT, SHAPE, BM, BN, NT>(a, splits, s);
  }
  return launch_tiles<gemm_kernel<T, CPLX, AT, CPLX && AT, BM, BN, BK, WM, WN, EPI, FT, MINB, M3,
                                  false>,
                      T, CPLX, EPI, FT, SHAPE, BM, BN, NT>(a, splits, s);
}

int gemm(bool cplx, bool prec32, bool at, bool epi_filter, bool out64, GemmShape shape,
         GemmArgs &a, int splits, hipStream_t s) {
  if (epi_filter) {  // filter steps: A = H read K-contiguous, big tiles
    if (prec32) {
      if (!out64) throw InvalidArg();
      if (cplx) return gemm_launch<float, true, true, EPI_FILTER, double, GEMM_BIG>(a, splits, s);
      return gemm_launch<float, false, true, EPI_FILTER, double, GEMM_BIG>(a, splits, s);
    }
    if (cplx) return gemm_launch<double, true, true, EPI_FILTER, double, GEMM_BIG>(a, splits, s);
    return gemm_launch<double, false, true, EPI_FILTER, double, GEMM_BIG>(a, splits, s);
  }
  if (prec32) throw InvalidArg();
#define G_CASE(C, A, S)                                                                  \
  if (cplx == C && at == A && shape == S)                                                \
    return gemm_launch<double, C, A, EPI_AXPBY, double, S>(a, splits, s);
  G_CASE(false, false, GEMM_BIG)
  G_CASE(false, true, GEMM_BIG)
  G_CASE(false, false, GEMM_SMALL)
  G_CASE(false, true, GEMM_SMALL)
  G_CASE(true, false, GEMM_BIG)
  G_CASE(true, true, GEMM_BIG)
  G_CASE(true, false, GEMM_SMALL)
  G_CASE(true, true, GEMM_SMALL)
#undef G_CASE
  throw InvalidArg();
}

}  // namespace chase
