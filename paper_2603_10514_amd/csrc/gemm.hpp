// One MFMA GEMM core for every dense contraction of the solver:
//   C(M x N) = op(A) B, reduction over K, with a fused epilogue.
//
//  * A is read either "K-contiguous" (AT = true: A(i,k) at A[i*lda + k], i.e.
//    the memory holds A^T column-major; with CONJA the element is conjugated)
//    or "M-contiguous" (AT = false: A(i,k) at A[k*lda + i], plain column-major).
//    The filter reads H this way with A(i,k) = conj(H[k + i*ldh]) = H(i,k) for a
//    Hermitian H, so both operands stream along contiguous columns.
//  * B is column-major K x N: B(k,j) at B[(col0 + j)*ldb + k].
//  * Complex products use three real MFMAs per block of 16x16 outputs on the
//    big tiles (M3, see gemm_kernel) and four elsewhere
//    (re = ar br - ai bi, im = ar bi + ai br).
//  * MFMA: v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32); both
//    take A(i = lane%16, k = lane/16) and B(k = lane/16, j = lane%16).  The
//    four results of a lane are D(i, j = lane%16) with i = 4*(lane/16) + r for
//    FP32 but i = lane/16 + 4*r for FP64 (r = 0..3; measured on gfx950).
//  * 256 threads = 4 waves in a 2 x 2 arrangement.  Two K loops:
//    - direct-load (both operands K-contiguous with 16-byte aligned rows: the
//      filter and the Rayleigh-Ritz H Q): K chunks copied by
//      global_load_lds_dwordx4 into a ring of LDS stages in a swizzled
//      row layout (dma_mainloop, dma_mainloop_real);
//    - register prefetch (everything else): LDS double-buffered tiles with a
//      register prefetch of the next K chunk, stored [k][i] with one element
//      of padding so that the transposing stores are conflict-free.
//  * Block -> tile mapping is XCD aware: consecutive hardware block ids go
//    round-robin to the 8 XCDs, so each XCD is handed a contiguous range of
//    logical tiles, ordered in bands of tile rows (tile_coords) so that the
//    blocks resident together share row and column panels in its L2.
//
// Epilogues:
//  EPI_AXPBY   C = alpha * acc + beta * C (beta == 0: C not read); with K
//              splits, split s writes C + s * split_stride.
//  EPI_FILTER  one step of the sigma-scaled Chebyshev recurrence (Alg. 4):
//              out = alpha * (acc - shift * Xcur) + beta * Xprev, where Xcur is
//              B itself (K == M); the columns are sorted by ascending degree,
//              so those whose degree equals this step (their last step,
//              Sec. 2.2) are the global columns below final_end: they go to
//              Ofinal, the others to Onext.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace chase {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4v acc;
  __device__ static __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  __device__ static __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef f4v acc;
  __device__ static __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  __device__ static __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Element types as the GEMM reads and writes them: T, or a native 2-vector
// (re, im) for complex data (bit-compatible with interleaved storage).
template <typename T, bool CPLX> struct MemT { typedef T type; };
template <typename T> struct MemT<T, true> { typedef T __attribute__((ext_vector_type(2))) type; };

template <typename T> __device__ __forceinline__ T mre(T v) { return v; }
template <typename T> __device__ __forceinline__ T mim(T) { return (T)0; }
__device__ __forceinline__ double mre(double __attribute__((ext_vector_type(2))) v) { return v.x; }
__device__ __forceinline__ double mim(double __attribute__((ext_vector_type(2))) v) { return v.y; }
__device__ __forceinline__ float mre(float __attribute__((ext_vector_type(2))) v) { return v.x; }
__device__ __forceinline__ float mim(float __attribute__((ext_vector_type(2))) v) { return v.y; }

template <typename M, typename T> __device__ __forceinline__ M mmake(T r, T i) {
  if constexpr (sizeof(M) == sizeof(T)) {
    return (M)r;
  } else {
    M v;
    v.x = r;
    v.y = i;
    return v;
  }
}

enum { EPI_AXPBY = 0, EPI_FILTER = 1 };

struct GemmArgs {
  const void *A; int64_t lda;
  const void *B; int64_t ldb;
  int M, N, K;
  int col0;              // first global column of B (and of the filter buffers)
  int ccol0;             // first global column of C (EPI_AXPBY)
  int tri;               // skip blocks strictly below the diagonal of C
  int kcap;              // B upper triangular: block column n uses k < col0 + n0 + BN
  int k_per_split;       // K range of one split (multiple of BK); grid.y = #splits
  int64_t split_stride;  // elements between the outputs of two splits
  void *C; int64_t ldc;  // EPI_AXPBY
  double alpha, beta;
  double shift;          // EPI_FILTER
  const void *Xprev; int64_t ldp;
  void *Onext; int64_t ldn;
  void *Ofinal; int64_t ldf;
  int final_end;          // EPI_FILTER: global columns < final_end are final
  const int *flag;       // non-null and *flag != 0: the launch does nothing
  // remainder split (set by the launcher): this launch covers logical tiles
  // [tile0, tile0 + ntiles) (ntiles == 0: all); with Pk set, every (tile,
  // split) writes its raw BM x BN partial sum to Pk and gemm_reduce_kernel
  // applies the epilogue.
  int tile0, ntiles;
  void *Pk;
  void *tail_ws; size_t tail_ws_bytes;  // scratch the launcher may use for Pk
};

// Logical tile g -> (tile row, tile column).  Tiles are grouped in bands of
// GM tile rows walked column by column, so that the blocks resident on one
// XCD at a time cover about GM rows x (resident / GM) columns and share both
// their H row panels and their X column panels in that XCD's L2.
#ifndef CHASE_TILE_GROUP
#define CHASE_TILE_GROUP 8
#endif
__device__ __forceinline__ void tile_coords(int g, int nbm, int nbn, int &bm, int &bn) {
  constexpr int GM = CHASE_TILE_GROUP;
  const int band = g / (GM * nbn);
  const int rows = min(GM, nbm - band * GM);
  const int r = g - band * GM * nbn;
  bm = band * GM + r % rows;
  bn = r / rows;
}

// The epilogue of one output element (row i, column j of this launch).
template <typename T, bool CPLX, int EPI, typename FT>
__device__ __forceinline__ void epilogue_store(const GemmArgs &p, int i, int j, T ar, T ai,
                                               int64_t split_off) {
  typedef typename MemT<T, CPLX>::type E;
  typedef const E __attribute__((address_space(1))) GE;
  typedef E __attribute__((address_space(1))) GEw;
  const T alpha = (T)p.alpha, beta = (T)p.beta;
  if constexpr (EPI == EPI_AXPBY) {
    GEw *Cg = (GEw *)p.C + split_off + (int64_t)(p.ccol0 + j) * p.ldc;
    T vr = alpha * ar, vi = alpha * ai;
    if (p.beta != 0.0) {
      const E c = Cg[i];
      vr += beta * mre(c);
      vi += beta * mim(c);
    }
    Cg[i] = mmake<E, T>(vr, vi);
  } else {
    typedef typename MemT<FT, CPLX>::type EF;
    typedef EF __attribute__((address_space(1))) GEF;
    const int jg = p.col0 + j;
    const T shift = (T)p.shift;
    const E x = ((const GE *)p.B)[(int64_t)jg * p.ldb + i];
    T vr = alpha * (ar - shift * mre(x));
    T vi = alpha * (ai - shift * mim(x));
    if (p.beta != 0.0) {
      const E xp = ((const GE *)p.Xprev)[(int64_t)jg * p.ldp + i];
      vr += beta * mre(xp);
      vi += beta * mim(xp);
    }
    if (jg < p.final_end)
      ((GEF *)p.Ofinal)[(int64_t)jg * p.ldf + i] = mmake<EF, FT>((FT)vr, (FT)vi);
    else
      ((GEw *)p.Onext)[(int64_t)jg * p.ldn + i] = mmake<E, T>(vr, vi);
  }
}

// ---------------------------------------------------- direct-load path --
// Complex tiles of 64 x 64 with both operands K-contiguous (the filter's H^H
// and X, and the Rayleigh-Ritz product H Q): a ring of three LDS stages fed
// by direct global -> LDS loads (global_load_lds_dwordx4: lane L of a wave
// writes its 16 bytes to the L-th slot after the wave's LDS base), so two K
// chunks are in flight while a third is multiplied, with no prefetch
// registers and no LDS store instructions.  A K chunk is 128 bytes of every
// row: 8 complex doubles or 16 complex floats, i.e. eight 16-byte slots of
// one (double) or two (float) elements.
#ifndef CHASE_GEMM_DMA
#define CHASE_GEMM_DMA 1
#endif
typedef double __attribute__((ext_vector_type(2))) dbl2;
typedef float __attribute__((ext_vector_type(4))) flt4;
typedef dbl2 __attribute__((address_space(3))) LdsD2;  // one 16-byte slot
typedef flt4 __attribute__((address_space(3))) LdsF4;

// LDS slot of (row r, slot column c) of a 64-row tile: rows of eight slots,
// c XOR-swizzled with bits 1..3 of the row so that the 16 rows one
// quarter-wave reads for a fixed c hit 16 different groups of four banks.
__device__ __forceinline__ int dma_slot(int r, int c) { return 8 * r + (c ^ ((r >> 1) & 7)); }

// One full K chunk [k0, k0 + 8 EPS) of A (rows m0..m0+ROWS-1) and B (columns
// n0..n0+ROWS-1) into the tiles LA, LB: each wave issues ROWS / 32 loads of
// 1 KB per tile, lane L of load q filling slot 64 q + L.  Rows (columns) past
// the matrix read the last one instead: they only feed outputs that are not
// stored.  ES is the element size in bytes, EPS = 16 / ES elements per slot.
template <int ES, int ROWS>
__device__ __forceinline__ void dma_chunk(const GemmArgs &p, int m0, int n0, int k0, int wave,
                                          int lane, LdsD2 *LA, LdsD2 *LB) {
  constexpr int EPS = 16 / ES, LPW = ROWS / 32;
  typedef const char __attribute__((address_space(1))) GC;
#pragma unroll
  for (int h = 0; h < LPW; ++h) {
    const int q = LPW * wave + h;
    const int s = 64 * q + lane;
    const int r = s >> 3;
    const int c = (s & 7) ^ ((r >> 1) & 7);
    const int gi = min(m0 + r, p.M - 1);
    const int gj = min(n0 + r, p.N - 1);
    const GC *a = (const GC *)p.A + ((int64_t)gi * p.lda + k0 + c * EPS) * ES;
    const GC *b = (const GC *)p.B + ((int64_t)(p.col0 + gj) * p.ldb + k0 + c * EPS) * ES;
    __builtin_amdgcn_global_load_lds(a, LA + 64 * q, 16, 0, 0);
    __builtin_amdgcn_global_load_lds(b, LB + 64 * q, 16, 0, 0);
  }
}

// The partial last chunk [k0, kend): ordinary loads with zero fill (k past
// kend must contribute nothing), packed into the same slots.  EL is the
// element type: double, or a 2-vector (re, im) of double or float.
template <typename EL, int ROWS>
__device__ __forceinline__ void reg_chunk(const GemmArgs &p, int m0, int n0, int k0, int kend,
                                          int tid, LdsD2 *LA, LdsD2 *LB) {
  typedef const EL __attribute__((address_space(1))) GE;
  constexpr int EPS = 16 / (int)sizeof(EL);
  const GE *Ag = (const GE *)p.A;
  const GE *Bg = (const GE *)p.B;
#pragma unroll
  for (int t = 0; t < ROWS / 32; ++t) {
    const int s = tid + 256 * t;
    const int r = s >> 3;
    const int c = (s & 7) ^ ((r >> 1) & 7);
    EL va[EPS], vb[EPS];
#pragma unroll
    for (int e = 0; e < EPS; ++e) {
      const int k = k0 + c * EPS + e;
      va[e] = (k < kend && m0 + r < p.M) ? Ag[(int64_t)(m0 + r) * p.lda + k] : EL{};
      vb[e] = (k < kend && n0 + r < p.N) ? Bg[(int64_t)(p.col0 + n0 + r) * p.ldb + k] : EL{};
    }
    dbl2 sa, sb;
    __builtin_memcpy(&sa, va, 16);
    __builtin_memcpy(&sb, vb, 16);
    LA[s] = sa;
    LB[s] = sb;
  }
}

// The K loop of the direct-load path.  The six stage tiles are restrict
// parameters of one inlined function, so the compiler knows that reading
// stage c % 3 does not depend on the loads just issued into the other stages
// and waits only for the loads of chunk c; the explicit wait before the
// barrier makes every wave's loads of chunk c visible to the others.
// K order inside a chunk: MFMA step t, lane group lk multiplies the element
// in slot column lk + 4 (t / EPS) (element t % EPS of the slot), the same
// for A and B, so every k of the chunk is used once.
template <typename T, bool CONJA, bool CPLX = true>
__device__ __forceinline__ void dma_mainloop(const GemmArgs &p, int m0, int n0, int kbeg, int kend,
                                             int tid, int wm, int wn,
                                             typename Mfma<T>::acc (&accR)[2][2],
                                             typename Mfma<T>::acc (&accI)[2][2],
                                             typename Mfma<T>::acc (&acc3)[2][2],
                                             LdsD2 *__restrict__ A0, LdsD2 *__restrict__ B0,
                                             LdsD2 *__restrict__ A1, LdsD2 *__restrict__ B1,
                                             LdsD2 *__restrict__ A2, LdsD2 *__restrict__ B2) {
  constexpr int ES = (CPLX ? 2 : 1) * (int)sizeof(T), EPS = 16 / ES, BK = 8 * EPS;
  static_assert(CPLX || sizeof(T) == 8, "real tiles of this loop are FP64");
  const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nch = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  auto full = [&](int c) { return kbeg + BK * c + BK <= kend; };
  auto issue = [&](int c, LdsD2 *LA, LdsD2 *LB) {
    const int k0 = kbeg + BK * c;
    typedef typename std::conditional<CPLX, T __attribute__((ext_vector_type(2))), T>::type EL;
    if (full(c))
      dma_chunk<ES, 64>(p, m0, n0, k0, wave_u, lane, LA, LB);
    else
      reg_chunk<EL, 64>(p, m0, n0, k0, kend, tid, LA, LB);
  };
  auto mma = [&](const T (&ar)[2], const T (&ai)[2], const T (&br)[2], const T (&bi)[2]) {
    T as_[2], bs_[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) as_[a] = CONJA ? ar[a] - ai[a] : ar[a] + ai[a];
#pragma unroll
    for (int b = 0; b < 2; ++b) bs_[b] = br[b] + bi[b];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accR[a][b] = Mfma<T>::op(ar[a], br[b], accR[a][b]);
        accI[a][b] = Mfma<T>::op(ai[a], bi[b], accI[a][b]);
        acc3[a][b] = Mfma<T>::op(as_[a], bs_[b], acc3[a][b]);
      }
  };
  auto compute = [&](const LdsD2 *LA, const LdsD2 *LB) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {  // slot columns lk and lk + 4
      const int c = lk + 4 * g;
      if constexpr (!CPLX) {  // real FP64: two k per slot
        dbl2 va[2], vb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) va[a] = LA[dma_slot(wm * 32 + a * 16 + lr, c)];
#pragma unroll
        for (int b = 0; b < 2; ++b) vb[b] = LB[dma_slot(wn * 32 + b * 16 + lr, c)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) accR[a][b] = Mfma<T>::op(va[a].x, vb[b].x, accR[a][b]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) accR[a][b] = Mfma<T>::op(va[a].y, vb[b].y, accR[a][b]);
      } else if constexpr (EPS == 1) {
        T ar[2], ai[2], br[2], bi[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const dbl2 v = LA[dma_slot(wm * 32 + a * 16 + lr, c)];
          ar[a] = v.x;
          ai[a] = v.y;
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const dbl2 v = LB[dma_slot(wn * 32 + b * 16 + lr, c)];
          br[b] = v.x;
          bi[b] = v.y;
        }
        mma(ar, ai, br, bi);
      } else {
        flt4 va[2], vb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) va[a] = ((const LdsF4 *)LA)[dma_slot(wm * 32 + a * 16 + lr, c)];
#pragma unroll
        for (int b = 0; b < 2; ++b) vb[b] = ((const LdsF4 *)LB)[dma_slot(wn * 32 + b * 16 + lr, c)];
        {
          const T ar[2] = {va[0].x, va[1].x}, ai[2] = {va[0].y, va[1].y};
          const T br[2] = {vb[0].x, vb[1].x}, bi[2] = {vb[0].y, vb[1].y};
          mma(ar, ai, br, bi);
        }
        {
          const T ar[2] = {va[0].z, va[1].z}, ai[2] = {va[0].w, va[1].w};
          const T br[2] = {vb[0].z, vb[1].z}, bi[2] = {vb[0].w, vb[1].w};
          mma(ar, ai, br, bi);
        }
      }
    }
  };
  // chunk c: wait for its loads (the next chunk's four, if direct, may stay
  // in flight), barrier (chunk c visible; every wave is done with chunk
  // c - 1, whose stage the load of chunk c + 2 reuses), multiply.
  auto step = [&](int c, const LdsD2 *Ac, const LdsD2 *Bc, LdsD2 *An, LdsD2 *Bn) {
    if (c + 1 < nch && full(c + 1))
      __builtin_amdgcn_s_waitcnt(0x0F74);  // vmcnt(4)
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // LDS barrier without the memory fence of __syncthreads, whose implied
    // vmcnt(0) would also drain the next chunk's loads; the clobber keeps
    // the compiler from moving memory accesses across it
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (c + 2 < nch) issue(c + 2, An, Bn);
    compute(Ac, Bc);
  };
  if (nch > 0) issue(0, A0, B0);
  if (nch > 1) issue(1, A1, B1);
  for (int c = 0; c < nch; c += 3) {
    step(c, A0, B0, A2, B2);
    if (c + 1 < nch) step(c + 1, A1, B1, A0, B0);
    if (c + 2 < nch) step(c + 2, A2, B2, A1, B1);
  }
}

// Real FP64 tiles of 128 x 128 (four waves of 64 x 64), K chunks of 16
// doubles (eight slots of two per row), two LDS stages of 32 KB fed by direct
// loads: the next chunk streams in while the current one is multiplied (64
// MFMAs per wave per chunk hide the load latency at two blocks per CU).
// Same structure as dma_mainloop, two stages: chunk c waits for its own
// loads (nothing else is in flight), barrier (every wave is done with chunk
// c - 1, whose stage the load of chunk c + 1 reuses), issue c + 1, multiply.
// K order inside a chunk: step 2 g + e, lane group lk multiplies element e of
// slot column lk + 4 g, for A and B alike.
__device__ __forceinline__ void dma_mainloop_real(const GemmArgs &p, int m0, int n0, int kbeg,
                                                  int kend, int tid, int wm, int wn,
                                                  d4v (&acc)[4][4], LdsD2 *__restrict__ A0,
                                                  LdsD2 *__restrict__ B0,
                                                  LdsD2 *__restrict__ A1,
                                                  LdsD2 *__restrict__ B1) {
  constexpr int BK = 16;
  const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nch = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  auto issue = [&](int c, LdsD2 *LA, LdsD2 *LB) {
    const int k0 = kbeg + BK * c;
    if (k0 + BK <= kend)
      dma_chunk<8, 128>(p, m0, n0, k0, wave_u, lane, LA, LB);
    else
      reg_chunk<double, 128>(p, m0, n0, k0, kend, tid, LA, LB);
  };
  auto compute = [&](const LdsD2 *LA, const LdsD2 *LB) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int c = lk + 4 * g;
      dbl2 va[4], vb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) va[a] = LA[dma_slot(wm * 64 + a * 16 + lr, c)];
#pragma unroll
      for (int b = 0; b < 4; ++b) vb[b] = LB[dma_slot(wn * 64 + b * 16 + lr, c)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<double>::op(va[a].x, vb[b].x, acc[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<double>::op(va[a].y, vb[b].y, acc[a][b]);
    }
  };
  auto step = [&](int c, const LdsD2 *Ac, const LdsD2 *Bc, LdsD2 *An, LdsD2 *Bn) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): chunk c
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (c + 1 < nch) issue(c + 1, An, Bn);
    compute(Ac, Bc);
  };
  if (nch > 0) issue(0, A0, B0);
  for (int c = 0; c < nch; c += 2) {
    step(c, A0, B0, A1, B1);
    if (c + 1 < nch) step(c + 1, A1, B1, A0, B0);
  }
}

// M3 (complex only): three real products per complex one,
// P1 = ar br, P2 = ai bi, P3 = (ar + ai)(br + bi); re = P1 - P2,
// im = P3 - P1 - P2 (a quarter fewer MFMAs than the four-product form).
// DMAP: use the direct-load K loop (complex 64 x 64 M3 tiles, real 64 x 64 or
// 128 x 128 tiles, A K-contiguous); the launcher selects it only when both
// operands have 16-byte aligned rows.
template <typename T, bool CPLX, bool AT, bool CONJA, int BM, int BN, int BK, int WM, int WN,
          int EPI, typename FT, int MINB, bool M3, bool DMAP>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), MINB) void gemm_kernel(const GemmArgs p) {
  typedef typename MemT<T, CPLX>::type E;
  typedef typename Mfma<T>::acc Acc;
  constexpr int NWM = BM / WM;
  constexpr int NT = 64 * NWM * (BN / WN);
  static_assert(!M3 || CPLX, "three-product form is for complex data");
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
  static_assert(AE * NT == BM * BK && BE * NT == BN * BK, "tile / thread mismatch");
  // direct-load paths (the launcher checks 16-byte alignment of the operands)
  constexpr bool DMA = DMAP && M3 && AT && BM == 64 && BN == 64 && WM == 32 && WN == 32 &&
                       BK == 128 / (2 * (int)sizeof(T));
  constexpr bool DMAR = DMAP && !CPLX && AT && sizeof(T) == 8 && BM == 128 && BN == 128 &&
                        WM == 64 && WN == 64 && BK == 16;
  constexpr bool DMAR64 = DMAP && !CPLX && AT && sizeof(T) == 8 && BM == 64 && BN == 64 &&
                          WM == 32 && WN == 32 && BK == 16;
  static_assert(!DMAP || DMA || DMAR || DMAR64, "no direct-load path for this tile configuration");

  if (p.flag != nullptr && *p.flag != 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % NWM, wn = wave / NWM;
  const int nbm = (p.M + BM - 1) / BM, nbn = (p.N + BN - 1) / BN;
  const int nb = p.ntiles > 0 ? p.ntiles : nbm * nbn;
  // XCD-aware remap of the hardware block id (bijective on [0, nb)).
  const int hb = blockIdx.x;
  const int xcd = hb & 7, q = hb >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int logical = p.tile0 + xcd * per + (xcd < rem ? xcd : rem) + q;
  int bm, bn;
  tile_coords(logical, nbm, nbn, bm, bn);
  const int m0 = bm * BM, n0 = bn * BN;
  if (p.tri && m0 > n0 + BN - 1) return;

  int kbeg = blockIdx.y * p.k_per_split;
  int kend = kbeg + p.k_per_split;
  if (kend > p.K) kend = p.K;
  if (p.kcap) {
    int cap = p.col0 + n0 + BN;
    if (kend > cap) kend = cap;
  }

  // global (address space 1) pointers: loads become global_load rather
  // than flat_load, which would also count against the LDS wait counter
  typedef const E __attribute__((address_space(1))) GE;
  typedef E __attribute__((address_space(1))) GEw;
  const GE *Ag = (const GE *)p.A;
  const GE *Bg = (const GE *)p.B;

  Acc accR[FM][FN];  // M3: P1
  Acc accI[FM][FN];  // M3: P2
  Acc acc3[M3 ? FM : 1][M3 ? FN : 1];  // M3: P3
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accR[a][b][r] = 0;
        accI[a][b][r] = 0;
        if constexpr (M3) acc3[a][b][r] = 0;
      }

  const int lr = lane & 15, lk = lane >> 4;
  if constexpr (DMAR) {
    __shared__ dbl2 R0[2][1024], R1[2][1024];
    dma_mainloop_real(p, m0, n0, kbeg, kend, tid, wm, wn, accR, (LdsD2 *)R0[0], (LdsD2 *)R0[1],
                      (LdsD2 *)R1[0], (LdsD2 *)R1[1]);
  } else if constexpr (DMAR64) {
    __shared__ dbl2 L0[2][512], L1[2][512], L2[2][512];
    dma_mainloop<T, false, false>(p, m0, n0, kbeg, kend, tid, wm, wn, accR, accR, accR,
                                  (LdsD2 *)L0[0], (LdsD2 *)L0[1], (LdsD2 *)L1[0],
                                  (LdsD2 *)L1[1], (LdsD2 *)L2[0], (LdsD2 *)L2[1]);
  } else if constexpr (DMA) {
    __shared__ dbl2 L0[2][512], L1[2][512], L2[2][512];
    dma_mainloop<T, CONJA>(p, m0, n0, kbeg, kend, tid, wm, wn, accR, accI, acc3,
                        (LdsD2 *)L0[0], (LdsD2 *)L0[1], (LdsD2 *)L1[0], (LdsD2 *)L1[1],
                        (LdsD2 *)L2[0], (LdsD2 *)L2[1]);
  } else {
  __shared__ T As[2][NP][BK][BM + 1];
  __shared__ T Bs[2][NP][BK][BN + 1];
  E ra[AE], rb[BE];
  const E zero = mmake<E, T>((T)0, (T)0);
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * NT;
      int i, k;
      if (AT) { k = idx % BK; i = idx / BK; } else { i = idx % BM; k = idx / BM; }
      const int gi = m0 + i, gk = k0 + k;
      if (gi < p.M && gk < kend)
        ra[e] = AT ? Ag[(int64_t)gi * p.lda + gk] : Ag[(int64_t)gk * p.lda + gi];
      else
        ra[e] = zero;
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * NT;
      const int k = idx % BK, j = idx / BK;
      const int gj = n0 + j, gk = k0 + k;
      if (gj < p.N && gk < kend)
        rb[e] = Bg[(int64_t)(p.col0 + gj) * p.ldb + gk];
      else
        rb[e] = zero;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * NT;
      int i, k;
      if (AT) { k = idx % BK; i = idx / BK; } else { i = idx % BM; k = idx / BM; }
      As[buf][0][k][i] = mre(ra[e]);
      if constexpr (CPLX) As[buf][NP - 1][k][i] = CONJA ? -mim(ra[e]) : mim(ra[e]);
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * NT;
      const int k = idx % BK, j = idx / BK;
      Bs[buf][0][k][j] = mre(rb[e]);
      if constexpr (CPLX) Bs[buf][NP - 1][k][j] = mim(rb[e]);
    }
  };

  int buf = 0;
  if (kbeg < kend) {
    load_tiles(kbeg);
    store_tiles(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = (k0 + BK) < kend;
    if (more) load_tiles(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        ar[a] = As[buf][0][kk + lk][wm * WM + a * 16 + lr];
        if constexpr (CPLX) ai[a] = As[buf][NP - 1][kk + lk][wm * WM + a * 16 + lr];
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        br[b] = Bs[buf][0][kk + lk][wn * WN + b * 16 + lr];
        if constexpr (CPLX) bi[b] = Bs[buf][NP - 1][kk + lk][wn * WN + b * 16 + lr];
      }
      if constexpr (M3) {
        T as_[FM], bs_[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) as_[a] = ar[a] + ai[a];
#pragma unroll
        for (int b = 0; b < FN; ++b) bs_[b] = br[b] + bi[b];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            accR[a][b] = Mfma<T>::op(ar[a], br[b], accR[a][b]);
            accI[a][b] = Mfma<T>::op(ai[a], bi[b], accI[a][b]);
            acc3[a][b] = Mfma<T>::op(as_[a], bs_[b], acc3[a][b]);
          }
      } else {
#pragma unroll
        for (int a = 0; a < FM; ++a) {
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            accR[a][b] = Mfma<T>::op(ar[a], br[b], accR[a][b]);
            if constexpr (CPLX) {
              accR[a][b] = Mfma<T>::op(-ai[a], bi[b], accR[a][b]);
              accI[a][b] = Mfma<T>::op(ar[a], bi[b], accI[a][b]);
              accI[a][b] = Mfma<T>::op(ai[a], br[b], accI[a][b]);
            }
          }
        }
      }
    }
    if (more) store_tiles(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  }

  // ---------------------------------------------------------- epilogue --
  if constexpr (M3) {  // (P1, P2, P3) -> (re, im)
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // the direct-load path multiplies the stored (unconjugated)
          // imaginary part of A: with CONJA, P2 = -ai bi and
          // P3 = (ar + ai)(br + bi) with ai the conjugate's part
          const T p1 = accR[a][b][r];
          const T p2 = (DMA && CONJA) ? -accI[a][b][r] : accI[a][b][r];
          accR[a][b][r] = p1 - p2;
          accI[a][b][r] = acc3[a][b][r] - p1 - p2;
        }
  }
  if (p.Pk != nullptr) {  // raw partial tile of one K split
    typedef E __attribute__((address_space(1))) GEw;
    GEw *Pt = (GEw *)p.Pk + ((int64_t)(logical - p.tile0) * gridDim.y + blockIdx.y) * (BM * BN);
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = wm * WM + a * 16 + Mfma<T>::row(lk, r);
          const int jj = wn * WN + b * 16 + lr;
          Pt[jj * BM + ii] = mmake<E, T>(accR[a][b][r], accI[a][b][r]);
        }
    return;
  }
  const int64_t split_off = (int64_t)blockIdx.y * p.split_stride;
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int j = n0 + wn * WN + b * 16 + lr;
    if (j >= p.N) continue;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * WM + a * 16 + Mfma<T>::row(lk, r);
        if (i >= p.M) continue;
        epilogue_store<T, CPLX, EPI, FT>(p, i, j, accR[a][b][r], accI[a][b][r], split_off);
      }
  }
}

// Sums the S partial tiles of the remainder tiles in a fixed order and
// applies the epilogue (deterministic).  One thread per tile element.
template <typename T, bool CPLX, int BM, int BN, int EPI, typename FT>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const GemmArgs p, int S) {
  typedef typename MemT<T, CPLX>::type E;
  typedef const E __attribute__((address_space(1))) GE;
  if (p.flag != nullptr && *p.flag != 0) return;  // same skip rule as the GEMM
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int tl = (int)(e / (BM * BN));
  const int w = (int)(e % (BM * BN));
  if (tl >= p.ntiles) return;
  const int ii = w % BM, jj = w / BM;
  const int nbm = (p.M + BM - 1) / BM, nbn = (p.N + BN - 1) / BN;
  int bm, bn;
  tile_coords(p.tile0 + tl, nbm, nbn, bm, bn);
  const int i = bm * BM + ii, j = bn * BN + jj;
  if (i >= p.M || j >= p.N) return;
  const GE *P = (const GE *)p.Pk + (int64_t)tl * S * (BM * BN) + w;
  T sr = 0, si = 0;
  for (int q = 0; q < S; ++q) {
    const E v = P[(int64_t)q * (BM * BN)];
    sr += mre(v);
    si += mim(v);
  }
  epilogue_store<T, CPLX, EPI, FT>(p, i, j, sr, si, 0);
}

}  // namespace chase
