// Host-side launchers of the gfx950 kernels (declarations).  All matrices are
// column-major; complex ones interleaved.  Every launcher enqueues on the
// given stream and never synchronises.
#pragma once
#include "common.hpp"

namespace chase {

enum GemmShape { GEMM_BIG = 0, GEMM_SMALL = 1 };

struct GemmArgs;

// dtype-erased GEMM dispatch.  prec32: operands are float / float2.
// at: A read K-contiguous (conjugated when complex); otherwise M-contiguous.
// epi_filter: EPI_FILTER epilogue (final outputs in FP64 when out64 is set).
// Returns the number of GEMM kernel dispatches (the remainder split adds
// one; its reduce kernel is not counted).
int gemm(bool cplx, bool prec32, bool at, bool epi_filter, bool out64, GemmShape shape,
         GemmArgs &args, int splits, hipStream_t s);
int gemm_bk();  // K chunk of the GEMM tiles (the split granularity)

// G (n x n) = sum over nsplit partials S, mirrored to a Hermitian /
// symmetric matrix with a real diagonal: from the upper triangle of S
// (average = 0) or as (S + S^H) / 2 (average = 1, S complete).
void reduce_hermitian(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int n,
                      void *G, int64_t ldg, int average, hipStream_t s);
// trace(G) -> trace_out[0]; when add_shift, G += coef * trace(G) * I and the
// shift is written to trace_out[1].
void trace_shift(bool cplx, void *G, int64_t ldg, int n, double coef, int add_shift,
                 double *trace_out, const int *flag, hipStream_t s);
// Factor the b x b diagonal block at (p0, p0) of G (upper triangle):
// R block and its inverse; flag[0] = failing column + 1, flag[1] = pass.
void chol_diag(bool cplx, void *G, int64_t ldg, void *R, int64_t ldr, void *Ri, int64_t ldi,
               int p0, int b, int *flag, int pass, int inject, hipStream_t s);
void fill_zero(bool cplx, void *A, int64_t lda, int rows, int cols, hipStream_t s);
// resid[a] = ||HV_a - theta_a V_a|| / ||V_a||
void residuals(bool cplx, const void *HV, int64_t ldhv, const void *V, int64_t ldv, int n,
               int ncols, const double *theta, double *resid, hipStream_t s);
// dst[:, a] = src[:, perm[a]] (perm may be null: identity); optional FP64->FP32.
void gather_cols(bool cplx, bool to32, const void *src, int64_t lds, void *dst, int64_t ldd,
                 int n, int ncols, const int *perm, hipStream_t s);
void copy_cols(bool cplx, const void *src, int64_t lds, void *dst, int64_t ldd, int n, int ncols,
               hipStream_t s);
// FP64 -> FP32 copy of a matrix.
void convert_to32(bool cplx, const void *src, int64_t lds, void *dst, int64_t ldd, int rows,
                  int cols, hipStream_t s);
// Gaussian block: real N(0,1); complex (N(0,1) + i N(0,1)) / sqrt(2).
void randn(bool cplx, void *V, int64_t ldv, int n, int ncols, uint64_t seed, hipStream_t s);
// Lanczos helpers.  Y (M x nv, ldy) = A (M x K, column-major, lda) X (K x nv, ldx), 1 <= nv <= 8,
// streaming A once; column-split partials use `scratch` (scratch_bytes).
void gemv_block(bool cplx, const void *A, int64_t lda, int M, int K, const void *X, int64_t ldx,
                int nv, void *Y, int64_t ldy, void *scratch, size_t scratch_bytes, hipStream_t s);
// out[c] = Re(v_c^H w_c); beta[c] = ||w_c|| and vout_c = w_c / beta[c]
// (one work-group per column).
void dot_re_cols(bool cplx, const void *v, const void *w, int64_t ld, int n, int ncols,
                 double *out, hipStream_t s);
void norm_scale_cols(bool cplx, const void *w, int64_t ldw, int n, int ncols, void *vout,
                     int64_t ldo, double *beta, hipStream_t s);
// out (rows x nv) = sum of nsplit partials, keeping row q only in column q % nv.
void sum_splits_diag(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                     int nv, void *out, int64_t ldo, hipStream_t s);

// One Lanczos step after the product for small orders (N <= kLzSmallMaxN,
// k + 1 <= kLzSmallMaxBasis): alpha, two classical Gram-Schmidt passes
// against the run's basis, beta and the next basis vector, one work-group
// per run (layout as in the solver's Lanczos).
constexpr int kLzSmallMaxN = 4096;
constexpr int kLzSmallMaxBasis = 128;
void lz_step_small(bool cplx, void *LV, int64_t ldv, int N, int j, int nv, void *W, int64_t ldw,
                   double *ab, int k, hipStream_t s);

// All k steps of the nv Lanczos runs in one cooperative launch for small
// orders (layout and outputs as lz_step_small's; V0: the normalised start
// vectors, LV's first nv columns; XV: N x nv exchange buffer; part: partial
// sums, 2 x blocks x (k + 1) x nv elements).  Resets the grid-barrier
// counter in hh_state; a barrier time-out sets its error flag.  Returns
// false (nothing launched) when a block's share does not fit its LDS or
// part is too small.
bool lanczos_coop(bool cplx, const void *H, int64_t ldh, int N, int k, int nv, const void *V0,
                  void *XV, double *ab, void *part, size_t part_bytes, void *hh_state,
                  hipStream_t s);

// Hermitian eigensolver of the Rayleigh-Ritz matrix (eig.hip).
constexpr int kEigSmallMax = 64;  // LDS-resident reduction / back transform up to this order
constexpr int kEigQrMax = 24;     // tridiagonal QR for the whole problem up to this order
constexpr int kEigMaxN = 2560;    // largest order (LDS arrays of the reduction)
constexpr int kDcLeaf = 16;       // largest leaf of the divide and conquer
constexpr int kDcGemmSmall = 256; // merges up to this order multiply in one batched launch
// A (n <= kEigSmallMax): eigenvalues ascending in theta, eigenvectors in
// place; info[0] = 1 if the tridiagonal QR did not converge.
void heev_small(bool cplx, void *A, int64_t lda, int n, double *theta, int *info, hipStream_t s);
// Launch j of the reduction to tridiagonal form (A n x n, lda; V: reflector
// j in column j below row j; tau; d, e: the tridiagonal; p vectors
// alternate between pin (read) and pout (written)).
void hetrd_step(bool cplx, void *A, int64_t lda, int n, int j, void *V, int64_t ldv, void *tau,
                double *d, double *e, const void *pin, void *pout, hipStream_t s);
// The last n - j0 <= kEigSmallMax columns of the reduction in one
// work-group (pin: the p vector of launch j0 - 1; unused when j0 == 0).
void hetrd_tail(bool cplx, const void *A, int64_t lda, int n, int j0, void *V, int64_t ldv,
                void *tau, double *d, double *e, const void *pin, hipStream_t s);
// X = H_0 ... H_{n-2} Z for n <= kEigSmallMax (one work-group).
void ormtr_small(bool cplx, const void *V, int64_t ldv, const void *tau, const double *Z,
                 int64_t ldz, int n, void *X, int64_t ldx, hipStream_t s);
// The products Zk = Qg U of every merge at depth t in one launch (merge
// orders up to kDcGemmSmall).
void dc_gemm_small(const double *Qg, const double *U, double *Zk, int n, int t, hipStream_t s);
// Divide and conquer on the tridiagonal (d, e) of order n: depth of the
// tree, the leaves (eigenvalues to w, eigenvectors to the diagonal blocks of
// Z, ld n, zero elsewhere), and per level t (D - 1 down to 0) the merge
// steps before (deflation, secular roots, Loewner, the rank-one problem's
// eigenvectors U, the gathered columns Qg) and after (sorted placement into
// Zn) the products Zk = Qg U of every merge, which the caller runs.
struct DcPtrs {
  double *dl, *zl, *tsec, *zh, *dval;
  int *org, *src_nd, *src_df, *srcbuf, *kcnt;
};
int dc_depth(int n);
void dc_leaves(const double *d, const double *e, int n, int D, double *w, double *Z, int *info,
               hipStream_t s);
void dc_merge_pre(const double *e, int n, int t, const double *w, double *Zc, double *Qg,
                  double *U, const DcPtrs &a, hipStream_t s);
void dc_merge_post(int n, int t, double *w, const double *Zk, const double *Zc, double *Zn,
                   const DcPtrs &a, hipStream_t s);
// X (n x n, ldx) = Z (real, ld n) as real or complex elements.
void real_to_elem(bool cplx, const double *Z, int n, void *X, int64_t ldx, hipStream_t s);

// Householder QR helpers (geqrf convention, panels of kHhNB columns).
constexpr int kHhNB = 32;         // columns of one panel of column steps
constexpr int kHhMaxOuter = 128;  // columns of one block reflector (T at most this wide)
// hh_state: the column steps' pivot rows and block sums (two each), then the
// panel kernel's pivot rows, barrier counter, error flag and block sums
constexpr int kHpMaxBlocks = 512;  // blocks of one panel launch
constexpr int kHpRows = 128;       // rows per block the panel launch aims at
constexpr int kHpMaxRows = 256;    // rows per block it accepts (LDS: 256 x 32 x 16 bytes)
constexpr size_t kHpStateBytes = (size_t)2 * 16 * kHhNB + 256 + 2 * (size_t)kHpMaxBlocks * kHhNB * 16;
constexpr size_t kHhStateBytes = ((size_t)320 << 10) + kHpStateBytes;
// One column step jj (0..nbp) of the panel P (Mp x nbp from its first
// diagonal element); Vb receives the explicit reflector vectors, tau the
// panel's tau entries.  Step jj + 1 reads what step jj left in hh_state, so
// the steps of one panel run in order on one stream.
void hh_column(bool cplx, void *P, int64_t ld, int Mp, int nbp, int jj, void *Vb, int64_t ldv,
               void *tau, void *hh_state, hipStream_t s);
// The whole column-step sequence of one panel in one cooperative launch
// (same results as steps 0..nbp of hh_column up to the order of the block
// sums).  Returns false, launching nothing, when the panel has too many rows
// for its blocks' LDS; *base is the barrier counter's value before the
// launch and is advanced past it.  hh_panel_reset zeroes the counter
// (before the first panel of a factorisation, base = 0).  hh_panel_error is
// the device address of an int that a barrier wait sets when it times out
// (every factorisation since is invalid); it stays set until
// hh_panel_clear_error.
bool hh_panel(bool cplx, void *P, int64_t ld, int Mp, int nbp, void *Vb, int64_t ldv, void *tau,
              void *hh_state, unsigned *base, hipStream_t s);
void hh_panel_reset(void *hh_state, hipStream_t s);
// Limit of a panel launch's barrier wait in wall-clock ticks (<= 0: two
// seconds); process-wide, for tests of the time-out path.
void hh_panel_set_wait_limit(long long ticks);
void hh_panel_clear_error(void *hh_state, hipStream_t s);
const void *hh_panel_error(const void *hh_state);
// T (nb x nb, nb <= kHhMaxOuter) of the compact WY form from S = V^H V and tau.
void hh_larft(bool cplx, const void *S, int64_t lds, const void *tau, void *T, int64_t ldt,
              int nb, hipStream_t s);
// out (rows x cols) = sum of nsplit partials.
void sum_splits(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                int cols, void *out, int64_t ldo, hipStream_t s);
void set_identity(bool cplx, void *A, int64_t lda, int rows, int cols, hipStream_t s);

}  // namespace chase
