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

// Eigenvalues (ascending, theta) and eigenvectors (in place, columns of A)
// of a Hermitian n x n matrix, n <= kJacobiMaxN, by one work-group (cyclic
// Jacobi, parallel order); info[0] = 1 if kJacobiMaxSweeps did not converge.
constexpr int kJacobiMaxN = 64;
constexpr int kJacobiMaxSweeps = 40;
void jacobi_eig(bool cplx, void *A, int64_t lda, int n, double *theta, int *info,
                hipStream_t s);

// Householder QR helpers (geqrf convention, panels of kHhNB columns).
constexpr int kHhNB = 32;         // columns of one panel of column steps
constexpr int kHhMaxOuter = 128;  // columns of one block reflector (T at most this wide)
constexpr size_t kHhStateBytes = (size_t)320 << 10;  // pivot rows, block sums (two each)
// One column step jj (0..nbp) of the panel P (Mp x nbp from its first
// diagonal element); Vb receives the explicit reflector vectors, tau the
// panel's tau entries.  Step jj + 1 reads what step jj left in hh_state, so
// the steps of one panel run in order on one stream.
void hh_column(bool cplx, void *P, int64_t ld, int Mp, int nbp, int jj, void *Vb, int64_t ldv,
               void *tau, void *hh_state, hipStream_t s);
// T (nb x nb, nb <= kHhMaxOuter) of the compact WY form from S = V^H V and tau.
void hh_larft(bool cplx, const void *S, int64_t lds, const void *tau, void *T, int64_t ldt,
              int nb, hipStream_t s);
// out (rows x cols) = sum of nsplit partials.
void sum_splits(bool cplx, const void *P, int nsplit, int64_t sstride, int64_t ldp, int rows,
                int cols, void *out, int64_t ldo, hipStream_t s);
void set_identity(bool cplx, void *A, int64_t lda, int rows, int cols, hipStream_t s);

}  // namespace chase
