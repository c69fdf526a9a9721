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
// Lanczos helpers (single work-group reductions).
void dot_re(bool cplx, const void *v, const void *w, int n, double *out, hipStream_t s);
void norm_scale(bool cplx, const void *w, int n, void *vout, double *beta_out, hipStream_t s);
void sum_splits(bool cplx, const void *P, int nsplit, int64_t sstride, int nelem, void *out,
                hipStream_t s);

}  // namespace chase
