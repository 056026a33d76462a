// FP32 block-CG kernels for the mixed-precision mode: the level-0 refinement
// solves run CG in FP32 on an FP32 copy of the edge-form matrix, inside an
// FP64 iterative-refinement loop (residual, update and stop test in FP64).
// Blocks are row-major with an even leading dimension so a lane can move two
// columns with one 8-byte access; per-column scalars and partial sums stay
// FP64 and reuse the FP64 scalar kernels (cg_init, cg_alpha, cg_beta).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace mmd {

struct CsrView32 {
  int n_rows = 0, n_cols = 0;
  int64_t nnz = 0;
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const float* val = nullptr;
  const float* diag = nullptr;  // non-null: edge form y = s x + sum w (x_i - x_j)
  // level-0 row-block tiling shared with the FP64 view (CsrView::t_*)
  int t_kind = 0;
  const int* t_row = nullptr;
  const int* t_uptr = nullptr;
  const int* t_urow = nullptr;
  const unsigned short* t_lcol = nullptr;
  int t_nblk = 0;
};

inline int even_ld(int b) { return (b + 1) & ~1; }

// Fused CG direction step in FP32 (same contract as spmm(..., fuse = true)):
// P = X + beta P, Y = A X + beta Y, partial[blk*b + c] = sum P.*Y (FP64).
// ldx, ldy, ldp must be even.  Returns the number of partials per column.
int spmm32_cg(const CsrView32& A, const float* X, int ldx, float* Y, int ldy, int b,
              bool first, const double* beta, float* P, int ldp, double* partial,
              hipStream_t s);
// partial[blk*b + c] = sum X.*Y (FP64 accumulation); returns #blocks.
int col_dot32(const float* X, int ldx, const float* Y, int ldy, int n, int b, double* partial,
              hipStream_t s);
// X += alpha P ; R -= alpha Q ; partial = R.*R (FP64); returns #blocks.
int cg_update32(float* X, int ldx, float* R, const float* P, const float* Q, int ld, int n,
                int b, const double* alpha, double* partial, hipStream_t s);
// Z(:, j) = (float) Y(:, idx[j]) for j < b; Z(:, j) = 0 for b <= j < ldz.
void gather_to32(const double* Y, int ldy, const int* idx, float* Z, int ldz, int n, int b,
                 hipStream_t s);
// Z(:, j) = Y(:, idx[j]) for j < b (FP32 compaction); padding columns zeroed.
void gather32(const float* Y, int ldy, const int* idx, float* Z, int ldz, int n, int b,
              hipStream_t s);
// X(:, dst[j]) += (double) D(:, src[j]) for j < m.
void scatter_add64(const float* D, int ldd, const int* src, const int* dst, double* X, int ldx,
                   int n, int m, hipStream_t s);
// Y = 0 (n x ld, FP32).
void zero32(float* Y, int n, int ld, hipStream_t s);
// FP32 copies of an FP64 array.
void to_f32(const double* x, float* y, int64_t n, hipStream_t s);

}  // namespace mmd
