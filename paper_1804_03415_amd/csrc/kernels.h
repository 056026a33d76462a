// Launchers of the device kernels (defined in kernels.hip).  All blocks of
// vectors are row-major: element (i, c) of an N x b block lives at
// X[i * ld + c].  Per-column scalars are device arrays of length b.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace mmd {

// Device CSR (int32 indices; nnz < 2^31).  For the level-0 edge form, val
// holds the positive edge weights w_ij = -a_ij of the off-diagonal entries and
// diag the self-loop weights s_i.
struct CsrView {
  int n_rows = 0, n_cols = 0;
  int64_t nnz = 0;
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const double* val = nullptr;
  const double* diag = nullptr;  // non-null: edge form y = s x + sum w (x_i - x_j)
  double avg_row = 1.0;
  // Row-block tiling of the edge form (level 0; t_uptr == nullptr: none),
  // built for tile shape kTileShapes[t_kind].  Block t owns rows
  // [t_row[t], t_row[t + 1]) (at most shape.rows); its column set U_t lists
  // those rows first, in order, then the other columns its rows touch,
  // ascending: t_urow[t_uptr[t] .. t_uptr[t + 1]).  t_lcol[q] is the position
  // in U_t of col[q].  Every |U_t| <= shape.cols and every block holds at
  // most shape.nnz entries.
  int t_kind = 0;
  const int* t_row = nullptr;
  const int* t_uptr = nullptr;
  const int* t_urow = nullptr;
  const unsigned short* t_lcol = nullptr;
  int t_nblk = 0;
};

// Tile shapes of the LDS-staged SpMMs: max rows per block, max distinct
// gathered rows (staged in LDS), max entries, and the workgroups per CU the
// LDS and register budget allow.  The level-0 tiling picks one per matrix by
// timing (build-time autotuning).
struct TileShape {
  int rows, cols, nnz, wgs_per_cu;
};
constexpr int kNumTileShapes = 3;
constexpr TileShape kTileShapes[kNumTileShapes] = {
    {32, 80, 1024, 3}, {32, 64, 768, 4}, {16, 48, 512, 5}};
constexpr int kTileRowsMax = 32;

// Patch Householder data of one level transfer (k-1 -> k).
struct HouseView {
  int npatch = 0;
  int nfine = 0;         // N^(k-1)
  int nred = 0;          // N^(k-1) - N^(k)
  const int* ptr = nullptr;      // [npatch+1] offsets into members / u
  const int* members = nullptr;  // fine dof of each patch slot
  const double* u = nullptr;     // Householder vector entries per slot
  const double* scale = nullptr; // 2 / u^T u per patch
};

// Work buffers for column reductions.
constexpr int kRedBlocks = 1024;  // max blocks of a reduction grid

// ---------------------------------------------------------------- SpMM
// Y = A X.  fuse != 0 selects the CG form:
//   Y <- A X + beta[c] * Y ;  P <- X + beta[c] * P ;  partial[blk*b+c] = sum P.*Y
// (first != 0: beta treated as 0 and the old Y / P are not read).
// dot_with != null (and fuse == 0): partial[blk*b+c] = sum dot_with .* Y.
// Returns the number of row blocks used (partials per column).
int spmm(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b,
         hipStream_t s, bool fuse = false, bool first = false, const double* beta = nullptr,
         double* P = nullptr, int ldp = 0, double* partial = nullptr,
         const double* dot_with = nullptr, int ld_dot = 0);

// One level-0 block-CG step with the previous step's update folded in
// (tiled edge form only: cg_tile_ok).  pend: X += alpha P and
// r = Ri - alpha Qi (alpha per column, the previous step's), written to Ro;
// then P = r + beta P, Qo = A r + beta Qi (first: P = r, Qo = A r).  A pending
// step needs Ro != Ri and Qo != Qi (other workgroups still gather the old
// rows); without pend Ro is unused and Qo may equal Qi.  Ri, Qi, Ro, Qo, P
// share the leading dimension ld.  partial receives four n_blk x b blocks,
// pstride (>= kRedBlocks * b) apart: p.q, r.q, q.q, r.r of the new vectors.
// Returns n_blk.
bool cg_tile_ok(const CsrView& A);
int cg_tile_step(const CsrView& A, double* X, int ldx, const double* Ri, const double* Qi,
                 double* Ro, double* Qo, double* P, int ld, int b, bool pend, bool first,
                 const double* alpha, const double* beta, double* partial, size_t pstride,
                 hipStream_t s);

// ---------------------------------------------------------------- Householder
// y_red = U^T x  (x: nfine x b, y: nred x b)
void house_ut(const HouseView& H, const double* x, int ldx, double* y, int ldy, int b,
              hipStream_t s);
// x = U y       (y: nred x b, x: nfine x b)
void house_u(const HouseView& H, const double* y, int ldy, double* x, int ldx, int b,
             hipStream_t s);

// ---------------------------------------------------------------- reductions
// partial[blk*b + c] = sum over the block's rows of X(i,c)*Y(i,c); returns #blocks.
int col_dot(const double* X, int ldx, const double* Y, int ldy, int n, int b,
            double* partial, hipStream_t s);
// two dots sharing X: partial1 = X.*Y1, partial2 = X.*Y2
int col_dot2(const double* X, int ldx, const double* Y1, const double* Y2, int ldy, int n,
             int b, double* partial1, double* partial2, hipStream_t s);
// out[c] = sum_blk partial[blk*b + c]
void reduce_partials(const double* partial, int nblk, int b, double* out, hipStream_t s);

// ---------------------------------------------------------------- CG scalars
struct ColScalars {
  double* rr;     // r^T r (plain CG) or r^T z (flexible PCG)
  double* rr2;    // plain r^T r for the stop test (PCG)
  double* alpha;
  double* beta;
  double* bn2;    // ||b||^2
  double* tol2;   // tol^2 (same for all columns)
  int* active;
  int* iters;
  int* notspd;    // set to 1 if p^T A p <= 0 on an active column
};
// init: bn2 = ||B||^2 (from partials), rr2 = ||R||^2 (from partials);
// active = bn2 > 0 && rr2 > tol2 * bn2; iters = 0; parent (nullable) masks.
void cg_init(ColScalars sc, const double* part_bn, const double* part_rr, int nblk, int b,
             double tol, const int* parent_active, hipStream_t s);
// alpha = active ? rr / sum(part_pq) : 0
void cg_alpha(ColScalars sc, const double* part_pq, int nblk, int b, hipStream_t s);
// plain CG: rr_new = sum(part); conv test; beta = rr_new/rr; rr = rr_new; iters++
void cg_beta(ColScalars sc, const double* part_rr, int nblk, int b, hipStream_t s);
// as cg_beta, but a column with rr_new <= tol2 * bn2 keeps iterating and sets
// upd[c] = 1 (request for an FP64 residual replacement)
void cg_beta_flag(ColScalars sc, const double* part_rr, int nblk, int b, int* upd,
                  hipStream_t s);
// residual replacement: rr = rr2 = bn2 = rr_true, beta *= rr_true / rr (old),
// or beta = 0 (restart) when rr_true > restart2 * rr or the column had stopped;
// tol2 = delta2, alpha = 0, active = 1, upd = 0
void reliable_scalars(ColScalars sc, const double* rr_true, double delta2, double restart2,
                      int b, int* upd, hipStream_t s);
// deferred-update step scalars (after cg_tile_step): alpha = r.r / p.q left
// pending, the next r.r from r.r - 2 alpha r.q + alpha^2 q.q for the stop test
// and beta; a column whose new r.r meets the tolerance stops with alpha = 0
void cg_defer_scalars(ColScalars sc, const double* part, size_t pstride, int nblk, int b,
                      hipStream_t s);
// after cg_update applied the pending alphas: alpha = 0; active columns take
// the direct r.r (part_rr), rescale beta to it and stop at the tolerance
void cg_defer_flush(ColScalars sc, const double* part_rr, int nblk, int b, hipStream_t s);
// flexible PCG stop test on ||r||^2 (part_rr); marks converged columns inactive
void pcg_conv(ColScalars sc, const double* part_rr, int nblk, int b, hipStream_t s);
// flexible PCG beta = (r.z - r.zold) / rz ; rz = r.z
void pcg_beta(ColScalars sc, const double* part_rz, const double* part_rzo, int nblk, int b,
              hipStream_t s);

// ---------------------------------------------------------------- elementwise
// X += alpha P ; R -= alpha Q ; partial = R.*R  (returns #blocks)
int cg_update(double* X, int ldx, double* R, const double* P, const double* Q, int ld, int n,
              int b, const double* alpha, double* partial, hipStream_t s);
// P = R + beta[c] P   (first: P = R)
void xpay(const double* R, int ldr, double* P, int ldp, int n, int b, const double* beta,
          bool first, hipStream_t s);
// Y = X (n x b)
void copy_block(const double* X, int ldx, double* Y, int ldy, int n, int b, hipStream_t s);
void zero_block(double* Y, int ldy, int n, int b, hipStream_t s);
// Y = X * diag(d) (+ Y if accumulate)
void scale_cols(const double* X, int ldx, const double* d, double* Y, int ldy, int n, int b,
                bool accumulate, hipStream_t s);
// X(i, c) *= d[i]  (n x b)
void scale_rows(double* X, int ldx, const double* d, int n, int b, hipStream_t s);
// Y = a X + c Y   (scalars on host)
void axpby(double a, const double* X, int ldx, double c, double* Y, int ldy, int n, int b,
           hipStream_t s);
// R = B - R   (after R = A X)
void rsub(const double* B, int ldb, double* R, int ldr, int n, int b, hipStream_t s);
// y = x / (*scal) (device scalar), n x 1 into column of a block
void scale_vec_dev(const double* x, const double* scal, bool inv_sqrt, double* y, int ldy,
                   int n, hipStream_t s);
// Y(:, idx[j]) gathered into Z(:, j)
void gather_cols(const double* Y, int ldy, const int* idx, double* Z, int ldz, int n, int b,
                 hipStream_t s);
// Y(:, j) scattered into Z(:, idx[j])
void scatter_cols(const double* Y, int ldy, const int* idx, double* Z, int ldz, int n, int b,
                  hipStream_t s);
// per-column CG scalars of columns idx[0..m) of src into columns 0..m of dst
// (notspd is not copied)
void gather_scalars(ColScalars src, ColScalars dst, const int* idx, int m, hipStream_t s);
// column-major output: out[c*n + perm[i]] = X[i*ldx + c] * colscale[c] (perm may be null)
void to_colmajor(const double* X, int ldx, const double* colscale, double* out, int n, int b,
                 const int* perm, hipStream_t s);
// per column: the entry of largest |X(i,c)| (ties: lowest perm[i], or i when perm is null);
// work_idx / work_val hold col_absmax_work_size(n, b) entries each
size_t col_absmax_work_size(int n, int b);
void col_absmax(const double* X, int ldx, int n, int b, int* idx, double* val,
                const int* perm, int* work_idx, double* work_val, hipStream_t s);
// rows: gather Y[i] = X[idx[i]] or scatter Y[idx[i]] = X[i] (n rows, b columns)
void permute_rows(const double* X, int ldx, double* Y, int ldy, int n, int b, const int* idx,
                  bool scatter, hipStream_t s);

// row-major out[i*ld + c] = in[c*n + (perm ? perm[i] : i)]  (column-major caller
// block to the internal row-major numbering)
void from_colmajor(const double* in, int n, int b, const int* perm, double* out, int ld,
                   hipStream_t s);
// Eigen-backward sampled product on a CSR pattern (rows of V, X row-major with
// leading dimension ld, nev columns): for every stored (i, j)
//   out[p] = sum_k glam[k] V(i,k) V(j,k) - (X(i,k) V(j,k) + V(i,k) X(j,k)) / 2
// glam may be null (no eigenvalue term), X may be null (no vector term).
void sddmm_eig(int n_rows, const int* rowptr, const int* col, const double* V, const double* X,
               int ld, int nev, const double* glam, double* out, hipStream_t s);

// int64 -> int32 copy of caller row pointers (the caller checks nnz < 2^31)
void i64_to_i32(const int64_t* src, int* dst, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- dense GEMMs (FP64)
// C (m x p, row-major ldc, device) = X^T Y, X: n x m (ldx), Y: n x p (ldy).
// work must hold splits*m*p doubles (see gram_work_size).
size_t gram_work_size(int n, int m, int p);
void gram(const double* X, int ldx, const double* Y, int ldy, int n, int m, int p, double* C,
          int ldc, double* work, hipStream_t s);
// Z (n x p, ldz) = alpha * X (n x m, ldx) * C (m x p, ldc, device) + beta * Z
void gemm_nn(const double* X, int ldx, const double* C, int ldc, double* Z, int ldz, int n,
             int m, int p, double alpha, double beta, hipStream_t s);
// matrix-vector forms for one column (Lanczos): h[m] = X^T y ; z -= X h.
// gemv_t splits the rows into at most kGemvChunks chunks; work holds
// kGemvChunks x m doubles.
constexpr int kGemvChunks = 1024;
void gemv_t(const double* X, int ldx, const double* y, int n, int m, double* h,
            double* work, hipStream_t s);
void gemv_n_sub(const double* X, int ldx, const double* h, int n, int m, double* z,
                hipStream_t s);

}  // namespace mmd
