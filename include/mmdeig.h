/*
 * mmdeig — leftmost eigenpairs of a sparse SPD matrix by the hierarchically
 * preconditioned eigensolver of Hou, Huang, Lam and Zhang, "A Fast
 * Hierarchically Preconditioned Eigensolver Based on Multiresolution Matrix
 * Decomposition" (arXiv 1804.03415), on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every function returns an int
 * status (MMD_OK = 0); on failure mmd_last_error() returns a thread-local
 * message describing the cause.  All device work is enqueued on the
 * caller's HIP stream (void* hip_stream, NULL = the default stream); results
 * in device buffers are valid once that stream has completed.  Host output
 * buffers are filled before the call returns.
 *
 * Memory ownership: the caller owns every buffer it passes; the library never
 * frees caller memory and keeps no caller pointer after a call returns.  A
 * handle owns the device copy of the decomposition and its workspaces until
 * mmd_free().  Calls that use the same handle must not overlap.
 */
#ifndef MMDEIG_H
#define MMDEIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define MMD_OK 0
#define MMD_EINVAL 1        /* bad argument: non-square, unsorted or asymmetric
                               pattern, NaN, nev out of range, bad level/op    */
#define MMD_ENOTSPD 2       /* nonpositive diagonal or CG curvature p^T A p <= 0 */
#define MMD_EUNSUPPORTED 3  /* positive off-diagonal / negative self-loop: no
                               edge-type energy decomposition (Section 2.1)    */
#define MMD_ENOCONV 4       /* iteration cap reached; partial results          */
#define MMD_ENOMEM 5        /* device or host allocation failed                */
#define MMD_EHIP 6          /* a HIP runtime call failed                       */

/* ------------------------------------------------------------------ inputs */
/* Symmetric sparse matrix in CSR form.  rowptr has n+1 entries (int64),
 * colind nnz sorted column indices per row (int32), val nnz float64 values.
 * mem = 0: the three arrays are host memory; mem = 1: device memory.
 * Optional geometry steers the partitioner: coords (host, n x coord_dim
 * row-major float64, may be NULL) for graphs; grid_dim = 2 or 3 with
 * grid[0..grid_dim-1] = (nx, ny[, nz]) for tensor grids whose vertex
 * (x, y, z) has index (z*ny + y)*nx + x (grid_dim = 0: not a grid). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* colind;
  const double* val;
  int32_t mem;
  int32_t coord_dim;
  const double* coords;
  int32_t grid_dim;
  int32_t grid[3];
} mmd_csr;

/* Decomposition options (Sections 2.2-2.3).  Zero-initialised fields take the
 * defaults given in brackets. */
typedef struct {
  int32_t levels;          /* number of coarse levels K [3]                      */
  int32_t n_targets;       /* entries used in targets[] [2: {4, 8}]              */
  int32_t targets[8];      /* greedy patch size of level k (last entry repeats)  */
  int32_t n_grid_blocks;   /* entries used in grid_blocks[] [2: {4, 2}]          */
  int32_t grid_blocks[8];  /* tensor block edge of level k for grids             */
  int32_t r_hops;          /* localisation radius of Psi in patch hops [1]       */
  int64_t exact_max_n;     /* levels whose fine size <= this use the exact Psi [0] */
  int32_t min_coarse;      /* stop coarsening below this many dofs [4]           */
  int32_t max_patch;       /* eps1 > 0: largest patch [32]                       */
  double eps1;             /* > 0: graphs are partitioned to prescribed accuracy
                              (Section 2.3): eps(P^(k)) <= eps1 / eta^(k-1) and
                              eps(P) delta(P) <= cbound, instead of targets.
                              Patches grow from Morton-ordered seeds, trying
                              the adjacent vertex of largest total coupling
                              sum |a_vp| first, with the split patch energy
                              A[P,P] - diag(sum_{j not in P} |a_ij|) on every
                              level; the localised Psi then needs a radius
                              r_hops that keeps the level accurate to eps_k
                              (5 on the SwissRoll graph of Section 7.1) [0] */
  double eta;              /* ratio eps_k / eps_(k+1) [0.1]                      */
  double cbound;           /* condition bound c [20]                             */
  int32_t r_hops_coarse;   /* localisation radius of Psi^(k), k >= 2 [r_hops]    */
} mmd_build_opts;

/* Solver options (Section 5 parameter choice).  Zero fields take defaults. */
typedef struct {
  double alpha;            /* mu_re^(k) = alpha eps_{k+1} [3]                    */
  double beta;             /* mu_ex^(k) = beta eps_k [1]                         */
  int32_t restart_mult;    /* c: shifts per restart = c d [1]                    */
  int32_t precision;       /* 0: FP64 throughout [0].  1: level-0 block solves
                              run CG in FP32 (FP32 matrix copy and vectors)
                              inside an FP64 iterative refinement (residual,
                              update and stop test in FP64, same tolerance);
                              everything else stays FP64                      */
  uint64_t seed;           /* Philox key of the random start vectors [0]         */
  int32_t max_restarts;    /* per extension [2000]                               */
  int32_t max_refine;      /* refinement iterations per level [200]              */
  int32_t streams;         /* eig_leftmost_batched: problems solved concurrently,
                              one HIP stream and host thread each [8]           */
  int32_t stop_level;      /* 0: solve down to level 0 [0].  k in 1..K: the
                              coarse-level approximation of Section 7.3 --
                              Alg. 6 (as printed it stops at level 1) stopped
                              after level k, returning lambda = 1/mu of the
                              level-k pairs and v = Psi^(1)...Psi^(k) z, within
                              eps_k of the true pairs (Lemma 3.3); tol is not
                              used                                             */
  int32_t d;               /* extension block size of every level (0: the
                              default max(1, min(N^(k)/10, nev/10)))            */
} eig_opts;

#define MMD_MAX_LEVELS 16
/* Per-level counters in the paper's statistics schema (Section 7.3). */
typedef struct {
  int32_t K;
  int32_t nconv;
  int64_t ref_in[MMD_MAX_LEVELS], ref_out[MMD_MAX_LEVELS], ref_iter[MMD_MAX_LEVELS];
  int64_t cg_B_calls[MMD_MAX_LEVELS], cg_B_iters[MMD_MAX_LEVELS];
  int64_t pcg_A_calls[MMD_MAX_LEVELS], pcg_A_iters[MMD_MAX_LEVELS];
  int64_t cg_M_iters[MMD_MAX_LEVELS];
  int64_t ext_in[MMD_MAX_LEVELS], ext_out[MMD_MAX_LEVELS];
  int64_t lanczos_steps[MMD_MAX_LEVELS], restarts[MMD_MAX_LEVELS];
  int64_t missed_swaps;
  double seconds_level[MMD_MAX_LEVELS];
  double seconds_total;
  /* wall time by phase, summed over levels: 0 refinement block PCG, 1 refinement
     B-CG, 2 refinement host dense work, 3 refinement QR/Gram/rotations,
     4 extension OP (PCG), 5 extension re-orthogonalisation, 6 restarts,
     7 output step and multiplicity check */
  double seconds_phase[8];
  /* the level-0 SpMM of the refinement block PCG (the dominant HBM kernel),
     timed with HIP events on the solve's stream: launches, summed duration in
     milliseconds, summed algorithmic bytes (matrix once, each block read or
     written once) and the block width of the last launch */
  int64_t spmm0_launches;
  double spmm0_ms;
  double spmm0_bytes;
  int32_t spmm0_b;
  /* precision = 1: level-0 block solves whose FP32 inner solves stopped
     reducing the FP64 residual and were finished by FP64 CG */
  int32_t mixed_fallbacks;
} eig_stats;

typedef struct mmd_handle mmd_handle;

/* Build the K-level multiresolution decomposition of A (Section 2.3, eq. MMD):
 * per level the patch partition, the local basis phi_j (smallest eigenvector
 * of the patch energy, q = 1, Section 2.2), one Householder reflector per
 * patch (the complement U, Lemma 2.3), the localised Psi (eq. psi_closedform
 * in its constrained-energy form, Appendix A) and A^(k) = Psi^T A^(k-1) Psi,
 * M^(k) = Psi^T M^(k-1) Psi.  Runs on the host, uploads the level operators
 * on hip_stream.  Errors: MMD_EINVAL, MMD_EUNSUPPORTED, MMD_ENOTSPD,
 * MMD_ENOMEM, MMD_EHIP.  *out is set only on success. */
int mmd_build(const mmd_csr* A, const mmd_build_opts* opts, void* hip_stream,
              mmd_handle** out);

/* Level sizes and error factors: K, N^(k) for k = 0..K (sizes[K+1]),
 * nnz(A^(k)) and nnz(M^(k)) (nnzA/nnzM[K+1], level 0: nnz(A), 0) and the
 * cumulative compression errors eps_k (eps[K+1], eps_0 = 0; Theorem 2.6).
 * Any output pointer may be NULL.  The arrays must hold MMD_MAX_LEVELS. */
int mmd_info(const mmd_handle* h, int32_t* K, int64_t* sizes, int64_t* nnzA,
             int64_t* nnzM, double* eps);

/* Copy one level object to host CSR buffers (for inspection and tests).
 * which: 0 = A^(k), 1 = M^(k) (k >= 1), 2 = Psi^(k) (k >= 1, N^(k-1) x N^(k)).
 * Pass rowptr = NULL to query n_rows / nnz only. */
int mmd_export(const mmd_handle* h, int32_t level, int32_t which, int64_t* n_rows,
               int64_t* n_cols, int64_t* nnz, int64_t* rowptr, int32_t* colind,
               double* val);

/* The nev smallest eigenpairs of A (Alg. 6, continued to level 0 with
 * A^(0) = A, M^(0) = I): coarsest-level generalised eigenproblem, then per
 * level reform (V <- Psi V), Eigenpair Refinement (Alg. 5) and Eigenpair
 * Extension (Alg. 4, operator OP = PCG with preconditioner M^(k), Section
 * 4), followed by a multiplicity check and an inverse-iteration +
 * Rayleigh-Ritz output step on level 0.
 *   tol    relative accuracy on level 0 (CG tolerance, Ritz residual
 *          relative to the Ritz value); coarse levels use 0.1 eps_k.
 *   evals  host float64 [nev], ascending.
 *   evecs  device float64, column-major n x nev (eigenvector i at
 *          evecs + i*n), unit 2-norm, largest-magnitude entry positive.
 *   st     optional counters.
 * Errors: MMD_EINVAL (nev out of range), MMD_ENOTSPD, MMD_ENOCONV, MMD_EHIP. */
int eig_leftmost(mmd_handle* h, int32_t nev, double tol, const eig_opts* opts,
                 double* evals, double* evecs, eig_stats* st, void* hip_stream);

/* Many independent problems at once: the same computation as eig_leftmost
 * for hs[b], nev[b], evals[b], evecs[b], b < B (distinct handles), with
 * opts->streams problems in flight at a time, each on its own HIP stream
 * driven by its own host thread, largest nnz x nev first.  Work on the
 * caller's stream that precedes the call is waited for; the results are
 * complete when the call returns.  Within a batch the persistent
 * single-vector solvers (cooperative launches with a grid barrier) run one at
 * a time; all other work of the problems overlaps.  st: NULL or an array of B
 * counters.  The first error of any problem is returned (the others are
 * still finished). */
int eig_leftmost_batched(int32_t B, mmd_handle* const* hs, const int32_t* nev, double tol,
                         const eig_opts* opts, double* const* evals, double* const* evecs,
                         eig_stats* st, void* hip_stream);
/* Reverse-mode derivative of the nev leftmost eigenpairs (the paper gives
 * none; first-order perturbation of a symmetric matrix).  Given the pairs
 * returned by eig_leftmost (evals host [nev] ascending, evecs device
 * column-major n x nev, orthonormal) and the adjoints of a loss L
 * (g_evals host [nev] and g_evecs device column-major n x nev, either may be
 * NULL), writes for every stored entry p = (i, j) of the caller's A, in the
 * caller's CSR order,
 *   g_vals[p] = S_ij,  S = sum_k g_evals[k] v_k v_k^T - sum_k sym(x_k v_k^T),
 *   x_k = sum_{j != k} v_j (v_j^T g_k)/(lambda_j - lambda_k)
 *         + (A - lambda_k I)^-1 on the complement of the evecs applied to
 *           (I - V V^T) g_k,
 * so that dL = sum_ij S_ij dA_ij for every symmetric perturbation dA (for an
 * edge weight w_ij of a Laplacian, dL/dw_ij = S_ii + S_jj - S_ij - S_ji).
 * The complement solves are CG with A - lambda_k I projected onto the
 * complement of V, stopped at relative residual tol.  g_vals: device
 * float64 [nnz].  Errors: MMD_EINVAL (nev out of range, a repeated eigenvalue
 * whose eigenvector adjoint couples the copies: the gradient is undefined),
 * MMD_ENOTSPD (the shifted operator is not positive on the complement: the
 * pairs are not the leftmost ones), MMD_ENOCONV, MMD_EHIP. */
int eig_backward(mmd_handle* h, int32_t nev, const double* evals, const double* evecs,
                 const double* g_evals, const double* g_evecs, double tol, double* g_vals,
                 void* hip_stream);
/* Apply one level operator to a block of b columns (device, row-major with
 * leading dimension b).  op: 0 = A^(k) (N^(k) -> N^(k)), 1 = M^(k),
 * 2 = B^(k+1) = U^T A^(k) U (reduced -> reduced, needs k < K),
 * 3 = U^(k+1) (reduced -> N^(k)), 4 = U^(k+1)^T (N^(k) -> reduced),
 * 5 = Psi^(k+1) (N^(k+1) -> N^(k)), 6 = A^(0) in FP32 arithmetic (level 0
 * only: X rounded to FP32, the FP32 matrix copy and kernel of the
 * mixed-precision solves, the result widened to FP64).  Level 0 A is applied
 * in edge form y_i = s_i x_i + sum_j w_ij (x_i - x_j) (Section 2.1 elements). */
int mmd_apply(mmd_handle* h, int32_t level, int32_t op, const double* X, double* Y,
              int32_t b, void* hip_stream);

/* Column-wise solves on one level, b independent right-hand sides (device,
 * row-major, leading dimension b).  kind 0: pcg(A^(k), rhs, M^(k), x0, tol)
 * of Section 4 (flexible PCG with an inner CG on M^(k) to 0.1 tol; plain CG on
 * level 0); kind 1: cg(B^(k+1), rhs, -, x0, tol) (Alg. 5 start block);
 * kind 2 (level 0 only): the same solve as kind 0 by FP32 CG inside an FP64
 * iterative refinement (the precision = 1 form of eig_opts).  X holds
 * x0 on entry (use_x0 != 0) and the solution on exit.  iters (host int32[b],
 * may be NULL) receives the outer iteration counts. */
int mmd_solve(mmd_handle* h, int32_t level, int32_t kind, const double* rhs, double* X,
              int32_t b, int32_t use_x0, double tol, int32_t* iters, void* hip_stream);

/* Y = A X for a caller-supplied device CSR (int64 rowptr, int32 colind,
 * float64 val; n_rows x n_cols) and a row-major block X [n_cols x b] ->
 * Y [n_rows x b] (CSR sparse-matrix times dense block, Section 7.3 "Main
 * Cost" unit). */
int mmdk_spmm(int64_t n_rows, int64_t n_cols, const int64_t* rowptr, const int32_t* colind,
              const double* val, const double* X, double* Y, int32_t b, void* hip_stream);

/* The dense tall-skinny products of the Rayleigh-Ritz and restart steps on
 * the FP64 matrix cores: C = X^T Y (the M-inner-product Gram matrices of the
 * M-orthogonal QR and S = W^T F of Alg. 5) and Z = alpha X C + beta Z (the
 * rotations V Q of Alg. 2 and Q P, F P of Alg. 5).  Device row-major
 * operands: X [n x m] (ld ldx >= m), Y [n x p] (ldy >= p), C [m x p]
 * (ldc >= p), Z [n x p] (ldz >= p).  mmdk_gram splits the n rows into chunks
 * whose partial products it sums in a library-allocated workspace.  Both
 * synchronise hip_stream before returning.  Errors: MMD_EINVAL, MMD_ENOMEM,
 * MMD_EHIP. */
int mmdk_gram(int64_t n, int32_t m, int32_t p, const double* X, int32_t ldx, const double* Y,
              int32_t ldy, double* C, int32_t ldc, void* hip_stream);
int mmdk_gemm(int64_t n, int32_t m, int32_t p, double alpha, const double* X, int32_t ldx,
              const double* C, int32_t ldc, double beta, double* Z, int32_t ldz,
              void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as mmdk_spmm, same arguments and layouts, with no hipMalloc, hipFree
 * or allocating library call.  The int32 copy of the row pointers goes to a
 * library-owned device array of fixed size (n_rows <= 4194304, 16 MiB held on
 * every GPU the library runs on until the process ends); larger inputs return
 * MMD_EINVAL before any device work.  Every call on one GPU shares that array:
 * calls that overlap on the same GPU race.  The call reads nnz from the
 * device row pointers and synchronises hip_stream, as mmdk_spmm does. */
int mmdk_spmm_noalloc(int64_t n_rows, int64_t n_cols, const int64_t* rowptr,
                      const int32_t* colind, const double* val, const double* X, double* Y,
                      int32_t b, void* hip_stream);

/* Release a handle and everything it owns (NULL is ignored). */
void mmd_free(mmd_handle* h);

/* Thread-local message for the last nonzero status on this thread. */
const char* mmd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MMDEIG_H */
