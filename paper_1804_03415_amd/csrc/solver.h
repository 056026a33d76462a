// The level driver of the hierarchical eigensolver (Alg. 2-6) on the device.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"
#include "pcg_persistent.h"

namespace mmd {

class OpBatcher;

// Device scratch owned by one solver call, reused across phases by name.
class Pool {
 public:
  double* d(const std::string& name, size_t count) { return dbl_[name].ensure(count), dbl_[name].p; }
  int* i(const std::string& name, size_t count) { return int_[name].ensure(count), int_[name].p; }
  float* f(const std::string& name, size_t count) { return flt_[name].ensure(count), flt_[name].p; }

 private:
  std::map<std::string, DBuf<double>> dbl_;
  std::map<std::string, DBuf<int>> int_;
  std::map<std::string, DBuf<float>> flt_;
};

// Per-column CG scalars backed by named pool buffers of length b.
ColScalars make_scalars(Pool& pool, const std::string& tag, int b);

struct SolveResult {
  std::vector<int> iters;
};

class Solver {
 public:
  Solver(mmd_handle& h, hipStream_t s, const eig_opts& o, eig_stats* st);
  ~Solver();

  // eig_leftmost: evals ascending (host), evecs column-major n x nev (device)
  void leftmost(int nev, double tol, double* evals, double* evecs);
  // off: single-vector solves use the block kernels instead of the
  // cooperative persistent ones (needed when other streams run concurrently:
  // a grid barrier must never wait on workgroups that cannot be resident)
  void set_persistent(bool on) { use_persistent_ = on; }
  // inside a batch: single-vector operator solves go through the batcher
  // (one cooperative launch for the solves pending across the batch), and
  // level-0 resident plans use few blocks so several solves fit at once
  void set_batcher(OpBatcher* b) { batcher_ = b; }

  // building blocks exposed through mmd_apply / mmd_solve
  void apply_op(int level, int op, const double* X, double* Y, int b);
  void solve(int level, int kind, const double* rhs, double* X, int b, bool use_x0, double tol,
             int* iters_out);
  // eig_backward: gradient per stored entry of the caller's A (device g_vals)
  void backward(int nev, const double* evals, const double* evecs, const double* g_evals,
                const double* g_evecs, double tol, double* g_vals);

 private:
  struct Block {  // row-major device block n x b (ld = b)
    double* p = nullptr;
    int n = 0, b = 0;
  };

  // level operators
  int nlev(int k) const { return h_.host[k].n; }
  void applyA(int k, const double* X, int ldx, double* Y, int ldy, int b);
  void applyM(int k, const double* X, int ldx, double* Y, int ldy, int b);
  void applyB(int k, const double* X, int ldx, double* Y, int ldy, int b);

  // solvers (columns independent, scalars on the device)
  enum class OpKind { A, M, B };
  void cg(int k, OpKind op, const double* B, int ldb, double* X, int ldx, int n, int b,
          double tol, bool use_x0, const int* parent_active, int fixed_iters,
          const std::string& tag, std::vector<int>* iters);
  // approximate eigenpairs (A q_j ~ q_j / mu_j) removed from the residual in
  // FP64 before each FP32 inner solve of the mixed-precision form
  struct Deflation {
    const double* Q = nullptr;  // n x m, row-major, leading dimension ld
    int ld = 0, m = 0;
    const double* mu = nullptr;  // device [m]
  };
  void pcg(int k, const double* B, int ldb, double* X, int ldx, int b, double tol, bool use_x0,
           std::vector<int>* iters, const Deflation* dfl = nullptr);
  bool pcg_single(int k, const double* B, double* X, double tol, bool use_x0,
                  std::vector<int>* iters);
  // level-0 block solve by FP32 CG inside FP64 iterative refinement
  void cg_mixed(const double* B, int ldb, double* X, int ldx, int b, double tol, bool use_x0,
                std::vector<int>* iters, const Deflation* dfl = nullptr);
  // FP32 CG (zero start) on the m columns of R32 (leading dimension even_ld(m),
  // consumed as the residual); the solutions are added to X(:, gcols[j]).
  void ensure32();
  // CG on P (A - diag shift) P, P = I - V V^T, for the columns of R (row-major
  // n x b, in V-perp); Y receives the solutions (zero start)
  void cg_shift_defl(const double* R, double* Y, int b, const double* shift_neg,
                     const double* V, int nev, double tol);

  // Lanczos / extension / refinement
  struct Lanczos;
  void lanczos_init(Lanczos& L, int k, const double* Vini, int mi, int cap_cols);
  void lanczos_random(Lanczos& L, double* out);
  void lanczos_orth(Lanczos& L, double* w, int jcols, std::vector<double>* hlast);
  double mnorm2(int k, const double* x);
  void lanczos_steps(Lanczos& L, int nsteps);
  bool ritz_converged(Lanczos& L, int nwant, double eps, bool relative);
  void restart(Lanczos& L, int kkeep, int p);
  void extend(int k, double*& V, std::vector<double>& D, int& m, int m_tar, double eps,
              double mu_ex, int d, bool relative);
  void multiplicity_check(int k, double*& V, std::vector<double>& D, int m, double eps, int d);
  void refine(int k, double*& V, std::vector<double>& D, int& m, double eps, double mu_h,
              double lam_max_M, double gamma);
  void mqr(int k, double* F, int n, int b, const std::string& tag);
  void final_pairs(double* V, const std::vector<double>& D, int m, int nev, double tol,
                   double* evals, double* evecs);
  // returned pairs: row-major level-0 block Vn (n x nev) -> caller's layout
  void emit_pairs(const double* Vn, const std::vector<double>& lam, int nev, double* evals,
                  double* evecs);
  // stop_level > 0: lift the level-k pairs to level 0 and return them
  void coarse_output(const double* V, const std::vector<double>& D, int m, int k, int nev,
                     double* evals, double* evecs);

  void sync() {
    MMD_HIP(hipStreamSynchronize(s_));
    harvest_timers();
  }
  // HIP-event timing of the level-0 block SpMM (only when stats are requested)
  void spmm0_begin();
  void spmm0_end(double bytes, int b);
  void harvest_timers();
  std::vector<hipEvent_t> ev_free_;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending_;
  std::vector<double> ev_bytes_;
  hipEvent_t ev_open_ = nullptr;
  template <typename T>
  void d2h(T* dst, const T* src, size_t n) {
    MMD_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s_));
  }
  template <typename T>
  void h2d(T* dst, const T* src, size_t n) {
    MMD_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s_));
  }

  mmd_handle& h_;
  hipStream_t s_;
  eig_opts o_;
  eig_stats* st_;
  Pool pool_;
  HBuf<double> hd_;
  HBuf<int> hi_;
  int inner_iters_ = 16;
  bool use_persistent_ = true;
  bool graphs_ = true;             // replay fixed CG chunks as HIP graphs (MMDEIG_GRAPHS=0: off)
  bool cg_defer_ = true;           // fold the level-0 CG update into the next step (MMDEIG_CG_DEFER=0: off)
  OpBatcher* batcher_ = nullptr;
  std::map<int, Pcg1Plan> plans_;  // resident plain-CG plan per level (level 0)
  double norm_a0_ = 0.0;           // ||A||_inf of level 0 (mixed-precision floor test)
  std::vector<double> tpcg_;       // relative PCG tolerance per level (k >= 1)
  int cur_level_ = 0;
  int64_t draws_[MMD_MAX_LEVELS] = {};
};

}  // namespace mmd
