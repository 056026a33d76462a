// Level driver of the hierarchical eigensolver on the device.
//
// Every length-N operation runs in the kernels of kernels.hip; the host keeps
// only small dense FP64 objects (the Lanczos matrix T, Ritz and Gram matrices,
// the coarsest-level operators) and the control flow of Alg. 2-6.  CG / PCG
// scalars live on the device per column; the host reads the convergence flags
// once per chunk of iterations, never per iteration.
#include "solver.h"

#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>

#include "batch.h"
#include "dense.h"
#include "mixed.h"
#include "pcg_persistent.h"

namespace mmd {

namespace {

// Philox4x32-10 (Salmon et al., SC'11); random start vectors of Alg. 3/4.
void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Entry i of draw `call` at `level`: counter (i/2, call, level, 0), values in
// [-0.5, 0.5).  With a renumbering, internal entry j is the caller's entry perm[j].
void uniform_vector(std::vector<double>& v, int n, uint64_t seed, int level, int64_t call,
                    const std::vector<int>* perm) {
  std::vector<double> u(n + 1);
  const double inv53 = 1.0 / 9007199254740992.0;
  for (int c = 0; 2 * c < n; ++c) {
    uint32_t ctr[4] = {static_cast<uint32_t>(c), static_cast<uint32_t>(call),
                       static_cast<uint32_t>(level), 0u};
    philox4x32_10(ctr, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const double a = (static_cast<double>(ctr[0] >> 5) * 67108864.0 + static_cast<double>(ctr[1] >> 6)) * inv53;
    const double b = (static_cast<double>(ctr[2] >> 5) * 67108864.0 + static_cast<double>(ctr[3] >> 6)) * inv53;
    u[2 * c] = a - 0.5;
    u[2 * c + 1] = b - 0.5;
  }
  v.resize(n);
  for (int j = 0; j < n; ++j) v[j] = perm ? u[(*perm)[j]] : u[j];
}


// Tridiagonal part of the dense Lanczos matrix (fill from restarts is rounding).
void tri_of(const std::vector<double>& T, int ld, int m, std::vector<double>& d,
            std::vector<double>& e) {
  d.resize(m);
  e.resize(m > 0 ? m - 1 : 0);
  for (int i = 0; i < m; ++i) d[i] = T[(size_t)i * ld + i];
  for (int i = 0; i + 1 < m; ++i) e[i] = T[(size_t)(i + 1) * ld + i];
}

// MMDEIG_LOG=1 prints per-level progress of the driver to stderr.
bool log_on() {
  static const bool on = [] {
    const char* e = std::getenv("MMDEIG_LOG");
    return e && e[0] && e[0] != '0';
  }();
  return on;
}

int keep_count(const std::vector<double>& D, int ml, double mu_h, double gamma) {
  int mh = 0;
  for (int i = 0; i < ml; ++i)
    if (D[i] >= mu_h) ++mh;
  while (mh > 0 && D[ml - 1] > gamma * D[mh - 1]) --mh;
  return mh;
}

// Wall-clock phase timer; syncs the stream at both ends only when stats are on.
struct PhaseTimer {
  eig_stats* st;
  int phase;
  hipStream_t s;
  std::chrono::steady_clock::time_point t0;
  PhaseTimer(eig_stats* st_, int ph, hipStream_t s_) : st(st_), phase(ph), s(s_) {
    if (st) {
      (void)hipStreamSynchronize(s);
      t0 = std::chrono::steady_clock::now();
    }
  }
  ~PhaseTimer() {
    if (st) {
      (void)hipStreamSynchronize(s);
      st->seconds_phase[phase] +=
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  }
};

}  // namespace

ColScalars make_scalars(Pool& pool, const std::string& tag, int b) {
  ColScalars sc;
  sc.rr = pool.d(tag + ":rr", b);
  sc.rr2 = pool.d(tag + ":rr2", b);
  sc.alpha = pool.d(tag + ":al", b);
  sc.beta = pool.d(tag + ":be", b);
  sc.bn2 = pool.d(tag + ":bn", b);
  sc.tol2 = pool.d(tag + ":tol", b);
  sc.active = pool.i(tag + ":act", b);
  sc.iters = pool.i(tag + ":it", b);
  sc.notspd = pool.i(tag + ":spd", 1);
  return sc;
}

struct Solver::Lanczos {
  int k = 0, n = 0;
  const double* Vini = nullptr;
  int mi = 0;
  double* V = nullptr;
  double* Vtmp = nullptr;
  int cap = 0;
  int j = 0;
  double* f = nullptr;
  double* w = nullptr;
  double* y = nullptr;
  std::vector<double> T;
  double beta_f = 0.0;
  double wnorm = 1.0;
  double eps_op = 0.0;
};

Solver::Solver(mmd_handle& h, hipStream_t s, const eig_opts& o, eig_stats* st)
    : h_(h), s_(s), o_(o), st_(st) {
  if (o_.alpha <= 0) o_.alpha = 3.0;
  if (o_.beta <= 0) o_.beta = 1.0;
  if (o_.restart_mult <= 0) o_.restart_mult = 1;
  if (o_.max_restarts <= 0) o_.max_restarts = 2000;
  if (o_.max_refine <= 0) o_.max_refine = 200;
  hd_.ensure(4096);
  hi_.ensure(4096);
  if (const char* e = std::getenv("MMDEIG_GRAPHS")) graphs_ = !(e[0] == '0' && e[1] == 0);
  if (const char* e = std::getenv("MMDEIG_CG_DEFER")) cg_defer_ = !(e[0] == '0' && e[1] == 0);
}

Solver::~Solver() {
  for (auto& pr : ev_pending_) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto e : ev_free_) (void)hipEventDestroy(e);
  if (ev_open_) (void)hipEventDestroy(ev_open_);
}

void Solver::spmm0_begin() {
  if (!st_) return;
  hipEvent_t e;
  if (ev_free_.empty()) {
    MMD_HIP(hipEventCreate(&e));
  } else {
    e = ev_free_.back();
    ev_free_.pop_back();
  }
  MMD_HIP(hipEventRecord(e, s_));
  ev_open_ = e;
}

void Solver::spmm0_end(double bytes, int b) {
  if (!st_ || !ev_open_) return;
  hipEvent_t e;
  if (ev_free_.empty()) {
    MMD_HIP(hipEventCreate(&e));
  } else {
    e = ev_free_.back();
    ev_free_.pop_back();
  }
  MMD_HIP(hipEventRecord(e, s_));
  ev_pending_.emplace_back(ev_open_, e);
  ev_bytes_.push_back(bytes);
  ev_open_ = nullptr;
  st_->spmm0_b = b;
}

void Solver::harvest_timers() {
  if (!st_) return;
  for (size_t i = 0; i < ev_pending_.size(); ++i) {
    float ms = 0.f;
    MMD_HIP(hipEventElapsedTime(&ms, ev_pending_[i].first, ev_pending_[i].second));
    st_->spmm0_ms += ms;
    st_->spmm0_bytes += ev_bytes_[i];
    st_->spmm0_launches += 1;
    ev_free_.push_back(ev_pending_[i].first);
    ev_free_.push_back(ev_pending_[i].second);
  }
  ev_pending_.clear();
  ev_bytes_.clear();
}

// ------------------------------------------------------------------ operators
void Solver::applyA(int k, const double* X, int ldx, double* Y, int ldy, int b) {
  spmm(h_.dev[k].A, X, ldx, Y, ldy, b, s_);
}

void Solver::applyM(int k, const double* X, int ldx, double* Y, int ldy, int b) {
  if (k == 0) copy_block(X, ldx, Y, ldy, nlev(0), b, s_);
  else spmm(h_.dev[k].M, X, ldx, Y, ldy, b, s_);
}

void Solver::applyB(int k, const double* X, int ldx, double* Y, int ldy, int b) {
  // B^(k+1) = U^T A^(k) U on the reduced space of the transfer k -> k+1
  const HouseView& H = h_.dev[k + 1].H;
  const int n = nlev(k);
  double* t1 = pool_.d("B:t1", (size_t)n * b);
  double* t2 = pool_.d("B:t2", (size_t)n * b);
  house_u(H, X, ldx, t1, b, b, s_);
  applyA(k, t1, b, t2, b, b);
  house_ut(H, t2, b, Y, ldy, b, s_);
}

// ------------------------------------------------------------------ CG
void Solver::cg(int k, OpKind op, const double* B, int ldb, double* X, int ldx, int n, int b,
                double tol, bool use_x0, const int* parent, int fixed_iters,
                const std::string& tag, std::vector<int>* iters) {
  if (b == 0 || n == 0) return;
  ColScalars sc = make_scalars(pool_, tag, b);
  double* R = pool_.d(tag + ":R", (size_t)n * b);
  double* P = pool_.d(tag + ":P", (size_t)n * b);
  double* Q = pool_.d(tag + ":Q", (size_t)n * b);
  double* p1 = pool_.d(tag + ":p1", (size_t)kRedBlocks * b);
  double* p2 = pool_.d(tag + ":p2", (size_t)kRedBlocks * b);
  const CsrView* csr = nullptr;
  if (op == OpKind::A) csr = &h_.dev[k].A;
  if (op == OpKind::M) csr = &h_.dev[k].M;
  // working set: bc columns (the unconverged ones once compacted); column j of
  // the working set is caller column cols[j], its iterate lives in Xw (ld ldw)
  int bc = b;
  double* Xw = X;
  int ldw = ldx;
  std::vector<int> cols(b);
  for (int c = 0; c < b; ++c) cols[c] = c;
  std::vector<int> it_host(b, 0);
  auto apply = [&](const double* x, int lx, double* y, int ly) {
    if (op == OpKind::A) applyA(k, x, lx, y, ly, bc);
    else if (op == OpKind::M) applyM(k, x, lx, y, ly, bc);
    else applyB(k, x, lx, y, ly, bc);
  };
  if (use_x0) {
    apply(X, ldx, R, b);
    rsub(B, ldb, R, b, n, b, s_);
  } else {
    copy_block(B, ldb, R, b, n, b, s_);
    zero_block(X, ldx, n, b, s_);
  }
  const int nb = col_dot(B, ldb, B, ldb, n, b, p1, s_);
  col_dot(R, b, R, b, n, b, p2, s_);
  cg_init(sc, p1, p2, nb, b, tol, parent, s_);
  MMD_HIP(hipMemsetAsync(sc.notspd, 0, sizeof(int), s_));
  int64_t n_wide = 0, n_narrow = 0, col_iters = 0;
  auto count_steps = [&](int steps) {
    if (bc > 32) n_wide += steps;
    else n_narrow += steps;
    col_iters += static_cast<int64_t>(bc) * steps;
  };
  auto iterate = [&](bool first) {
    int np;
    if (csr) {
      // fused: P = R + beta P, Q = A R + beta Q (= A P), partial p.q per block
      const bool timed = k == 0 && op == OpKind::A && bc > 32;
      if (timed) spmm0_begin();
      np = spmm(*csr, R, bc, Q, bc, bc, s_, true, first, sc.beta, P, bc, p1);
      if (timed) {
        // matrix once (weights + columns, row pointers, self-loops), R read once,
        // P and Q read and written once
        const double nnz = static_cast<double>(csr->nnz);
        const double bytes = 12.0 * nnz + 12.0 * n + 40.0 * n * static_cast<double>(bc) +
                             (first ? -16.0 * n * static_cast<double>(bc) : 0.0);
        spmm0_end(bytes, bc);
      }
    } else {
      xpay(R, bc, P, bc, n, bc, sc.beta, first, s_);
      apply(P, bc, Q, bc);
      np = col_dot(P, bc, Q, bc, n, bc, p1, s_);
    }
    cg_alpha(sc, p1, np, bc, s_);
    const int nu = cg_update(Xw, ldw, R, P, Q, bc, n, bc, sc.alpha, p2, s_);
    cg_beta(sc, p2, nu, bc, s_);
  };
  if (fixed_iters > 0) {
    for (int t = 0; t < fixed_iters; ++t) iterate(t == 0);
    return;
  }
  // Level-0 wide steps on the tiled form fold each step's X and R update
  // into the next step's SpMM (cg_tile_step): the step length stays pending
  // until that kernel, or a flush (k_cg_update) before the working set is
  // compacted or the loop ends, applies it.
  // A pending step reads R, Q and writes the new ones to Ra, Qa (other
  // workgroups still gather the old rows); the pairs swap after it.
  const bool defer_ok = csr && k == 0 && op == OpKind::A && cg_defer_ && cg_tile_ok(*csr);
  double* p4 = defer_ok ? pool_.d(tag + ":p4", (size_t)4 * kRedBlocks * b) : nullptr;
  double* Ra = defer_ok ? pool_.d(tag + ":Ra", (size_t)n * b) : nullptr;
  double* Qa = defer_ok ? pool_.d(tag + ":Qa", (size_t)n * b) : nullptr;
  bool pending = false;
  auto defer_step = [&](bool first_step) {
    spmm0_begin();
    const size_t ps = (size_t)kRedBlocks * bc;
    const int np = pending
        ? cg_tile_step(*csr, Xw, ldw, R, Q, Ra, Qa, P, bc, bc, true, false, sc.alpha, sc.beta,
                       p4, ps, s_)
        : cg_tile_step(*csr, Xw, ldw, R, Q, R, Q, P, bc, bc, false, first_step, sc.alpha,
                       sc.beta, p4, ps, s_);
    if (pending) {
      std::swap(R, Ra);
      std::swap(Q, Qa);
    }
    // matrix once (weights + columns, row pointers, self-loops); pending: X, R,
    // P, Q read and written once; else R read, P and Q read (not on a first
    // step) and written
    const double nnz = static_cast<double>(csr->nnz);
    const double vec = pending ? 64.0 : first_step ? 24.0 : 40.0;
    spmm0_end(12.0 * nnz + 12.0 * n + vec * n * static_cast<double>(bc), bc);
    cg_defer_scalars(sc, p4, ps, np, bc, s_);
    pending = true;
  };
  auto flush_pending = [&]() {
    if (!pending) return;
    const int nu = cg_update(Xw, ldw, R, P, Q, bc, n, bc, sc.alpha, p2, s_);
    cg_defer_flush(sc, p2, nu, bc, s_);
    pending = false;
  };
  // A chunk of steps on an unchanged working set is the same kernel sequence
  // with the same arguments every time, so after the first chunk it is
  // captured once per working set (stage) as a HIP graph and replayed.  The level-0 wide
  // steps are not captured: their SpMM launches carry the library's own
  // event timing, and at ~300 us each their launch gaps do not matter.
  hipGraphExec_t gexec = nullptr;
  int gstage = -1, gchunk = 0;
  auto drop_graph = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  };
  struct GraphGuard {
    std::function<void()> f;
    ~GraphGuard() { f(); }
  } graph_guard{drop_graph};
  // the working state moves to a compact copy once a quarter of its columns
  // have converged; converged columns keep their final iterate in X
  int* d_idx = pool_.i(tag + ":cidx", b);
  int* d_cols = pool_.i(tag + ":ccol", b);
  int stage = 0;
  auto flush_x = [&]() {  // working iterates back to the caller's columns
    if (Xw == X) return;
    h2d(d_cols, cols.data(), bc);
    scatter_cols(Xw, ldw, d_cols, X, ldx, n, bc, s_);
    sync();  // the host index list must outlive the copy
  };
  auto take_iters = [&]() {
    hi_.ensure(bc);
    d2h(hi_.p, sc.iters, bc);
    sync();
    for (int c = 0; c < bc; ++c) it_host[cols[c]] = hi_.p[c];
  };
  // The columns are checked on the host before the first step (columns whose
  // start already meets the tolerance never iterate) and then every 8 steps
  // (16 once the block is narrow); the working set is compacted as soon as an
  // eighth of it has converged.  A compaction moves about as many bytes as
  // one step, and the columns of a refinement block need from 0 to ~100
  // steps each, so the width tracks the unconverged columns closely.
  const int maxit = 100000;
  int done = 0;
  bool first = true;
  while (true) {
    hi_.ensure(bc + 1);
    d2h(hi_.p, sc.active, bc);
    d2h(hi_.p + bc, sc.notspd, 1);
    sync();
    MMD_REQUIRE(hi_.p[bc] == 0, MMD_ENOTSPD, "CG curvature p^T A p <= 0");
    std::vector<int> keep;
    for (int c = 0; c < bc; ++c)
      if (hi_.p[c] != 0) keep.push_back(c);
    if (keep.empty()) break;
    MMD_REQUIRE(done < maxit, MMD_ENOCONV, "CG reached the iteration cap");
    const int na = static_cast<int>(keep.size());
    if (bc >= 16 && 8 * na <= 7 * bc) {
      flush_pending();
      take_iters();
      flush_x();
      ++stage;
      const std::string st = tag + ":c" + std::to_string(stage & 1);
      double* R2 = pool_.d(st + "R", (size_t)n * na);
      double* P2 = pool_.d(st + "P", (size_t)n * na);
      double* Q2 = pool_.d(st + "Q", (size_t)n * na);
      double* X2 = pool_.d(st + "X", (size_t)n * na);
      ColScalars sc2 = make_scalars(pool_, st, b);
      sc2.notspd = sc.notspd;
      h2d(d_idx, keep.data(), na);
      gather_cols(R, bc, d_idx, R2, na, n, na, s_);
      if (!first) {  // before the first step P and Q hold nothing yet
        gather_cols(P, bc, d_idx, P2, na, n, na, s_);
        gather_cols(Q, bc, d_idx, Q2, na, n, na, s_);
      }
      gather_cols(Xw, ldw, d_idx, X2, na, n, na, s_);
      gather_scalars(sc, sc2, d_idx, na, s_);
      sync();  // keep (host) must outlive its copy
      std::vector<int> cols2(na);
      for (int j = 0; j < na; ++j) cols2[j] = cols[keep[j]];
      cols.swap(cols2);
      R = R2;
      P = P2;
      Q = Q2;
      Xw = X2;
      if (defer_ok) {  // spare pair of this stage: never the source of the next gather
        Ra = pool_.d(st + "Ra", (size_t)n * na);
        Qa = pool_.d(st + "Qa", (size_t)n * na);
      }
      ldw = na;
      sc = sc2;
      bc = na;
    }
    const int chunk = bc > 32 ? 8 : 16;
    const bool timed = k == 0 && op == OpKind::A && bc > 32;
    const bool defer = defer_ok && timed;
    if (!defer) flush_pending();
    // the legacy default stream cannot be captured: graphs run on the
    // caller's (or the batch's) own streams only
    if (graphs_ && s_ != nullptr && !first && !timed) {
      if (!gexec || gstage != stage || gchunk != chunk) {
        drop_graph();
        MMD_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
        hipGraph_t g = nullptr;
        try {
          for (int t = 0; t < chunk; ++t) iterate(false);
        } catch (...) {
          (void)hipStreamEndCapture(s_, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        MMD_HIP(hipStreamEndCapture(s_, &g));
        const hipError_t e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        MMD_REQUIRE(e == hipSuccess, MMD_EHIP, "hipGraphInstantiate failed");
        gstage = stage;
        gchunk = chunk;
      }
      MMD_HIP(hipGraphLaunch(gexec, s_));
    } else if (defer) {
      for (int t = 0; t < chunk; ++t) {
        defer_step(first);
        first = false;
      }
    } else {
      for (int t = 0; t < chunk; ++t) {
        iterate(first);
        first = false;
      }
    }
    count_steps(chunk);
    done += chunk;
  }
  flush_pending();
  take_iters();
  flush_x();
  if (log_on() && k == 0 && op == OpKind::A && b > 32) {
    std::vector<int> h = it_host;
    std::sort(h.begin(), h.end());
    std::fprintf(stderr, "[mmdeig] cg0 %s b %d iters min %d med %d max %d; steps wide %lld narrow %lld; column-steps %lld\n",
                 tag.c_str(), b, h.front(), h[h.size() / 2], h.back(), (long long)n_wide,
                 (long long)n_narrow, (long long)col_iters);
  }
  if (iters) *iters = it_host;
}

bool Solver::pcg_single(int k, const double* B, double* X, double tol, bool use_x0,
                        std::vector<int>* iters) {
  const int n = nlev(k);
  Pcg1Args a;
  a.A = h_.dev[k].A;
  if (k > 0) a.M = h_.dev[k].M;
  a.n = n;
  a.b = B;
  a.x = X;
  a.r = pool_.d("p1:r", n);
  a.z = pool_.d("p1:z", n);
  a.zo = pool_.d("p1:zo", n);
  a.p = pool_.d("p1:p", n);
  a.q = pool_.d("p1:q", n);
  a.ri = pool_.d("p1:ri", n);
  a.pi = pool_.d("p1:pi", n);
  a.qi = pool_.d("p1:qi", n);
  a.red = pool_.d("p1:red", pcg1_red_size());
  a.bar = reinterpret_cast<unsigned*>(pool_.i("p1:bar", 64));
  a.tol = tol;
  a.tol_in = 0.1 * tol;
  a.use_x0 = use_x0 ? 1 : 0;
  a.out = pool_.i("p1:out", 3);
  a.res = pool_.d("p1:res", 2);
  const Pcg1Plan* plan = nullptr;
  {
    auto it = plans_.find(k);
    if (it == plans_.end()) {
      std::vector<int> rp(n + 1);
      d2h(rp.data(), a.A.rowptr, n + 1);
      sync();
      it = plans_.emplace(k, Pcg1Plan()).first;
      if (k == 0) {
        pcg1_plan(a.A, rp, it->second, s_, batcher_ ? 32 : 112);
      } else {
        std::vector<int> rpm(n + 1);
        d2h(rpm.data(), a.M.rowptr, n + 1);
        sync();
        pcg1_plan_flex(a.A, rp, a.M, rpm, it->second, s_);
      }
    }
    plan = &it->second;
  }
  if (batcher_) {
    // the right-hand side is complete before the batched launch reads it;
    // the batcher returns after that launch has finished
    sync();
    batcher_->solve(pcg1_request(a, plan));
  } else {
    pcg1(a, s_, plan);
  }
  hi_.ensure(4);
  d2h(hi_.p, a.out, 3);
  sync();
  MMD_REQUIRE(hi_.p[2] != 1, MMD_ENOTSPD, "PCG curvature p^T A p <= 0");
  MMD_REQUIRE(hi_.p[2] != 2, MMD_ENOCONV, "PCG reached the iteration cap");
  if (st_ && k > 0) st_->cg_M_iters[k] += hi_.p[1];
  if (iters) iters->assign(1, hi_.p[0]);
  return true;
}

// ------------------------------------------------------------------ mixed precision
void Solver::ensure32() {
  LevelDev& D = h_.dev[0];
  if (D.has32) return;
  const CsrView& A = D.A;
  D.a_val32.ensure(std::max<int64_t>(1, A.nnz));
  to_f32(A.val, D.a_val32.p, A.nnz, s_);
  if (A.diag) {
    D.a_diag32.ensure(std::max(1, A.n_rows));
    to_f32(A.diag, D.a_diag32.p, A.n_rows, s_);
  }
  D.A32.n_rows = A.n_rows;
  D.A32.n_cols = A.n_cols;
  D.A32.nnz = A.nnz;
  D.A32.rowptr = A.rowptr;
  D.A32.col = A.col;
  D.A32.val = D.a_val32.p;
  D.A32.diag = A.diag ? D.a_diag32.p : nullptr;
  D.A32.t_kind = A.t_kind;
  D.A32.t_row = A.t_row;
  D.A32.t_uptr = A.t_uptr;
  D.A32.t_urow = A.t_urow;
  D.A32.t_lcol = A.t_lcol;
  D.A32.t_nblk = A.t_nblk;
  D.has32 = true;
}

// Mixed-precision level-0 block CG with reliable updates (residual
// replacement, Sleijpen and van der Vorst 1996; the mixed-precision form of
// Clark et al. 2010): CG iterates in FP32 on the FP32 copy of the edge-form
// matrix (directions P, products Q = A P, recursive residual R, increment D),
// while X, the true residual B - A X, the stop test and the deflation stay
// FP64.  When a column's recursive residual has fallen by the factor delta
// since its last replacement, the increments of all working columns are
// added to X in FP64, the true residuals replace the recursive ones, and
// iteration continues on the same search directions (beta rescaled to the
// replaced residual), so the Krylov space is not thrown away as in a
// restarted refinement.  A column stops when its true residual meets tol, or
// at the FP64 floor of a true residual; a column whose true residual stops
// shrinking across replacements hands the remaining columns to FP64 CG.
void Solver::cg_mixed(const double* B, int ldb, double* X, int ldx, int b, double tol,
                      bool use_x0, std::vector<int>* iters, const Deflation* dfl) {
  const int n = nlev(0);
  ensure32();
  const CsrView32& A32 = h_.dev[0].A32;
  if (!use_x0) zero_block(X, ldx, n, b, s_);
  if (norm_a0_ <= 0.0) {  // ||A||_inf of the level-0 matrix for the floor test
    const HostCSR& A0 = h_.host[0].A;
    for (int i = 0; i < A0.n_rows; ++i) {
      double t = 0.0;
      for (int64_t q = A0.ptr[i]; q < A0.ptr[i + 1]; ++q) t += std::fabs(A0.val[q]);
      norm_a0_ = std::max(norm_a0_, t);
    }
  }
  // FP64 work of the replacements (working columns gathered contiguously)
  double* Xw = pool_.d("mx:X", (size_t)n * b);
  double* Bw = pool_.d("mx:B", (size_t)n * b);
  double* Rw = pool_.d("mx:R", (size_t)n * b);
  double* part = pool_.d("mx:part", (size_t)kRedBlocks * b);
  double* nrm = pool_.d("mx:nrm", b);
  double* d_rt = pool_.d("mx:rt", b);
  int* d_gl = pool_.i("mx:gl", b);
  int* d_idx = pool_.i("mx:idx", b);
  int* d_src = pool_.i("mx:src", b);
  double* p1 = pool_.d("m32:p1", (size_t)kRedBlocks * b);
  double* p2 = pool_.d("m32:p2", (size_t)kRedBlocks * b);
  // delta: a replacement per 10x drop of the recursive residual norm (the
  // recursive FP32 residual then never drifts far from the true one); at most
  // kSince FP32 steps between replacements; a column whose true residual
  // norm is more than 2x its recursive one restarts its direction
  const double delta2 = 1e-2, restart2 = 4.0;
  constexpr int kStall = 4;      // replacements without a 2x true-residual drop
  constexpr int kMaxUpdates = 400;
  constexpr int kSince = 256;
  constexpr int kMaxCurv = 3;    // FP32 curvature breakdowns before FP64 takes over
  int curv = 0;

  std::vector<double> bn2(b);
  {
    const int g = col_dot(B, ldb, B, ldb, n, b, part, s_);
    reduce_partials(part, g, b, nrm, s_);
    d2h(bn2.data(), nrm, b);
    sync();
  }
  std::vector<int> total(b, 0);
  std::vector<std::vector<double>> hist(b);
  std::vector<int> gl(b);  // working column -> global column
  for (int c = 0; c < b; ++c) gl[c] = c;
  int m = b, ldw = even_ld(b), stage = 0;
  float* R = nullptr;
  float* P = nullptr;
  float* Q = nullptr;
  float* D = nullptr;
  int* upd = nullptr;
  ColScalars sc{};
  bool first = true, fallback = false;
  std::vector<double> rr, xx;
  std::vector<int> hv(b + 1), src_host(b);  // host lists live until the next sync
  auto alloc_stage = [&](int mm) {
    const std::string st = "m32:s" + std::to_string(stage & 1);
    const int ld = even_ld(mm);
    float* R2 = pool_.f(st + "R", (size_t)n * ld);
    float* P2 = pool_.f(st + "P", (size_t)n * ld);
    float* Q2 = pool_.f(st + "Q", (size_t)n * ld);
    float* D2 = pool_.f(st + "D", (size_t)n * ld);
    int* u2 = pool_.i(st + "upd", std::max(mm, 1));
    ColScalars s2 = make_scalars(pool_, st, std::max(mm, 1));
    ++stage;
    return std::make_tuple(R2, P2, Q2, D2, u2, s2, ld);
  };
  int updates = 0;
  while (true) {
    // ---- residual replacement over the working columns (FP64)
    if (D) {
      for (int c = 0; c < m; ++c) src_host[c] = c;
      h2d(d_src, src_host.data(), m);
      h2d(d_gl, gl.data(), m);
      scatter_add64(D, ldw, d_src, d_gl, X, ldx, n, m, s_);
    } else {
      h2d(d_gl, gl.data(), m);
    }
    const bool ident = m == b && ldx == b && ldb == b;  // no gather needed
    const double* Xc = X;
    const double* Bc = B;
    int ldxc = ldx, ldbc = ldb;
    if (!ident) {
      gather_cols(X, ldx, d_gl, Xw, m, n, m, s_);
      gather_cols(B, ldb, d_gl, Bw, m, n, m, s_);
      Xc = Xw;
      Bc = Bw;
      ldxc = ldbc = m;
    }
    applyA(0, Xc, ldxc, Rw, m, m);
    rsub(Bc, ldbc, Rw, m, n, m, s_);
    if (dfl && dfl->m > 0) {
      // C = Q^T R ; R -= Q C ; X += Q diag(mu) C   (all FP64)
      const int mq = dfl->m;
      double* C = pool_.d("mx:C", (size_t)mq * m);
      double* gw = pool_.d("mx:gw", gram_work_size(n, mq, m));
      if (ident) {
        copy_block(X, ldx, Xw, m, n, m, s_);
      } else if (Xc != Xw) {
        gather_cols(X, ldx, d_gl, Xw, m, n, m, s_);
      }
      gram(dfl->Q, dfl->ld, Rw, m, n, mq, m, C, m, gw, s_);
      gemm_nn(dfl->Q, dfl->ld, C, m, Rw, m, n, mq, m, -1.0, 1.0, s_);
      scale_rows(C, m, dfl->mu, mq, m, s_);
      gemm_nn(dfl->Q, dfl->ld, C, m, Xw, m, n, mq, m, 1.0, 1.0, s_);
      scatter_cols(Xw, m, d_gl, X, ldx, n, m, s_);
      Xc = Xw;
      ldxc = m;
    }
    {
      int g = col_dot(Rw, m, Rw, m, n, m, part, s_);
      reduce_partials(part, g, m, nrm, s_);
      rr.resize(m);
      d2h(rr.data(), nrm, m);
      g = col_dot(Xc, ldxc, Xc, ldxc, n, m, part, s_);
      reduce_partials(part, g, m, nrm, s_);
      xx.resize(m);
      d2h(xx.data(), nrm, m);
      if (sc.iters) {
        hi_.ensure(m);
        d2h(hi_.p, sc.iters, m);
      }
      sync();
      if (sc.iters)
        for (int c = 0; c < m; ++c) total[gl[c]] = hi_.p[c];
    }
    std::vector<int> keep;
    for (int c = 0; c < m; ++c) {
      const int g = gl[c];
      const double floor = 64.0 * 2.2e-16 * norm_a0_ * std::sqrt(xx[c]);
      const bool at_floor = !hist[g].empty() && rr[c] > 0.25 * hist[g].back() &&
                            rr[c] <= floor * floor;
      if (!(bn2[g] > 0.0) || rr[c] <= tol * tol * bn2[g] || at_floor) continue;
      hist[g].push_back(rr[c]);
      const size_t h = hist[g].size();
      if (h > kStall && hist[g][h - 1] > 0.25 * hist[g][h - 1 - kStall]) fallback = true;
      keep.push_back(c);
    }
    if (keep.empty()) break;
    if (fallback || updates >= kMaxUpdates) {
      fallback = true;
      break;
    }
    ++updates;
    // ---- FP32 working state of the kept columns
    const int na = static_cast<int>(keep.size());
    std::vector<double> rt(na);
    for (int j = 0; j < na; ++j) rt[j] = rr[keep[j]];
    auto [R2, P2, Q2, D2, u2, sc2, ld2] = alloc_stage(na);
    h2d(d_idx, keep.data(), na);
    h2d(d_rt, rt.data(), na);
    gather_to32(Rw, m, d_idx, R2, ld2, n, na, s_);
    zero32(D2, n, ld2, s_);
    if (first) {
      zero32(P2, n, ld2, s_);
      zero32(Q2, n, ld2, s_);
      const int nb = col_dot32(R2, ld2, R2, ld2, n, na, p1, s_);
      cg_init(sc2, p1, nullptr, nb, na, std::sqrt(delta2), nullptr, s_);
      MMD_HIP(hipMemsetAsync(sc2.notspd, 0, sizeof(int), s_));
      MMD_HIP(hipMemsetAsync(u2, 0, sizeof(int) * na, s_));
    } else {
      gather32(P, ldw, d_idx, P2, ld2, n, na, s_);
      gather32(Q, ldw, d_idx, Q2, ld2, n, na, s_);
      gather_scalars(sc, sc2, d_idx, na, s_);
      sc2.notspd = sc.notspd;
      reliable_scalars(sc2, d_rt, delta2, restart2, na, u2, s_);
    }
    std::vector<int> gl2(na);
    for (int j = 0; j < na; ++j) gl2[j] = gl[keep[j]];
    sync();  // host index lists must outlive their copies
    gl.swap(gl2);
    R = R2;
    P = P2;
    Q = Q2;
    D = D2;
    upd = u2;
    sc = sc2;
    ldw = ld2;
    m = na;
    // ---- FP32 CG until some column asks for a replacement
    int chunk = 4, since = 0;
    while (true) {
      for (int t = 0; t < chunk; ++t) {
        const bool timed = m > 64;
        if (timed) spmm0_begin();
        const int np = spmm32_cg(A32, R, ldw, Q, ldw, m, first, sc.beta, P, ldw, p1, s_);
        if (timed) {
          // matrix once (4-byte weights and columns, row pointers, self-loops),
          // R read once, P and Q read and written once (FP32)
          const double nnz = static_cast<double>(A32.nnz);
          const double bytes = 8.0 * nnz + 8.0 * n + 20.0 * n * static_cast<double>(m) +
                               (first ? -8.0 * n * static_cast<double>(m) : 0.0);
          spmm0_end(bytes, m);
        }
        first = false;
        cg_alpha(sc, p1, np, m, s_);
        const int nu = cg_update32(D, ldw, R, P, Q, ldw, n, m, sc.alpha, p2, s_);
        cg_beta_flag(sc, p2, nu, m, upd, s_);
      }
      since += chunk;
      d2h(hv.data(), upd, m);
      d2h(hv.data() + m, sc.notspd, 1);
      sync();
      bool any = false;
      for (int c = 0; c < m; ++c) any |= hv[c] != 0;
      if (hv[m] != 0) {
        // p^T A p <= 0 in FP32 (a direction at the FP32 resolution of a
        // near-singular matrix): the column stopped; the replacement restarts
        // it from its true residual, repeated breakdowns go to FP64
        MMD_HIP(hipMemsetAsync(sc.notspd, 0, sizeof(int), s_));
        if (++curv > kMaxCurv) fallback = true;
        break;
      }
      if (any || since >= kSince) break;
      chunk = std::min(chunk * 2, 32);
    }
    if (fallback) {
      // add the open increments before FP64 CG continues from X
      for (int c = 0; c < m; ++c) src_host[c] = c;
      h2d(d_src, src_host.data(), m);
      h2d(d_gl, gl.data(), m);
      scatter_add64(D, ldw, d_src, d_gl, X, ldx, n, m, s_);
      hi_.ensure(m);
      d2h(hi_.p, sc.iters, m);
      sync();
      for (int c = 0; c < m; ++c) total[gl[c]] = hi_.p[c];
      break;
    }
  }
  if (fallback) {
    std::vector<int> its64;
    cg(0, OpKind::A, B, ldb, X, ldx, n, b, tol, true, nullptr, 0, "mxfb", &its64);
    for (int c = 0; c < b; ++c) total[c] += its64[c];
    if (st_) st_->mixed_fallbacks += 1;
    if (log_on())
      std::fprintf(stderr, "[mmdeig] mixed refinement: FP64 CG finishes the open columns "
                           "after %d residual replacements\n", updates);
  }
  if (iters) *iters = total;
}

void Solver::pcg(int k, const double* B, int ldb, double* X, int ldx, int b, double tol,
                 bool use_x0, std::vector<int>* iters, const Deflation* dfl) {
  const int n = nlev(k);
  if (b == 1 && ldb == 1 && ldx == 1 && use_persistent_) {
    pcg_single(k, B, X, tol, use_x0, iters);
    return;
  }
  if (k == 0) {
    if (o_.precision == 1)
      cg_mixed(B, ldb, X, ldx, b, tol, use_x0, iters, dfl);
    else
      cg(0, OpKind::A, B, ldb, X, ldx, n, b, tol, use_x0, nullptr, 0, "cg0", iters);
    return;
  }
  if (b == 0) return;
  const std::string tag = "pcg";
  ColScalars sc = make_scalars(pool_, tag, b);
  double* R = pool_.d(tag + ":R", (size_t)n * b);
  double* Z = pool_.d(tag + ":Z", (size_t)n * b);
  double* Zo = pool_.d(tag + ":Zo", (size_t)n * b);
  double* P = pool_.d(tag + ":P", (size_t)n * b);
  double* Q = pool_.d(tag + ":Q", (size_t)n * b);
  double* p1 = pool_.d(tag + ":p1", (size_t)kRedBlocks * b);
  double* p2 = pool_.d(tag + ":p2", (size_t)kRedBlocks * b);
  double* p3 = pool_.d(tag + ":p3", (size_t)kRedBlocks * b);
  if (use_x0) {
    applyA(k, X, ldx, R, b, b);
    rsub(B, ldb, R, b, n, b, s_);
  } else {
    copy_block(B, ldb, R, b, n, b, s_);
    zero_block(X, ldx, n, b, s_);
  }
  const int nb = col_dot(B, ldb, B, ldb, n, b, p1, s_);
  col_dot(R, b, R, b, n, b, p2, s_);
  cg_init(sc, p1, p2, nb, b, tol, nullptr, s_);
  MMD_HIP(hipMemsetAsync(sc.notspd, 0, sizeof(int), s_));
  const double tol_in = 0.1 * tol;
  auto minv = [&](double* Zout) {
    cg(k, OpKind::M, R, b, Zout, b, n, b, tol_in, false, sc.active, inner_iters_, "inner", nullptr);
  };
  minv(Z);
  {
    const int nz = col_dot(R, b, Z, b, n, b, p1, s_);
    reduce_partials(p1, nz, b, sc.rr, s_);  // rz
  }
  const int maxit = 100000;
  int done = 0, chunk = 4;
  bool first = true;
  int64_t inner_total = 0;
  while (true) {
    for (int t = 0; t < chunk; ++t) {
      int np;
      if (b <= 32) {
        np = spmm(h_.dev[k].A, Z, b, Q, b, b, s_, true, first, sc.beta, P, b, p1);
      } else {
        spmm(h_.dev[k].A, Z, b, Q, b, b, s_, true, first, sc.beta, P, b, nullptr);
        np = col_dot(P, b, Q, b, n, b, p1, s_);
      }
      cg_alpha(sc, p1, np, b, s_);
      const int nu = cg_update(X, ldx, R, P, Q, b, n, b, sc.alpha, p2, s_);
      pcg_conv(sc, p2, nu, b, s_);
      std::swap(Z, Zo);
      minv(Z);
      const int nd = col_dot2(R, b, Z, Zo, b, n, b, p1, p3, s_);
      pcg_beta(sc, p1, p3, nd, b, s_);
      first = false;
    }
    done += chunk;
    inner_total += chunk;
    hi_.ensure(2 * b + 2);
    d2h(hi_.p, sc.active, b);
    d2h(hi_.p + b, sc.notspd, 1);
    d2h(hi_.p + b + 1, pool_.i("inner:act", b), b);
    sync();
    MMD_REQUIRE(hi_.p[b] == 0, MMD_ENOTSPD, "PCG curvature p^T A p <= 0");
    bool any = false, inner_open = false;
    for (int c = 0; c < b; ++c) {
      any |= hi_.p[c] != 0;
      inner_open |= hi_.p[b + 1 + c] != 0;
    }
    if (inner_open && inner_iters_ < 64) inner_iters_ += 4;
    if (!any) break;
    MMD_REQUIRE(done < maxit, MMD_ENOCONV, "PCG reached the iteration cap");
    chunk = std::min(chunk * 2, 32);
  }
  if (st_) st_->cg_M_iters[k] += inner_total * inner_iters_ * b;
  if (iters) {
    iters->resize(b);
    d2h(hi_.p, sc.iters, b);
    sync();
    std::copy(hi_.p, hi_.p + b, iters->begin());
  }
}

// ------------------------------------------------------------------ Lanczos (Alg. 3)
double Solver::mnorm2(int k, const double* x) {
  const int n = nlev(k);
  double* p = pool_.d("mn:p", kRedBlocks);
  double* out = pool_.d("mn:o", 1);
  int nb;
  if (k == 0) {
    nb = col_dot(x, 1, x, 1, n, 1, p, s_);
  } else {
    double* y = pool_.d("mn:y", n);
    applyM(k, x, 1, y, 1, 1);
    nb = col_dot(x, 1, y, 1, n, 1, p, s_);
  }
  reduce_partials(p, nb, 1, out, s_);
  d2h(hd_.p, out, 1);
  sync();
  return hd_.p[0];
}

void Solver::lanczos_orth(Lanczos& L, double* w, int jcols, std::vector<double>* hlast) {
  const int n = L.n;
  double* y = L.y;
  double* h1 = pool_.d("lz:h1", std::max(L.mi, 1));
  double* h2 = pool_.d("lz:h2", std::max(jcols, 1));
  double* work = pool_.d("lz:gw", (size_t)kGemvChunks * std::max(std::max(L.mi, jcols), 1));
  double last = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    if (L.k == 0) copy_block(w, 1, y, 1, n, 1, s_);
    else applyM(L.k, w, 1, y, 1, 1);
    if (L.mi > 0) {
      gemv_t(L.Vini, L.mi, y, n, L.mi, h1, work, s_);
      gemv_n_sub(L.Vini, L.mi, h1, n, L.mi, w, s_);
    }
    if (jcols > 0) {
      gemv_t(L.V, L.cap, y, n, jcols, h2, work, s_);
      gemv_n_sub(L.V, L.cap, h2, n, jcols, w, s_);
      if (hlast) {
        d2h(hd_.p + pass, h2 + jcols - 1, 1);
      }
    }
  }
  if (hlast && jcols > 0) {
    sync();
    last = hd_.p[0] + hd_.p[1];
    hlast->assign(1, last);
  }
}

void Solver::lanczos_random(Lanczos& L, double* out) {
  std::vector<double> v;
  uniform_vector(v, L.n, o_.seed, L.k, draws_[L.k]++,
                 (L.k == 0 && !h_.perm.empty()) ? &h_.perm : nullptr);
  h2d(out, v.data(), L.n);
  lanczos_orth(L, out, L.j, nullptr);
  sync();  // v goes out of scope
}

void Solver::lanczos_init(Lanczos& L, int k, const double* Vini, int mi, int cap_cols) {
  L.k = k;
  L.n = nlev(k);
  L.Vini = Vini;
  L.mi = mi;
  L.cap = std::max(cap_cols, 1);
  L.j = 0;
  L.V = pool_.d("lz:V", (size_t)L.n * L.cap);
  L.Vtmp = pool_.d("lz:Vt", (size_t)L.n * L.cap);
  L.f = pool_.d("lz:f", L.n);
  L.w = pool_.d("lz:w", L.n);
  L.y = pool_.d("lz:y", L.n);
  L.T.assign((size_t)L.cap * L.cap, 0.0);
  L.wnorm = 1.0;
  lanczos_random(L, L.f);
  L.beta_f = std::sqrt(mnorm2(k, L.f));
}

void Solver::lanczos_steps(Lanczos& L, int nsteps) {
  const int n = L.n;
  double* v = pool_.d("lz:v", n);
  double* rhs = pool_.d("lz:rhs", n);
  for (int t = 0; t < nsteps; ++t) {
    const int j = L.j;
    MMD_REQUIRE(j < L.cap, MMD_EINVAL, "Lanczos basis capacity exceeded");
    double coupling;
    if (j > 0 && L.beta_f <= 1e-12 * L.wnorm) {
      lanczos_random(L, L.f);
      const double b2 = std::sqrt(mnorm2(L.k, L.f));
      axpby(1.0 / b2, L.f, 1, 0.0, v, 1, n, 1, s_);
      coupling = 0.0;
    } else {
      axpby(1.0 / L.beta_f, L.f, 1, 0.0, v, 1, n, 1, s_);
      coupling = L.beta_f;
    }
    copy_block(v, 1, L.V + j, L.cap, n, 1, s_);
    if (j > 0) {
      L.T[(size_t)j * L.cap + j - 1] = coupling;
      L.T[(size_t)(j - 1) * L.cap + j] = coupling;
    }
    // w = OP(v) = pcg(A, M v, M, 0, eps)
    if (L.k == 0) copy_block(v, 1, rhs, 1, n, 1, s_);
    else applyM(L.k, v, 1, rhs, 1, 1);
    std::vector<int> it;
    {
      PhaseTimer pt(st_, 4, s_);
      pcg(L.k, rhs, 1, L.w, 1, 1, L.eps_op, false, st_ ? &it : nullptr);
    }
    if (st_) {
      st_->pcg_A_calls[L.k] += 1;
      st_->pcg_A_iters[L.k] += it.empty() ? 0 : it[0];
    }
    {
      PhaseTimer pt(st_, 5, s_);
      L.wnorm = std::sqrt(mnorm2(L.k, L.w));
      std::vector<double> hl;
      lanczos_orth(L, L.w, j + 1, &hl);
      L.T[(size_t)j * L.cap + j] = hl[0];
      std::swap(L.f, L.w);
      L.beta_f = std::sqrt(mnorm2(L.k, L.f));
    }
    L.j = j + 1;
    if (st_) st_->lanczos_steps[L.k] += 1;
  }
}

bool Solver::ritz_converged(Lanczos& L, int nwant, double eps, bool relative) {
  const int m = L.j;
  std::vector<double> d, e, w;
  tri_of(L.T, L.cap, m, d, e);
  std::vector<double> last(m, 0.0);
  last[m - 1] = 1.0;
  dense::tridiag_eig(m, d.data(), e.data(), w, last.data(), 1);
  for (int q = 0; q < nwant; ++q) {
    const int i = m - 1 - q;  // largest first
    const double res = L.beta_f * std::fabs(last[i]);
    const double lim = relative ? eps * std::fabs(w[i]) : eps;
    if (!(res <= lim)) return false;
  }
  return true;
}

void Solver::restart(Lanczos& L, int kkeep, int p) {
  PhaseTimer pt(st_, 6, s_);
  const int m = L.j;
  MMD_REQUIRE(m == kkeep + p, MMD_EINVAL, "restart size mismatch");
  std::vector<double> T((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) T[(size_t)i * m + j] = L.T[(size_t)i * L.cap + j];
  std::vector<double> d, e, theta;
  tri_of(L.T, L.cap, m, d, e);
  dense::tridiag_eig(m, d.data(), e.data(), theta, nullptr, 0);
  std::vector<double> Q((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
  for (int q = 0; q < p; ++q) dense::shifted_qr_step(m, T.data(), theta[q], Q.data());
  const double bk = T[(size_t)kkeep * m + kkeep - 1];
  const double sk = Q[(size_t)(m - 1) * m + kkeep - 1];
  // f <- V Q(:, k+1) T(k+1, k) + f Q(m, k)   (with the basis before truncation)
  std::vector<double> g(m), qk((size_t)m * kkeep);
  for (int i = 0; i < m; ++i) g[i] = -Q[(size_t)i * m + kkeep] * bk;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < kkeep; ++j) qk[(size_t)i * kkeep + j] = Q[(size_t)i * m + j];
  double* gd = pool_.d("rs:g", m);
  double* qd = pool_.d("rs:q", (size_t)m * kkeep);
  h2d(gd, g.data(), m);
  h2d(qd, qk.data(), (size_t)m * kkeep);
  axpby(sk, L.f, 1, 0.0, L.f, 1, L.n, 1, s_);
  gemv_n_sub(L.V, L.cap, gd, L.n, m, L.f, s_);
  gemm_nn(L.V, L.cap, qd, kkeep, L.Vtmp, L.cap, L.n, m, kkeep, 1.0, 0.0, s_);
  std::swap(L.V, L.Vtmp);
  std::vector<double> Tn((size_t)L.cap * L.cap, 0.0);
  for (int i = 0; i < kkeep; ++i)
    for (int j = 0; j < kkeep; ++j) Tn[(size_t)i * L.cap + j] = T[(size_t)i * m + j];
  L.T.swap(Tn);
  L.j = kkeep;
  L.beta_f = std::sqrt(mnorm2(L.k, L.f));  // also waits for the host arrays above
  if (st_) st_->restarts[L.k] += 1;
}

// ------------------------------------------------------------------ extension (Alg. 4)
void Solver::extend(int k, double*& V, std::vector<double>& D, int& m, int m_tar, double eps,
                    double mu_ex, int d, bool relative) {
  const int n = nlev(k);
  const int mi = m;
  if (st_) st_->ext_in[k] += mi;
  const int want = m_tar - mi;
  const int cap = n - mi;
  if (want <= 0 || cap <= 0) {
    if (st_) st_->ext_out[k] += mi;
    return;
  }
  const int c = o_.restart_mult;
  const int vcap = std::min(cap, want + c * std::max(want, d));
  Lanczos L;
  L.eps_op = k == 0 ? eps : tpcg_[k];
  lanczos_init(L, k, V, mi, vcap);
  int kcur = 0, restarts = 0;
  auto converge = [&](int kk, int p) {
    while (!ritz_converged(L, kk, eps, relative)) {
      if (p <= 0) break;
      lanczos_steps(L, p);
      restart(L, kk, p);
      MMD_REQUIRE(++restarts <= o_.max_restarts, MMD_ENOCONV, "extension: restart cap reached");
    }
  };
  while (true) {
    const int kk = std::min(std::min(kcur + d, want), cap);
    const int p = std::min(c * d, cap - kk);
    lanczos_steps(L, kk - L.j);
    converge(kk, p);
    kcur = kk;
    std::vector<double> dd, ee, th;
    tri_of(L.T, L.cap, L.j, dd, ee);
    dense::tridiag_eig(L.j, dd.data(), ee.data(), th, nullptr, 0);
    const double mu_hat = th[std::min(d, kcur) - 1];
    if (log_on())
      std::fprintf(stderr, "[mmdeig] extend L%d explored %d of %d, restarts %d, mu_hat %.6g\n",
                   k, kcur, want, restarts, mu_hat);
    if (mu_hat < mu_ex || kcur >= want || kcur >= cap) break;
  }
  const int mnew = kcur;
  converge(mnew, std::min(c * mnew, cap - mnew));
  if (log_on())
    std::fprintf(stderr, "[mmdeig] extend L%d in %d new %d restarts %d steps %d\n", k, mi, mnew,
                 restarts, L.j);
  // Schur (symmetric eig) of T, descending
  std::vector<double> T((size_t)mnew * mnew);
  for (int i = 0; i < mnew; ++i)
    for (int j = 0; j < mnew; ++j) T[(size_t)i * mnew + j] = L.T[(size_t)i * L.cap + j];
  std::vector<double> w, Z;
  dense::sym_eig(mnew, T.data(), w, &Z);
  std::vector<double> Y((size_t)mnew * mnew);
  for (int i = 0; i < mnew; ++i)
    for (int j = 0; j < mnew; ++j) Y[(size_t)i * mnew + j] = Z[(size_t)i * mnew + (mnew - 1 - j)];
  double* Yd = pool_.d("ex:Y", (size_t)mnew * mnew);
  h2d(Yd, Y.data(), Y.size());
  const int mo = mi + mnew;
  double* Vn = pool_.d(V == pool_.d("VA", 0) ? "VB" : "VA", (size_t)n * mo);
  double* tmp = pool_.d("ex:tmp", (size_t)n * mo);
  copy_block(V, mi, tmp, mo, n, mi, s_);
  gemm_nn(L.V, L.cap, Yd, mnew, tmp + mi, mo, n, mnew, mnew, 1.0, 0.0, s_);
  std::vector<double> Dn(D.begin(), D.begin() + mi);
  for (int j = 0; j < mnew; ++j) Dn.push_back(w[mnew - 1 - j]);
  std::vector<int> order(mo);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return Dn[a] > Dn[b]; });
  int* od = pool_.i("ex:ord", mo);
  h2d(od, order.data(), mo);
  gather_cols(tmp, mo, od, Vn, mo, n, mo, s_);
  D.resize(mo);
  for (int j = 0; j < mo; ++j) D[j] = Dn[order[j]];
  sync();
  V = Vn;
  m = mo;
  if (st_) st_->ext_out[k] += mo;
}

void Solver::multiplicity_check(int k, double*& V, std::vector<double>& D, int m, double eps,
                                int d) {
  // level 0: relative tests (eps * theta); coarse levels: absolute in mu
  const bool relative = k == 0;
  const int n = nlev(k);
  const int cap = n - m;
  if (cap <= 0 || m == 0) return;
  const int c = o_.restart_mult;
  for (int swaps = 0; swaps < 64; ++swaps) {
    const int s = std::min(d + 10, cap);
    const int p = std::min(c * d, cap - 1);
    Lanczos L;
    L.eps_op = k == 0 ? eps : tpcg_[k];
    lanczos_init(L, k, V, m, std::max(s, 1 + p));
    lanczos_steps(L, s);
    std::vector<double> dd, ee, th;
    tri_of(L.T, L.cap, L.j, dd, ee);
    dense::tridiag_eig(L.j, dd.data(), ee.data(), th, nullptr, 0);
    const double lim = relative ? D[m - 1] * (1.0 + eps) : D[m - 1] + eps;
    if (th.back() <= lim) return;
    while (p > 0 && !ritz_converged(L, 1, eps, relative)) {
      restart(L, 1, L.j - 1);
      lanczos_steps(L, p);
    }
    const int mm = L.j;
    std::vector<double> T((size_t)mm * mm), w, Z;
    for (int i = 0; i < mm; ++i)
      for (int j = 0; j < mm; ++j) T[(size_t)i * mm + j] = L.T[(size_t)i * L.cap + j];
    dense::sym_eig(mm, T.data(), w, &Z);
    std::vector<double> y(mm);
    for (int i = 0; i < mm; ++i) y[i] = Z[(size_t)i * mm + (mm - 1)];
    double* yd = pool_.d("mc:y", mm);
    h2d(yd, y.data(), mm);
    double* u = pool_.d("mc:u", n);
    gemm_nn(L.V, L.cap, yd, 1, u, 1, n, mm, 1, 1.0, 0.0, s_);
    copy_block(u, 1, V + (m - 1), m, n, 1, s_);
    D[m - 1] = w[mm - 1];
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return D[a] > D[b]; });
    int* od = pool_.i("mc:ord", m);
    h2d(od, order.data(), m);
    double* tmp = pool_.d("mc:tmp", (size_t)n * m);
    copy_block(V, m, tmp, m, n, m, s_);
    gather_cols(tmp, m, od, V, m, n, m, s_);
    std::vector<double> Dn(m);
    for (int j = 0; j < m; ++j) Dn[j] = D[order[j]];
    D.swap(Dn);
    sync();
    if (st_) st_->missed_swaps += 1;
  }
  throw Error(MMD_ENOCONV, "multiplicity check: too many swaps");
}

// ------------------------------------------------------------------ refinement (Alg. 5)
void Solver::mqr(int k, double* F, int n, int b, const std::string& tag) {
  double* MF = pool_.d(tag + ":MF", (size_t)n * b);
  double* G = pool_.d(tag + ":G", (size_t)b * b);
  double* Rd = pool_.d(tag + ":R", (size_t)b * b);
  double* T = pool_.d(tag + ":T", (size_t)n * b);
  double* work = pool_.d("gram:w", gram_work_size(n, b, b));
  std::vector<double> Gh((size_t)b * b), R, Ri;
  for (int pass = 0; pass < 2; ++pass) {
    if (k == 0) gram(F, b, F, b, n, b, b, G, b, work, s_);
    else {
      applyM(k, F, b, MF, b, b);
      gram(F, b, MF, b, n, b, b, G, b, work, s_);
    }
    d2h(Gh.data(), G, Gh.size());
    sync();
    MMD_REQUIRE(dense::cholesky_upper(b, Gh.data(), R), MMD_ENOCONV,
                "M-orthogonal QR: Gram matrix not positive definite");
    dense::upper_inverse(b, R.data(), Ri);
    h2d(Rd, Ri.data(), Ri.size());
    gemm_nn(F, b, Rd, b, T, b, n, b, b, 1.0, 0.0, s_);
    copy_block(T, b, F, b, n, b, s_);
    sync();
  }
}

void Solver::refine(int k, double*& V, std::vector<double>& D, int& m, double eps, double mu_h,
                    double lam_max_M, double gamma) {
  const int ml = m;
  if (st_) st_->ref_in[k] += ml;
  if (ml == 0) return;
  const int n = nlev(k);
  const HouseView& H = h_.dev[k + 1].H;
  const int nred = H.nred;
  double* MQ = pool_.d("rf:MQ", (size_t)n * ml);
  double* RB = pool_.d("rf:RB", (size_t)std::max(nred, 1) * ml);
  double* G = pool_.d("rf:G", (size_t)std::max(nred, 1) * ml);
  double* F = pool_.d("rf:F", (size_t)n * ml);
  double* F2 = pool_.d("rf:F2", (size_t)n * ml);
  double* Q = pool_.d("rf:Q", (size_t)n * ml);
  double* W = pool_.d("rf:W", (size_t)n * ml);
  double* Tm = pool_.d("rf:T", (size_t)n * ml);
  double* Qp = pool_.d("rf:Qp", (size_t)n * ml);
  double* E = pool_.d("rf:E", (size_t)n * ml);
  double* Dd = pool_.d("rf:D", ml);
  double* Pd = pool_.d("rf:P", (size_t)ml * ml);
  double* Sd = pool_.d("rf:S", (size_t)ml * ml);
  double* work = pool_.d("gram:w", gram_work_size(n, ml, ml));
  // on level 0 the solves run at 0.1 eps so the stop test lies above their noise;
  // coarse levels use the relative PCG tolerance of the level
  const double eps_solve = k == 0 ? 0.1 * eps : tpcg_[k];
  // start block F = Q D + U G, g_i = cg(B, U^T M q_i, 0, eps)
  applyM(k, V, ml, MQ, ml, ml);
  if (nred > 0) {
    house_ut(H, MQ, ml, RB, ml, ml, s_);
    PhaseTimer pt(st_, 1, s_);
    std::vector<int> it;
    cg(k, OpKind::B, RB, ml, G, ml, nred, ml, eps_solve, false, nullptr, 0, "bcg",
       st_ ? &it : nullptr);
    if (st_) {
      st_->cg_B_calls[k] += ml;
      for (int x : it) st_->cg_B_iters[k] += x;
    }
    house_u(H, G, ml, F, ml, ml, s_);
  } else {
    zero_block(F, ml, n, ml, s_);
  }
  h2d(Dd, D.data(), ml);
  scale_cols(V, ml, Dd, F, ml, n, ml, true, s_);
  std::vector<double> mu_prev(D.begin(), D.begin() + ml), Dn(ml);
  bool have_prev = false;
  int mh = 0;
  const double thresh = eps / std::sqrt(lam_max_M);
  std::vector<double> hist;
  std::vector<double> Sh((size_t)ml * ml), w, Z, Ph((size_t)ml * ml);
  int it = 0;
  for (it = 1; it <= o_.max_refine; ++it) {
    {
      PhaseTimer pt(st_, 3, s_);
      mqr(k, F, n, ml, "rq");
      copy_block(F, ml, Q, ml, n, ml, s_);
      applyM(k, Q, ml, W, ml, ml);
      h2d(Dd, mu_prev.data(), ml);
      scale_cols(Q, ml, Dd, F2, ml, n, ml, false, s_);
    }
    std::vector<int> its;
    {
      PhaseTimer pt(st_, 0, s_);
      Deflation dfl;  // used by the mixed-precision level-0 solve only
      dfl.Q = Q;
      dfl.ld = ml;
      dfl.m = ml;
      dfl.mu = Dd;
      pcg(k, W, ml, F2, ml, ml, eps_solve, true, st_ ? &its : nullptr, &dfl);
    }
    if (st_) {
      st_->pcg_A_calls[k] += ml;
      for (int x : its) st_->pcg_A_iters[k] += x;
    }
    {
      PhaseTimer pt(st_, 3, s_);
      gram(W, ml, F2, ml, n, ml, ml, Sd, ml, work, s_);
      d2h(Sh.data(), Sd, Sh.size());
    }
    {
      PhaseTimer pt(st_, 2, s_);
      dense::sym_eig(ml, Sh.data(), w, &Z);
    }
    for (int j = 0; j < ml; ++j) {
      Dn[j] = w[ml - 1 - j];
      for (int i = 0; i < ml; ++i) Ph[(size_t)i * ml + j] = Z[(size_t)i * ml + (ml - 1 - j)];
    }
    mh = keep_count(Dn, ml, mu_h, gamma);
    h2d(Pd, Ph.data(), Ph.size());
    gemm_nn(Q, ml, Pd, ml, Tm, ml, n, ml, ml, 1.0, 0.0, s_);
    std::swap(Q, Tm);
    gemm_nn(F2, ml, Pd, ml, Tm, ml, n, ml, ml, 1.0, 0.0, s_);
    std::swap(F2, Tm);
    if (st_) st_->ref_iter[k] += 1;
    bool done = false;
    if (have_prev && mh > 0) {
      applyM(k, Q, ml, MQ, ml, ml);
      double* X = pool_.d("rf:X", (size_t)mh * mh);
      double* wk = pool_.d("gram:w2", gram_work_size(n, mh, mh));
      gram(Qp, ml, MQ, ml, n, mh, mh, X, mh, wk, s_);
      copy_block(Q, ml, E, mh, n, mh, s_);
      gemm_nn(Qp, ml, X, mh, E, mh, n, mh, mh, -1.0, 1.0, s_);
      double* pr = pool_.d("rf:pr", (size_t)kRedBlocks * mh);
      double* cn = pool_.d("rf:cn", mh);
      const int nb = col_dot(E, mh, E, mh, n, mh, pr, s_);
      reduce_partials(pr, nb, mh, cn, s_);
      std::vector<double> cnh(mh);
      d2h(cnh.data(), cn, mh);
      sync();
      double fro = 0.0;
      for (double x : cnh) fro += x;
      const double dist = std::sqrt(fro);
      hist.push_back(dist);
      // stop at the threshold, or at a stagnated floor below 10x the threshold
      done = dist < thresh || (hist.size() > 5 && dist < 10 * thresh &&
                               dist > 0.9 * hist[hist.size() - 6]);
      if (log_on())
        std::fprintf(stderr, "[mmdeig] refine L%d it %d ml %d mh %d dist %.3e thresh %.3e mu[0] %.6g mu[mh-1] %.6g mu[ml-1] %.6g\n",
                     k, it, ml, mh, dist, thresh, Dn[0], Dn[std::max(mh - 1, 0)], Dn[ml - 1]);
    } else if (have_prev && mh == 0) {
      done = true;
    }
    copy_block(Q, ml, Qp, ml, n, ml, s_);
    have_prev = true;
    mu_prev = Dn;
    std::swap(F, F2);
    if (done) break;
  }
  MMD_REQUIRE(it <= o_.max_refine, MMD_ENOCONV, "refinement: iteration cap reached");
  double* Vo = pool_.d(V == pool_.d("VA", 0) ? "VB" : "VA", (size_t)n * std::max(mh, 1));
  copy_block(Q, ml, Vo, mh, n, mh, s_);
  sync();
  V = Vo;
  m = mh;
  D.assign(Dn.begin(), Dn.begin() + mh);
  if (st_) st_->ref_out[k] += mh;
}

// ------------------------------------------------------------------ output step
void Solver::final_pairs(double* V, const std::vector<double>& D0, int m, int nev, double tol,
                         double* evals, double* evecs) {
  const int n = nlev(0);
  MMD_REQUIRE(m >= nev, MMD_ENOCONV, "fewer converged pairs than requested");
  double* F = pool_.d("fp:F", (size_t)n * m);
  double* Dd = pool_.d("fp:D", m);
  double* AQ = pool_.d("fp:AQ", (size_t)n * m);
  double* Hd = pool_.d("fp:H", (size_t)m * m);
  double* Yd = pool_.d("fp:Y", (size_t)m * m);
  double* Vo = pool_.d("fp:V", (size_t)n * m);
  double* Rr = pool_.d("fp:Rr", (size_t)n * nev);
  double* work = pool_.d("gram:w", gram_work_size(n, m, m));
  double* pr = pool_.d("fp:pr", (size_t)kRedBlocks * m);
  double* cn = pool_.d("fp:cn", m);
  double* ld = pool_.d("fp:ld", m);
  std::vector<double> D(D0.begin(), D0.begin() + m), lam, Z;
  // Inverse iteration + Rayleigh-Ritz with A on the block, repeated while a
  // returned pair misses ||A v - lambda v|| <= 10 tol lambda ||v|| and the
  // largest such residual still falls by 10% per pass.
  const int max_passes = 30;
  double prev = std::numeric_limits<double>::infinity();
  for (int pass = 0;; ++pass) {
    h2d(Dd, D.data(), m);
    scale_cols(V, m, Dd, F, m, n, m, false, s_);
    std::vector<int> its;
    cg(0, OpKind::A, V, m, F, m, n, m, tol, true, nullptr, 0, "cg0", st_ ? &its : nullptr);
    if (st_) {
      st_->pcg_A_calls[0] += m;
      for (int x : its) st_->pcg_A_iters[0] += x;
    }
    mqr(0, F, n, m, "fq");
    applyA(0, F, m, AQ, m, m);
    gram(F, m, AQ, m, n, m, m, Hd, m, work, s_);
    std::vector<double> Hh((size_t)m * m);
    d2h(Hh.data(), Hd, Hh.size());
    sync();
    dense::sym_eig(m, Hh.data(), lam, &Z);
    h2d(Yd, Z.data(), Z.size());
    gemm_nn(F, m, Yd, m, Vo, m, n, m, m, 1.0, 0.0, s_);
    // residual norms of the nev returned pairs: R = A V - V diag(lambda)
    h2d(ld, lam.data(), nev);
    applyA(0, Vo, m, Rr, nev, nev);
    double* Tv = AQ;  // free again: V diag(lambda) for the nev columns
    scale_cols(Vo, m, ld, Tv, nev, n, nev, false, s_);
    axpby(-1.0, Tv, nev, 1.0, Rr, nev, n, nev, s_);
    int nb = col_dot(Rr, nev, Rr, nev, n, nev, pr, s_);
    reduce_partials(pr, nb, nev, cn, s_);
    nb = col_dot(Vo, m, Vo, m, n, nev, pr, s_);
    reduce_partials(pr, nb, nev, ld, s_);
    std::vector<double> rn(nev), vn(nev);
    d2h(rn.data(), cn, nev);
    d2h(vn.data(), ld, nev);
    sync();
    double worst = 0.0;
    for (int j = 0; j < nev; ++j)
      worst = std::max(worst, std::sqrt(rn[j]) / (std::fabs(lam[j]) * std::sqrt(vn[j])));
    if (log_on())
      std::fprintf(stderr, "[mmdeig] output pass %d: max relative residual %.3e\n", pass, worst);
    if (worst <= 10.0 * tol || worst > 0.9 * prev || pass + 1 >= max_passes) break;
    prev = worst;
    // next pass: the Ritz block (all m columns) and its mu = 1 / lambda
    copy_block(Vo, m, V, m, n, m, s_);
    for (int j = 0; j < m; ++j) D[j] = 1.0 / lam[j];
  }
  double* Vn = pool_.d("fp:Vn", (size_t)n * nev);
  copy_block(Vo, m, Vn, nev, n, nev, s_);
  emit_pairs(Vn, lam, nev, evals, evecs);
}

void Solver::emit_pairs(const double* Vn, const std::vector<double>& lam, int nev, double* evals,
                        double* evecs) {
  // unit 2-norm, largest-magnitude entry positive (lowest caller index on
  // ties), column-major in the caller's numbering
  const int n = nlev(0);
  double* pr = pool_.d("ep:pr", (size_t)kRedBlocks * nev);
  double* cn = pool_.d("ep:cn", nev);
  int* ai = pool_.i("ep:ai", nev);
  double* av = pool_.d("ep:av", nev);
  const int nb = col_dot(Vn, nev, Vn, nev, n, nev, pr, s_);
  reduce_partials(pr, nb, nev, cn, s_);
  const int* perm = h_.perm.empty() ? nullptr : h_.d_perm.p;
  const size_t aw = col_absmax_work_size(n, nev);
  col_absmax(Vn, nev, n, nev, ai, av, perm, pool_.i("ep:awi", aw), pool_.d("ep:awv", aw), s_);
  std::vector<double> nrm(nev), amax(nev), scale(nev);
  d2h(nrm.data(), cn, nev);
  d2h(amax.data(), av, nev);
  sync();
  for (int j = 0; j < nev; ++j) scale[j] = (amax[j] < 0 ? -1.0 : 1.0) / std::sqrt(nrm[j]);
  double* sd = pool_.d("ep:sc", nev);
  h2d(sd, scale.data(), nev);
  to_colmajor(Vn, nev, sd, evecs, n, nev, perm, s_);
  for (int j = 0; j < nev; ++j) evals[j] = lam[j];
  sync();
}

void Solver::coarse_output(const double* V, const std::vector<double>& D, int m, int k, int nev,
                           double* evals, double* evecs) {
  // Section 7.3: lambda = 1 / mu of the level-k pairs, v = Psi^(1) ... Psi^(k) z
  MMD_REQUIRE(m >= nev, MMD_ENOCONV,
              "coarse-level approximation: level " + std::to_string(k) + " produced " +
                  std::to_string(m) + " pairs, fewer than nev");
  const double* cur = V;
  int ld = m;
  for (int j = k; j >= 1; --j) {
    const int nf = nlev(j - 1);
    double* nxt = pool_.d(j % 2 ? "co:a" : "co:b", (size_t)nf * nev);
    spmm(h_.dev[j].Psi, cur, ld, nxt, nev, nev, s_);
    cur = nxt;
    ld = nev;
  }
  std::vector<double> lam(nev);
  for (int j = 0; j < nev; ++j) lam[j] = 1.0 / D[j];
  emit_pairs(cur, lam, nev, evals, evecs);
}

// ------------------------------------------------------------------ driver (Alg. 6)
void Solver::leftmost(int nev, double tol, double* evals, double* evecs) {
  const auto t0 = std::chrono::steady_clock::now();
  const int K = h_.K;
  const int n0 = nlev(0);
  MMD_REQUIRE(nev > 0 && nev <= n0, MMD_EINVAL, "nev out of range");
  MMD_REQUIRE(tol > 0 && tol < 1, MMD_EINVAL, "tol must be in (0, 1)");
  const double alpha = o_.alpha, beta = o_.beta, gamma = (1.0 + beta) / alpha;
  std::vector<double> eps_op(K + 1), mu_re(K + 1), mu_ex(K + 1);
  std::vector<int> dd(K + 1);
  // PCG solves stop at the relative residual eps^(k); without the paper's
  // scaling (lambda_1 = 1) eps^(k) = 0.1 eps_k can exceed 1, where x = 0
  // already passes and OP vanishes: levels k >= 1 use min(eps^(k), 0.1)
  tpcg_.assign(K + 1, tol);
  for (int k = 1; k <= K; ++k) tpcg_[k] = std::min(0.1, 0.1 * h_.eps[k]);
  for (int k = 0; k <= K; ++k) {
    eps_op[k] = k == 0 ? tol : 0.1 * h_.eps[k];
    mu_re[k] = k + 1 <= K ? alpha * h_.eps[k + 1] : 0.0;
    mu_ex[k] = beta * h_.eps[k];
    dd[k] = o_.d > 0 ? std::min(o_.d, nlev(k)) : std::max(1, std::min(nlev(k) / 10, nev / 10));
  }
  const int stop = o_.stop_level;
  MMD_REQUIRE(stop >= 0 && stop <= K, MMD_EINVAL,
              "stop_level must lie between 0 and the number of coarse levels");
  if (st_) {
    std::memset(st_, 0, sizeof(eig_stats));
    st_->K = K;
  }
  ev_pending_.clear();
  ev_bytes_.clear();
  double* V = pool_.d("VA", 1);
  std::vector<double> D;
  int m = 0;
  if (K > 0) {
    // Alg. 6 first step: coarsest generalised eigenproblem (dense, host)
    const LevelHost& L = h_.host[K];
    const int nk = L.n;
    std::vector<double> A((size_t)nk * nk, 0.0), M((size_t)nk * nk, 0.0);
    for (int i = 0; i < nk; ++i) {
      for (int64_t q = L.A.ptr[i]; q < L.A.ptr[i + 1]; ++q) A[(size_t)i * nk + L.A.col[q]] = L.A.val[q];
      for (int64_t q = L.M.ptr[i]; q < L.M.ptr[i + 1]; ++q) M[(size_t)i * nk + L.M.col[q]] = L.M.val[q];
    }
    std::vector<double> lam, Z;
    MMD_REQUIRE(dense::gen_eig(nk, A.data(), M.data(), lam, Z), MMD_ENOTSPD,
                "coarsest M not positive definite");
    int keep = 0;
    for (int i = 0; i < nk; ++i)
      if (1.0 / lam[i] >= mu_ex[K]) ++keep;
    // the coarse-level approximation on the coarsest level itself returns the
    // nev leading pairs of the dense problem (Section 7.3), no threshold
    if (stop == K) keep = nk;
    keep = std::min(keep, nev);
    std::vector<double> Zk((size_t)nk * std::max(keep, 1));
    for (int i = 0; i < nk; ++i)
      for (int j = 0; j < keep; ++j) Zk[(size_t)i * keep + j] = Z[(size_t)i * nk + j];
    V = pool_.d("VA", (size_t)nk * std::max(keep, 1));
    h2d(V, Zk.data(), (size_t)nk * keep);
    D.resize(keep);
    for (int j = 0; j < keep; ++j) D[j] = 1.0 / lam[j];
    m = keep;
    sync();
    if (st_) st_->ext_out[K] = keep;
  }
  for (int k = K - 1; k >= stop; --k) {
    const auto tl = std::chrono::steady_clock::now();
    cur_level_ = k;
    // the level returned by the coarse-level approximation: OP accurate to
    // eps^(k) in mu units, i.e. relative eps^(k) / mu_1 (mu_1 = 1 under the
    // paper's scaling, where the two readings coincide)
    if (k == stop && k > 0 && m > 0) tpcg_[k] = std::min(0.1, eps_op[k] / D[0]);
    // reform V <- Psi^(k+1) V
    const int nk = nlev(k);
    double* Vn = pool_.d(V == pool_.d("VA", 0) ? "VB" : "VA", (size_t)nk * std::max(m, 1));
    if (m > 0) spmm(h_.dev[k + 1].Psi, V, m, Vn, m, m, s_);
    V = Vn;
    refine(k, V, D, m, eps_op[k], mu_re[k], h_.host[k].lam_max_M, gamma);
    extend(k, V, D, m, nev, eps_op[k], mu_ex[k], dd[k], k == 0);
    if (st_) st_->seconds_level[k] = std::chrono::duration<double>(std::chrono::steady_clock::now() - tl).count();
  }
  if (stop > 0) {
    // coarse-level approximation: the level-stop pairs (with missed copies
    // of repeated eigenvalues swapped in), lifted to level 0
    if (stop < K) {
      PhaseTimer pt(st_, 7, s_);
      multiplicity_check(stop, V, D, m, eps_op[stop], dd[stop]);
    }
    coarse_output(V, D, m, stop, nev, evals, evecs);
    if (st_) {
      st_->nconv = nev;
      st_->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return;
  }
  if (K == 0) extend(0, V, D, m, nev, tol, 0.0, dd[0], true);
  {
    PhaseTimer pt(st_, 7, s_);
    multiplicity_check(0, V, D, m, tol, dd[0]);
    final_pairs(V, D, m, nev, tol, evals, evecs);
  }
  if (st_) {
    st_->nconv = nev;
    st_->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
}

// ------------------------------------------------------------------ exposed blocks
void Solver::apply_op(int level, int op, const double* Xu, double* Yu, int b) {
  MMD_REQUIRE(level >= 0 && level <= h_.K, MMD_EINVAL, "level out of range");
  MMD_REQUIRE(b > 0, MMD_EINVAL, "b must be positive");
  MMD_REQUIRE(op >= 0 && op <= 6, MMD_EINVAL, "unknown operator");
  MMD_REQUIRE(op != 6 || level == 0, MMD_EINVAL, "the FP32 operator exists on level 0 only");
  // level-0 vectors are in the caller's numbering at the boundary
  const bool perm = level == 0 && !h_.perm.empty();
  const int n0 = nlev(0);
  const bool in0 = perm && (op == 0 || op == 1 || op == 4 || op == 6);
  const bool out0 = perm && (op == 0 || op == 1 || op == 3 || op == 5 || op == 6);
  const double* X = Xu;
  double* Y = Yu;
  if (in0) {
    double* t = pool_.d("ap:in", (size_t)n0 * b);
    permute_rows(Xu, b, t, b, n0, b, h_.d_perm.p, false, s_);
    X = t;
  }
  if (out0) Y = pool_.d("ap:out", (size_t)n0 * b);
  switch (op) {
    case 0: applyA(level, X, b, Y, b, b); break;
    case 1: applyM(level, X, b, Y, b, b); break;
    case 2:
      MMD_REQUIRE(level < h_.K, MMD_EINVAL, "B needs a coarser level");
      applyB(level, X, b, Y, b, b);
      break;
    case 3:
      MMD_REQUIRE(level < h_.K, MMD_EINVAL, "U needs a coarser level");
      house_u(h_.dev[level + 1].H, X, b, Y, b, b, s_);
      break;
    case 4:
      MMD_REQUIRE(level < h_.K, MMD_EINVAL, "U^T needs a coarser level");
      house_ut(h_.dev[level + 1].H, X, b, Y, b, b, s_);
      break;
    case 5:
      MMD_REQUIRE(level < h_.K, MMD_EINVAL, "Psi needs a coarser level");
      spmm(h_.dev[level + 1].Psi, X, b, Y, b, b, s_);
      break;
    case 6: {
      // the FP32 kernel of the mixed-precision solves: X rounded to FP32, the
      // first (beta-free) fused CG step Y = A32 X32, Y widened to FP64
      ensure32();
      const int ld32 = even_ld(b);
      float* X32 = pool_.f("ap:x32", (size_t)n0 * ld32);
      float* Y32 = pool_.f("ap:y32", (size_t)n0 * ld32);
      float* P32 = pool_.f("ap:p32", (size_t)n0 * ld32);
      double* part = pool_.d("ap:part", (size_t)kRedBlocks * b);
      double* bet = pool_.d("ap:beta", b);
      int* ids = pool_.i("ap:ids", b);
      std::vector<int> id(b);
      std::iota(id.begin(), id.end(), 0);
      h2d(ids, id.data(), b);
      gather_to32(X, b, ids, X32, ld32, n0, b, s_);
      spmm32_cg(h_.dev[0].A32, X32, ld32, Y32, ld32, b, true, bet, P32, ld32, part, s_);
      zero_block(Y, b, n0, b, s_);
      scatter_add64(Y32, ld32, ids, ids, Y, b, n0, b, s_);
      sync();  // id (host) must outlive its copy
      break;
    }
    default: throw Error(MMD_EINVAL, "unknown operator");
  }
  if (out0) permute_rows(Y, b, Yu, b, n0, b, h_.d_perm.p, true, s_);
}

void Solver::solve(int level, int kind, const double* rhs, double* X, int b, bool use_x0,
                   double tol, int* iters_out) {
  MMD_REQUIRE(level >= 0 && level <= h_.K, MMD_EINVAL, "level out of range");
  MMD_REQUIRE(b > 0, MMD_EINVAL, "b must be positive");
  MMD_REQUIRE(tol > 0 && tol < 1, MMD_EINVAL, "tol must be in (0, 1)");
  std::vector<int> it;
  if (kind == 0) {
    if (level == 0 && !h_.perm.empty()) {
      const int n0 = nlev(0);
      double* r = pool_.d("sv:rhs", (size_t)n0 * b);
      double* x = pool_.d("sv:x", (size_t)n0 * b);
      permute_rows(rhs, b, r, b, n0, b, h_.d_perm.p, false, s_);
      if (use_x0) permute_rows(X, b, x, b, n0, b, h_.d_perm.p, false, s_);
      pcg(level, r, b, x, b, b, tol, use_x0, &it);
      permute_rows(x, b, X, b, n0, b, h_.d_perm.p, true, s_);
    } else {
      pcg(level, rhs, b, X, b, b, tol, use_x0, &it);
    }
  } else if (kind == 2) {
    MMD_REQUIRE(level == 0, MMD_EINVAL, "the mixed-precision solve is a level-0 solve");
    const int n0 = nlev(0);
    if (!h_.perm.empty()) {
      double* r = pool_.d("sv:rhs", (size_t)n0 * b);
      double* x = pool_.d("sv:x", (size_t)n0 * b);
      permute_rows(rhs, b, r, b, n0, b, h_.d_perm.p, false, s_);
      if (use_x0) permute_rows(X, b, x, b, n0, b, h_.d_perm.p, false, s_);
      cg_mixed(r, b, x, b, b, tol, use_x0, &it);
      permute_rows(x, b, X, b, n0, b, h_.d_perm.p, true, s_);
    } else {
      cg_mixed(rhs, b, X, b, b, tol, use_x0, &it);
    }
  } else if (kind == 1) {
    MMD_REQUIRE(level < h_.K, MMD_EINVAL, "B needs a coarser level");
    const int nred = h_.dev[level + 1].H.nred;
    cg(level, OpKind::B, rhs, b, X, b, nred, b, tol, use_x0, nullptr, 0, "bcg", &it);
  } else {
    throw Error(MMD_EINVAL, "unknown solve kind");
  }
  sync();
  if (iters_out) std::copy(it.begin(), it.end(), iters_out);
}

}  // namespace mmd
