// Persistent cooperative CG / flexible PCG for one right-hand side.
#pragma once

#include <vector>

#include "common.h"
#include "kernels.h"

namespace mmd {

struct Pcg1Args {
  CsrView A;          // level operator (edge form on level 0)
  CsrView M;          // preconditioner M^(k); rowptr == nullptr: plain CG
  int n = 0;
  const double* b = nullptr;
  double* x = nullptr;  // x0 on entry when use_x0, solution on exit
  double *r = nullptr, *z = nullptr, *zo = nullptr, *p = nullptr, *q = nullptr;
  double *ri = nullptr, *pi = nullptr, *qi = nullptr;  // inner CG work
  double* red = nullptr;  // pcg1_red_size() doubles
  unsigned* bar = nullptr;  // one arrival counter (zeroed by pcg1 before the launch)
  double tol = 0.0, tol_in = 0.0;
  int maxit = 100000, maxit_in = 500, use_x0 = 0;
  int lpr_a = 8, lpr_m = 8;
  int fold = 1;  // resident plain CG: one barrier per iteration (1) or two (0); from the plan
  int* out = nullptr;     // [3]: outer iterations, inner iterations, flag (1 not SPD, 2 cap)
  double* res = nullptr;  // [2]: final ||r||^2, ||b||^2
};

// Row partition and LDS size for the resident plain-CG kernel on A (host copy
// rp of its row pointers).  resident == false: A does not fit, use k_pcg1.
struct Pcg1Plan {
  bool resident = false;
  bool flex = false;  // resident flexible PCG (A and M slices in LDS)
  bool fold = true;   // plain CG: one barrier per iteration (most gathers block-local)
  int grid = 0;
  size_t lds = 0;
  DBuf<int> part;  // grid + 1 row boundaries
};
// grid_cap: preferred block count (more are taken when the slices need the
// LDS of more blocks).  The block partition is copied on stream s (ordered
// with the solver's work; no legacy-stream copy, so another thread may be
// capturing a graph meanwhile) and s is synchronised.
void pcg1_plan(const CsrView& A, const std::vector<int>& rp, Pcg1Plan& plan, hipStream_t s,
               int grid_cap = 112);
// Plan for the resident flexible PCG on (A, M) (host row pointers rpa, rpm):
// the fewest blocks (multiple of 8, at least 16) whose slices fit in LDS.
void pcg1_plan_flex(const CsrView& A, const std::vector<int>& rpa, const CsrView& M,
                    const std::vector<int>& rpm, Pcg1Plan& plan, hipStream_t s);

// Launch on stream s (asynchronous).  Stop rule ||r|| <= tol ||b||; the inner
// CG stops at ||r_in|| <= tol_in ||r||.  Plain CG (no M) runs the resident
// kernel when plan says it fits.
void pcg1(Pcg1Args a, hipStream_t s, const Pcg1Plan* plan = nullptr);

// One solve of a batched launch: the same arguments and plan as pcg1, the
// kernel body and block count pcg1 would choose, and the request's block
// range [off, off + nblk) in the batch grid.
struct Pcg1Req {
  Pcg1Args a;
  const int* part = nullptr;  // resident plans: row boundaries per block
  int kind = 0;               // 0 resident plain CG, 1 resident flexible PCG, 2 from global memory
  int off = 0, nblk = 0;
  size_t lds = 0;             // dynamic LDS bytes per block
};
Pcg1Req pcg1_request(Pcg1Args a, const Pcg1Plan* plan);
// Blocks that can be co-resident in one batched launch with lds bytes of
// dynamic LDS per block.
int pcg1_multi_capacity(size_t lds);
// One cooperative launch of all reqs (offsets assigned here, multiples of 8);
// h_reqs (pinned) and d_reqs hold reqs.size() entries; every request's
// arrival counter is cleared on s before the launch.  The caller checks that
// the total block count fits pcg1_multi_capacity.
void pcg1_multi(std::vector<Pcg1Req>& reqs, Pcg1Req* h_reqs, Pcg1Req* d_reqs, hipStream_t s);
size_t pcg1_red_size();
int pcg1_grid();

}  // namespace mmd
