// Single-right-hand-side CG / flexible PCG as one persistent cooperative kernel.
//
// The Lanczos operator OP (Section 4) applies pcg(A, M v, M, 0, eps) to one
// vector per step; launched as separate kernels every CG iteration costs
// several kernel boundaries, so the whole solve (outer PCG and the inner CG
// on M) runs here in one cooperative launch with grid-wide barriers.
//
// Barrier discipline: every block executes exactly the same sequence of grid
// barriers.  Each loop decision (convergence, curvature check, iteration
// caps) is taken from scalars that every block computes from the same global
// partial sums in the same order, so all blocks agree.
//
// Cross-XCD synchronisation costs about 30 ns per arriving block on MI355X,
// so the kernel runs few fat workgroups (1024 threads) with a single arrival
// counter; the cooperative launch guarantees they are co-resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "pcg_persistent.h"

namespace mmd {

namespace {

constexpr int kThreads = 1024;
constexpr int kWave = 64;

struct Ctx {
  unsigned* bar;  // arrival counter, zero at launch
  unsigned gen;   // barriers passed so far
  int nblk, blk, gtid, gsize, gwave, nwave, lane;
  double* red;   // two disjoint slots of 4*nblk partial sums
  int slot;
};

// Grid barrier: every block adds one arrival (release), then waits until all
// c.nblk arrivals of this generation are in (relaxed spin, acquire fence).
// c.nblk is the number of blocks of this solve (the whole grid, or one
// request's block range in a batched launch).
__device__ inline void grid_barrier(Ctx& c) {
  __syncthreads();
  c.gen += 1;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(c.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    // modular comparison: the counter may wrap past 2^32 in a long solve, the
    // distance to the target never exceeds c.nblk
    const unsigned target = c.gen * (unsigned)c.nblk;
    while ((int)(__hip_atomic_load(c.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0)
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Sum of v over the block, result valid in every thread.
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < kThreads / kWave; ++q) t += sh[q];
  __syncthreads();
  return t;
}

// Grid-wide sum: each block contributes its partial, barrier, then every block
// adds the partials in the same fixed order.
__device__ inline double grid_sum(Ctx& c, double part, double* sh) {
  const double b = block_sum(part, sh);
  // every grid sum uses slot regions of 4 nblk doubles (the widest sum's), so
  // consecutive sums, which take alternate slots, never share partials
  double* r = c.red + (size_t)c.slot * 4 * c.nblk;
  if (threadIdx.x == 0) r[c.blk] = b;
  grid_barrier(c);
  // the first wavefront adds the partials (same order in every block) and
  // hands the sum to the others through LDS: one block barrier instead of a
  // full block reduction
  if (threadIdx.x < kWave) {
    double t = 0.0;
    for (int j = threadIdx.x; j < c.nblk; j += kWave) t += r[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, kWave);
    if (threadIdx.x == 0) sh[0] = t;
  }
  __syncthreads();
  const double s = sh[0];
  c.slot ^= 1;
  return s;
}

// Two grid sums sharing one barrier.
__device__ inline void grid_sum2(Ctx& c, double p1, double p2, double* sh, double& s1,
                                 double& s2) {
  const double b1 = block_sum(p1, sh);
  const double b2 = block_sum(p2, sh);
  double* r = c.red + (size_t)c.slot * 4 * c.nblk;
  if (threadIdx.x == 0) {
    r[c.blk] = b1;
    r[c.nblk + c.blk] = b2;
  }
  grid_barrier(c);
  if (threadIdx.x < kWave) {
    double t1 = 0.0, t2 = 0.0;
    for (int j = threadIdx.x; j < c.nblk; j += kWave) {
      t1 += r[j];
      t2 += r[c.nblk + j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      t1 += __shfl_xor(t1, off, kWave);
      t2 += __shfl_xor(t2, off, kWave);
    }
    if (threadIdx.x == 0) {
      sh[0] = t1;
      sh[1] = t2;
    }
  }
  __syncthreads();
  s1 = sh[0];
  s2 = sh[1];
  c.slot ^= 1;
}

// Four grid sums sharing one barrier; sh4 holds 4 * kThreads / kWave + 4
// doubles.  Thread 0 publishes the block's four partials (the thread that
// releases the barrier), slot regions of 4 * nblk doubles alternate.
__device__ inline void grid_sum4(Ctx& c, double p0, double p1, double p2, double p3,
                                 double* sh4, double (&s)[4]) {
  constexpr int W = kThreads / kWave;
  double v[4] = {p0, p1, p2, p3};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] += __shfl_xor(v[m], off, kWave);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) sh4[m * W + w] = v[m];
  __syncthreads();
  double* r = c.red + (size_t)c.slot * 4 * c.nblk;
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double t = 0.0;
      for (int q = 0; q < W; ++q) t += sh4[m * W + q];
      r[(size_t)m * c.nblk + c.blk] = t;
    }
  grid_barrier(c);
  if (threadIdx.x < kWave) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < c.nblk; j += kWave)
#pragma unroll
      for (int m = 0; m < 4; ++m) t[m] += r[(size_t)m * c.nblk + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int m = 0; m < 4; ++m) t[m] += __shfl_xor(t[m], off, kWave);
    if (threadIdx.x == 0)
#pragma unroll
      for (int m = 0; m < 4; ++m) sh4[4 * W + m] = t[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) s[m] = sh4[4 * W + m];
  c.slot ^= 1;
}

// Rows handled by one wave per pass: kUnroll row-groups of kWave / lpr rows,
// their gathers interleaved so a wave keeps several loads in flight.
constexpr int kUnroll = 4;

// acc[u] = (A x)_row(u) for the kUnroll row-groups g0 + u * nwave of this wave
// (edge form when A.diag != null: s_i x_i + sum_j w_ij (x_i - x_j)).  All lanes
// of the wave call this together; lanes of rows past the end get zero.
__device__ inline void rows_apply(const Ctx& c, const CsrView& A, const double* __restrict__ x,
                                  int lpr, int g0, int groups, int row[kUnroll],
                                  double acc[kUnroll]) {
  const int R = kWave / lpr;
  const int s = c.lane % lpr;
  const int r = c.lane / lpr;
  int lo[kUnroll], hi[kUnroll];
  double xi[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int g = g0 + u * c.nwave;
    row[u] = g * R + r;
    const bool ok = g < groups && row[u] < A.n_rows;
    if (!ok) row[u] = -1;
    lo[u] = ok ? A.rowptr[row[u]] + s : 0;
    hi[u] = ok ? A.rowptr[row[u] + 1] : 0;
    xi[u] = (ok && A.diag) ? x[row[u]] : 0.0;
    acc[u] = 0.0;
  }
  for (int t = 0;; t += lpr) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int k = lo[u] + t;
      if (k < hi[u]) {
        any = true;
        const double xj = x[A.col[k]];
        acc[u] += A.diag ? A.val[k] * (xi[u] - xj) : A.val[k] * xj;
      }
    }
    if (!any) break;
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    for (int off = 1; off < lpr; off <<= 1) acc[u] += __shfl_xor(acc[u], off, kWave);
    if (A.diag && row[u] >= 0) acc[u] += A.diag[row[u]] * xi[u];
  }
}

// Fused CG direction step: w = A rr (all rows of rr complete), then per row
// p = rr + beta p, q = w + beta q; returns this thread's share of p.q.
__device__ inline double dir_step(Ctx& c, const CsrView& A, int lpr, const double* rr, double* p,
                                  double* q, double beta, bool first) {
  const int R = kWave / lpr;
  const int s = c.lane % lpr;
  const int groups = (A.n_rows + R - 1) / R;
  double part = 0.0;
  for (int g0 = c.gwave; g0 < groups; g0 += kUnroll * c.nwave) {
    int row[kUnroll];
    double w[kUnroll];
    rows_apply(c, A, rr, lpr, g0, groups, row, w);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (row[u] >= 0 && s == 0) {
        const int i = row[u];
        const double pn = first ? rr[i] : rr[i] + beta * p[i];
        const double qn = first ? w[u] : w[u] + beta * q[i];
        p[i] = pn;
        q[i] = qn;
        part += pn * qn;
      }
    }
  }
  return part;
}

__device__ inline void body_pcg1(const Pcg1Args& a, const int gblk, const int gnb, double* sh) {
  // rows are dealt per XCD-contiguous block number (workgroups go round-robin to XCDs)
  const int bx = (gnb % 8) ? (int)gblk
                                 : (int)((gblk % 8) * (gnb / 8) + gblk / 8);
  Ctx c{a.bar, 0u, (int)gnb, (int)gblk,
        (int)(bx * blockDim.x + threadIdx.x), (int)(gnb * blockDim.x),
        (int)((bx * blockDim.x + threadIdx.x) / kWave),
        (int)((gnb * blockDim.x) / kWave), (int)(threadIdx.x & (kWave - 1)), a.red, 0};
  const int n = a.n;
  const bool pre = a.M.rowptr != nullptr;
  // r = b - A x0 (or b with x = 0); ||b||^2, ||r||^2
  double pb = 0.0, pr = 0.0;
  if (a.use_x0) {
    // w = A x0 stored in q temporarily
    const int R = kWave / a.lpr_a;
    const int s = c.lane % a.lpr_a;
    const int groups = (n + R - 1) / R;
    for (int g0 = c.gwave; g0 < groups; g0 += kUnroll * c.nwave) {
      int row[kUnroll];
      double w[kUnroll];
      rows_apply(c, a.A, a.x, a.lpr_a, g0, groups, row, w);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (row[u] >= 0 && s == 0) a.q[row[u]] = w[u];
    }
    grid_barrier(c);
    for (int i = c.gtid; i < n; i += c.gsize) {
      const double ri = a.b[i] - a.q[i];
      a.r[i] = ri;
      pb += a.b[i] * a.b[i];
      pr += ri * ri;
    }
  } else {
    for (int i = c.gtid; i < n; i += c.gsize) {
      a.x[i] = 0.0;
      a.r[i] = a.b[i];
      pb += a.b[i] * a.b[i];
    }
    pr = pb;
  }
  double bn2, rr2;
  grid_sum2(c, pb, pr, sh, bn2, rr2);
  const double tol2 = a.tol * a.tol * bn2;
  int it = 0, inner_total = 0, flag = 0;
  bool done = !(bn2 > 0.0) || rr2 <= tol2;
  if (!pre) {
    // ---------------- plain CG
    double rr = rr2, beta = 0.0;
    bool first = true;
    while (!done) {
      const double ppq = dir_step(c, a.A, a.lpr_a, a.r, a.p, a.q, beta, first);
      first = false;
      const double pq = grid_sum(c, ppq, sh);
      if (!(pq > 0.0)) {
        flag = 1;
        break;
      }
      const double al = rr / pq;
      double prr = 0.0;
      for (int i = c.gtid; i < n; i += c.gsize) {
        a.x[i] += al * a.p[i];
        const double ri = a.r[i] - al * a.q[i];
        a.r[i] = ri;
        prr += ri * ri;
      }
      const double rn = grid_sum(c, prr, sh);
      ++it;
      beta = rn / rr;
      rr = rn;
      rr2 = rn;
      if (rn <= tol2) break;
      if (it >= a.maxit) {
        flag = 2;
        break;
      }
    }
  } else {
    // ---------------- flexible PCG with an inner CG on M (zero start)
    const double tol_in2 = a.tol_in * a.tol_in;
    auto inner = [&](double rnorm2) {
      // z = M^-1 r approximately; ri = r, pi/qi directions, z accumulates
      for (int i = c.gtid; i < n; i += c.gsize) {
        a.z[i] = 0.0;
        a.ri[i] = a.r[i];
      }
      grid_barrier(c);
      double rri = rnorm2, bi = 0.0;
      bool f = true;
      int k = 0;
      while (rri > tol_in2 * rnorm2 && k < a.maxit_in) {
        const double ppq = dir_step(c, a.M, a.lpr_m, a.ri, a.pi, a.qi, bi, f);
        f = false;
        const double pq = grid_sum(c, ppq, sh);
        if (!(pq > 0.0)) break;
        const double al = rri / pq;
        double prr = 0.0;
        for (int i = c.gtid; i < n; i += c.gsize) {
          a.z[i] += al * a.pi[i];
          const double ri = a.ri[i] - al * a.qi[i];
          a.ri[i] = ri;
          prr += ri * ri;
        }
        const double rn = grid_sum(c, prr, sh);
        bi = rn / rri;
        rri = rn;
        ++k;
      }
      inner_total += k;
    };
    if (!done) {
      inner(rr2);
      double prz = 0.0;
      for (int i = c.gtid; i < n; i += c.gsize) prz += a.r[i] * a.z[i];
      double rz = grid_sum(c, prz, sh);
      double beta = 0.0;
      bool first = true;
      while (true) {
        const double ppq = dir_step(c, a.A, a.lpr_a, a.z, a.p, a.q, beta, first);
        first = false;
        const double pq = grid_sum(c, ppq, sh);
        if (!(pq > 0.0)) {
          flag = 1;
          break;
        }
        const double al = rz / pq;
        double prr = 0.0;
        for (int i = c.gtid; i < n; i += c.gsize) {
          a.x[i] += al * a.p[i];
          const double ri = a.r[i] - al * a.q[i];
          a.r[i] = ri;
          a.zo[i] = a.z[i];
          prr += ri * ri;
        }
        const double rn = grid_sum(c, prr, sh);
        ++it;
        rr2 = rn;
        if (rn <= tol2) break;
        if (it >= a.maxit) {
          flag = 2;
          break;
        }
        inner(rn);
        double p1 = 0.0, p2 = 0.0;
        for (int i = c.gtid; i < n; i += c.gsize) {
          p1 += a.r[i] * a.z[i];
          p2 += a.r[i] * a.zo[i];
        }
        double rzn, rzo;
        grid_sum2(c, p1, p2, sh, rzn, rzo);
        beta = (rzn - rzo) / rz;
        rz = rzn;
      }
    }
  }
  if (c.gtid == 0) {
    a.out[0] = it;
    a.out[1] = inner_total;
    a.out[2] = flag;
    a.res[0] = rr2;
    a.res[1] = bn2;
  }
}

// ---------------------------------------------------------------------------
// Resident plain CG (no preconditioner; the level-0 operator).  Block bx owns
// the contiguous rows [part[bx], part[bx+1]) (balanced by nonzeros + rows on
// the host) and keeps their slice of the matrix in LDS for the whole solve;
// thread t owns local rows t, t + 1024, ... and holds x, r, p, q of those rows
// in registers.  CG with one grid barrier per iteration: an iteration first
// applies the previous step's update to its own rows (x += alpha p,
// r -= alpha q), forms A r gathering the neighbours' new r as r_j - alpha q_j
// from the previous iteration's copies of r and q in global memory, updates
// p = r + beta p, q = A r + beta q, writes r and q to the other buffer pair,
// and ends in one grid sum of p.q, r.q, q.q and r.r.  alpha = r.r / p.q, and
// the next residual norm, needed for beta and the stop test before the next
// update is applied, is |r - alpha q|^2 = r.r - 2 alpha r.q + alpha^2 q.q.
// The buffer pairs alternate, so the one barrier both publishes an
// iteration's r and q and ends every read of the pair the next iteration
// overwrites.  The iterates are those of plain CG; the expansion differs from
// the summed norm by rounding relative to the previous r.r (it is not
// trusted to stop the solve below 64 eps of it; the next direct r.r is).
// The second gathered vector pays off when the gathers stay mostly within a
// block's own rows (the patch-ordered level 0); for a matrix in an order
// that scatters them the plan selects the two-barrier form (a.fold = 0):
// plain CG with one gathered vector, grid sums of p.q and of r.r.
constexpr int kMaxU = 4;  // rows per thread

// (A r)_i of local row l with r_i = ri (edge form when ldg != null).
__device__ inline double row_res(int l, double ri, const int* lrp, const int* lcol,
                                 const double* lval, const double* ldg, const double* r) {
  const int lo = lrp[l], hi = lrp[l + 1];
  double a0 = 0.0, a1 = 0.0;
  int k = lo;
  if (ldg) {
    for (; k + 3 < hi; k += 4) {
      const double x0 = r[lcol[k]], x1 = r[lcol[k + 1]], x2 = r[lcol[k + 2]], x3 = r[lcol[k + 3]];
      a0 += lval[k] * (ri - x0) + lval[k + 1] * (ri - x1);
      a1 += lval[k + 2] * (ri - x2) + lval[k + 3] * (ri - x3);
    }
    for (; k < hi; ++k) a0 += lval[k] * (ri - r[lcol[k]]);
    return ldg[l] * ri + (a0 + a1);
  }
  for (; k + 3 < hi; k += 4) {
    const double x0 = r[lcol[k]], x1 = r[lcol[k + 1]], x2 = r[lcol[k + 2]], x3 = r[lcol[k + 3]];
    a0 += lval[k] * x0 + lval[k + 1] * x1;
    a1 += lval[k + 2] * x2 + lval[k + 3] * x3;
  }
  for (; k < hi; ++k) a0 += lval[k] * r[lcol[k]];
  return a0 + a1;
}

// (A r')_i of local row l with r'_i = ri and the neighbours' r'_j formed as
// r_j - al q_j (the same fused multiply-add as the owner's update of r_j).
__device__ inline double row_res_pend(int l, double ri, const int* lrp, const int* lcol,
                                      const double* lval, const double* ldg,
                                      const double* r, const double* q, double al) {
  const int lo = lrp[l], hi = lrp[l + 1];
  double a0 = 0.0, a1 = 0.0;
  int k = lo;
  auto g = [&](int j) { return __builtin_fma(-al, q[j], r[j]); };
  if (ldg) {
    for (; k + 3 < hi; k += 4) {
      const double x0 = g(lcol[k]), x1 = g(lcol[k + 1]), x2 = g(lcol[k + 2]), x3 = g(lcol[k + 3]);
      a0 += lval[k] * (ri - x0) + lval[k + 1] * (ri - x1);
      a1 += lval[k + 2] * (ri - x2) + lval[k + 3] * (ri - x3);
    }
    for (; k < hi; ++k) a0 += lval[k] * (ri - g(lcol[k]));
    return ldg[l] * ri + (a0 + a1);
  }
  for (; k + 3 < hi; k += 4) {
    const double x0 = g(lcol[k]), x1 = g(lcol[k + 1]), x2 = g(lcol[k + 2]), x3 = g(lcol[k + 3]);
    a0 += lval[k] * x0 + lval[k + 1] * x1;
    a1 += lval[k + 2] * x2 + lval[k + 3] * x3;
  }
  for (; k < hi; ++k) a0 += lval[k] * g(lcol[k]);
  return a0 + a1;
}

__device__ inline void body_cg1_res(const Pcg1Args& a, const int* __restrict__ part,
                                    const int gblk, const int gnb, double* lds, double* sh,
                                    double* sh4) {
  const int bx = (gnb % 8) ? (int)gblk
                                 : (int)((gblk % 8) * (gnb / 8) + gblk / 8);
  Ctx c{a.bar, 0u, (int)gnb, (int)gblk, 0, 0, 0, 0, (int)(threadIdx.x & (kWave - 1)),
        a.red, 0};
  const CsrView& A = a.A;
  const int r0 = part[bx], r1 = part[bx + 1], nr = r1 - r0;
  const int e0 = A.rowptr[r0], ne = A.rowptr[r1] - e0;
  const bool edge = A.diag != nullptr;
  double* lval = lds;
  double* ldg = lval + ne;
  int* lrp = reinterpret_cast<int*>(ldg + (edge ? nr : 0));
  int* lcol = lrp + nr + 1;
  for (int t = threadIdx.x; t < ne; t += kThreads) {
    lval[t] = A.val[e0 + t];
    lcol[t] = A.col[e0 + t];
  }
  for (int t = threadIdx.x; t <= nr; t += kThreads) lrp[t] = A.rowptr[r0 + t] - e0;
  if (edge)
    for (int t = threadIdx.x; t < nr; t += kThreads) ldg[t] = A.diag[r0 + t];
  __syncthreads();
  const double* dg = edge ? ldg : nullptr;
  double* r = a.r;
  double xr[kMaxU], rr_[kMaxU], pr[kMaxU], qr[kMaxU];
  double pb = 0.0, prr0 = 0.0;
#pragma unroll
  for (int u = 0; u < kMaxU; ++u) {
    xr[u] = rr_[u] = pr[u] = qr[u] = 0.0;
    const int l = threadIdx.x + u * kThreads;
    if (l < nr) {
      const double bi = a.b[r0 + l];
      pb += bi * bi;
      if (a.use_x0) {
        xr[u] = a.x[r0 + l];
      } else {
        rr_[u] = bi;
        r[r0 + l] = bi;
      }
    }
  }
  if (a.use_x0) {
    // r = b - A x0, x0 gathered from global memory (complete at launch)
#pragma unroll
    for (int u = 0; u < kMaxU; ++u) {
      const int l = threadIdx.x + u * kThreads;
      if (l < nr) {
        const double ri = a.b[r0 + l] - row_res(l, xr[u], lrp, lcol, lval, dg, a.x);
        rr_[u] = ri;
        r[r0 + l] = ri;
        prr0 += ri * ri;
      }
    }
  } else {
    prr0 = pb;
  }
  double bn2, rr2;
  grid_sum2(c, pb, prr0, sh, bn2, rr2);
  const double tol2 = a.tol * a.tol * bn2;
  int it = 0, flag = 0;
  bool done = !(bn2 > 0.0) || rr2 <= tol2;
  // r and q copies read by the neighbours: iteration t reads pair t % 2 and
  // writes pair (t + 1) % 2 (a.r holds the initial residual)
  double* const r0b = a.r;
  double* const r1b = a.z;
  double* const q0b = a.q;
  double* const q1b = a.p;
  int cur = 0;
  double beta = 0.0, al = 0.0;  // al: the step length still to be applied
  bool first = true;
  if (!a.fold) {
    // two grid barriers per iteration (p.q, then r.r) and one gathered vector:
    // the plan's choice when most gathered rows belong to other blocks, where
    // a second gathered vector costs more than the barrier it saves
    double rho = rr2;
    while (!done) {
      double ppq = 0.0;
#pragma unroll
      for (int u = 0; u < kMaxU; ++u) {
        const int l = threadIdx.x + u * kThreads;
        if (l < nr) {
          const double w = row_res(l, rr_[u], lrp, lcol, lval, dg, r0b);
          const double pn = first ? rr_[u] : rr_[u] + beta * pr[u];
          const double qn = first ? w : w + beta * qr[u];
          pr[u] = pn;
          qr[u] = qn;
          ppq += pn * qn;
        }
      }
      first = false;
      const double pq = grid_sum(c, ppq, sh);
      if (!(pq > 0.0)) {
        flag = 1;
        break;
      }
      const double a2 = rho / pq;
      double prr = 0.0;
#pragma unroll
      for (int u = 0; u < kMaxU; ++u) {
        const int l = threadIdx.x + u * kThreads;
        if (l < nr) {
          xr[u] += a2 * pr[u];
          const double ri = rr_[u] - a2 * qr[u];
          rr_[u] = ri;
          r0b[r0 + l] = ri;
          prr += ri * ri;
        }
      }
      const double rn = grid_sum(c, prr, sh);
      ++it;
      beta = rn / rho;
      rho = rn;
      rr2 = rn;
      if (rn <= tol2) break;
      if (it >= a.maxit) {
        flag = 2;
        break;
      }
    }
    done = true;  // al stays 0: x is complete
  }
  while (!done) {
    const double* rin = cur ? r1b : r0b;
    const double* qin = cur ? q1b : q0b;
    double* rout = cur ? r0b : r1b;
    double* qout = cur ? q0b : q1b;
    double spq = 0.0, srq = 0.0, sqq = 0.0, srr = 0.0;
#pragma unroll
    for (int u = 0; u < kMaxU; ++u) {
      const int l = threadIdx.x + u * kThreads;
      if (l < nr) {
        double ri, w;
        if (first) {
          ri = rr_[u];
          w = row_res(l, ri, lrp, lcol, lval, dg, rin);
        } else {
          xr[u] = __builtin_fma(al, pr[u], xr[u]);
          ri = __builtin_fma(-al, qr[u], rr_[u]);
          w = row_res_pend(l, ri, lrp, lcol, lval, dg, rin, qin, al);
        }
        const double pn = first ? ri : ri + beta * pr[u];
        const double qn = first ? w : w + beta * qr[u];
        rr_[u] = ri;
        pr[u] = pn;
        qr[u] = qn;
        rout[r0 + l] = ri;
        qout[r0 + l] = qn;
        spq += pn * qn;
        srq += ri * qn;
        sqq += qn * qn;
        srr += ri * ri;
      }
    }
    first = false;
    double sum[4];
    grid_sum4(c, spq, srq, sqq, srr, sh4, sum);
    cur ^= 1;
    const double pq = sum[0], rq = sum[1], qq = sum[2], rr = sum[3];
    al = 0.0;
    rr2 = rr;
    if (rr <= tol2) break;  // the update just applied met the tolerance
    if (!(pq > 0.0)) {
      flag = 1;
      break;
    }
    al = rr / pq;
    ++it;
    const double rn = rr - 2.0 * al * rq + al * al * qq;
    const double rp = rn > 0.0 ? rn : 0.0;
    rr2 = rp;
    if (rn >= 64.0 * 2.220446049250313e-16 * rr && rn <= tol2) break;
    if (it >= a.maxit) {
      flag = 2;
      break;
    }
    beta = rp / rr;
  }
  // the last step's update of x (r is not needed any more)
#pragma unroll
  for (int u = 0; u < kMaxU; ++u) {
    const int l = threadIdx.x + u * kThreads;
    if (l < nr) a.x[r0 + l] = __builtin_fma(al, pr[u], xr[u]);
  }
  if (bx == 0 && threadIdx.x == 0) {
    a.out[0] = it;
    a.out[1] = 0;
    a.out[2] = flag;
    a.res[0] = rr2;
    a.res[1] = bn2;
  }
}

// ---------------------------------------------------------------------------
// Resident flexible PCG (levels k >= 1): the block's rows of A^(k) and M^(k)
// both live in LDS, the row state (x, r, z, z_old, p, q and the inner
// ri, pi, qi) in registers; only z (gathered by A z) and the inner ri and
// qi (gathered by M ri, double-buffered) go through global memory.  Coarse
// rows hold tens of entries, so kLpr lanes share a row (strided over its
// entries, combined with xor shuffles); every lane of the group keeps the
// row's state, lane 0 of the group writes it out and contributes it to the
// dot products.  Same method as k_pcg1's flexible branch: Polak-Ribiere
// beta, inner CG on M from zero to tol_in ||r||, the inner CG with one grid
// barrier per iteration (below).
constexpr int kLpr = 8;
constexpr int kSlots = kThreads / kLpr;  // rows per pass
constexpr int kMaxU2 = 2;                // passes: rows per block <= 256

// (B x)_l for local row l (all lanes of the group call it; invalid rows give 0)
__device__ inline double row_lpr(bool ok, int l, int sub, const int* lrp, const int* lcol,
                                 const double* lval, const double* x) {
  double acc = 0.0;
  if (ok)
    for (int k = lrp[l] + sub; k < lrp[l + 1]; k += kLpr) acc += lval[k] * x[lcol[k]];
#pragma unroll
  for (int off = 1; off < kLpr; off <<= 1) acc += __shfl_xor(acc, off, kWave);
  return acc;
}

// (B x')_l with x'_j = x_j - al q_j (the same fused multiply-add as the row
// owner's update of x_j)
__device__ inline double row_lpr_pend(bool ok, int l, int sub, const int* lrp, const int* lcol,
                                      const double* lval, const double* x, const double* q,
                                      double al) {
  double acc = 0.0;
  if (ok)
    for (int k = lrp[l] + sub; k < lrp[l + 1]; k += kLpr) {
      const int j = lcol[k];
      acc += lval[k] * __builtin_fma(-al, q[j], x[j]);
    }
#pragma unroll
  for (int off = 1; off < kLpr; off <<= 1) acc += __shfl_xor(acc, off, kWave);
  return acc;
}

__device__ inline void body_pcg1_res(const Pcg1Args& a, const int* __restrict__ part,
                                     const int gblk, const int gnb, double* lds, double* sh,
                                     double* sh4) {
  const int bx = (gnb % 8) ? (int)gblk
                                 : (int)((gblk % 8) * (gnb / 8) + gblk / 8);
  Ctx c{a.bar, 0u, (int)gnb, (int)gblk, 0, 0, 0, 0, (int)(threadIdx.x & (kWave - 1)),
        a.red, 0};
  const CsrView& A = a.A;
  const CsrView& M = a.M;
  const int r0 = part[bx], r1 = part[bx + 1], nr = r1 - r0;
  const int ea = A.rowptr[r0], na = A.rowptr[r1] - ea;
  const int em = M.rowptr[r0], nm = M.rowptr[r1] - em;
  double* aval = lds;
  double* mval = aval + na;
  int* arp = reinterpret_cast<int*>(mval + nm);
  int* mrp = arp + nr + 1;
  int* acol = mrp + nr + 1;
  int* mcol = acol + na;
  for (int t = threadIdx.x; t < na; t += kThreads) {
    aval[t] = A.val[ea + t];
    acol[t] = A.col[ea + t];
  }
  for (int t = threadIdx.x; t < nm; t += kThreads) {
    mval[t] = M.val[em + t];
    mcol[t] = M.col[em + t];
  }
  for (int t = threadIdx.x; t <= nr; t += kThreads) {
    arp[t] = A.rowptr[r0 + t] - ea;
    mrp[t] = M.rowptr[r0 + t] - em;
  }
  __syncthreads();
  const int sub = threadIdx.x % kLpr, slot = threadIdx.x / kLpr;
  const bool lead = sub == 0;
  double* zg = a.z;    // gathered by A z
  // x stays in global memory (its owner updates it once per outer step),
  // the rest of the row state in registers
  double r[kMaxU2], z[kMaxU2], zo[kMaxU2], p[kMaxU2], q[kMaxU2];
  double ri[kMaxU2], pi[kMaxU2], qi[kMaxU2];
  bool ok[kMaxU2];
  int lrow[kMaxU2];
  double pb = 0.0, prr0 = 0.0;
#pragma unroll
  for (int u = 0; u < kMaxU2; ++u) {
    r[u] = z[u] = zo[u] = p[u] = q[u] = ri[u] = pi[u] = qi[u] = 0.0;
    lrow[u] = slot + u * kSlots;
    ok[u] = lrow[u] < nr;
    if (ok[u]) {
      const double bi = a.b[r0 + lrow[u]];
      if (lead) pb += bi * bi;
      if (!a.use_x0) {
        r[u] = bi;
        if (lead) a.x[r0 + lrow[u]] = 0.0;  // no block gathers x without x0
      }
    }
  }
  if (a.use_x0) {
#pragma unroll
    for (int u = 0; u < kMaxU2; ++u) {
      const double w = row_lpr(ok[u], lrow[u], sub, arp, acol, aval, a.x);
      if (ok[u]) {
        r[u] = a.b[r0 + lrow[u]] - w;
        if (lead) prr0 += r[u] * r[u];
      }
    }
  } else {
    prr0 = pb;
  }
  double bn2, rr2;
  grid_sum2(c, pb, prr0, sh, bn2, rr2);
  const double tol2 = a.tol * a.tol * bn2;
  const double tol_in2 = a.tol_in * a.tol_in;
  int it = 0, inner_total = 0, flag = 0;
  bool done = !(bn2 > 0.0) || rr2 <= tol2;
  // z = M^-1 r approximately (inner CG from zero); z ends in registers and zg
  // z = M^-1 r approximately (inner CG from zero); z ends in registers and zg.
  // One grid barrier per inner iteration, as in the level-0 resident CG: an
  // iteration applies the previous step to its own rows, gathers the
  // neighbours' new ri as ri_j - al qi_j from the previous iteration's copies
  // (ri and qi double-buffered), and ends in one grid sum of p.q, r.q, q.q
  // and r.r; the next r.r for beta and the stop test is expanded from them.
  double* const ri0 = a.ri;
  double* const ri1 = a.pi;
  double* const qi0 = a.qi;
  double* const qi1 = a.q;
  auto inner = [&](double rnorm2) {
#pragma unroll
    for (int u = 0; u < kMaxU2; ++u) {
      z[u] = 0.0;
      ri[u] = r[u];
      if (ok[u] && lead) ri0[r0 + lrow[u]] = ri[u];
    }
    grid_barrier(c);
    const double stop_in = tol_in2 * rnorm2;
    double bi = 0.0, al = 0.0;  // al: the step length still to be applied
    bool f = true;
    int k = 0, cur = 0;
    if (rnorm2 > stop_in && k < a.maxit_in) {
      while (true) {
        const double* rin = cur ? ri1 : ri0;
        const double* qin = cur ? qi1 : qi0;
        double* rout = cur ? ri0 : ri1;
        double* qout = cur ? qi0 : qi1;
        double spq = 0.0, srq = 0.0, sqq = 0.0, srr = 0.0;
#pragma unroll
        for (int u = 0; u < kMaxU2; ++u) {
          if (!f && ok[u]) {
            z[u] = __builtin_fma(al, pi[u], z[u]);
            ri[u] = __builtin_fma(-al, qi[u], ri[u]);
          }
          const double w = f ? row_lpr(ok[u], lrow[u], sub, mrp, mcol, mval, rin)
                             : row_lpr_pend(ok[u], lrow[u], sub, mrp, mcol, mval, rin, qin, al);
          if (ok[u]) {
            pi[u] = f ? ri[u] : ri[u] + bi * pi[u];
            qi[u] = f ? w : w + bi * qi[u];
            if (lead) {
              rout[r0 + lrow[u]] = ri[u];
              qout[r0 + lrow[u]] = qi[u];
              spq += pi[u] * qi[u];
              srq += ri[u] * qi[u];
              sqq += qi[u] * qi[u];
              srr += ri[u] * ri[u];
            }
          }
        }
        f = false;
        double sum[4];
        grid_sum4(c, spq, srq, sqq, srr, sh4, sum);
        cur ^= 1;
        const double pq = sum[0], rq = sum[1], qq = sum[2], rr = sum[3];
        al = 0.0;
        if (rr <= stop_in) break;
        if (!(pq > 0.0)) break;
        al = rr / pq;
        ++k;
        const double rn = rr - 2.0 * al * rq + al * al * qq;
        if (rn >= 64.0 * 2.220446049250313e-16 * rr && rn <= stop_in) break;
        if (k >= a.maxit_in) break;
        bi = (rn > 0.0 ? rn : 0.0) / rr;
      }
    }
#pragma unroll
    for (int u = 0; u < kMaxU2; ++u) {
      if (ok[u]) z[u] = __builtin_fma(al, pi[u], z[u]);  // the last step's update
      if (ok[u] && lead) zg[r0 + lrow[u]] = z[u];
    }
    inner_total += k;
  };
  if (!done) {
    inner(rr2);
    double prz = 0.0;
#pragma unroll
    for (int u = 0; u < kMaxU2; ++u)
      if (ok[u] && lead) prz += r[u] * z[u];
    double rz = grid_sum(c, prz, sh);
    double beta = 0.0;
    bool first = true;
    while (true) {
      double ppq = 0.0;
#pragma unroll
      for (int u = 0; u < kMaxU2; ++u) {
        const double w = row_lpr(ok[u], lrow[u], sub, arp, acol, aval, zg);
        if (ok[u]) {
          p[u] = first ? z[u] : z[u] + beta * p[u];
          q[u] = first ? w : w + beta * q[u];
          if (lead) ppq += p[u] * q[u];
        }
      }
      first = false;
      const double pq = grid_sum(c, ppq, sh);
      if (!(pq > 0.0)) {
        flag = 1;
        break;
      }
      const double al = rz / pq;
      double prr = 0.0;
#pragma unroll
      for (int u = 0; u < kMaxU2; ++u) {
        if (ok[u]) {
          if (lead) a.x[r0 + lrow[u]] += al * p[u];
          r[u] -= al * q[u];
          zo[u] = z[u];
          if (lead) prr += r[u] * r[u];
        }
      }
      const double rn = grid_sum(c, prr, sh);
      ++it;
      rr2 = rn;
      if (rn <= tol2) break;
      if (it >= a.maxit) {
        flag = 2;
        break;
      }
      inner(rn);
      double p1 = 0.0, p2 = 0.0;
#pragma unroll
      for (int u = 0; u < kMaxU2; ++u)
        if (ok[u] && lead) {
          p1 += r[u] * z[u];
          p2 += r[u] * zo[u];
        }
      double rzn, rzo;
      grid_sum2(c, p1, p2, sh, rzn, rzo);
      beta = (rzn - rzo) / rz;
      rz = rzn;
    }
  }
  if (bx == 0 && threadIdx.x == 0) {
    a.out[0] = it;
    a.out[1] = inner_total;
    a.out[2] = flag;
    a.res[0] = rr2;
    a.res[1] = bn2;
  }
}

// Static LDS of the bodies, declared once per kernel and handed down, so a
// batched launch that may run any body holds one copy: the block-sum slots
// (sh) and the four-way sum slots plus their results (sh4).
constexpr int kSh = kThreads / kWave;
constexpr int kSh4 = 4 * kThreads / kWave + 4;

__global__ __launch_bounds__(kThreads) void k_pcg1(Pcg1Args a) {
  __shared__ double sh[kSh];
  body_pcg1(a, (int)blockIdx.x, (int)gridDim.x, sh);
}

__global__ __launch_bounds__(kThreads) void k_cg1_res(Pcg1Args a, const int* __restrict__ part) {
  extern __shared__ double lds[];
  __shared__ double sh[kSh];
  __shared__ double sh4[kSh4];
  body_cg1_res(a, part, (int)blockIdx.x, (int)gridDim.x, lds, sh, sh4);
}

__global__ __launch_bounds__(kThreads) void k_pcg1_res(Pcg1Args a, const int* __restrict__ part) {
  extern __shared__ double lds[];
  __shared__ double sh[kSh];
  __shared__ double sh4[kSh4];
  body_pcg1_res(a, part, (int)blockIdx.x, (int)gridDim.x, lds, sh, sh4);
}

// Several independent single-vector solves in one cooperative launch: request
// r owns the blocks [off_r, off_r + nblk_r) and runs the body its plan selects
// on them, with its own arrival counter and reduction slots, so the requests
// never wait for each other.  Offsets are multiples of 8, so local block j of
// a request sits on XCD j % 8 as in a launch of its own.
__global__ __launch_bounds__(kThreads) void k_pcg1_multi(const Pcg1Req* __restrict__ reqs,
                                                         int nreq) {
  extern __shared__ double lds[];
  __shared__ double sh[kSh];
  __shared__ double sh4[kSh4];
  int r = 0;
  while (r + 1 < nreq && (int)blockIdx.x >= reqs[r + 1].off) ++r;
  const Pcg1Req& q = reqs[r];
  const int gblk = (int)blockIdx.x - q.off;
  if (gblk >= q.nblk) return;  // padding to a whole XCD round: not part of the solve
  if (q.kind == 0)
    body_cg1_res(q.a, q.part, gblk, q.nblk, lds, sh, sh4);
  else if (q.kind == 1)
    body_pcg1_res(q.a, q.part, gblk, q.nblk, lds, sh, sh4);
  else
    body_pcg1(q.a, gblk, q.nblk, sh);
}

int lanes_for(double avg) {
  if (avg <= 10.0) return 8;
  if (avg <= 24.0) return 16;
  if (avg <= 48.0) return 32;
  return 64;
}

}  // namespace

int pcg1_grid() {
  // computed once per process (thread-safe initialisation)
  static const int cached = [] {
    int dev = 0;
    MMD_HIP(hipGetDevice(&dev));
    int coop = 0;
    MMD_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    MMD_REQUIRE(coop != 0, MMD_EHIP, "device does not support cooperative launches");
    int cus = 0;
    MMD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per = 0;
    MMD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pcg1, kThreads, 0));
    MMD_REQUIRE(per > 0, MMD_EHIP, "persistent PCG kernel cannot be resident");
    return cus * per;  // upper bound for co-residency
  }();
  return cached;
}

Pcg1Req pcg1_request(Pcg1Args a, const Pcg1Plan* plan) {
  Pcg1Req q;
  if (plan && plan->resident && (a.M.rowptr != nullptr) == plan->flex) {
    q.kind = plan->flex ? 1 : 0;
    a.fold = plan->fold ? 1 : 0;
    q.part = plan->part.p;
    q.nblk = plan->grid;
    q.lds = plan->lds;
  } else {
    const int64_t work = a.A.nnz + (a.M.rowptr ? a.M.nnz : 0);
    int grid = static_cast<int>(std::min<int64_t>(128, std::max<int64_t>(16, work / 16384)));
    grid = std::min(grid, pcg1_grid());
    grid = std::min(grid, std::max(1, (a.n + kThreads - 1) / kThreads * 4));
    grid = std::max(8, grid / 8 * 8);
    a.lpr_a = lanes_for(a.A.avg_row);
    a.lpr_m = a.M.rowptr ? lanes_for(a.M.avg_row) : 8;
    q.kind = 2;
    q.nblk = grid;
    q.lds = 0;
  }
  q.a = a;
  return q;
}

int pcg1_multi_capacity(size_t lds) {
  int dev = 0;
  MMD_HIP(hipGetDevice(&dev));
  int cus = 0;
  MMD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  MMD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_pcg1_multi),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  int per = 0;
  MMD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pcg1_multi, kThreads, lds));
  return per * cus;
}

void pcg1_multi(std::vector<Pcg1Req>& reqs, Pcg1Req* h_reqs, Pcg1Req* d_reqs, hipStream_t s) {
  if (reqs.empty()) return;
  int off = 0;
  size_t lds = 0;
  for (auto& q : reqs) {
    q.off = off;
    off += (q.nblk + 7) / 8 * 8;  // whole XCD rounds per request
    lds = std::max(lds, q.lds);
  }
  for (size_t i = 0; i < reqs.size(); ++i) h_reqs[i] = reqs[i];
  MMD_HIP(hipMemcpyAsync(d_reqs, h_reqs, sizeof(Pcg1Req) * reqs.size(), hipMemcpyHostToDevice, s));
  for (auto& q : reqs) MMD_HIP(hipMemsetAsync(q.a.bar, 0, sizeof(unsigned), s));
  int nreq = static_cast<int>(reqs.size());
  void* args[] = {&d_reqs, &nreq};
  MMD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_pcg1_multi),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  MMD_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_pcg1_multi), dim3(off),
                                     dim3(kThreads), args, static_cast<unsigned>(lds), s));
}

void pcg1(Pcg1Args a, hipStream_t s, const Pcg1Plan* plan) {
  MMD_HIP(hipMemsetAsync(a.bar, 0, sizeof(unsigned), s));
  void* args[] = {&a};
  if (plan && plan->resident && (a.M.rowptr != nullptr) == plan->flex) {
    const int* part = plan->part.p;
    a.fold = plan->fold ? 1 : 0;
    void* rargs[] = {&a, &part};
    const void* fn = plan->flex ? reinterpret_cast<const void*>(k_pcg1_res)
                                : reinterpret_cast<const void*>(k_cg1_res);
    MMD_HIP(hipLaunchCooperativeKernel(fn, dim3(plan->grid), dim3(kThreads), rargs,
                                       static_cast<unsigned>(plan->lds), s));
    return;
  }
  // blocks: barrier cost (~30 ns per block) against memory-level parallelism
  const int64_t work = a.A.nnz + (a.M.rowptr ? a.M.nnz : 0);
  int grid = static_cast<int>(std::min<int64_t>(128, std::max<int64_t>(16, work / 16384)));
  if (const char* e = std::getenv("MMDEIG_COOP_BLOCKS")) grid = std::max(1, std::atoi(e));
  grid = std::min(grid, pcg1_grid());
  grid = std::min(grid, std::max(1, (a.n + kThreads - 1) / kThreads * 4));
  if (grid >= 8) grid = grid / 8 * 8;  // whole XCD rounds
  a.lpr_a = lanes_for(a.A.avg_row);
  a.lpr_m = a.M.rowptr ? lanes_for(a.M.avg_row) : 8;
  MMD_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_pcg1), dim3(grid),
                                     dim3(kThreads), args, 0, s));
}

void pcg1_plan(const CsrView& A, const std::vector<int>& rp, Pcg1Plan& plan, hipStream_t s,
               int grid_cap) {
  plan.resident = false;
  const int n = A.n_rows;
  if (n == 0 || (int)rp.size() != n + 1) return;
  if (const char* e = std::getenv("MMDEIG_NO_RESIDENT"))
    if (std::atoi(e) != 0) return;
  // 14 blocks per XCD measured best for the n = 1e5 RGG (barrier cost grows
  // with the block count, the per-thread row count with fewer blocks); a
  // matrix whose slices do not fit that many blocks' LDS takes the fewest
  // blocks (multiple of 8) that hold it, up to what can be co-resident
  int grid0 = grid_cap;
  if (const char* e = std::getenv("MMDEIG_RES_BLOCKS")) grid0 = std::max(8, std::atoi(e));
  grid0 = std::max(8, grid0 / 8 * 8);
  grid0 = std::min(grid0, std::max(8, (n + 63) / 64 / 8 * 8));
  int dev = 0;
  MMD_HIP(hipGetDevice(&dev));
  int maxsh = 0, cus = 0;
  MMD_HIP(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  MMD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // room for the static LDS of every kernel that may run the plan (the
  // batched kernel holds the reduction arrays of all three bodies)
  const size_t static_lds = 1024;
  const bool edge = A.diag != nullptr;
  const double tot = static_cast<double>(rp[n]) + n;
  std::vector<int> part;
  size_t lds = 0;
  int grid = grid0;
  for (;; grid += 8) {
    if (grid > cus) return;  // one 1024-thread block per CU at these LDS sizes
    // balance nonzeros + rows: block j starts at the first row whose prefix
    // weight reaches j / grid of the total
    part.assign(grid + 1, n);
    part[0] = 0;
    int i = 0;
    for (int j = 1; j < grid; ++j) {
      const double target = tot * j / grid;
      while (i < n && static_cast<double>(rp[i]) + i < target) ++i;
      part[j] = i;
    }
    lds = 0;
    int max_rows = 0;
    for (int j = 0; j < grid; ++j) {
      const int nr = part[j + 1] - part[j];
      const size_t ne = static_cast<size_t>(rp[part[j + 1]] - rp[part[j]]);
      const size_t b = ne * 12 + (edge ? 8 * (size_t)nr : 0) + 4 * (size_t)(nr + 1);
      lds = std::max(lds, b);
      max_rows = std::max(max_rows, nr);
    }
    if (max_rows <= kMaxU * kThreads &&
        (lds + 255) / 256 * 256 + static_lds <= static_cast<size_t>(maxsh))
      break;
  }
  lds = (lds + 255) / 256 * 256;
  MMD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg1_res),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  int per = 0;
  MMD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg1_res, kThreads, lds));
  if (per <= 0 || grid > per * cus) return;
  // gather locality: the share of entries whose column lies in the row's own
  // block picks the one-barrier form (at least half) or the two-barrier form
  // (MMDEIG_CG1_FOLD=0/1 forces one)
  {
    std::vector<int> col(static_cast<size_t>(rp[n]));
    if (!col.empty()) {
      MMD_HIP(hipMemcpyAsync(col.data(), A.col, sizeof(int) * col.size(), hipMemcpyDeviceToHost,
                             s));
      MMD_HIP(hipStreamSynchronize(s));
    }
    int64_t local = 0;
    for (int j = 0; j < grid; ++j)
      for (int k = rp[part[j]]; k < rp[part[j + 1]]; ++k)
        local += (col[k] >= part[j] && col[k] < part[j + 1]) ? 1 : 0;
    plan.fold = col.empty() || 2 * local >= static_cast<int64_t>(col.size());
    if (const char* e = std::getenv("MMDEIG_CG1_FOLD"))
      if (e[0]) plan.fold = std::atoi(e) != 0;
    if (const char* e = std::getenv("MMDEIG_LOG"))
      if (std::atoi(e) != 0)
        std::fprintf(stderr, "[mmdeig] resident CG plan: n %d, %d blocks, block-local entries %.3f, %s\n",
                     n, grid, col.empty() ? 1.0 : static_cast<double>(local) / col.size(),
                     plan.fold ? "one barrier per iteration" : "two barriers per iteration");
  }
  plan.part.ensure(grid + 1);
  MMD_HIP(hipMemcpyAsync(plan.part.p, part.data(), sizeof(int) * (grid + 1),
                         hipMemcpyHostToDevice, s));
  MMD_HIP(hipStreamSynchronize(s));  // part (host) must outlive the copy
  plan.grid = grid;
  plan.lds = lds;
  plan.resident = true;
}

void pcg1_plan_flex(const CsrView& A, const std::vector<int>& rpa, const CsrView& M,
                    const std::vector<int>& rpm, Pcg1Plan& plan, hipStream_t s) {
  plan.resident = false;
  plan.flex = true;
  const int n = A.n_rows;
  if (n == 0 || (int)rpa.size() != n + 1 || (int)rpm.size() != n + 1 || M.n_rows != n) return;
  if (const char* e = std::getenv("MMDEIG_NO_RESIDENT"))
    if (std::atoi(e) != 0) return;
  int dev = 0;
  MMD_HIP(hipGetDevice(&dev));
  int maxsh = 0, cus = 0;
  MMD_HIP(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  MMD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t avail = static_cast<size_t>(maxsh) - 1024 - 256;
  const double tot_bytes = 12.0 * (rpa[n] + rpm[n]) + 8.0 * n;
  const int max_rows = kMaxU2 * kSlots;
  int grid = std::max(16, (n + max_rows - 1) / max_rows);
  grid = std::max(grid, static_cast<int>(std::ceil(tot_bytes / (0.95 * avail))));
  grid = (grid + 7) / 8 * 8;
  // balance entries of A and M plus rows
  const double tot = static_cast<double>(rpa[n]) + rpm[n] + n;
  std::vector<int> part;
  size_t lds = 0;
  for (; grid <= 4 * cus; grid += 8) {
    part.assign(grid + 1, n);
    part[0] = 0;
    int i = 0;
    for (int j = 1; j < grid; ++j) {
      const double target = tot * j / grid;
      while (i < n && static_cast<double>(rpa[i]) + rpm[i] + i < target) ++i;
      part[j] = i;
    }
    lds = 0;
    int mr = 0;
    for (int j = 0; j < grid; ++j) {
      const int nr = part[j + 1] - part[j];
      const size_t ne = static_cast<size_t>(rpa[part[j + 1]] - rpa[part[j]]) +
                        static_cast<size_t>(rpm[part[j + 1]] - rpm[part[j]]);
      lds = std::max(lds, ne * 12 + 8 * static_cast<size_t>(nr + 1));
      mr = std::max(mr, nr);
    }
    if (lds <= avail && mr <= max_rows) break;
  }
  if (grid > 4 * cus) return;
  lds = (lds + 255) / 256 * 256;
  MMD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_pcg1_res),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  int per = 0;
  MMD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pcg1_res, kThreads, lds));
  if (per <= 0 || grid > per * cus) return;
  plan.part.ensure(grid + 1);
  MMD_HIP(hipMemcpyAsync(plan.part.p, part.data(), sizeof(int) * (grid + 1),
                         hipMemcpyHostToDevice, s));
  MMD_HIP(hipStreamSynchronize(s));  // part (host) must outlive the copy
  plan.grid = grid;
  plan.lds = lds;
  plan.resident = true;
}

size_t pcg1_red_size() { return 8 * (size_t)1024; }

}  // namespace mmd
