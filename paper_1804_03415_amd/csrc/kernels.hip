// Device kernels of the hierarchical eigensolver for CDNA4 (gfx950, wave64).
//
// Hot path (Section 4, operator OP, and Alg. 5): CSR SpMM with A^(k), M^(k)
// and Psi, the patch Householder transforms that realise U and U^T, the
// vector updates and column dot products of CG / flexible PCG, and the
// tall-skinny FP64 products of the Lanczos re-orthogonalisation and the
// Rayleigh-Ritz steps.  Blocks of vectors are row-major (N x b, leading
// dimension ld) so one gathered row of X serves all b right-hand sides with
// one coalesced load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.h"
#include "kernels.h"

namespace mmd {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

inline void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(MMD_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// ------------------------------------------------------------------ SpMM
// One wavefront handles R = 64 / (LPR * CT) rows and a tile of CT columns;
// lane = (r, s, c): c = lane % CT, s = (lane / CT) % LPR, r = lane / (CT*LPR).
// The LPR lanes of a (row, column) pair stride over the row's nonzeros and are
// combined with xor shuffles.  A block walks several row groups so it can keep
// per-column partial dot products for the fused CG epilogue.
template <int LPR, int CT, bool EDGE, bool FUSE, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm(
    int n_rows, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ diag,
    const double* __restrict__ X, int ldx, double* __restrict__ Y, int ldy, int b,
    int first, const double* __restrict__ beta, double* __restrict__ P, int ldp,
    double* __restrict__ partial, const double* __restrict__ dotw, int lddot) {
  constexpr int R = kWave / (LPR * CT);
  constexpr int WPB = kBlock / kWave;
  __shared__ double red[WPB * R * CT];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int c = lane % CT;
  const int s = (lane / CT) % LPR;
  const int r = lane / (CT * LPR);
  const int c0 = blockIdx.y * CT;
  const int colx = c0 + c;
  const bool cok = colx < b;
  const double bt = (FUSE && cok && !first) ? beta[colx] : 0.0;
  double dsum = 0.0;
  const int groups = (n_rows + R - 1) / R;
  // each XCD (workgroups are dealt to the 8 XCDs round-robin) sweeps its own
  // contiguous eighth of the row groups, its resident blocks moving through it
  // as one band
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int xcd = blockIdx.x % nx, bl = blockIdx.x / nx;
  const int gpx = (groups + nx - 1) / nx;
  const int g_hi = min(groups, (xcd + 1) * gpx);
  for (int g = xcd * gpx + bl * WPB + wid; g < g_hi; g += bpx * WPB) {
    const int row = g * R + r;
    double acc = 0.0;
    double xi = 0.0;
    if (row < n_rows && cok) {
      const int lo = rowptr[row], hi = rowptr[row + 1];
      if (EDGE) xi = X[(size_t)row * ldx + colx];
      int k = lo + s;
      // four gathers in flight per lane
      for (; k + 3 * LPR < hi; k += 4 * LPR) {
        const int j0 = col[k], j1 = col[k + LPR], j2 = col[k + 2 * LPR], j3 = col[k + 3 * LPR];
        const double v0 = val[k], v1 = val[k + LPR], v2 = val[k + 2 * LPR], v3 = val[k + 3 * LPR];
        const double x0 = X[(size_t)j0 * ldx + colx], x1 = X[(size_t)j1 * ldx + colx];
        const double x2 = X[(size_t)j2 * ldx + colx], x3 = X[(size_t)j3 * ldx + colx];
        if (EDGE)
          acc += v0 * (xi - x0) + v1 * (xi - x1) + v2 * (xi - x2) + v3 * (xi - x3);
        else
          acc += v0 * x0 + v1 * x1 + v2 * x2 + v3 * x3;
      }
      for (; k < hi; k += LPR) {
        const double xj = X[(size_t)col[k] * ldx + colx];
        if (EDGE)
          acc += val[k] * (xi - xj);
        else
          acc += val[k] * xj;
      }
    }
#pragma unroll
    for (int off = CT; off < CT * LPR; off <<= 1) acc += __shfl_xor(acc, off, kWave);
    if (s == 0 && row < n_rows && cok) {
      double y = EDGE ? diag[row] * xi + acc : acc;
      if (FUSE) {  // partial == nullptr: direction update only, p.q taken separately
        const size_t iy = (size_t)row * ldy + colx;
        const size_t ip = (size_t)row * ldp + colx;
        double pn;
        if (first) {
          pn = X[(size_t)row * ldx + colx];
        } else {
          y += bt * Y[iy];
          pn = X[(size_t)row * ldx + colx] + bt * P[ip];
        }
        P[ip] = pn;
        dsum += pn * y;
      } else if (DOT) {
        dsum += dotw[(size_t)row * lddot + colx] * y;
      }
      Y[(size_t)row * ldy + colx] = y;
    }
  }
  if ((FUSE && partial != nullptr) || DOT) {
    // lanes with s == 0 hold (r, c) partial sums; combine over r and waves
    if (s == 0) red[(wid * R + r) * CT + c] = dsum;
    __syncthreads();
    if (threadIdx.x < CT) {
      double t = 0.0;
      for (int q = 0; q < WPB * R; ++q) t += red[q * CT + threadIdx.x];
      const int cc = c0 + threadIdx.x;
      if (cc < b) partial[(size_t)blockIdx.x * b + cc] = t;
    }
  }
}

// Blocks of more than 32 columns: one wavefront per (row, 64-column tile),
// U rows per wavefront in flight (one at the launch used).  The lanes first
// load up to 64 of the row's column indices and weights with one vector load,
// then broadcast them with readlane, so the gathers of the row are issued in
// steps of STEP without waiting on an index load each.  Slots past the end of a row's nonzeros gather
// row 0 with weight 0.  Each XCD (workgroups are dealt round-robin to the
// 8 XCDs) sweeps its own contiguous eighth of the rows.  Fused CG epilogue as
// in k_spmm.
constexpr int kStep = 8;

__device__ inline double readlane_d(double v, int k) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u), k));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), k));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// eight wavefronts per SIMD (at most 64 VGPRs): the kernel is bound by the
// latency of its dependent load rounds, so resident waves count more than
// rows in flight per wave
template <bool EDGE, bool FUSE, int U, int STEP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_spmm_r64(
    int n_rows, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ diag,
    const double* __restrict__ X, int ldx, double* __restrict__ Y, int ldy, int b, int first,
    const double* __restrict__ beta, double* __restrict__ P, int ldp,
    double* __restrict__ partial) {
  constexpr int WPB = kBlock / kWave;
  __shared__ double red[WPB * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cc = blockIdx.y * kWave + lane;
  const bool cok = cc < b;
  const int cx = cok ? cc : 0;  // lanes past b read column 0 and store nothing
  const double bt = (FUSE && cok && !first) ? beta[cc] : 0.0;
  double dsum = 0.0;
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int xcd = blockIdx.x % nx, bl = blockIdx.x / nx;
  const int rpx = (n_rows + nx - 1) / nx;
  const int rhi = min(n_rows, (xcd + 1) * rpx);
  const int stride = bpx * WPB;
  // a wavefront takes U rows one band stride apart
  const int first0 = xcd * rpx + bl * WPB + wid;
  const int rstep = U * stride;
  // software pipeline: the row pointers of the next row group are loaded while
  // the current group gathers, and every load of a group that does not depend
  // on its gathers (own X row, old Y and P, the first index chunk) is issued
  // before the gathers, so a group costs about three memory latencies
  int lo_n[U], hi_n[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = first0 + u * stride;
    lo_n[u] = r < rhi ? rowptr[r] : 0;
    hi_n[u] = r < rhi ? rowptr[r + 1] : 0;
  }
  for (int row0 = first0; row0 < rhi; row0 += rstep) {
    int row[U], lo[U], hi[U];
    bool ok[U];
    double xi[U], acc[U], yo[U], po[U], dg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      row[u] = row0 + u * stride;
      ok[u] = row[u] < rhi;
      lo[u] = lo_n[u];
      hi[u] = hi_n[u];
      // own-row reads only for square forms (edge form, fused CG): X has
      // n_cols rows, which may be fewer than n_rows otherwise
      const size_t rx = (size_t)(ok[u] ? row[u] : 0);
      xi[u] = (EDGE || FUSE) ? X[rx * ldx + cx] : 0.0;
      dg[u] = EDGE ? diag[rx] : 0.0;
      // P and Y stream through once: non-temporal, so they do not evict the
      // gathered rows of X from L2
      yo[u] = (FUSE && !first) ? __builtin_nontemporal_load(Y + rx * ldy + cx) : 0.0;
      po[u] = (FUSE && !first) ? __builtin_nontemporal_load(P + rx * ldp + cx) : 0.0;
      acc[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = row[u] + rstep;
      lo_n[u] = r < rhi ? rowptr[r] : 0;
      hi_n[u] = r < rhi ? rowptr[r + 1] : 0;
    }
    for (int base = 0;; base += kWave) {
      int m = 0;
      int jv[U];
      double vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int nu = max(0, min(kWave, hi[u] - lo[u] - base));
        m = max(m, nu);
        jv[u] = lane < nu ? col[lo[u] + base + lane] : 0;
        vv[u] = lane < nu ? val[lo[u] + base + lane] : 0.0;
      }
      if (m == 0) break;
      // steps of STEP slots with a fixed trip count, so all U * STEP gathers
      // of a step are in flight together (padding slots carry weight 0)
      for (int k0 = 0; k0 < m; k0 += STEP) {
        double xs[U][STEP], ws[U][STEP];
#pragma unroll
        for (int q = 0; q < STEP; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int j = __builtin_amdgcn_readlane(jv[u], k0 + q);
            ws[u][q] = readlane_d(vv[u], k0 + q);
            xs[u][q] = X[(size_t)j * ldx + cx];
          }
#pragma unroll
        for (int q = 0; q < STEP; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u)
            acc[u] += EDGE ? ws[u][q] * (xi[u] - xs[u][q]) : ws[u][q] * xs[u][q];
      }
      if (m < kWave) break;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u] && cok) {
        double y = EDGE ? dg[u] * xi[u] + acc[u] : acc[u];
        const size_t iy = (size_t)row[u] * ldy + cc;
        if (FUSE) {
          const size_t ip = (size_t)row[u] * ldp + cc;
          double pn;
          if (first) {
            pn = xi[u];
          } else {
            y += bt * yo[u];
            pn = xi[u] + bt * po[u];
          }
          __builtin_nontemporal_store(pn, P + ip);
          dsum += pn * y;
        }
        __builtin_nontemporal_store(y, Y + iy);
      }
    }
  }
  if (FUSE && partial != nullptr) {
    red[wid * kWave + lane] = dsum;
    __syncthreads();
    if (threadIdx.x < kWave) {
      double t = 0.0;
      for (int w = 0; w < WPB; ++w) t += red[w * kWave + threadIdx.x];
      const int c = blockIdx.y * kWave + threadIdx.x;
      if (c < b) partial[(size_t)blockIdx.x * b + c] = t;
    }
  }
}

// LDS-staged block SpMM on the tiled level-0 edge form (CsrView::t_uptr):
// a workgroup takes a tile of up to shape.rows consecutive rows whose entries
// touch at most shape.cols rows, and one 64-column slice, copies the X rows
// its entries touch (own rows first, then the halo) into LDS with one
// coalesced 512-byte load per row, together with the tile's weights, local
// column positions and row pointers, and then forms every row from LDS.
// 40 KB of LDS and at most 128 VGPRs per workgroup: four workgroups (16
// wavefronts) per CU.  Caps measured on the n = 1e5 RGG: 128 staged rows
// (two workgroups per CU) 337 us per launch, 80 rows (three) 296 us, 64 rows
// (four) 282 us, 48 rows with 16-row tiles (five) 285 us.  Each gathered row of X leaves L2 once per tile
// instead of once per entry (about 2.3 reads per row against 11 for the
// RGG in Morton order).  Tiles are dealt to the 8 XCDs in contiguous ranges,
// so neighbouring tiles that share halo rows run on the same L2.  Fused CG
// epilogue as in k_spmm_r64.
template <bool FUSE, int KIND>
__global__ __launch_bounds__(kBlock, kTileShapes[KIND].wgs_per_cu) void k_spmm_tile(
    int n_rows, const int* __restrict__ rowptr, const double* __restrict__ val,
    const double* __restrict__ diag, const int* __restrict__ trow,
    const int* __restrict__ uptr, const int* __restrict__ urow,
    const unsigned short* __restrict__ lcol, int nblk,
    const double* __restrict__ X, int ldx, double* __restrict__ Y, int ldy, int b, int first,
    const double* __restrict__ beta, double* __restrict__ P, int ldp,
    double* __restrict__ partial) {
  constexpr int WPB = kBlock / kWave;
  constexpr int kTileRows = kTileShapes[KIND].rows;
  constexpr int kTileCols = kTileShapes[KIND].cols;
  constexpr int kTileNnz = kTileShapes[KIND].nnz;
  constexpr int RPW = kTileRows / WPB;  // rows per wavefront and tile
  __shared__ double sx[kTileCols * kWave];  // also the partial-sum buffer at the end
  __shared__ double sv[kTileNnz];
  __shared__ unsigned short sc[kTileNnz];
  __shared__ int sp[kTileRows + 1];
  double* red = sx;
  static_assert(kTileCols >= WPB, "the reduction reuses the staging buffer");
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cc = blockIdx.y * kWave + lane;
  const bool cok = cc < b;
  const int cx = cok ? cc : 0;  // lanes past b read column 0 and store nothing
  const double bt = (FUSE && cok && !first) ? beta[cc] : 0.0;
  double dsum = 0.0;
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int xcd = blockIdx.x % nx, bl = blockIdx.x / nx;
  const int tpx = (nblk + nx - 1) / nx;
  const int thi = min(nblk, (xcd + 1) * tpx);
  for (int t = xcd * tpx + bl; t < thi; t += bpx) {
    const int r0 = trow[t];
    const int r1 = trow[t + 1];
    const int u0 = uptr[t], nu = uptr[t + 1] - u0;
    const int e0 = rowptr[r0], ne = rowptr[r1] - e0;
    // own-row streams of this wavefront's rows first: they do not wait for
    // the staging
    double yo[RPW], po[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int i = r0 + wid + k * WPB;
      const bool ok = FUSE && !first && i < r1;
      const size_t ri = (size_t)(ok ? i : 0);
      yo[k] = ok ? __builtin_nontemporal_load(Y + ri * ldy + cx) : 0.0;
      po[k] = ok ? __builtin_nontemporal_load(P + ri * ldp + cx) : 0.0;
    }
    // staging of the tile: every global load of the tile is issued before
    // the first LDS store, so the tile waits for one memory round trip.
    // The entries (weights, local positions) come first, then the X rows:
    // lane j of wavefront w holds the row of slot w + 4 j, broadcast with
    // readlane, and all of the wavefront's slots are loaded in one batch.
    {
      constexpr int EPT = kTileNnz / kBlock;  // entries per thread
      double ev[EPT];
      unsigned short ec[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = threadIdx.x + q * kBlock;
        ev[q] = e < ne ? val[e0 + e] : 0.0;
        ec[q] = e < ne ? lcol[e0 + e] : 0;
      }
      const int rp = threadIdx.x <= r1 - r0 ? rowptr[r0 + threadIdx.x] - e0 : 0;
      constexpr int SPW = kTileCols / WPB;  // slots per wavefront
      const int myu = wid + WPB * lane;
      const int ridx = (lane < SPW && myu < nu) ? urow[u0 + myu] : -1;
      double v[SPW];
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        const int j = __builtin_amdgcn_readlane(ridx, q);
        v[q] = j >= 0 ? X[(size_t)j * ldx + cx] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = threadIdx.x + q * kBlock;
        if (e < ne) {
          sv[e] = ev[q];
          sc[e] = ec[q];
        }
      }
      if (threadIdx.x <= r1 - r0) sp[threadIdx.x] = rp;
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        const int u = wid + WPB * q;
        if (u < nu) sx[u * kWave + lane] = v[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int i = r0 + wid + k * WPB;
      if (i < r1) {
        const int l = i - r0;
        const double xi = sx[l * kWave + lane];
        const int lo = sp[l], hi = sp[l + 1];
        double a0 = 0.0;
        // lane j holds entry lo + base + j of the row (position and weight),
        // broadcast with readlane, so the row's LDS gathers issue together
        for (int base = 0; base < hi - lo; base += kWave) {
          const int m = min(kWave, hi - lo - base);
          const int jv = lane < m ? static_cast<int>(sc[lo + base + lane]) : 0;
          const double wv = lane < m ? sv[lo + base + lane] : 0.0;
          for (int k0 = 0; k0 < m; k0 += 8) {
            double xs[8], ws[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int j = __builtin_amdgcn_readlane(jv, k0 + q);
              ws[q] = readlane_d(wv, k0 + q);
              xs[q] = sx[j * kWave + lane];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) a0 += ws[q] * (xi - xs[q]);
          }
        }
        double y = diag[i] * xi + a0;
        if (cok) {
          if (FUSE) {
            double pn;
            if (first) {
              pn = xi;
            } else {
              y += bt * yo[k];
              pn = xi + bt * po[k];
            }
            __builtin_nontemporal_store(pn, P + (size_t)i * ldp + cc);
            dsum += pn * y;
          }
          __builtin_nontemporal_store(y, Y + (size_t)i * ldy + cc);
        }
      }
    }
    __syncthreads();  // the next tile overwrites the staging
  }
  if (FUSE && partial != nullptr) {
    red[wid * kWave + lane] = dsum;
    __syncthreads();
    if (threadIdx.x < kWave) {
      double s = 0.0;
      for (int w = 0; w < WPB; ++w) s += red[w * kWave + threadIdx.x];
      const int c = blockIdx.y * kWave + threadIdx.x;
      if (c < b) partial[(size_t)blockIdx.x * b + c] = s;
    }
  }
}

template <int KIND>
void launch_tile_kind(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b,
                      hipStream_t s, bool fuse, bool first, const double* beta, double* P,
                      int ldp, double* partial, dim3 grid) {
  if (fuse)
    hipLaunchKernelGGL((k_spmm_tile<true, KIND>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr,
                       A.val, A.diag, A.t_row, A.t_uptr, A.t_urow, A.t_lcol, A.t_nblk, X, ldx, Y,
                       ldy, b, first ? 1 : 0, beta, P, ldp, partial);
  else
    hipLaunchKernelGGL((k_spmm_tile<false, KIND>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr,
                       A.val, A.diag, A.t_row, A.t_uptr, A.t_urow, A.t_lcol, A.t_nblk, X, ldx, Y,
                       ldy, b, first ? 1 : 0, beta, P, ldp, partial);
}

int launch_spmm_tile(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b,
                     hipStream_t s, bool fuse, bool first, const double* beta, double* P,
                     int ldp, double* partial) {
  int gx = A.t_nblk;
  if (fuse && partial) gx = std::min(gx, kRedBlocks);
  if (gx >= 8) gx = gx / 8 * 8;  // whole XCD rounds
  dim3 grid(gx, ceil_div(b, kWave));
  switch (A.t_kind) {
    case 0: launch_tile_kind<0>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, grid); break;
    case 1: launch_tile_kind<1>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, grid); break;
    default: launch_tile_kind<2>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, grid); break;
  }
  check_launch();
  return gx;
}

// One block-CG step on the tiled level-0 edge form with the previous step's
// iterate and residual update folded in.  With a pending step length
// a = alpha[c] (PEND), every own row does
//   x += a p ;  r -= a q ;  p = r + beta p ;  q = A r + beta q
// and the gathered rows of r are formed as r - a q while they are staged, so
// the update needs no pass over the block of its own (one pass fewer over R,
// P and Q per step than the fused SpMM followed by k_cg_update).  Own rows of
// Q come from the row loads that the q update needs anyway; only the halo
// rows load Q a second time.  Other workgroups stage these rows of R and Q
// as halo while this one updates them, so a pending step reads Ri, Qi and
// writes the new r, q to Ro, Qo (separate buffers, swapped by the caller
// every step); P and X are read and written only by the row's owner.  A
// step without PEND writes no r and may take Qo == Qi: the halo entries of
// Qi it loads are never used.  Four partial sums per block and column, of the
// new vectors: p.q, r.q, q.q and r.r (k_cg_defer_scalars turns them into
// alpha and, through |r - alpha q|^2 = r.r - 2 alpha r.q + alpha^2 q.q, the
// next beta).  Without PEND (first step, or the step after a flush) r is
// staged as stored and x, r are neither read nor written.  Tiling, staging
// order and XCD mapping as in k_spmm_tile.
template <bool PEND, int KIND>
__global__ __launch_bounds__(kBlock, kTileShapes[KIND].wgs_per_cu) void k_cg_tile(
    const int* __restrict__ rowptr, const double* __restrict__ val,
    const double* __restrict__ diag, const int* __restrict__ trow,
    const int* __restrict__ uptr, const int* __restrict__ urow,
    const unsigned short* __restrict__ lcol, int nblk, double* __restrict__ X, int ldx,
    const double* __restrict__ Ri, const double* Qi, double* __restrict__ Ro, double* Qo,
    double* __restrict__ P, int ld, int b,
    int first_arg, const double* __restrict__ alpha, const double* __restrict__ beta,
    double* __restrict__ partial, size_t pstride) {
  constexpr int WPB = kBlock / kWave;
  constexpr int kTileRows = kTileShapes[KIND].rows;
  constexpr int kTileCols = kTileShapes[KIND].cols;
  constexpr int kTileNnz = kTileShapes[KIND].nnz;
  constexpr int RPW = kTileRows / WPB;
  constexpr int SPW = kTileCols / WPB;
  __shared__ double sx[kTileCols * kWave];  // also the partial-sum buffer at the end
  __shared__ double sv[kTileNnz];
  __shared__ unsigned short sc[kTileNnz];
  __shared__ int sp[kTileRows + 1];
  static_assert(kTileCols >= 4 * WPB, "the four reductions reuse the staging buffer");
  static_assert(kBlock == 4 * kWave, "one wavefront per partial sum in the reduction");
  const bool first = !PEND && first_arg != 0;  // a pending step is never the first
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cc = blockIdx.y * kWave + lane;
  const bool cok = cc < b;
  const int cx = cok ? cc : 0;  // lanes past b read column 0 and store nothing
  const double bt = (cok && !first) ? beta[cc] : 0.0;
  const double al = (PEND && cok) ? alpha[cc] : 0.0;
  double s_pq = 0.0, s_rq = 0.0, s_qq = 0.0, s_rr = 0.0;
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int xcd = blockIdx.x % nx, bl = blockIdx.x / nx;
  const int tpx = (nblk + nx - 1) / nx;
  const int thi = min(nblk, (xcd + 1) * tpx);
  for (int t = xcd * tpx + bl; t < thi; t += bpx) {
    const int r0 = trow[t];
    const int r1 = trow[t + 1];
    const int nr = r1 - r0;
    const int u0 = uptr[t], nu = uptr[t + 1] - u0;
    const int e0 = rowptr[r0], ne = rowptr[r1] - e0;
    // w[q] = old q (= A p) of the row in slot wid + WPB q.  The slots below
    // nr are the own rows in order, so w[k] (k < RPW) is also the old q of own
    // row r0 + wid + k WPB, kept for the q update; the other entries serve
    // the residual update of the halo rows (PEND only).
    double w[SPW];
    {
      constexpr int EPT = kTileNnz / kBlock;
      double ev[EPT];
      unsigned short ec[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = threadIdx.x + q * kBlock;
        ev[q] = e < ne ? val[e0 + e] : 0.0;
        ec[q] = e < ne ? lcol[e0 + e] : 0;
      }
      const int rp = threadIdx.x <= nr ? rowptr[r0 + threadIdx.x] - e0 : 0;
      // slot wid + WPB q of the tile is held by lane q of this wavefront
      const int myu = wid + WPB * lane;
      const int ridx = (lane < SPW && myu < nu) ? urow[u0 + myu] : -1;
      double v[SPW];
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        const int j = __builtin_amdgcn_readlane(ridx, q);
        v[q] = j >= 0 ? Ri[(size_t)j * ld + cx] : 0.0;
        w[q] = ((PEND || (!first && q < RPW)) && j >= 0) ? Qi[(size_t)j * ld + cx] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = threadIdx.x + q * kBlock;
        if (e < ne) {
          sv[e] = ev[q];
          sc[e] = ec[q];
        }
      }
      if (threadIdx.x <= nr) sp[threadIdx.x] = rp;
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        const int u = wid + WPB * q;
        if (u < nu) sx[u * kWave + lane] = PEND ? v[q] - al * w[q] : v[q];
      }
    }
    __syncthreads();
    double po[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int i = r0 + wid + k * WPB;
      const size_t ri = (size_t)(i < r1 ? i : r0);
      po[k] = (!first && i < r1) ? __builtin_nontemporal_load(P + ri * ld + cx) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int i = r0 + wid + k * WPB;
      if (i < r1) {
        const int l = i - r0;
        // the iterate's row: loaded here so that its latency overlaps the
        // row's gathers rather than holding registers across the tile
        const double xo = (PEND && cok) ? __builtin_nontemporal_load(X + (size_t)i * ldx + cc) : 0.0;
        const double xi = sx[l * kWave + lane];
        const int lo = sp[l], hi = sp[l + 1];
        double a0 = 0.0;
        for (int base = 0; base < hi - lo; base += kWave) {
          const int m = min(kWave, hi - lo - base);
          const int jv = lane < m ? static_cast<int>(sc[lo + base + lane]) : 0;
          const double wv = lane < m ? sv[lo + base + lane] : 0.0;
          for (int k0 = 0; k0 < m; k0 += 8) {
            double xs[8], ws[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int j = __builtin_amdgcn_readlane(jv, k0 + q);
              ws[q] = readlane_d(wv, k0 + q);
              xs[q] = sx[j * kWave + lane];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) a0 += ws[q] * (xi - xs[q]);
          }
        }
        const double y = diag[i] * xi + a0 + bt * w[k];
        const double pn = xi + bt * po[k];
        if (cok) {
          const size_t iv = (size_t)i * ld + cc;
          __builtin_nontemporal_store(pn, P + iv);
          __builtin_nontemporal_store(y, Qo + iv);
          if (PEND) {
            __builtin_nontemporal_store(xi, Ro + iv);
            __builtin_nontemporal_store(xo + al * po[k], X + (size_t)i * ldx + cc);
          }
          s_pq += pn * y;
          s_rq += xi * y;
          s_qq += y * y;
          s_rr += xi * xi;
        }
      }
    }
    __syncthreads();  // the next tile overwrites the staging
  }
  double* red = sx;
  red[(0 * WPB + wid) * kWave + lane] = s_pq;
  red[(1 * WPB + wid) * kWave + lane] = s_rq;
  red[(2 * WPB + wid) * kWave + lane] = s_qq;
  red[(3 * WPB + wid) * kWave + lane] = s_rr;
  __syncthreads();
  {
    const int m = wid;  // wavefront m sums partial m
    double s = 0.0;
    for (int w = 0; w < WPB; ++w) s += red[(m * WPB + w) * kWave + lane];
    if (cok) partial[(size_t)m * pstride + (size_t)blockIdx.x * b + cc] = s;
  }
}

template <int KIND>
void launch_cg_tile_kind(const CsrView& A, double* X, int ldx, const double* Ri, const double* Qi,
                         double* Ro, double* Qo, double* P, int ld, int b, bool pend,
                         bool first, const double* alpha,
                         const double* beta, double* partial, size_t pstride, dim3 grid,
                         hipStream_t s) {
  if (pend)
    hipLaunchKernelGGL((k_cg_tile<true, KIND>), grid, dim3(kBlock), 0, s, A.rowptr, A.val,
                       A.diag, A.t_row, A.t_uptr, A.t_urow, A.t_lcol, A.t_nblk, X, ldx, Ri, Qi, Ro,
                       Qo, P, ld, b, 0, alpha, beta, partial, pstride);
  else
    hipLaunchKernelGGL((k_cg_tile<false, KIND>), grid, dim3(kBlock), 0, s, A.rowptr, A.val,
                       A.diag, A.t_row, A.t_uptr, A.t_urow, A.t_lcol, A.t_nblk, X, ldx, Ri, Qi, Ro,
                       Qo, P, ld, b, first ? 1 : 0, alpha, beta, partial, pstride);
}

int launch_cg_tile(const CsrView& A, double* X, int ldx, const double* Ri, const double* Qi,
                   double* Ro, double* Qo, double* P, int ld, int b, bool pend, bool first,
                   const double* alpha,
                   const double* beta, double* partial, size_t pstride, hipStream_t s) {
  int gx = std::min(A.t_nblk, kRedBlocks);
  if (gx >= 8) gx = gx / 8 * 8;  // whole XCD rounds
  dim3 grid(gx, ceil_div(b, kWave));
  switch (A.t_kind) {
    case 0: launch_cg_tile_kind<0>(A, X, ldx, Ri, Qi, Ro, Qo, P, ld, b, pend, first, alpha, beta, partial, pstride, grid, s); break;
    case 1: launch_cg_tile_kind<1>(A, X, ldx, Ri, Qi, Ro, Qo, P, ld, b, pend, first, alpha, beta, partial, pstride, grid, s); break;
    default: launch_cg_tile_kind<2>(A, X, ldx, Ri, Qi, Ro, Qo, P, ld, b, pend, first, alpha, beta, partial, pstride, grid, s); break;
  }
  check_launch();
  return gx;
}

template <int U, int STEP>
int launch_r64_t(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b,
                 hipStream_t s, bool fuse, bool first, const double* beta, double* P, int ldp,
                 double* partial) {
  constexpr int WPB = kBlock / kWave;
  int gx = std::max(1, ceil_div(A.n_rows, U * WPB));
  if (fuse && partial) gx = std::min(gx, kRedBlocks);
  if (gx >= 8) gx = gx / 8 * 8;  // whole XCD rounds
  dim3 grid(gx, ceil_div(b, kWave));
  const bool edge = A.diag != nullptr;
#define MMD_R64_CASE(E, F)                                                                   \
  hipLaunchKernelGGL((k_spmm_r64<E, F, U, STEP>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr, \
                     A.col, A.val, A.diag, X, ldx, Y, ldy, b, first ? 1 : 0, beta, P, ldp,     \
                     partial)
  if (edge) {
    if (fuse) MMD_R64_CASE(true, true);
    else MMD_R64_CASE(true, false);
  } else {
    if (fuse) MMD_R64_CASE(false, true);
    else MMD_R64_CASE(false, false);
  }
#undef MMD_R64_CASE
  check_launch();
  return gx;
}

int launch_spmm_r64(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b,
                    hipStream_t s, bool fuse, bool first, const double* beta, double* P,
                    int ldp, double* partial) {
  // one row per wavefront, gathers in steps of 4 slots, 8 waves per SIMD:
  // measured best of 1-4 rows x 2-8 slots at 5-8 waves per SIMD
  return launch_r64_t<1, 4>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial);
}

template <int LPR, int CT>
int launch_spmm_t(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b,
                  hipStream_t s, bool fuse, bool first, const double* beta, double* P, int ldp,
                  double* partial, const double* dotw, int lddot) {
  constexpr int R = kWave / (LPR * CT);
  constexpr int WPB = kBlock / kWave;
  const int groups = ceil_div(A.n_rows, R);
  int gx = ceil_div(groups, WPB);
  const bool red = (fuse && partial != nullptr) || dotw != nullptr;
  if (red) gx = std::min(gx, kRedBlocks);
  gx = std::max(gx, 1);
  if (gx >= 8) gx = (gx + 7) / 8 * 8;  // whole XCD rounds
  if (red) gx = std::min(gx, kRedBlocks);
  dim3 grid(gx, ceil_div(b, CT));
  const bool edge = A.diag != nullptr;
#define MMD_SPMM_CASE(E, F, D)                                                             \
  hipLaunchKernelGGL((k_spmm<LPR, CT, E, F, D>), grid, dim3(kBlock), 0, s, A.n_rows,       \
                     A.rowptr, A.col, A.val, A.diag, X, ldx, Y, ldy, b, first ? 1 : 0, beta, \
                     P, ldp, partial, dotw, lddot)
  if (edge) {
    if (fuse) MMD_SPMM_CASE(true, true, false);
    else if (dotw) MMD_SPMM_CASE(true, false, true);
    else MMD_SPMM_CASE(true, false, false);
  } else {
    if (fuse) MMD_SPMM_CASE(false, true, false);
    else if (dotw) MMD_SPMM_CASE(false, false, true);
    else MMD_SPMM_CASE(false, false, false);
  }
#undef MMD_SPMM_CASE
  check_launch();
  return gx;
}

// ------------------------------------------------------------------ Householder
__global__ void k_house_ut(int npatch, const int* __restrict__ ptr, const int* __restrict__ mem,
                           const double* __restrict__ u, const double* __restrict__ scale,
                           const double* __restrict__ x, int ldx, double* __restrict__ y,
                           int ldy, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)npatch * b) return;
  const int j = static_cast<int>(t / b);
  const int c = static_cast<int>(t % b);
  const int lo = ptr[j], hi = ptr[j + 1];
  double d = 0.0;
  for (int q = lo; q < hi; ++q) d += u[q] * x[(size_t)mem[q] * ldx + c];
  const double sc = scale[j] * d;
  const int base = lo - j - 1;  // reduced index of slot q is base + (q - lo)
  for (int q = lo + 1; q < hi; ++q)
    y[(size_t)(base + (q - lo)) * ldy + c] = x[(size_t)mem[q] * ldx + c] - sc * u[q];
}

__global__ void k_house_u(int npatch, const int* __restrict__ ptr, const int* __restrict__ mem,
                          const double* __restrict__ u, const double* __restrict__ scale,
                          const double* __restrict__ y, int ldy, double* __restrict__ x,
                          int ldx, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)npatch * b) return;
  const int j = static_cast<int>(t / b);
  const int c = static_cast<int>(t % b);
  const int lo = ptr[j], hi = ptr[j + 1];
  const int base = lo - j - 1;
  double d = 0.0;
  for (int q = lo + 1; q < hi; ++q) d += u[q] * y[(size_t)(base + (q - lo)) * ldy + c];
  const double sc = scale[j] * d;
  x[(size_t)mem[lo] * ldx + c] = -sc * u[lo];
  for (int q = lo + 1; q < hi; ++q)
    x[(size_t)mem[q] * ldx + c] = y[(size_t)(base + (q - lo)) * ldy + c] - sc * u[q];
}

// ------------------------------------------------------------------ column reductions
// Thread layout shared by the reduction kernels: for b <= 256 a block uses
// tb = (256 / b) * b threads, thread t owns column t % b and row offset t / b;
// for b > 256 the block walks column tiles of 256 with one row per step.
struct ColMap {
  int b, tb, rstep, col, roff;
  bool act;
};

// blockDim.x == kBlock for b <= 256; for 256 < b <= 1024 the block has one
// thread per column (rounded up to a wave) and walks rows one at a time.
__device__ inline ColMap colmap(int b, int tile_c0) {
  ColMap m;
  m.b = b;
  if (b > kBlock && (int)blockDim.x >= b) {
    m.tb = blockDim.x;
    m.rstep = 1;
    m.col = threadIdx.x;
    m.roff = 0;
    m.act = threadIdx.x < b;
    return m;
  }
  if (b <= kBlock) {
    m.tb = (kBlock / b) * b;
    m.rstep = kBlock / b;
    m.col = threadIdx.x % b;
    m.roff = threadIdx.x / b;
    m.act = threadIdx.x < m.tb;
  } else {
    m.tb = kBlock;
    m.rstep = 1;
    m.col = tile_c0 + threadIdx.x;
    m.roff = 0;
    m.act = m.col < b;
  }
  return m;
}

__device__ inline void block_col_store(double v, const ColMap& m, double* partial) {
  __shared__ double sh[kBlock];
  if (m.b > kBlock) {  // one thread per column: no block reduction needed
    if (m.act) partial[(size_t)blockIdx.x * m.b + m.col] = v;
    return;
  }
  sh[threadIdx.x] = m.act ? v : 0.0;
  __syncthreads();
  if (m.b <= kBlock) {
    if (threadIdx.x < m.b) {
      double t = 0.0;
      for (int q = threadIdx.x; q < m.tb; q += m.b) t += sh[q];
      partial[(size_t)blockIdx.x * m.b + threadIdx.x] = t;
    }
  } else if (m.act) {
    partial[(size_t)blockIdx.x * m.b + m.col] = sh[threadIdx.x];
  }
  __syncthreads();
}

template <int MODE>  // 0: X.*Y ; 1: two dots X.*Y1, X.*Y2
__global__ __launch_bounds__(1024) void k_coldot(const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ Y1,
                                                   const double* __restrict__ Y2, int ldy,
                                                   int n, int b, double* __restrict__ p1,
                                                   double* __restrict__ p2) {
  const int ntile = (b <= kBlock || (int)blockDim.x >= b) ? 1 : (b + kBlock - 1) / kBlock;
  for (int tile = 0; tile < ntile; ++tile) {
    ColMap m = colmap(b, tile * kBlock);
    double a1 = 0.0, a2 = 0.0;
    if (m.act) {
      for (int i = blockIdx.x * m.rstep + m.roff; i < n; i += gridDim.x * m.rstep) {
        const double x = X[(size_t)i * ldx + m.col];
        a1 += x * Y1[(size_t)i * ldy + m.col];
        if (MODE == 1) a2 += x * Y2[(size_t)i * ldy + m.col];
      }
    }
    block_col_store(a1, m, p1);
    if (MODE == 1) block_col_store(a2, m, p2);
  }
}

// Per-column sums of a partial-sum array partial[q * b + c], q < nblk.  A block
// of kScThreads threads serves kScCols consecutive columns: lane t reads column
// t % kScCols of slices q = t / kScCols, t / kScCols + kScSlices, ... (one
// 128-byte line per slice row), the slice sums are combined in LDS in a fixed
// order, and the result is valid in threads t < kScCols.
constexpr int kScCols = 16;
constexpr int kScThreads = 1024;
constexpr int kScSlices = kScThreads / kScCols;

__device__ inline double col_sum(const double* __restrict__ p, int nblk, int b, bool want) {
  __shared__ double sh[kScThreads];
  const int c = blockIdx.x * kScCols + threadIdx.x % kScCols;
  const int sl = threadIdx.x / kScCols;
  double t = 0.0;
  if (want && c < b) {
    double t1 = 0.0;
    int q = sl;
    for (; q + kScSlices < nblk; q += 2 * kScSlices) {
      t += p[(size_t)q * b + c];
      t1 += p[(size_t)(q + kScSlices) * b + c];
    }
    if (q < nblk) t += p[(size_t)q * b + c];
    t += t1;
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < kScCols)
    for (int q = 0; q < kScSlices; ++q) r += sh[q * kScCols + threadIdx.x];
  __syncthreads();
  return r;
}

// Four column sums at once (arrays ps apart): each thread adds its slices of
// all four, the four slices of a column inside a wavefront combine by
// shuffles, and 16 threads add the 16 wavefronts' results.  Valid in threads
// below kScCols.
__device__ inline void col_sum4(const double* __restrict__ p, size_t ps, int nblk, int b,
                                bool want, double (&out)[4]) {
  constexpr int W = kScThreads / 64;
  __shared__ double sh4[4 * W * kScCols];
  const int c = blockIdx.x * kScCols + threadIdx.x % kScCols;
  const int sl = threadIdx.x / kScCols;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  if (want && c < b)
    for (int q = sl; q < nblk; q += kScSlices)
#pragma unroll
      for (int m = 0; m < 4; ++m) t[m] += p[m * ps + (size_t)q * b + c];
  // lanes l, l ^ 16, l ^ 32, l ^ 48 of a wavefront hold slices of one column
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    t[m] += __shfl_xor(t[m], 16, 64);
    t[m] += __shfl_xor(t[m], 32, 64);
  }
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane < kScCols)
#pragma unroll
    for (int m = 0; m < 4; ++m) sh4[(m * W + w) * kScCols + lane] = t[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    out[m] = 0.0;
    if (threadIdx.x < kScCols)
      for (int v = 0; v < W; ++v) out[m] += sh4[(m * W + v) * kScCols + threadIdx.x];
  }
  __syncthreads();
}

inline int sc_grid(int b) { return ceil_div(b, kScCols); }

__device__ inline int sc_col() { return blockIdx.x * kScCols + threadIdx.x; }

__global__ __launch_bounds__(kScThreads) void k_reduce_partials(
    const double* __restrict__ partial, int nblk, int b, double* __restrict__ out) {
  const double v = col_sum(partial, nblk, b, true);
  const int c = sc_col();
  if (threadIdx.x < kScCols && c < b) out[c] = v;
}

// The activity flag of column c as seen by all lanes of the block (inactive
// columns skip their reads).
__device__ inline bool col_active(const ColScalars& sc, int b) {
  const int c = blockIdx.x * kScCols + threadIdx.x % kScCols;
  return c < b && sc.active[c] != 0;
}

// ------------------------------------------------------------------ CG scalars
__global__ __launch_bounds__(kScThreads) void k_cg_init(ColScalars sc,
                                                        const double* __restrict__ pbn,
                                                        const double* __restrict__ prr,
                                                        int nblk, int b, double tol,
                                                        const int* __restrict__ parent) {
  const double bn2 = col_sum(pbn, nblk, b, true);
  const double rr = prr ? col_sum(prr, nblk, b, true) : bn2;
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  sc.bn2[c] = bn2;
  sc.rr2[c] = rr;
  sc.rr[c] = rr;
  sc.tol2[c] = tol * tol;
  sc.alpha[c] = 0.0;
  sc.beta[c] = 0.0;
  sc.iters[c] = 0;
  const bool par = parent ? parent[c] != 0 : true;
  sc.active[c] = (par && bn2 > 0.0 && rr > tol * tol * bn2) ? 1 : 0;
}

__global__ __launch_bounds__(kScThreads) void k_cg_alpha(ColScalars sc,
                                                         const double* __restrict__ ppq,
                                                         int nblk, int b) {
  const bool act = col_active(sc, b);
  const double pq = col_sum(ppq, nblk, b, act);
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  if (!act) {
    sc.alpha[c] = 0.0;
    return;
  }
  if (!(pq > 0.0)) {
    sc.notspd[0] = 1;
    sc.active[c] = 0;
    sc.alpha[c] = 0.0;
    return;
  }
  sc.alpha[c] = sc.rr[c] / pq;
}

__global__ __launch_bounds__(kScThreads) void k_cg_beta(ColScalars sc,
                                                        const double* __restrict__ prr,
                                                        int nblk, int b) {
  const bool act = col_active(sc, b);
  const double rn = col_sum(prr, nblk, b, act);
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  if (!act) {
    sc.beta[c] = 0.0;
    return;
  }
  sc.iters[c] += 1;
  sc.rr2[c] = rn;
  if (rn <= sc.tol2[c] * sc.bn2[c]) {
    sc.active[c] = 0;
    sc.beta[c] = 0.0;
    return;
  }
  sc.beta[c] = rn / sc.rr[c];
  sc.rr[c] = rn;
}

// CG scalars of the reliable-update mixed solve: as k_cg_beta, but a column
// whose recursive residual has dropped below tol2 * bn2 keeps iterating and
// raises upd[c], which asks the host for an FP64 residual replacement.
// Scalars of a deferred-update step (k_cg_tile): partial sums p.q, r.q, q.q
// and r.r of the step's new vectors, pstride apart.  A column whose new
// residual (direct r.r) already meets the tolerance stops with no step
// pending (alpha = 0).  Otherwise alpha = r.r / p.q is left pending for the
// next step or flush, and the next residual norm |r - alpha q|^2 is taken
// from the expansion r.r - 2 alpha r.q + alpha^2 q.q for the stop test and
// beta.  The expansion cancels when the residual drops by about 1/eps in
// one step; below 64 eps r.r it is not trusted to stop the column (the next
// step's direct r.r decides).
__global__ __launch_bounds__(kScThreads) void k_cg_defer_scalars(ColScalars sc,
                                                                 const double* __restrict__ part,
                                                                 size_t pstride, int nblk,
                                                                 int b) {
  const bool act = col_active(sc, b);
  double sum[4];
  col_sum4(part, pstride, nblk, b, act, sum);
  const double pq = sum[0], rq = sum[1], qq = sum[2], rr = sum[3];
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  sc.alpha[c] = 0.0;
  sc.beta[c] = 0.0;
  if (!act) return;
  sc.rr[c] = rr;
  sc.rr2[c] = rr;
  const double stop2 = sc.tol2[c] * sc.bn2[c];
  if (rr <= stop2) {
    sc.active[c] = 0;
    return;
  }
  if (!(pq > 0.0)) {
    sc.notspd[0] = 1;
    sc.active[c] = 0;
    return;
  }
  const double a = rr / pq;
  sc.alpha[c] = a;
  sc.iters[c] += 1;
  const double rn = rr - 2.0 * a * rq + a * a * qq;
  const double rp = rn > 0.0 ? rn : 0.0;
  sc.rr2[c] = rp;
  if (rn >= 64.0 * 2.220446049250313e-16 * rr && rn <= stop2) {
    sc.active[c] = 0;  // alpha stays pending: the next step or flush applies it
    return;
  }
  sc.beta[c] = rp / rr;
  sc.rr[c] = rp;
}

// After k_cg_update has applied the pending alphas (partial = new r.r):
// alpha = 0 everywhere; an active column takes its direct r.r, rescales beta
// from the expanded norm to it, and stops if it meets the tolerance.
__global__ __launch_bounds__(kScThreads) void k_cg_defer_flush(ColScalars sc,
                                                               const double* __restrict__ prr,
                                                               int nblk, int b) {
  const bool act = col_active(sc, b);
  const double rr = col_sum(prr, nblk, b, act);
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  sc.alpha[c] = 0.0;
  if (!act) return;
  const double old = sc.rr[c];
  sc.rr2[c] = rr;
  if (rr <= sc.tol2[c] * sc.bn2[c]) {
    sc.active[c] = 0;
    sc.beta[c] = 0.0;
    return;
  }
  if (old > 0.0) sc.beta[c] *= rr / old;
  sc.rr[c] = rr;
}

__global__ __launch_bounds__(kScThreads) void k_cg_beta_flag(ColScalars sc,
                                                             const double* __restrict__ prr,
                                                             int nblk, int b,
                                                             int* __restrict__ upd) {
  const bool act = col_active(sc, b);
  const double rn = col_sum(prr, nblk, b, act);
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  if (!act) {
    sc.beta[c] = 0.0;
    return;
  }
  sc.iters[c] += 1;
  sc.rr2[c] = rn;
  if (rn <= sc.tol2[c] * sc.bn2[c]) upd[c] = 1;
  sc.beta[c] = rn / sc.rr[c];
  sc.rr[c] = rn;
}

// Residual replacement: the recursive residual r (with r.r = rr) is replaced
// by the true residual with r.r = rr_true.  The next direction p = r + beta p
// takes beta = rr_true / (r.r of the step before), i.e. the old beta scaled
// by rr_true / rr; the column stays active, its next flag threshold is
// delta2 * rr_true.  A column whose true residual exceeds restart2 times the
// recursive one (the directions no longer match the residual), or that
// stopped on a non-positive curvature, restarts with p = r (beta = 0).
__global__ void k_reliable_scalars(ColScalars sc, const double* __restrict__ rr_true,
                                   double delta2, double restart2, int b,
                                   int* __restrict__ upd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b) return;
  const double rt = rr_true[c];
  const double rn = sc.rr[c];
  const bool restart = !(rn > 0.0) || !sc.active[c] || rt > restart2 * rn;
  sc.beta[c] = restart ? 0.0 : sc.beta[c] * (rt / rn);
  sc.rr[c] = rt;
  sc.rr2[c] = rt;
  sc.bn2[c] = rt;
  sc.tol2[c] = delta2;
  sc.alpha[c] = 0.0;
  sc.active[c] = 1;
  upd[c] = 0;
}

__global__ __launch_bounds__(kScThreads) void k_pcg_conv(ColScalars sc,
                                                         const double* __restrict__ prr,
                                                         int nblk, int b) {
  const bool act = col_active(sc, b);
  const double rn = col_sum(prr, nblk, b, act);
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b || !act) return;
  sc.iters[c] += 1;
  sc.rr2[c] = rn;
  if (rn <= sc.tol2[c] * sc.bn2[c]) {
    sc.active[c] = 0;
    sc.beta[c] = 0.0;
  }
}

__global__ __launch_bounds__(kScThreads) void k_pcg_beta(ColScalars sc,
                                                         const double* __restrict__ prz,
                                                         const double* __restrict__ przo,
                                                         int nblk, int b) {
  const bool act = col_active(sc, b);
  const double rz = col_sum(prz, nblk, b, act);
  const double rzo = col_sum(przo, nblk, b, act);
  const int c = sc_col();
  if (threadIdx.x >= kScCols || c >= b) return;
  if (!act) {
    sc.beta[c] = 0.0;
    return;
  }
  sc.beta[c] = (rz - rzo) / sc.rr[c];
  sc.rr[c] = rz;
}

// ------------------------------------------------------------------ elementwise
__global__ __launch_bounds__(1024) void k_cg_update(double* __restrict__ X, int ldx,
                                                      double* __restrict__ R,
                                                      const double* __restrict__ P,
                                                      const double* __restrict__ Q, int ld,
                                                      int n, int b,
                                                      const double* __restrict__ alpha,
                                                      double* __restrict__ partial) {
  const int ntile = (b <= kBlock || (int)blockDim.x >= b) ? 1 : (b + kBlock - 1) / kBlock;
  for (int tile = 0; tile < ntile; ++tile) {
    ColMap m = colmap(b, tile * kBlock);
    double acc = 0.0;
    if (m.act) {
      const double a = alpha[m.col];
      const int step = gridDim.x * m.rstep;
      int i = blockIdx.x * m.rstep + m.roff;
      for (; i < n; i += step) {
        const size_t idx = (size_t)i * ld + m.col;
        double r = R[idx];
        if (a != 0.0) {
          X[(size_t)i * ldx + m.col] += a * P[idx];
          r -= a * Q[idx];
          R[idx] = r;
        }
        acc += r * r;
      }
    }
    block_col_store(acc, m, partial);
  }
}

__global__ void k_xpay(const double* __restrict__ R, int ldr, double* __restrict__ P, int ldp,
                       int n, int b, const double* __restrict__ beta, int first) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  const double r = R[i * ldr + c];
  P[i * ldp + c] = first ? r : r + beta[c] * P[i * ldp + c];
}

__global__ void k_scale_rows(double* __restrict__ X, int ldx, const double* __restrict__ d, int n,
                             int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  X[i * ldx + c] *= d[i];
}

__global__ void k_copy(const double* __restrict__ X, int ldx, double* __restrict__ Y, int ldy,
                       int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  Y[i * ldy + c] = X[i * ldx + c];
}

__global__ void k_zero(double* __restrict__ Y, int ldy, int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  Y[i * ldy + c] = 0.0;
}

__global__ void k_scale_cols(const double* __restrict__ X, int ldx, const double* __restrict__ d,
                             double* __restrict__ Y, int ldy, int n, int b, int acc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  const double v = X[i * ldx + c] * d[c];
  if (acc)
    Y[i * ldy + c] += v;
  else
    Y[i * ldy + c] = v;
}

__global__ void k_axpby(double a, const double* __restrict__ X, int ldx, double cc,
                        double* __restrict__ Y, int ldy, int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  const double y = cc == 0.0 ? 0.0 : cc * Y[i * ldy + c];
  Y[i * ldy + c] = a * X[i * ldx + c] + y;
}

__global__ void k_rsub(const double* __restrict__ B, int ldb, double* __restrict__ R, int ldr,
                       int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  R[i * ldr + c] = B[i * ldb + c] - R[i * ldr + c];
}

__global__ void k_scale_vec_dev(const double* __restrict__ x, const double* __restrict__ sc,
                                int inv_sqrt, double* __restrict__ y, int ldy, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = inv_sqrt ? 1.0 / sqrt(sc[0]) : 1.0 / sc[0];
  y[(size_t)i * ldy] = x[i] * f;
}

__global__ void k_gather_cols(const double* __restrict__ Y, int ldy, const int* __restrict__ idx,
                              double* __restrict__ Z, int ldz, int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  Z[i * ldz + c] = Y[i * ldy + idx[c]];
}

__global__ void k_scatter_cols(const double* __restrict__ Y, int ldy, const int* __restrict__ idx,
                               double* __restrict__ Z, int ldz, int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  Z[i * ldz + idx[c]] = Y[i * ldy + c];
}

__global__ void k_gather_scalars(ColScalars a, ColScalars d, const int* __restrict__ idx, int m) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int c = idx[j];
  d.rr[j] = a.rr[c];
  d.rr2[j] = a.rr2[c];
  d.alpha[j] = a.alpha[c];
  d.beta[j] = a.beta[c];
  d.bn2[j] = a.bn2[c];
  d.tol2[j] = a.tol2[c];
  d.active[j] = a.active[c];
  d.iters[j] = a.iters[c];
}

__global__ void k_to_colmajor(const double* __restrict__ X, int ldx,
                              const double* __restrict__ scale, double* __restrict__ out, int n,
                              int b, const int* __restrict__ perm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t c = t / n, i = t % n;
  const int64_t o = perm ? perm[i] : i;
  out[c * n + o] = X[i * ldx + c] * scale[c];
}

__global__ void k_from_colmajor(const double* __restrict__ in, int n, int b,
                                const int* __restrict__ perm, double* __restrict__ out, int ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  const int64_t src = perm ? perm[i] : i;
  out[i * ld + c] = in[c * n + src];
}

// One wavefront per row, lanes over the row's nonzeros; the row's own factor
// entries are the same address for every lane (one broadcast load each).
__global__ __launch_bounds__(kBlock) void k_sddmm_eig(int n_rows, const int* __restrict__ rowptr,
                                                      const int* __restrict__ col,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ X, int ld,
                                                      int nev, const double* __restrict__ glam,
                                                      double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int row = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (row >= n_rows) return;
  const int lo = rowptr[row], hi = rowptr[row + 1];
  const double* vi = V + (size_t)row * ld;
  const double* xi = X ? X + (size_t)row * ld : nullptr;
  for (int p = lo + lane; p < hi; p += kWave) {
    const int j = col[p];
    const double* vj = V + (size_t)j * ld;
    double acc = 0.0;
    if (glam)
      for (int k = 0; k < nev; ++k) acc += glam[k] * vi[k] * vj[k];
    if (X) {
      const double* xj = X + (size_t)j * ld;
      double t = 0.0;
      for (int k = 0; k < nev; ++k) t += xi[k] * vj[k] + vi[k] * xj[k];
      acc -= 0.5 * t;
    }
    out[p] = acc;
  }
}

__global__ void k_permute_rows(const double* __restrict__ X, int ldx, double* __restrict__ Y,
                               int ldy, int n, int b, const int* __restrict__ idx, int scatter) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * b) return;
  const int64_t i = t / b, c = t % b;
  if (scatter)
    Y[(int64_t)idx[i] * ldy + c] = X[i * ldx + c];
  else
    Y[i * ldy + c] = X[(int64_t)idx[i] * ldx + c];
}

__global__ void k_absmax_part(const double* __restrict__ X, int ldx, int n, int b, int chunk,
                              int* __restrict__ pidx, double* __restrict__ pval,
                              const int* __restrict__ perm) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= b) return;
  const int lo = blockIdx.x * chunk;
  const int hi = min(n, lo + chunk);
  double best = -1.0, bv = 0.0;
  int bi = n;
  for (int i = lo; i < hi; ++i) {
    const double v = X[(size_t)i * ldx + c];
    const int ui = perm ? perm[i] : i;
    if (fabs(v) > best || (fabs(v) == best && ui < bi)) {
      best = fabs(v);
      bv = v;
      bi = ui;
    }
  }
  pidx[(size_t)blockIdx.x * b + c] = bi;
  pval[(size_t)blockIdx.x * b + c] = bv;
}

__global__ void k_absmax_fin(const int* __restrict__ pidx, const double* __restrict__ pval,
                             int nch, int b, int* __restrict__ idx, double* __restrict__ val) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b) return;
  double best = -1.0, bv = 0.0;
  int bi = 0x7fffffff;
  for (int q = 0; q < nch; ++q) {
    const double v = pval[(size_t)q * b + c];
    const int ui = pidx[(size_t)q * b + c];
    if (fabs(v) > best || (fabs(v) == best && ui < bi)) {  // ties: lowest caller index
      best = fabs(v);
      bv = v;
      bi = ui;
    }
  }
  idx[c] = bi;
  val[c] = bv;
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ src, int* __restrict__ dst, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = static_cast<int>(src[t]);
}

// ------------------------------------------------------------------ FP64 GEMMs
// Both tall-skinny products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64, D[16x16] += A[16x4] B[4x16]).  A workgroup of four
// wavefronts owns a 64 x 64 output tile; the two operand tiles are staged
// through LDS 16 deep along the contracted index, and each wavefront
// accumulates one 32 x 32 quadrant as 2 x 2 MFMA tiles, 4 MFMA steps per stage.
// Lane layout of the instruction (lane l = 0..63): A[l % 16][l / 16],
// B[l / 16][l % 16], D[l / 16 + 4 r][l % 16] in accumulator element r
// (measured on gfx950).
constexpr int TM = 64, TK = 16;
typedef double v4d __attribute__((ext_vector_type(4)));

// acc[ti][tj] += sum_k as[k][row0 + 16 ti + i] * bs[k][col0 + 16 tj + j] over the
// TK staged values of k (as, bs: [TK][ld] in LDS)
template <int LDA, int LDB>
__device__ inline void mfma_quadrant(const double (*as)[LDA], const double (*bs)[LDB], int row0,
                                     int col0, v4d acc[2][2]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < TK; k0 += 4) {
    const double a0 = as[k0 + kq][row0 + i];
    const double a1 = as[k0 + kq][row0 + 16 + i];
    const double b0 = bs[k0 + kq][col0 + i];
    const double b1 = bs[k0 + kq][col0 + 16 + i];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__global__ __launch_bounds__(kBlock) void k_gram(const double* __restrict__ X, int ldx,
                                                 const double* __restrict__ Y, int ldy, int n,
                                                 int m, int p, int chunk,
                                                 double* __restrict__ work) {
  __shared__ double xs[TK][TM];
  __shared__ double ys[TK][TM];
  const int i0 = blockIdx.x * TM, j0 = blockIdx.y * TM;
  const int r0 = blockIdx.z * chunk;
  const int r1 = min(n, r0 + chunk);
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int qi = 32 * (w >> 1), qj = 32 * (w & 1);  // this wavefront's quadrant
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = r0; k0 < r1; k0 += TK) {
    for (int q = threadIdx.x; q < TK * TM; q += kBlock) {
      const int kk = q / TM, cc = q % TM;
      const int row = k0 + kk;
      xs[kk][cc] = (row < r1 && i0 + cc < m) ? X[(size_t)row * ldx + i0 + cc] : 0.0;
      ys[kk][cc] = (row < r1 && j0 + cc < p) ? Y[(size_t)row * ldy + j0 + cc] : 0.0;
    }
    __syncthreads();
    mfma_quadrant<TM, TM>(xs, ys, qi, qj, acc);
    __syncthreads();
  }
  double* wk = work + (size_t)blockIdx.z * m * p;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + qi + 16 * a + (lane >> 4) + 4 * r;
        const int j = j0 + qj + 16 * b + (lane & 15);
        if (i < m && j < p) wk[(size_t)i * p + j] = acc[a][b][r];
      }
}

__global__ void k_gram_reduce(const double* __restrict__ work, int splits, int m, int p,
                              double* __restrict__ C, int ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * p) return;
  double s = 0.0;
  for (int q = 0; q < splits; ++q) s += work[(size_t)q * m * p + t];
  C[(t / p) * ldc + (t % p)] = s;
}

__global__ __launch_bounds__(kBlock) void k_gemm_nn(const double* __restrict__ X, int ldx,
                                                    const double* __restrict__ C, int ldc,
                                                    double* __restrict__ Z, int ldz, int n,
                                                    int m, int p, double alpha, double beta) {
  __shared__ double xs[TK][TM + 1];
  __shared__ double cs[TK][TM];
  const int i0 = blockIdx.x * TM, j0 = blockIdx.y * TM;
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int qi = 32 * (w >> 1), qj = 32 * (w & 1);
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += TK) {
    for (int q = threadIdx.x; q < TK * TM; q += kBlock) {
      const int rr = q / TK, kk = q % TK;  // X tile: 64 rows x 16 k, k fastest
      const int row = i0 + rr, k = k0 + kk;
      xs[kk][rr] = (row < n && k < m) ? X[(size_t)row * ldx + k] : 0.0;
      const int kc = q / TM, cc = q % TM;  // C tile: 16 k x 64 cols
      const int k2 = k0 + kc, j = j0 + cc;
      cs[kc][cc] = (k2 < m && j < p) ? C[(size_t)k2 * ldc + j] : 0.0;
    }
    __syncthreads();
    mfma_quadrant<TM + 1, TM>(xs, cs, qi, qj, acc);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + qi + 16 * a + (lane >> 4) + 4 * r;
        const int j = j0 + qj + 16 * b + (lane & 15);
        if (i < n && j < p) {
          const size_t iz = (size_t)i * ldz + j;
          const double old = beta == 0.0 ? 0.0 : beta * Z[iz];
          Z[iz] = alpha * acc[a][b][r] + old;
        }
      }
}

// thread c of a block sums its column over one chunk of rows, four rows per
// pass with separate accumulators so four loads are in flight
__global__ __launch_bounds__(kBlock) void k_gemv_t(const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ y, int n, int m,
                                                   int chunk, double* __restrict__ work) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = lo;
  for (; i + 3 < hi; i += 4) {
    a0 += X[(size_t)i * ldx + c] * y[i];
    a1 += X[(size_t)(i + 1) * ldx + c] * y[i + 1];
    a2 += X[(size_t)(i + 2) * ldx + c] * y[i + 2];
    a3 += X[(size_t)(i + 3) * ldx + c] * y[i + 3];
  }
  for (; i < hi; ++i) a0 += X[(size_t)i * ldx + c] * y[i];
  work[(size_t)blockIdx.x * m + c] = (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(kBlock) void k_gemv_n_sub(const double* __restrict__ X, int ldx,
                                                       const double* __restrict__ h, int n,
                                                       int m, double* __restrict__ z) {
  const int lane = threadIdx.x & (kWave - 1);
  const int row = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (row >= n) return;
  double acc = 0.0;
  for (int c = lane; c < m; c += kWave) acc += X[(size_t)row * ldx + c] * h[c];
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) acc += __shfl_xor(acc, off, kWave);
  if (lane == 0) z[row] -= acc;
}

// threads per block of the column-reduction kernels (see colmap)
inline int red_threads(int b) {
  if (b > kBlock && b <= 1024) return (b + kWave - 1) / kWave * kWave;
  return kBlock;
}

inline int red_grid(int n, int b) {
  const int rows_per_block = b <= kBlock ? kBlock / b : 1;
  const int want = ceil_div((int64_t)n, (int64_t)rows_per_block * 8);
  return std::max(1, std::min(kRedBlocks, want));
}

inline int ew_grid(int64_t count) { return std::max(1, ceil_div(count, kBlock)); }

// MMDEIG_NO_TILE=1 runs the plain row-per-wavefront kernel on tiled operators
bool tile_off() {
  static const bool off = [] {
    const char* e = std::getenv("MMDEIG_NO_TILE");
    return e && e[0] && e[0] != '0';
  }();
  return off;
}

}  // namespace

// ======================================================================= launchers
int spmm(const CsrView& A, const double* X, int ldx, double* Y, int ldy, int b, hipStream_t s,
         bool fuse, bool first, const double* beta, double* P, int ldp, double* partial,
         const double* dot_with, int ld_dot) {
  if (A.n_rows == 0 || b == 0) return 0;
  if (b == 1) {
    if (A.avg_row <= 10.0) return launch_spmm_t<8, 1>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, dot_with, ld_dot);
    if (A.avg_row <= 24.0) return launch_spmm_t<16, 1>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, dot_with, ld_dot);
    return launch_spmm_t<64, 1>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, dot_with, ld_dot);
  }
  if (b <= 4) return launch_spmm_t<16, 4>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, dot_with, ld_dot);
  if (b <= 32) return launch_spmm_t<4, 16>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, dot_with, ld_dot);
  if (!dot_with && A.t_uptr && A.diag && !tile_off())
    return launch_spmm_tile(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial);
  if (!dot_with) return launch_spmm_r64(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial);
  return launch_spmm_t<1, 64>(A, X, ldx, Y, ldy, b, s, fuse, first, beta, P, ldp, partial, dot_with, ld_dot);
}

void house_ut(const HouseView& H, const double* x, int ldx, double* y, int ldy, int b,
              hipStream_t s) {
  if (H.npatch == 0 || b == 0) return;
  const int64_t cnt = (int64_t)H.npatch * b;
  hipLaunchKernelGGL(k_house_ut, dim3(ew_grid(cnt)), dim3(kBlock), 0, s, H.npatch, H.ptr,
                     H.members, H.u, H.scale, x, ldx, y, ldy, b);
  check_launch();
}

void house_u(const HouseView& H, const double* y, int ldy, double* x, int ldx, int b,
             hipStream_t s) {
  if (H.npatch == 0 || b == 0) return;
  const int64_t cnt = (int64_t)H.npatch * b;
  hipLaunchKernelGGL(k_house_u, dim3(ew_grid(cnt)), dim3(kBlock), 0, s, H.npatch, H.ptr,
                     H.members, H.u, H.scale, y, ldy, x, ldx, b);
  check_launch();
}

int col_dot(const double* X, int ldx, const double* Y, int ldy, int n, int b, double* partial,
            hipStream_t s) {
  const int g = red_grid(n, b);
  hipLaunchKernelGGL(k_coldot<0>, dim3(g), dim3(red_threads(b)), 0, s, X, ldx, Y, nullptr, ldy, n, b,
                     partial, nullptr);
  check_launch();
  return g;
}

int col_dot2(const double* X, int ldx, const double* Y1, const double* Y2, int ldy, int n,
             int b, double* partial1, double* partial2, hipStream_t s) {
  const int g = red_grid(n, b);
  hipLaunchKernelGGL(k_coldot<1>, dim3(g), dim3(red_threads(b)), 0, s, X, ldx, Y1, Y2, ldy, n, b,
                     partial1, partial2);
  check_launch();
  return g;
}

void reduce_partials(const double* partial, int nblk, int b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(sc_grid(b)), dim3(kScThreads), 0, s, partial,
                     nblk, b, out);
  check_launch();
}

void cg_init(ColScalars sc, const double* part_bn, const double* part_rr, int nblk, int b,
             double tol, const int* parent_active, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_bn,
                     part_rr, nblk, b, tol, parent_active);
  check_launch();
}

void cg_alpha(ColScalars sc, const double* part_pq, int nblk, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_pq,
                     nblk, b);
  check_launch();
}

void cg_beta(ColScalars sc, const double* part_rr, int nblk, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_rr,
                     nblk, b);
  check_launch();
}

bool cg_tile_ok(const CsrView& A) { return A.t_uptr && A.diag && !tile_off(); }

int cg_tile_step(const CsrView& A, double* X, int ldx, const double* Ri, const double* Qi,
                 double* Ro, double* Qo, double* P, int ld, int b, bool pend, bool first,
                 const double* alpha, const double* beta, double* partial, size_t pstride,
                 hipStream_t s) {
  MMD_REQUIRE(cg_tile_ok(A), MMD_EINVAL, "deferred CG step needs the tiled edge form");
  MMD_REQUIRE(!(pend && first), MMD_EINVAL, "a first step has no pending update");
  MMD_REQUIRE(!pend || (Ro != Ri && Qo != Qi), MMD_EINVAL,
              "a pending step writes r and q to buffers other than the ones it gathers");
  MMD_REQUIRE(pstride >= (size_t)kRedBlocks * b, MMD_EINVAL, "partial stride too small");
  if (A.n_rows == 0 || b == 0) return 0;
  return launch_cg_tile(A, X, ldx, Ri, Qi, Ro, Qo, P, ld, b, pend, first, alpha, beta, partial,
                        pstride, s);
}

void cg_defer_scalars(ColScalars sc, const double* part, size_t pstride, int nblk, int b,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_cg_defer_scalars, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part,
                     pstride, nblk, b);
  check_launch();
}

void cg_defer_flush(ColScalars sc, const double* part_rr, int nblk, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_defer_flush, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_rr,
                     nblk, b);
  check_launch();
}

void cg_beta_flag(ColScalars sc, const double* part_rr, int nblk, int b, int* upd,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta_flag, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_rr,
                     nblk, b, upd);
  check_launch();
}

void reliable_scalars(ColScalars sc, const double* rr_true, double delta2, double restart2,
                      int b, int* upd, hipStream_t s) {
  if (b == 0) return;
  hipLaunchKernelGGL(k_reliable_scalars, dim3(ceil_div(b, kBlock)), dim3(kBlock), 0, s, sc,
                     rr_true, delta2, restart2, b, upd);
  check_launch();
}

void pcg_conv(ColScalars sc, const double* part_rr, int nblk, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_conv, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_rr,
                     nblk, b);
  check_launch();
}

void pcg_beta(ColScalars sc, const double* part_rz, const double* part_rzo, int nblk, int b,
              hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_beta, dim3(sc_grid(b)), dim3(kScThreads), 0, s, sc, part_rz,
                     part_rzo, nblk, b);
  check_launch();
}

int cg_update(double* X, int ldx, double* R, const double* P, const double* Q, int ld, int n,
              int b, const double* alpha, double* partial, hipStream_t s) {
  const int g = red_grid(n, b);
  hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(red_threads(b)), 0, s, X, ldx, R, P, Q, ld, n, b, alpha,
                     partial);
  check_launch();
  return g;
}

void scale_rows(double* X, int ldx, const double* d, int n, int b, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_scale_rows, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, X, ldx, d,
                     n, b);
  check_launch();
}

void xpay(const double* R, int ldr, double* P, int ldp, int n, int b, const double* beta,
          bool first, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_xpay, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, R, ldr, P, ldp,
                     n, b, beta, first ? 1 : 0);
  check_launch();
}

void copy_block(const double* X, int ldx, double* Y, int ldy, int n, int b, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_copy, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, X, ldx, Y, ldy,
                     n, b);
  check_launch();
}

void zero_block(double* Y, int ldy, int n, int b, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_zero, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, Y, ldy, n, b);
  check_launch();
}

void scale_cols(const double* X, int ldx, const double* d, double* Y, int ldy, int n, int b,
                bool accumulate, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_scale_cols, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, X, ldx, d,
                     Y, ldy, n, b, accumulate ? 1 : 0);
  check_launch();
}

void axpby(double a, const double* X, int ldx, double c, double* Y, int ldy, int n, int b,
           hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, a, X, ldx, c,
                     Y, ldy, n, b);
  check_launch();
}

void rsub(const double* B, int ldb, double* R, int ldr, int n, int b, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_rsub, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, B, ldb, R, ldr,
                     n, b);
  check_launch();
}

void scale_vec_dev(const double* x, const double* scal, bool inv_sqrt, double* y, int ldy,
                   int n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_scale_vec_dev, dim3(ew_grid(n)), dim3(kBlock), 0, s, x, scal,
                     inv_sqrt ? 1 : 0, y, ldy, n);
  check_launch();
}

void gather_cols(const double* Y, int ldy, const int* idx, double* Z, int ldz, int n, int b,
                 hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_gather_cols, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, Y, ldy,
                     idx, Z, ldz, n, b);
  check_launch();
}

void scatter_cols(const double* Y, int ldy, const int* idx, double* Z, int ldz, int n, int b,
                  hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_scatter_cols, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, Y, ldy,
                     idx, Z, ldz, n, b);
  check_launch();
}

void gather_scalars(ColScalars src, ColScalars dst, const int* idx, int m, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_gather_scalars, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, s, src, dst,
                     idx, m);
  check_launch();
}

void from_colmajor(const double* in, int n, int b, const int* perm, double* out, int ld,
                   hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_from_colmajor, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, in, n, b,
                     perm, out, ld);
  check_launch();
}

void sddmm_eig(int n_rows, const int* rowptr, const int* col, const double* V, const double* X,
               int ld, int nev, const double* glam, double* out, hipStream_t s) {
  if (n_rows == 0) return;
  hipLaunchKernelGGL(k_sddmm_eig, dim3(ceil_div(n_rows, kBlock / kWave)), dim3(kBlock), 0, s,
                     n_rows, rowptr, col, V, X, ld, nev, glam, out);
  check_launch();
}

void to_colmajor(const double* X, int ldx, const double* colscale, double* out, int n, int b,
                 const int* perm, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_to_colmajor, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, X, ldx,
                     colscale, out, n, b, perm);
  check_launch();
}

void permute_rows(const double* X, int ldx, double* Y, int ldy, int n, int b, const int* idx,
                  bool scatter, hipStream_t s) {
  if ((int64_t)n * b == 0) return;
  hipLaunchKernelGGL(k_permute_rows, dim3(ew_grid((int64_t)n * b)), dim3(kBlock), 0, s, X, ldx,
                     Y, ldy, n, b, idx, scatter ? 1 : 0);
  check_launch();
}

static int absmax_chunks(int n) {
  const int chunk = std::max(256, ceil_div(n, 256));
  return std::max(1, ceil_div(n, chunk));
}

size_t col_absmax_work_size(int n, int b) { return (size_t)absmax_chunks(n) * b; }

void col_absmax(const double* X, int ldx, int n, int b, int* idx, double* val, const int* perm,
                int* work_idx, double* work_val, hipStream_t s) {
  // per-chunk candidates go to the caller's work arrays (col_absmax_work_size each)
  const int chunk = std::max(256, ceil_div(n, 256));
  const int nch = absmax_chunks(n);
  hipLaunchKernelGGL(k_absmax_part, dim3(nch, ceil_div(b, kBlock)), dim3(kBlock), 0, s, X, ldx,
                     n, b, chunk, work_idx, work_val, perm);
  check_launch();
  hipLaunchKernelGGL(k_absmax_fin, dim3(ceil_div(b, kBlock)), dim3(kBlock), 0, s, work_idx,
                     work_val, nch, b, idx, val);
  check_launch();
}

void i64_to_i32(const int64_t* src, int* dst, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_i64_to_i32, dim3(ew_grid(n)), dim3(kBlock), 0, s, src, dst, n);
  check_launch();
}

static int gram_splits(int n, int m, int p) {
  const int tiles = ceil_div(m, TM) * ceil_div(p, TM);
  int splits = std::max(1, 1024 / std::max(1, tiles));
  splits = std::min(splits, std::max(1, ceil_div(n, 256)));
  return splits;
}

size_t gram_work_size(int n, int m, int p) {
  return (size_t)gram_splits(n, m, p) * m * p;
}

void gram(const double* X, int ldx, const double* Y, int ldy, int n, int m, int p, double* C,
          int ldc, double* work, hipStream_t s) {
  if (m == 0 || p == 0) return;
  const int splits = gram_splits(n, m, p);
  const int chunk = ceil_div(n, splits);
  hipLaunchKernelGGL(k_gram, dim3(ceil_div(m, TM), ceil_div(p, TM), splits), dim3(kBlock), 0, s,
                     X, ldx, Y, ldy, n, m, p, chunk, work);
  check_launch();
  hipLaunchKernelGGL(k_gram_reduce, dim3(ew_grid((int64_t)m * p)), dim3(kBlock), 0, s, work,
                     splits, m, p, C, ldc);
  check_launch();
}

void gemm_nn(const double* X, int ldx, const double* C, int ldc, double* Z, int ldz, int n,
             int m, int p, double alpha, double beta, hipStream_t s) {
  if (n == 0 || p == 0) return;
  hipLaunchKernelGGL(k_gemm_nn, dim3(ceil_div(n, TM), ceil_div(p, TM)), dim3(kBlock), 0, s, X,
                     ldx, C, ldc, Z, ldz, n, m, p, alpha, beta);
  check_launch();
}

void gemv_t(const double* X, int ldx, const double* y, int n, int m, double* h, double* work,
            hipStream_t s) {
  if (m == 0) return;
  const int chunk = std::max(32, ceil_div(n, kGemvChunks));
  const int nch = ceil_div(n, chunk);
  const int threads = std::min(kBlock, ceil_div(m, kWave) * kWave);
  hipLaunchKernelGGL(k_gemv_t, dim3(nch, ceil_div(m, threads)), dim3(threads), 0, s, X, ldx, y,
                     n, m, chunk, work);
  check_launch();
  reduce_partials(work, nch, m, h, s);
}

void gemv_n_sub(const double* X, int ldx, const double* h, int n, int m, double* z,
                hipStream_t s) {
  if (m == 0 || n == 0) return;
  hipLaunchKernelGGL(k_gemv_n_sub, dim3(ceil_div(n, kBlock / kWave)), dim3(kBlock), 0, s, X, ldx,
                     h, n, m, z);
  check_launch();
}

}  // namespace mmd
