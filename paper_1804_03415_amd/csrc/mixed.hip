// FP32 block-CG kernels of the mixed-precision mode (see mixed.h).
//
// The SpMM follows the FP64 design of kernels.hip (XCD row bands, index
// broadcast with readlane, two rows per wavefront in flight) with each lane
// moving two adjacent columns as one float2, so a wavefront covers 128
// columns of a row.  Narrow blocks (<= 64 columns) pack several rows into a
// wavefront instead.  Partial dot products are accumulated in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "mixed.h"

namespace mmd {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWpb = kBlock / kWave;
constexpr int kStep = 8;

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

inline void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(MMD_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

__device__ inline float readlane_f(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

__device__ inline float2 ld2(const float* p) { return *reinterpret_cast<const float2*>(p); }

// Row range of this block's XCD and the block's position in it (workgroups
// are dealt to the 8 XCDs round-robin).
struct Band {
  int lo, hi, first, stride;
};

__device__ inline Band band(int units, int per_wave_unit) {
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int xcd = blockIdx.x % nx, bl = blockIdx.x / nx;
  const int upx = (units + nx - 1) / nx;
  Band r;
  r.lo = xcd * upx;
  r.hi = min(units, (xcd + 1) * upx);
  r.first = r.lo + bl * kWpb * per_wave_unit + (threadIdx.x / kWave) * per_wave_unit;
  r.stride = bpx * kWpb * per_wave_unit;
  return r;
}

// Block-combine per-lane partials (two columns per lane) into
// partial[blockIdx.x * b + c] for the tile's columns.  R rows per wave share a
// column slot; lanes (r, l) with the same l hold the same column pair.
template <int L>
__device__ inline void store_partials(double d0, double d1, int c0, int b, double* partial) {
  constexpr int R = kWave / L;
  __shared__ double red[2][kWpb * R * L];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  red[0][wid * kWave + lane] = d0;
  red[1][wid * kWave + lane] = d1;
  __syncthreads();
  if (threadIdx.x < 2 * L) {
    const int l = threadIdx.x >> 1, h = threadIdx.x & 1;
    double t = 0.0;
    for (int q = 0; q < kWpb * R; ++q) t += red[h][q * L + l];
    const int c = c0 + 2 * l + h;
    if (c < b) partial[(size_t)blockIdx.x * b + c] = t;
  }
}

// Wide form: one wavefront per (row, 128-column tile), two rows in flight,
// indices broadcast with readlane (slots past a row's end gather row 0 with
// weight 0).
template <bool EDGE>
__global__ __launch_bounds__(kBlock) void k_spmm32_w(
    int n_rows, const int* __restrict__ rowptr, const int* __restrict__ col,
    const float* __restrict__ val, const float* __restrict__ diag, const float* __restrict__ X,
    int ldx, float* __restrict__ Y, int ldy, int b, int first, const double* __restrict__ beta,
    float* __restrict__ P, int ldp, double* __restrict__ partial) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c0 = blockIdx.y * 2 * kWave;
  const int c = c0 + 2 * lane;
  const bool ok0 = c < b, ok1 = c + 1 < b;
  const int cx = ok0 ? c : 0;
  const float bt0 = (!first && ok0) ? static_cast<float>(beta[c]) : 0.f;
  const float bt1 = (!first && ok1) ? static_cast<float>(beta[c + 1]) : 0.f;
  double d0 = 0.0, d1 = 0.0;
  const Band bd = band(n_rows, 1);
  for (int row0 = bd.first; row0 < bd.hi; row0 += 2 * bd.stride) {
    const int row1 = row0 + bd.stride;
    const bool has1 = row1 < bd.hi;
    const int r1 = has1 ? row1 : row0;
    const int lo0 = rowptr[row0], hi0 = rowptr[row0 + 1];
    const int lo1 = has1 ? rowptr[row1] : 0, hi1 = has1 ? rowptr[row1 + 1] : 0;
    const float2 xi0 = EDGE ? ld2(X + (size_t)row0 * ldx + cx) : make_float2(0.f, 0.f);
    const float2 xi1 = EDGE ? ld2(X + (size_t)r1 * ldx + cx) : make_float2(0.f, 0.f);
    float a0x = 0.f, a0y = 0.f, a1x = 0.f, a1y = 0.f;
    for (int b0 = lo0, b1 = lo1; b0 < hi0 || b1 < hi1; b0 += kWave, b1 += kWave) {
      const int n0 = max(0, min(kWave, hi0 - b0)), n1 = max(0, min(kWave, hi1 - b1));
      const int jv0 = lane < n0 ? col[b0 + lane] : 0;
      const float vv0 = lane < n0 ? val[b0 + lane] : 0.f;
      const int jv1 = lane < n1 ? col[b1 + lane] : 0;
      const float vv1 = lane < n1 ? val[b1 + lane] : 0.f;
      const int m = max(n0, n1);
      for (int k0 = 0; k0 < m; k0 += kStep) {
        float2 x0[kStep], x1[kStep];
        float w0[kStep], w1[kStep];
#pragma unroll
        for (int q = 0; q < kStep; ++q) {
          const int j0 = __builtin_amdgcn_readlane(jv0, k0 + q);
          const int j1 = __builtin_amdgcn_readlane(jv1, k0 + q);
          w0[q] = readlane_f(vv0, k0 + q);
          w1[q] = readlane_f(vv1, k0 + q);
          x0[q] = ld2(X + (size_t)j0 * ldx + cx);
          x1[q] = ld2(X + (size_t)j1 * ldx + cx);
        }
#pragma unroll
        for (int q = 0; q < kStep; ++q) {
          if (EDGE) {
            a0x += w0[q] * (xi0.x - x0[q].x);
            a0y += w0[q] * (xi0.y - x0[q].y);
            a1x += w1[q] * (xi1.x - x1[q].x);
            a1y += w1[q] * (xi1.y - x1[q].y);
          } else {
            a0x += w0[q] * x0[q].x;
            a0y += w0[q] * x0[q].y;
            a1x += w1[q] * x1[q].x;
            a1y += w1[q] * x1[q].y;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int row = u ? row1 : row0;
      if ((u == 0 || has1) && ok0) {
        const float2 xi = u ? xi1 : xi0;
        const float dg = EDGE ? diag[row] : 0.f;
        float yx = (EDGE ? dg * xi.x : 0.f) + (u ? a1x : a0x);
        float yy = (EDGE ? dg * xi.y : 0.f) + (u ? a1y : a0y);
        float* yp = Y + (size_t)row * ldy + c;
        float* pp = P + (size_t)row * ldp + c;
        const float2 xr = ld2(X + (size_t)row * ldx + c);
        float px, py;
        if (first) {
          px = xr.x;
          py = xr.y;
        } else {
          const float2 yo = ld2(yp), po = ld2(pp);
          yx += bt0 * yo.x;
          yy += bt1 * yo.y;
          px = xr.x + bt0 * po.x;
          py = xr.y + bt1 * po.y;
        }
        if (!ok1) {
          py = 0.f;
          yy = 0.f;
        }
        *reinterpret_cast<float2*>(pp) = make_float2(px, py);
        *reinterpret_cast<float2*>(yp) = make_float2(yx, yy);
        d0 += static_cast<double>(px) * yx;
        d1 += static_cast<double>(py) * yy;
      }
    }
  }
  store_partials<kWave>(d0, d1, c0, b, partial);
}

// LDS-staged form on the tiled level-0 edge form, the FP32 counterpart of
// kernels.hip's k_spmm_tile: a workgroup takes one tile (CsrView32::t_row)
// and one 128-column slice (a lane moves two columns as a float2), issues
// every global load of the tile in one batch (own-row streams, entries,
// row pointers, the touched X rows), stages them in LDS and forms each row
// from LDS.  Same tile shapes (and workgroups per CU) as the FP64 kernel.
template <int KIND>
__global__ __launch_bounds__(kBlock, kTileShapes[KIND].wgs_per_cu) void k_spmm32_tile(
    const int* __restrict__ rowptr, const float* __restrict__ val,
    const float* __restrict__ diag, const int* __restrict__ trow,
    const int* __restrict__ uptr, const int* __restrict__ urow,
    const unsigned short* __restrict__ lcol, int nblk, const float* __restrict__ X, int ldx,
    float* __restrict__ Y, int ldy, int b, int first, const double* __restrict__ beta,
    float* __restrict__ P, int ldp, double* __restrict__ partial) {
  constexpr int kTileRows = kTileShapes[KIND].rows;
  constexpr int kTileCols = kTileShapes[KIND].cols;
  constexpr int kTileNnz = kTileShapes[KIND].nnz;
  constexpr int RPW = kTileRows / kWpb;  // rows per wavefront and tile
  __shared__ float2 sx[kTileCols * kWave];  // also the partial-sum buffer at the end
  __shared__ float sv[kTileNnz];
  __shared__ unsigned short sc[kTileNnz];
  __shared__ int sp[kTileRows + 1];
  static_assert(sizeof(sx) >= 2 * kBlock * sizeof(double), "partials reuse the staging");
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int c0 = blockIdx.y * 2 * kWave;
  const int c = c0 + 2 * lane;
  const bool ok0 = c < b, ok1 = c + 1 < b;
  const int cx = ok0 ? c : 0;  // lanes past b read column 0 and store nothing
  const float bt0 = (!first && ok0) ? static_cast<float>(beta[c]) : 0.f;
  const float bt1 = (!first && ok1) ? static_cast<float>(beta[c + 1]) : 0.f;
  double d0 = 0.0, d1 = 0.0;
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int xcd = blockIdx.x % nx, bl = blockIdx.x / nx;
  const int tpx = (nblk + nx - 1) / nx;
  const int thi = min(nblk, (xcd + 1) * tpx);
  for (int t = xcd * tpx + bl; t < thi; t += bpx) {
    const int r0 = trow[t], r1 = trow[t + 1];
    const int u0 = uptr[t], nu = uptr[t + 1] - u0;
    const int e0 = rowptr[r0], ne = rowptr[r1] - e0;
    float2 yo[RPW], po[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int i = r0 + wid + k * kWpb;
      const bool ok = !first && i < r1;
      const size_t ri = (size_t)(ok ? i : 0);
      yo[k] = ok ? ld2(Y + ri * ldy + cx) : make_float2(0.f, 0.f);
      po[k] = ok ? ld2(P + ri * ldp + cx) : make_float2(0.f, 0.f);
    }
    {
      constexpr int EPT = kTileNnz / kBlock;  // entries per thread
      float ev[EPT];
      unsigned short ec[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = threadIdx.x + q * kBlock;
        ev[q] = e < ne ? val[e0 + e] : 0.f;
        ec[q] = e < ne ? lcol[e0 + e] : 0;
      }
      const int rp = threadIdx.x <= r1 - r0 ? rowptr[r0 + threadIdx.x] - e0 : 0;
      constexpr int SPW = kTileCols / kWpb;  // slots per wavefront
      const int myu = wid + kWpb * lane;
      const int ridx = (lane < SPW && myu < nu) ? urow[u0 + myu] : -1;
      float2 v[SPW];
#pragma unroll
      for (int q = 0; q < SPW; ++q) {
        const int j = __builtin_amdgcn_readlane(ridx, q);
        v[q] = j >= 0 ? ld2(X + (size_t)j * ldx + cx) : make_float2(0.f, 0.f);
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
        const int u = wid + kWpb * q;
        if (u < nu) sx[u * kWave + lane] = v[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int i = r0 + wid + k * kWpb;
      if (i < r1) {
        const int l = i - r0;
        const float2 xi = sx[l * kWave + lane];
        const int lo = sp[l], hi = sp[l + 1];
        float ax = 0.f, ay = 0.f;
        for (int base = 0; base < hi - lo; base += kWave) {
          const int m = min(kWave, hi - lo - base);
          const int jv = lane < m ? static_cast<int>(sc[lo + base + lane]) : 0;
          const float wv = lane < m ? sv[lo + base + lane] : 0.f;
          for (int k0 = 0; k0 < m; k0 += 8) {
            float2 xs[8];
            float ws[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int j = __builtin_amdgcn_readlane(jv, k0 + q);
              ws[q] = readlane_f(wv, k0 + q);
              xs[q] = sx[j * kWave + lane];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              ax += ws[q] * (xi.x - xs[q].x);
              ay += ws[q] * (xi.y - xs[q].y);
            }
          }
        }
        if (ok0) {
          const float dg = diag[i];
          float yx = dg * xi.x + ax, yy = dg * xi.y + ay;
          float px, py;
          if (first) {
            px = xi.x;
            py = xi.y;
          } else {
            yx += bt0 * yo[k].x;
            yy += bt1 * yo[k].y;
            px = xi.x + bt0 * po[k].x;
            py = xi.y + bt1 * po[k].y;
          }
          if (!ok1) {
            py = 0.f;
            yy = 0.f;
          }
          *reinterpret_cast<float2*>(P + (size_t)i * ldp + c) = make_float2(px, py);
          *reinterpret_cast<float2*>(Y + (size_t)i * ldy + c) = make_float2(yx, yy);
          d0 += static_cast<double>(px) * yx;
          d1 += static_cast<double>(py) * yy;
        }
      }
    }
    __syncthreads();  // the next tile overwrites the staging
  }
  double* red = reinterpret_cast<double*>(sx);
  red[wid * kWave + lane] = d0;
  red[kBlock + wid * kWave + lane] = d1;
  __syncthreads();
  if (threadIdx.x < 2 * kWave) {
    const int l = threadIdx.x >> 1, h = threadIdx.x & 1;
    double tsum = 0.0;
    for (int w = 0; w < kWpb; ++w) tsum += red[h * kBlock + w * kWave + l];
    const int cc = c0 + 2 * l + h;
    if (cc < b) partial[(size_t)blockIdx.x * b + cc] = tsum;
  }
}

// Narrow form: L lanes per row (2L columns per tile), R = 64 / L rows per
// wavefront, direct index loads, four gathers in flight per lane.
template <int L, bool EDGE>
__global__ __launch_bounds__(kBlock) void k_spmm32_n(
    int n_rows, const int* __restrict__ rowptr, const int* __restrict__ col,
    const float* __restrict__ val, const float* __restrict__ diag, const float* __restrict__ X,
    int ldx, float* __restrict__ Y, int ldy, int b, int first, const double* __restrict__ beta,
    float* __restrict__ P, int ldp, double* __restrict__ partial) {
  constexpr int R = kWave / L;
  const int lane = threadIdx.x & (kWave - 1);
  const int l = lane % L, r = lane / L;
  const int c0 = blockIdx.y * 2 * L;
  const int c = c0 + 2 * l;
  const bool ok0 = c < b, ok1 = c + 1 < b;
  const int cx = ok0 ? c : 0;
  const float bt0 = (!first && ok0) ? static_cast<float>(beta[c]) : 0.f;
  const float bt1 = (!first && ok1) ? static_cast<float>(beta[c + 1]) : 0.f;
  double d0 = 0.0, d1 = 0.0;
  const int groups = (n_rows + R - 1) / R;
  const Band bd = band(groups, 1);
  for (int g = bd.first; g < bd.hi; g += bd.stride) {
    const int row = g * R + r;
    if (row >= n_rows || !ok0) continue;
    const int lo = rowptr[row], hi = rowptr[row + 1];
    const float2 xi = ld2(X + (size_t)row * ldx + cx);
    float ax = 0.f, ay = 0.f;
    int k = lo;
    for (; k + 3 < hi; k += 4) {
      const int j0 = col[k], j1 = col[k + 1], j2 = col[k + 2], j3 = col[k + 3];
      const float v0 = val[k], v1 = val[k + 1], v2 = val[k + 2], v3 = val[k + 3];
      const float2 x0 = ld2(X + (size_t)j0 * ldx + cx), x1 = ld2(X + (size_t)j1 * ldx + cx);
      const float2 x2 = ld2(X + (size_t)j2 * ldx + cx), x3 = ld2(X + (size_t)j3 * ldx + cx);
      if (EDGE) {
        ax += v0 * (xi.x - x0.x) + v1 * (xi.x - x1.x) + v2 * (xi.x - x2.x) + v3 * (xi.x - x3.x);
        ay += v0 * (xi.y - x0.y) + v1 * (xi.y - x1.y) + v2 * (xi.y - x2.y) + v3 * (xi.y - x3.y);
      } else {
        ax += v0 * x0.x + v1 * x1.x + v2 * x2.x + v3 * x3.x;
        ay += v0 * x0.y + v1 * x1.y + v2 * x2.y + v3 * x3.y;
      }
    }
    for (; k < hi; ++k) {
      const float v = val[k];
      const float2 x = ld2(X + (size_t)col[k] * ldx + cx);
      ax += EDGE ? v * (xi.x - x.x) : v * x.x;
      ay += EDGE ? v * (xi.y - x.y) : v * x.y;
    }
    const float dg = EDGE ? diag[row] : 0.f;
    float yx = (EDGE ? dg * xi.x : 0.f) + ax;
    float yy = (EDGE ? dg * xi.y : 0.f) + ay;
    float* yp = Y + (size_t)row * ldy + c;
    float* pp = P + (size_t)row * ldp + c;
    float px, py;
    if (first) {
      px = xi.x;
      py = xi.y;
    } else {
      const float2 yo = ld2(yp), po = ld2(pp);
      yx += bt0 * yo.x;
      yy += bt1 * yo.y;
      px = xi.x + bt0 * po.x;
      py = xi.y + bt1 * po.y;
    }
    if (!ok1) {
      py = 0.f;
      yy = 0.f;
    }
    *reinterpret_cast<float2*>(pp) = make_float2(px, py);
    *reinterpret_cast<float2*>(yp) = make_float2(yx, yy);
    d0 += static_cast<double>(px) * yx;
    d1 += static_cast<double>(py) * yy;
  }
  store_partials<L>(d0, d1, c0, b, partial);
}

// Column-pair reductions and updates: 32 lanes cover 64 columns of a row,
// 8 rows per block step.
constexpr int kPairs = 32;
constexpr int kRowsPerStep = kBlock / kPairs;

__device__ inline void pair_partials(double s0, double s1, int c, int b, double* partial) {
  __shared__ double sh[2][kBlock];
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  __syncthreads();
  if (threadIdx.x < 2 * kPairs) {
    const int p = threadIdx.x >> 1, h = threadIdx.x & 1;
    double t = 0.0;
    for (int q = 0; q < kRowsPerStep; ++q) t += sh[h][q * kPairs + p];
    const int cc = blockIdx.y * 2 * kPairs + 2 * p + h;
    if (cc < b) partial[(size_t)blockIdx.x * b + cc] = t;
  }
  (void)c;
}

__global__ __launch_bounds__(kBlock) void k_coldot32(const float* __restrict__ X, int ldx,
                                                     const float* __restrict__ Y, int ldy, int n,
                                                     int b, double* __restrict__ partial) {
  const int p = threadIdx.x % kPairs, ty = threadIdx.x / kPairs;
  const int c = blockIdx.y * 2 * kPairs + 2 * p;
  double s0 = 0.0, s1 = 0.0;
  if (c < b) {
    for (int i = blockIdx.x * kRowsPerStep + ty; i < n; i += gridDim.x * kRowsPerStep) {
      const float2 x = ld2(X + (size_t)i * ldx + c), y = ld2(Y + (size_t)i * ldy + c);
      s0 += static_cast<double>(x.x) * y.x;
      s1 += static_cast<double>(x.y) * y.y;
    }
  }
  pair_partials(s0, s1, c, b, partial);
}

__global__ __launch_bounds__(kBlock) void k_cg_update32(float* __restrict__ X, int ldx,
                                                        float* __restrict__ R,
                                                        const float* __restrict__ P,
                                                        const float* __restrict__ Q, int ld,
                                                        int n, int b,
                                                        const double* __restrict__ alpha,
                                                        double* __restrict__ partial) {
  const int p = threadIdx.x % kPairs, ty = threadIdx.x / kPairs;
  const int c = blockIdx.y * 2 * kPairs + 2 * p;
  double s0 = 0.0, s1 = 0.0;
  if (c < b) {
    const float a0 = static_cast<float>(alpha[c]);
    const float a1 = c + 1 < b ? static_cast<float>(alpha[c + 1]) : 0.f;
    const bool upd = a0 != 0.f || a1 != 0.f;
    for (int i = blockIdx.x * kRowsPerStep + ty; i < n; i += gridDim.x * kRowsPerStep) {
      float2 r = ld2(R + (size_t)i * ld + c);
      if (upd) {
        const float2 pv = ld2(P + (size_t)i * ld + c), qv = ld2(Q + (size_t)i * ld + c);
        float2 x = ld2(X + (size_t)i * ldx + c);
        x.x += a0 * pv.x;
        x.y += a1 * pv.y;
        r.x -= a0 * qv.x;
        r.y -= a1 * qv.y;
        *reinterpret_cast<float2*>(X + (size_t)i * ldx + c) = x;
        *reinterpret_cast<float2*>(R + (size_t)i * ld + c) = r;
      }
      s0 += static_cast<double>(r.x) * r.x;
      s1 += static_cast<double>(r.y) * r.y;
    }
  }
  pair_partials(s0, s1, c, b, partial);
}

__global__ void k_gather_to32(const double* __restrict__ Y, int ldy, const int* __restrict__ idx,
                              float* __restrict__ Z, int ldz, int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * ldz) return;
  const int64_t i = t / ldz, c = t % ldz;
  Z[i * ldz + c] = c < b ? static_cast<float>(Y[i * ldy + idx[c]]) : 0.f;
}

__global__ void k_gather32(const float* __restrict__ Y, int ldy, const int* __restrict__ idx,
                           float* __restrict__ Z, int ldz, int n, int b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * ldz) return;
  const int64_t i = t / ldz, c = t % ldz;
  Z[i * ldz + c] = c < b ? Y[i * ldy + idx[c]] : 0.f;
}

__global__ void k_scatter_add64(const float* __restrict__ D, int ldd, const int* __restrict__ src,
                                const int* __restrict__ dst, double* __restrict__ X, int ldx,
                                int n, int m) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * m) return;
  const int64_t i = t / m, j = t % m;
  X[i * ldx + dst[j]] += static_cast<double>(D[i * ldd + src[j]]);
}

__global__ void k_zero32(float* __restrict__ Y, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) Y[t] = 0.f;
}

__global__ void k_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = static_cast<float>(x[t]);
}

inline int ew_grid(int64_t count) { return std::max(1, ceil_div(count, kBlock)); }

inline int pair_grid(int n) {
  return std::max(1, std::min(kRedBlocks, ceil_div(n, kRowsPerStep * 4)));
}

template <int L>
int launch_n(const CsrView32& A, const float* X, int ldx, float* Y, int ldy, int b, bool first,
             const double* beta, float* P, int ldp, double* partial, hipStream_t s) {
  constexpr int R = kWave / L;
  const int groups = ceil_div(A.n_rows, R);
  int gx = std::max(1, std::min(kRedBlocks, ceil_div(groups, kWpb)));
  if (gx >= 8) gx = gx / 8 * 8;
  dim3 grid(gx, ceil_div(b, 2 * L));
  if (A.diag)
    hipLaunchKernelGGL((k_spmm32_n<L, true>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr,
                       A.col, A.val, A.diag, X, ldx, Y, ldy, b, first ? 1 : 0, beta, P, ldp,
                       partial);
  else
    hipLaunchKernelGGL((k_spmm32_n<L, false>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr,
                       A.col, A.val, A.diag, X, ldx, Y, ldy, b, first ? 1 : 0, beta, P, ldp,
                       partial);
  check_launch();
  return gx;
}

}  // namespace

int spmm32_cg(const CsrView32& A, const float* X, int ldx, float* Y, int ldy, int b, bool first,
              const double* beta, float* P, int ldp, double* partial, hipStream_t s) {
  if (A.n_rows == 0 || b == 0) return 0;
  MMD_REQUIRE(ldx % 2 == 0 && ldy % 2 == 0 && ldp % 2 == 0, MMD_EINVAL,
              "FP32 blocks need an even leading dimension");
  if (b <= 2) return launch_n<1>(A, X, ldx, Y, ldy, b, first, beta, P, ldp, partial, s);
  if (b <= 4) return launch_n<2>(A, X, ldx, Y, ldy, b, first, beta, P, ldp, partial, s);
  if (b <= 8) return launch_n<4>(A, X, ldx, Y, ldy, b, first, beta, P, ldp, partial, s);
  if (b <= 16) return launch_n<8>(A, X, ldx, Y, ldy, b, first, beta, P, ldp, partial, s);
  if (b <= 32) return launch_n<16>(A, X, ldx, Y, ldy, b, first, beta, P, ldp, partial, s);
  if (b <= 64) return launch_n<32>(A, X, ldx, Y, ldy, b, first, beta, P, ldp, partial, s);
  if (A.t_uptr && A.t_row && A.diag) {
    int gx = std::min(A.t_nblk, kRedBlocks);
    if (gx >= 8) gx = gx / 8 * 8;
    dim3 grid(gx, ceil_div(b, 2 * kWave));
#define MMD_TILE32(KIND)                                                                  \
  hipLaunchKernelGGL(k_spmm32_tile<KIND>, grid, dim3(kBlock), 0, s, A.rowptr, A.val, A.diag, \
                     A.t_row, A.t_uptr, A.t_urow, A.t_lcol, A.t_nblk, X, ldx, Y, ldy, b,     \
                     first ? 1 : 0, beta, P, ldp, partial)
    switch (A.t_kind) {
      case 0: MMD_TILE32(0); break;
      case 1: MMD_TILE32(1); break;
      default: MMD_TILE32(2); break;
    }
#undef MMD_TILE32
    check_launch();
    return gx;
  }
  int gx = std::max(1, std::min(kRedBlocks, ceil_div(A.n_rows, 2 * kWpb)));
  if (gx >= 8) gx = gx / 8 * 8;
  dim3 grid(gx, ceil_div(b, 2 * kWave));
  if (A.diag)
    hipLaunchKernelGGL((k_spmm32_w<true>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr, A.col,
                       A.val, A.diag, X, ldx, Y, ldy, b, first ? 1 : 0, beta, P, ldp, partial);
  else
    hipLaunchKernelGGL((k_spmm32_w<false>), grid, dim3(kBlock), 0, s, A.n_rows, A.rowptr, A.col,
                       A.val, A.diag, X, ldx, Y, ldy, b, first ? 1 : 0, beta, P, ldp, partial);
  check_launch();
  return gx;
}

int col_dot32(const float* X, int ldx, const float* Y, int ldy, int n, int b, double* partial,
              hipStream_t s) {
  const int g = pair_grid(n);
  hipLaunchKernelGGL(k_coldot32, dim3(g, ceil_div(b, 2 * kPairs)), dim3(kBlock), 0, s, X, ldx,
                     Y, ldy, n, b, partial);
  check_launch();
  return g;
}

int cg_update32(float* X, int ldx, float* R, const float* P, const float* Q, int ld, int n,
                int b, const double* alpha, double* partial, hipStream_t s) {
  const int g = pair_grid(n);
  hipLaunchKernelGGL(k_cg_update32, dim3(g, ceil_div(b, 2 * kPairs)), dim3(kBlock), 0, s, X,
                     ldx, R, P, Q, ld, n, b, alpha, partial);
  check_launch();
  return g;
}

void gather_to32(const double* Y, int ldy, const int* idx, float* Z, int ldz, int n, int b,
                 hipStream_t s) {
  if ((int64_t)n * ldz == 0) return;
  hipLaunchKernelGGL(k_gather_to32, dim3(ew_grid((int64_t)n * ldz)), dim3(kBlock), 0, s, Y, ldy,
                     idx, Z, ldz, n, b);
  check_launch();
}

void gather32(const float* Y, int ldy, const int* idx, float* Z, int ldz, int n, int b,
              hipStream_t s) {
  if ((int64_t)n * ldz == 0) return;
  hipLaunchKernelGGL(k_gather32, dim3(ew_grid((int64_t)n * ldz)), dim3(kBlock), 0, s, Y, ldy,
                     idx, Z, ldz, n, b);
  check_launch();
}

void scatter_add64(const float* D, int ldd, const int* src, const int* dst, double* X, int ldx,
                   int n, int m, hipStream_t s) {
  if ((int64_t)n * m == 0) return;
  hipLaunchKernelGGL(k_scatter_add64, dim3(ew_grid((int64_t)n * m)), dim3(kBlock), 0, s, D, ldd,
                     src, dst, X, ldx, n, m);
  check_launch();
}

void zero32(float* Y, int n, int ld, hipStream_t s) {
  const int64_t cnt = (int64_t)n * ld;
  if (cnt == 0) return;
  hipLaunchKernelGGL(k_zero32, dim3(ew_grid(cnt)), dim3(kBlock), 0, s, Y, cnt);
  check_launch();
}

void to_f32(const double* x, float* y, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(n)), dim3(kBlock), 0, s, x, y, n);
  check_launch();
}

}  // namespace mmd
