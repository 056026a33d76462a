// Host construction of the multiresolution matrix decomposition
// (Sections 2.1-2.3): partition, local basis phi (q = 1), Householder
// complement U, localised Psi (constrained-energy form, Appendix A),
// Galerkin level operators A^(k), M^(k), and their upload to the device.
#include <omp.h>

#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <string>

#include "dense.h"
#include "handle.h"

namespace mmd {

namespace {

// ---------------------------------------------------------------- input checks
void validate_and_copy(const mmd_csr& in, HostCSR& A, std::vector<double>& s) {
  MMD_REQUIRE(in.n > 0 && in.n < (int64_t(1) << 31), MMD_EINVAL, "n out of range");
  MMD_REQUIRE(in.nnz >= in.n && in.nnz < (int64_t(1) << 31), MMD_EINVAL, "nnz out of range");
  const int n = static_cast<int>(in.n);
  A.n_rows = A.n_cols = n;
  A.ptr.resize(n + 1);
  A.col.resize(in.nnz);
  A.val.resize(in.nnz);
  if (in.mem == 1) {
    MMD_HIP(hipMemcpy(A.ptr.data(), in.rowptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    MMD_HIP(hipMemcpy(A.col.data(), in.colind, in.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    MMD_HIP(hipMemcpy(A.val.data(), in.val, in.nnz * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::copy(in.rowptr, in.rowptr + n + 1, A.ptr.begin());
    std::copy(in.colind, in.colind + in.nnz, A.col.begin());
    std::copy(in.val, in.val + in.nnz, A.val.begin());
  }
  MMD_REQUIRE(A.ptr[0] == 0 && A.ptr[n] == in.nnz, MMD_EINVAL, "rowptr does not span nnz");
  s.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    MMD_REQUIRE(A.ptr[i] <= A.ptr[i + 1], MMD_EINVAL, "rowptr not monotone");
    double diag = 0.0, off = 0.0;
    bool has_diag = false;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int j = A.col[k];
      const double v = A.val[k];
      MMD_REQUIRE(j >= 0 && j < n, MMD_EINVAL, "column index out of range");
      MMD_REQUIRE(k == A.ptr[i] || A.col[k - 1] < j, MMD_EINVAL, "columns not sorted/unique");
      MMD_REQUIRE(std::isfinite(v), MMD_EINVAL, "non-finite value");
      if (j == i) {
        diag = v;
        has_diag = true;
      } else {
        MMD_REQUIRE(v <= 0.0, MMD_EUNSUPPORTED,
                    "positive off-diagonal: no edge-type energy decomposition");
        off += v;
        // symmetric counterpart
        auto b = A.col.begin() + A.ptr[j], e = A.col.begin() + A.ptr[j + 1];
        auto it = std::lower_bound(b, e, i);
        MMD_REQUIRE(it != e && *it == i && A.val[it - A.col.begin()] == v, MMD_EINVAL,
                    "matrix is not symmetric");
      }
    }
    MMD_REQUIRE(has_diag && diag > 0.0, MMD_ENOTSPD, "nonpositive diagonal entry");
    double si = diag + off;
    MMD_REQUIRE(si >= -1e-14 * diag, MMD_EUNSUPPORTED,
                "negative self-loop weight (not diagonally dominant)");
    s[i] = si < 0.0 ? 0.0 : si;
  }
}

// ---------------------------------------------------------------- partitions
using Patches = std::vector<std::vector<int>>;

Patches grid_patches(const std::vector<int>& shape, int blk, std::vector<int>& cshape) {
  const int d = static_cast<int>(shape.size());
  cshape.resize(d);
  for (int a = 0; a < d; ++a) cshape[a] = (shape[a] + blk - 1) / blk;
  int np = 1;
  for (int a = 0; a < d; ++a) np *= cshape[a];
  Patches P(np);
  const int nx = shape[0], ny = shape[1], nz = d == 3 ? shape[2] : 1;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int v = (z * ny + y) * nx + x;
        int pid = (y / blk) * cshape[0] + (x / blk);
        if (d == 3) pid = ((z / blk) * cshape[1] + (y / blk)) * cshape[0] + (x / blk);
        P[pid].push_back(v);  // ascending vertex order by construction
      }
  return P;
}

std::vector<int> morton_order(const std::vector<double>& xyz, int n, int d) {
  const int bits = d == 2 ? 16 : 10;
  const double scale = static_cast<double>(1 << bits);
  std::vector<int64_t> code(n, 0);
  for (int a = 0; a < d; ++a) {
    double lo = std::numeric_limits<double>::infinity(), hi = -lo;
    for (int i = 0; i < n; ++i) {
      lo = std::min(lo, xyz[(size_t)i * d + a]);
      hi = std::max(hi, xyz[(size_t)i * d + a]);
    }
    if (!(hi > lo)) continue;
    for (int i = 0; i < n; ++i) {
      double t = std::floor((xyz[(size_t)i * d + a] - lo) / (hi - lo) * scale);
      int64_t q = static_cast<int64_t>(std::min(std::max(t, 0.0), scale - 1.0));
      for (int b = 0; b < bits; ++b) code[i] |= ((q >> b) & 1) << (d * b + a);
    }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return code[x] < code[y]; });
  return ord;
}

// Greedy breadth-first aggregation in Morton order, then merge of patches
// smaller than target/2 into the neighbour sharing the most entries.
Patches greedy_patches(const HostCSR& A, const std::vector<double>& xyz, int d, int target) {
  const int n = A.n_rows;
  std::vector<int> order;
  if (d > 0) order = morton_order(xyz, n, d);
  else {
    order.resize(n);
    std::iota(order.begin(), order.end(), 0);
  }
  std::vector<int> pid(n, -1);
  Patches P;
  for (int s : order) {
    if (pid[s] >= 0) continue;
    const int cur = static_cast<int>(P.size());
    std::vector<int> mem{s};
    pid[s] = cur;
    size_t head = 0;
    while (head < mem.size() && static_cast<int>(mem.size()) < target) {
      const int v = mem[head++];
      for (int64_t k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
        const int u = A.col[k];
        if (pid[u] < 0) {
          pid[u] = cur;
          mem.push_back(u);
          if (static_cast<int>(mem.size()) >= target) break;
        }
      }
    }
    P.push_back(std::move(mem));
  }
  for (size_t p = 0; p < P.size(); ++p) {
    if (P[p].empty() || 2 * static_cast<int>(P[p].size()) >= target) continue;
    std::vector<std::pair<int, int>> cnt;  // (patch, count), small
    for (int v : P[p])
      for (int64_t k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
        const int q = pid[A.col[k]];
        if (q == static_cast<int>(p)) continue;
        auto it = std::find_if(cnt.begin(), cnt.end(), [&](auto& c) { return c.first == q; });
        if (it == cnt.end()) cnt.emplace_back(q, 1);
        else it->second++;
      }
    if (cnt.empty()) continue;
    int best = -1, bc = -1;
    for (auto& c : cnt)
      if (c.second > bc || (c.second == bc && c.first < best)) {
        best = c.first;
        bc = c.second;
      }
    for (int v : P[p]) pid[v] = best;
    P[best].insert(P[best].end(), P[p].begin(), P[p].end());
    P[p].clear();
  }
  Patches out;
  for (auto& m : P)
    if (!m.empty()) {
      std::sort(m.begin(), m.end());
      out.push_back(std::move(m));
    }
  return out;
}

// ---------------------------------------------------------------- patch energies
// Patch energies (Section 2.2): interior (level 1 of a target-size
// partition: generalised edges inside P + clamped remainder), closed
// (its levels >= 2: the principal submatrix), or split (every level of a
// partition to prescribed accuracy: A[P, P] - diag(sum_{j not in P} |a_ij|),
// whose sum over patches is bounded by A because the rest is diagonally
// dominant).
enum class Energy { Interior, Closed, Split };

std::vector<double> patch_energy(const HostCSR& A, const std::vector<int>& mem, Energy kind) {
  const bool closed = kind == Energy::Closed;
  const int p = static_cast<int>(mem.size());
  std::vector<double> E((size_t)p * p, 0.0);
  for (int a = 0; a < p; ++a) {
    const int i = mem[a];
    double diag = 0.0, offabs = 0.0, inner = 0.0;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int c = A.col[k];
      const double v = A.val[k];
      if (c == i) {
        diag += v;
        continue;
      }
      offabs += std::fabs(v);
      auto it = std::lower_bound(mem.begin(), mem.end(), c);
      if (it != mem.end() && *it == c) {
        E[(size_t)a * p + (it - mem.begin())] = v;
        inner += std::fabs(v);
      }
    }
    E[(size_t)a * p + a] = closed                   ? diag
                           : kind == Energy::Split ? diag - (offabs - inner)
                                                   : inner + std::max(diag - offabs, 0.0);
  }
  return E;
}

// Partition with prescribed accuracy (Section 2.3: eps(P) <= eps_k and
// eps(P) delta(P) <= c).  Seeds in Morton order (vertex order without
// coordinates); a seed opens a patch that grows greedily: among the unassigned
// vertices adjacent to the patch and not yet refused by it, the one with the
// largest total coupling sum_{p in P} |a_vp| to the patch is tried next (ties:
// smaller vertex id).  It joins when the enlarged patch keeps
// eps(P) = 1 / lambda_2(E_P) <= eps_k (E_P the split patch energy) and
// eps(P) delta(P) <= c, where delta(P) = 1 / (phi^T Abar_P^-1 phi) with phi
// the eigenvector of lambda_1(E_P) and Abar_P the principal submatrix;
// otherwise the patch refuses it.  The patch closes when no candidate is left
// or it holds max_size vertices.  Couplings accumulate member by member in
// join order and CSR order within a row.
Patches eps_patches(const HostCSR& A, const std::vector<double>& xyz, int d, double eps_k,
                    double cbound, Energy energy, int max_size) {
  const int n = A.n_rows;
  std::vector<int> order;
  if (d > 0) order = morton_order(xyz, n, d);
  else {
    order.resize(n);
    std::iota(order.begin(), order.end(), 0);
  }
  std::vector<int> pid(n, -1), stamp(n, -1), refused(n, -1);
  std::vector<double> coup(n, 0.0);
  Patches P;
  std::vector<int> cands, cand;
  for (int s0 : order) {
    if (pid[s0] >= 0) continue;
    const int cur = static_cast<int>(P.size());
    std::vector<int> mem{s0};
    pid[s0] = cur;
    cands.clear();
    auto add_couplings = [&](int v) {
      for (int64_t k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
        const int u = A.col[k];
        if (u == v || pid[u] >= 0) continue;
        if (stamp[u] != cur) {
          stamp[u] = cur;
          coup[u] = 0.0;
          cands.push_back(u);
        }
        coup[u] += std::fabs(A.val[k]);
      }
    };
    add_couplings(s0);
    while (static_cast<int>(mem.size()) < max_size) {
      int u = -1;
      for (int c : cands) {
        if (pid[c] >= 0 || refused[c] == cur) continue;
        if (u < 0 || coup[c] > coup[u] || (coup[c] == coup[u] && c < u)) u = c;
      }
      if (u < 0) break;
      cand = mem;
      cand.push_back(u);
      std::sort(cand.begin(), cand.end());
      const int p = static_cast<int>(cand.size());
      const std::vector<double> E = patch_energy(A, cand, energy);
      std::vector<double> w, Z;
      dense::sym_eig(p, E.data(), w, &Z);
      bool ok = false;
      std::vector<double> R;
      const std::vector<double> Ab = patch_energy(A, cand, Energy::Closed);
      if (w[1] > 0.0 && dense::cholesky_upper(p, Ab.data(), R)) {
        const double eps = 1.0 / w[1];
        // phi^T Abar^-1 phi by Cholesky of the principal submatrix
        std::vector<double> y(p);
        for (int i = 0; i < p; ++i) {  // R^T y = phi
          double t = Z[(size_t)i * p];
          for (int j = 0; j < i; ++j) t -= R[(size_t)j * p + i] * y[j];
          y[i] = t / R[(size_t)i * p + i];
        }
        double q = 0.0;
        for (int i = 0; i < p; ++i) q += y[i] * y[i];
        const double delta = 1.0 / q;
        ok = eps <= eps_k && eps * delta <= cbound;
      }
      if (ok) {
        mem.push_back(u);
        pid[u] = cur;
        add_couplings(u);
      } else {
        refused[u] = cur;
      }
    }
    std::sort(mem.begin(), mem.end());
    P.push_back(std::move(mem));
  }
  return P;
}

// ---------------------------------------------------------------- sparse helpers
// Remove stored entries that are exactly zero (a basis vector's support is the
// set of its nonzero entries, so no coupling is derived from a stored zero).
void drop_zeros(HostCSR& X) {
  int64_t q = 0;
  for (int i = 0; i < X.n_rows; ++i) {
    const int64_t b = X.ptr[i], e = X.ptr[i + 1];
    X.ptr[i] = q;
    for (int64_t k = b; k < e; ++k)
      if (X.val[k] != 0.0) {
        X.col[q] = X.col[k];
        X.val[q] = X.val[k];
        ++q;
      }
  }
  X.ptr[X.n_rows] = q;
  X.col.resize(q);
  X.val.resize(q);
}

HostCSR transpose(const HostCSR& X) {
  HostCSR T;
  T.n_rows = X.n_cols;
  T.n_cols = X.n_rows;
  T.ptr.assign(T.n_rows + 1, 0);
  for (int64_t k = 0; k < X.nnz(); ++k) T.ptr[X.col[k] + 1]++;
  for (int i = 0; i < T.n_rows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(X.nnz());
  T.val.resize(X.nnz());
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int i = 0; i < X.n_rows; ++i)
    for (int64_t k = X.ptr[i]; k < X.ptr[i + 1]; ++k) {
      const int64_t q = pos[X.col[k]]++;
      T.col[q] = i;
      T.val[q] = X.val[k];
    }
  return T;
}

// Z = X * Y with the structural pattern (every touched column is kept).
HostCSR spgemm(const HostCSR& X, const HostCSR& Y) {
  HostCSR Z;
  Z.n_rows = X.n_rows;
  Z.n_cols = Y.n_cols;
  const int nr = X.n_rows;
  std::vector<std::vector<int>> rc(nr);
  std::vector<std::vector<double>> rv(nr);
#pragma omp parallel
  {
    std::vector<double> acc(Y.n_cols, 0.0);
    std::vector<char> mark(Y.n_cols, 0);
    std::vector<int> cols;
#pragma omp for schedule(dynamic, 64)
    for (int i = 0; i < nr; ++i) {
      cols.clear();
      for (int64_t k = X.ptr[i]; k < X.ptr[i + 1]; ++k) {
        const int r = X.col[k];
        const double xv = X.val[k];
        for (int64_t q = Y.ptr[r]; q < Y.ptr[r + 1]; ++q) {
          const int c = Y.col[q];
          if (!mark[c]) {
            mark[c] = 1;
            cols.push_back(c);
          }
          acc[c] += xv * Y.val[q];
        }
      }
      std::sort(cols.begin(), cols.end());
      rc[i] = cols;
      rv[i].resize(cols.size());
      for (size_t t = 0; t < cols.size(); ++t) {
        rv[i][t] = acc[cols[t]];
        acc[cols[t]] = 0.0;
        mark[cols[t]] = 0;
      }
    }
  }
  Z.ptr.assign(nr + 1, 0);
  for (int i = 0; i < nr; ++i) Z.ptr[i + 1] = Z.ptr[i] + static_cast<int64_t>(rc[i].size());
  Z.col.resize(Z.ptr[nr]);
  Z.val.resize(Z.ptr[nr]);
  for (int i = 0; i < nr; ++i) {
    std::copy(rc[i].begin(), rc[i].end(), Z.col.begin() + Z.ptr[i]);
    std::copy(rv[i].begin(), rv[i].end(), Z.val.begin() + Z.ptr[i]);
  }
  return Z;
}

// 0.5 (C + C^T) on C's (structurally symmetric) pattern.
void symmetrize(HostCSR& C) {
  std::vector<double> out(C.val.size());
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < C.n_rows; ++i)
    for (int64_t k = C.ptr[i]; k < C.ptr[i + 1]; ++k) {
      const int j = C.col[k];
      auto b = C.col.begin() + C.ptr[j], e = C.col.begin() + C.ptr[j + 1];
      auto it = std::lower_bound(b, e, i);
      const double cji = (it != e && *it == i) ? C.val[it - C.col.begin()] : 0.0;
      out[k] = 0.5 * (C.val[k] + cji);
    }
  C.val.swap(out);
}

// Psi^T X Psi (X == nullptr: identity), symmetrised.
HostCSR galerkin(const HostCSR& Psi, const HostCSR* X) {
  HostCSR Pt = transpose(Psi);
  HostCSR C = X ? spgemm(Pt, spgemm(*X, Psi)) : spgemm(Pt, Psi);
  symmetrize(C);
  return C;
}

double gershgorin(const HostCSR& M) {
  double best = 0.0;
  for (int i = 0; i < M.n_rows; ++i) {
    double s = 0.0;
    for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) s += std::fabs(M.val[k]);
    best = std::max(best, s);
  }
  return best;
}

// dense principal submatrix A[S, S] (S sorted)
void dense_sub(const HostCSR& A, const std::vector<int>& S, std::vector<double>& D) {
  const int m = static_cast<int>(S.size());
  D.assign((size_t)m * m, 0.0);
  for (int a = 0; a < m; ++a) {
    const int i = S[a];
    int64_t k = A.ptr[i];
    const int64_t ke = A.ptr[i + 1];
    int b = 0;
    while (k < ke && b < m) {  // merge of two sorted lists
      if (A.col[k] == S[b]) {
        D[(size_t)a * m + b] = A.val[k];
        ++k;
        ++b;
      } else if (A.col[k] < S[b]) {
        ++k;
      } else {
        ++b;
      }
    }
  }
}

// solve (R^T R) X = B in place for nrhs columns of the row-major m x nrhs B
void chol_solve(int m, const std::vector<double>& R, double* B, int nrhs) {
  // R^T y = b, then R x = y, for all right-hand sides at once (rows of B are
  // contiguous over the right-hand sides)
  for (int i = 0; i < m; ++i) {
    double* bi = B + (size_t)i * nrhs;
    const double inv = 1.0 / R[(size_t)i * m + i];
    for (int c = 0; c < nrhs; ++c) bi[c] *= inv;
    for (int k = i + 1; k < m; ++k) {
      const double f = R[(size_t)i * m + k];
      if (f == 0.0) continue;
      double* bk = B + (size_t)k * nrhs;
      for (int c = 0; c < nrhs; ++c) bk[c] -= f * bi[c];
    }
  }
  for (int i = m - 1; i >= 0; --i) {
    double* bi = B + (size_t)i * nrhs;
    for (int k = i + 1; k < m; ++k) {
      const double f = R[(size_t)i * m + k];
      if (f == 0.0) continue;
      const double* bk = B + (size_t)k * nrhs;
      for (int c = 0; c < nrhs; ++c) bi[c] -= f * bk[c];
    }
    const double inv = 1.0 / R[(size_t)i * m + i];
    for (int c = 0; c < nrhs; ++c) bi[c] *= inv;
  }
}

// ---------------------------------------------------------------- Psi
HostCSR psi_exact(const HostCSR& A, const Patches& P, const std::vector<double>& phi,
                  const std::vector<int>& pptr) {
  const int n = A.n_rows, m = static_cast<int>(P.size());
  std::vector<int> all(n);
  std::iota(all.begin(), all.end(), 0);
  std::vector<double> D;
  dense_sub(A, all, D);
  std::vector<double> R;
  MMD_REQUIRE(dense::cholesky_upper(n, D.data(), R), MMD_ENOTSPD, "level matrix not SPD");
  std::vector<double> Y((size_t)n * m, 0.0);
  for (int j = 0; j < m; ++j)
    for (size_t t = 0; t < P[j].size(); ++t) Y[(size_t)P[j][t] * m + j] = phi[pptr[j] + t];
  std::vector<double> Phi = Y;
  chol_solve(n, R, Y.data(), m);
  std::vector<double> G((size_t)m * m, 0.0);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      double s = 0.0;
      for (size_t t = 0; t < P[a].size(); ++t)
        s += phi[pptr[a] + t] * Y[(size_t)P[a][t] * m + b];
      G[(size_t)a * m + b] = s;
    }
  for (int a = 0; a < m; ++a)
    for (int b = a + 1; b < m; ++b) {
      const double v = 0.5 * (G[(size_t)a * m + b] + G[(size_t)b * m + a]);
      G[(size_t)a * m + b] = G[(size_t)b * m + a] = v;
    }
  std::vector<double> RG;
  MMD_REQUIRE(dense::cholesky_upper(m, G.data(), RG), MMD_ENOTSPD, "Phi^T A^-1 Phi not SPD");
  // Psi = Y G^-1 : rows of Psi^T = G^-1 Y^T -> solve G Z = Y^T (columns = rows of Y)
  std::vector<double> Yt((size_t)m * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) Yt[(size_t)j * n + i] = Y[(size_t)i * m + j];
  chol_solve(m, RG, Yt.data(), n);
  HostCSR Psi;
  Psi.n_rows = n;
  Psi.n_cols = m;
  Psi.ptr.resize(n + 1);
  Psi.col.resize((size_t)n * m);
  Psi.val.resize((size_t)n * m);
  for (int i = 0; i <= n; ++i) Psi.ptr[i] = (int64_t)i * m;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      Psi.col[(size_t)i * m + j] = j;
      Psi.val[(size_t)i * m + j] = Yt[(size_t)j * n + i];
    }
  (void)Phi;
  return Psi;
}

HostCSR psi_localized(const HostCSR& A, const Patches& P, const std::vector<double>& phi,
                      const std::vector<int>& pptr, int r_hops) {
  const int n = A.n_rows, m = static_cast<int>(P.size());
  std::vector<int> pid(n);
  for (int j = 0; j < m; ++j)
    for (int v : P[j]) pid[v] = j;
  std::vector<std::vector<int>> nbr(m);
#pragma omp parallel for schedule(dynamic, 64)
  for (int j = 0; j < m; ++j) {
    std::vector<int> s;
    for (int v : P[j])
      for (int64_t k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
        const int q = pid[A.col[k]];
        if (q != j) s.push_back(q);
      }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    nbr[j] = std::move(s);
  }
  std::vector<std::vector<int>> cols(m);  // support rows of column j
  std::vector<std::vector<double>> vals(m);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : bad)
  for (int j = 0; j < m; ++j) {
    // patches within r hops
    std::vector<int> C{j}, frontier{j};
    std::vector<int> seen{j};
    for (int h = 0; h < r_hops; ++h) {
      std::vector<int> nxt;
      for (int a : frontier)
        for (int b : nbr[a])
          if (std::find(seen.begin(), seen.end(), b) == seen.end()) {
            seen.push_back(b);
            nxt.push_back(b);
          }
      frontier.swap(nxt);
    }
    C = seen;
    std::sort(C.begin(), C.end());
    std::vector<int> S;
    for (int a : C) S.insert(S.end(), P[a].begin(), P[a].end());
    std::sort(S.begin(), S.end());
    const int ms = static_cast<int>(S.size()), mc = static_cast<int>(C.size());
    std::vector<double> D;
    dense_sub(A, S, D);
    std::vector<double> R;
    if (!dense::cholesky_upper(ms, D.data(), R)) {
      bad += 1;
      continue;
    }
    std::vector<double> Y((size_t)ms * mc, 0.0);
    for (int b = 0; b < mc; ++b) {
      const int a = C[b];
      for (size_t t = 0; t < P[a].size(); ++t) {
        const int pos = static_cast<int>(std::lower_bound(S.begin(), S.end(), P[a][t]) - S.begin());
        Y[(size_t)pos * mc + b] = phi[pptr[a] + t];
      }
    }
    std::vector<double> PhiC = Y;
    chol_solve(ms, R, Y.data(), mc);
    std::vector<double> G((size_t)mc * mc, 0.0);  // G = PhiC^T Y, row updates
    for (int i = 0; i < ms; ++i) {
      const double* yi = Y.data() + (size_t)i * mc;
      for (int a = 0; a < mc; ++a) {
        const double f = PhiC[(size_t)i * mc + a];
        if (f == 0.0) continue;
        double* ga = G.data() + (size_t)a * mc;
        for (int b = 0; b < mc; ++b) ga[b] += f * yi[b];
      }
    }
    for (int a = 0; a < mc; ++a)
      for (int b = a + 1; b < mc; ++b) {
        const double v = 0.5 * (G[(size_t)a * mc + b] + G[(size_t)b * mc + a]);
        G[(size_t)a * mc + b] = G[(size_t)b * mc + a] = v;
      }
    std::vector<double> RG;
    if (!dense::cholesky_upper(mc, G.data(), RG)) {
      bad += 1;
      continue;
    }
    std::vector<double> e(mc, 0.0);
    e[std::lower_bound(C.begin(), C.end(), j) - C.begin()] = 1.0;
    chol_solve(mc, RG, e.data(), 1);
    std::vector<double> psi(ms, 0.0);
    for (int i = 0; i < ms; ++i) {
      double s = 0.0;
      for (int b = 0; b < mc; ++b) s += Y[(size_t)i * mc + b] * e[b];
      psi[i] = s;
    }
    cols[j] = std::move(S);
    vals[j] = std::move(psi);
  }
  MMD_REQUIRE(bad == 0, MMD_ENOTSPD, "local KKT system not positive definite");
  // assemble column lists into CSR (rows = fine dofs)
  HostCSR PsiT;
  PsiT.n_rows = m;
  PsiT.n_cols = n;
  PsiT.ptr.assign(m + 1, 0);
  for (int j = 0; j < m; ++j) PsiT.ptr[j + 1] = PsiT.ptr[j] + static_cast<int64_t>(cols[j].size());
  PsiT.col.resize(PsiT.ptr[m]);
  PsiT.val.resize(PsiT.ptr[m]);
  for (int j = 0; j < m; ++j) {
    std::copy(cols[j].begin(), cols[j].end(), PsiT.col.begin() + PsiT.ptr[j]);
    std::copy(vals[j].begin(), vals[j].end(), PsiT.val.begin() + PsiT.ptr[j]);
  }
  return transpose(PsiT);
}

}  // namespace

// Renumber level 0 patch-major: patches in reverse Cuthill-McKee order of the
// patch graph, members ascending.  The SpMM gathers of level 0 then touch
// nearby rows (L2 reuse) and every patch is a contiguous index range; patch
// ids (the level-1 numbering) do not change.  The first-level patches are
// rewritten in the new numbering; the caller's numbering is restored at the
// API boundary.
// Reverse Cuthill-McKee order of the patch graph (patches adjacent when an
// entry of A joins them): breadth-first from a pseudo-peripheral patch of each
// component, neighbours by ascending degree, reversed.  Neighbouring patches
// end up close in the order, so the rows a block or an XCD sweeps gather
// from a narrow band of rows.
std::vector<int> patch_rcm(const HostCSR& A, const Patches& P) {
  const int m = static_cast<int>(P.size());
  std::vector<int> pid(A.n_rows);
  for (int j = 0; j < m; ++j)
    for (int v : P[j]) pid[v] = j;
  std::vector<std::vector<int>> adj(m);
#pragma omp parallel for schedule(dynamic, 256)
  for (int j = 0; j < m; ++j) {
    std::vector<int> s;
    for (int v : P[j])
      for (int64_t q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
        const int t = pid[A.col[q]];
        if (t != j) s.push_back(t);
      }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    adj[j] = std::move(s);
  }
  auto deg = [&](int j) { return static_cast<int>(adj[j].size()); };
  std::vector<int> level(m, -1), order;
  order.reserve(m);
  std::vector<char> done(m, 0);
  auto bfs = [&](int root, std::vector<int>& out) {  // plain BFS, returns last level's node
    out.clear();
    out.push_back(root);
    level[root] = 0;
    for (size_t h = 0; h < out.size(); ++h)
      for (int t : adj[out[h]])
        if (level[t] < 0) {
          level[t] = level[out[h]] + 1;
          out.push_back(t);
        }
    int far = out.back();
    for (int v : out) {
      if (level[v] == level[far] && deg(v) < deg(far)) far = v;
      level[v] = -1;
    }
    return far;
  };
  std::vector<int> comp;
  for (int r = 0; r < m; ++r) {
    if (done[r]) continue;
    // pseudo-peripheral start: two sweeps from r
    int a = bfs(r, comp);
    a = bfs(a, comp);
    const size_t first = order.size();
    order.push_back(a);
    done[a] = 1;
    for (size_t h = first; h < order.size(); ++h) {
      std::vector<int> nb;
      for (int t : adj[order[h]])
        if (!done[t]) {
          done[t] = 1;
          nb.push_back(t);
        }
      std::stable_sort(nb.begin(), nb.end(), [&](int x, int y) { return deg(x) < deg(y); });
      order.insert(order.end(), nb.begin(), nb.end());
    }
    std::reverse(order.begin() + first, order.end());
  }
  return order;
}

// Strip order of the patches of a 2-D point set: patch centroids in
// vertical strips about two patch diameters wide, bottom to top and top to
// bottom in alternate strips.  Every neighbour of a row then lies within about
// one and a half strip lengths of it in the order, a band that stays in one
// XCD's L2 while the XCD sweeps its contiguous range of rows.
std::vector<int> patch_strips(const std::vector<double>& xy, const Patches& P) {
  const int m = static_cast<int>(P.size());
  std::vector<double> cx(m), cy(m);
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int j = 0; j < m; ++j) {
    double a = 0.0, b = 0.0;
    for (int v : P[j]) {
      a += xy[2 * (size_t)v];
      b += xy[2 * (size_t)v + 1];
    }
    cx[j] = a / P[j].size();
    cy[j] = b / P[j].size();
    x0 = std::min(x0, cx[j]);
    x1 = std::max(x1, cx[j]);
    y0 = std::min(y0, cy[j]);
    y1 = std::max(y1, cy[j]);
  }
  const double area = std::max((x1 - x0) * (y1 - y0), 1e-300);
  const double w = 2.0 * std::sqrt(area / std::max(m, 1));
  std::vector<int> strip(m), order(m);
  for (int j = 0; j < m; ++j) strip[j] = static_cast<int>((cx[j] - x0) / w);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (strip[a] != strip[b]) return strip[a] < strip[b];
    return (strip[a] & 1) ? cy[a] > cy[b] : cy[a] < cy[b];
  });
  return order;
}

void renumber_level0(mmd_handle& h, Patches& P) {
  LevelHost& L0 = h.host[0];
  const int n = L0.n;
  std::vector<int> perm;
  perm.reserve(n);
  // with coordinates the patches keep their construction order (Morton order
  // of their seeds): a run of consecutive rows is then a compact region, and
  // the tiles of the block SpMM gather few distinct rows; without coordinates
  // reverse Cuthill-McKee keeps neighbouring patches close
  std::vector<int> order;
  const char* env = std::getenv("MMDEIG_L0_ORDER");
  const std::string mode = env ? env : "";
  if (!L0.coords.empty() && L0.cdim == 2 && mode == "strip") {
    order = patch_strips(L0.coords, P);
  } else if (!L0.coords.empty() && mode != "rcm") {
    order.resize(P.size());
    std::iota(order.begin(), order.end(), 0);
  } else {
    order = patch_rcm(L0.A, P);
  }
  for (int j : order) perm.insert(perm.end(), P[j].begin(), P[j].end());
  std::vector<int> iperm(n);
  for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
  h.A_user = L0.A;
  HostCSR B;
  B.n_rows = B.n_cols = n;
  B.ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) B.ptr[i + 1] = B.ptr[i] + (L0.A.ptr[perm[i] + 1] - L0.A.ptr[perm[i]]);
  B.col.resize(L0.A.nnz());
  B.val.resize(L0.A.nnz());
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < n; ++i) {
    const int o = perm[i];
    std::vector<std::pair<int, double>> row;
    for (int64_t q = L0.A.ptr[o]; q < L0.A.ptr[o + 1]; ++q) row.emplace_back(iperm[L0.A.col[q]], L0.A.val[q]);
    std::sort(row.begin(), row.end());
    for (size_t t = 0; t < row.size(); ++t) {
      B.col[B.ptr[i] + t] = row[t].first;
      B.val[B.ptr[i] + t] = row[t].second;
    }
  }
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i) s[i] = L0.s[perm[i]];
  L0.A = std::move(B);
  L0.s = std::move(s);
  if (!L0.coords.empty()) {
    std::vector<double> c(L0.coords.size());
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < L0.cdim; ++a) c[(size_t)i * L0.cdim + a] = L0.coords[(size_t)perm[i] * L0.cdim + a];
    L0.coords = std::move(c);
  }
  for (auto& m : P) {
    for (int& v : m) v = iperm[v];
    std::sort(m.begin(), m.end());
  }
  h.perm = std::move(perm);
}

// ======================================================================= build
void build_hierarchy(mmd_handle& h, const mmd_csr& in, const mmd_build_opts& o) {
  const int levels = o.levels > 0 ? o.levels : (o.levels < 0 ? 0 : 3);
  std::vector<int> targets, blocks;
  if (o.n_targets > 0) targets.assign(o.targets, o.targets + std::min(o.n_targets, 8));
  else targets = {4, 8};
  if (o.n_grid_blocks > 0) blocks.assign(o.grid_blocks, o.grid_blocks + std::min(o.n_grid_blocks, 8));
  else blocks = {4, 2};
  const int r_hops = o.r_hops > 0 ? o.r_hops : 1;
  const int min_coarse = o.min_coarse > 0 ? o.min_coarse : 4;
  MMD_REQUIRE(levels < MMD_MAX_LEVELS, MMD_EINVAL, "too many levels");
  for (int t : targets) MMD_REQUIRE(t >= 2, MMD_EINVAL, "patch target must be >= 2");
  for (int t : blocks) MMD_REQUIRE(t >= 2, MMD_EINVAL, "grid block must be >= 2");

  h.host.clear();
  h.host.emplace_back();
  LevelHost& L0 = h.host[0];
  validate_and_copy(in, L0.A, L0.s);
  L0.n = L0.A.n_rows;
  h.n = L0.n;
  if (in.coords && in.coord_dim > 0) {
    MMD_REQUIRE(in.coord_dim == 2 || in.coord_dim == 3, MMD_EINVAL, "coord_dim must be 2 or 3");
    L0.cdim = in.coord_dim;
    L0.coords.assign(in.coords, in.coords + (size_t)L0.n * in.coord_dim);
  }
  if (in.grid_dim > 0) {
    MMD_REQUIRE(in.grid_dim == 2 || in.grid_dim == 3, MMD_EINVAL, "grid_dim must be 2 or 3");
    int64_t prod = 1;
    for (int a = 0; a < in.grid_dim; ++a) {
      MMD_REQUIRE(in.grid[a] > 0, MMD_EINVAL, "grid extent must be positive");
      prod *= in.grid[a];
    }
    MMD_REQUIRE(prod == L0.n, MMD_EINVAL, "grid shape does not match n");
    L0.grid.assign(in.grid, in.grid + in.grid_dim);
  }
  h.eps.assign(1, 0.0);
  h.perm.clear();
  h.A_user = HostCSR();

  for (int k = 1; k <= levels; ++k) {
    const double t_level = omp_get_wtime();
    const LevelHost& prev = h.host[k - 1];
    const HostCSR& Ak = prev.A;
    Patches P;
    std::vector<int> cgrid;
    if (!prev.grid.empty()) {
      const int blk = blocks[std::min<size_t>(k - 1, blocks.size() - 1)];
      P = grid_patches(prev.grid, blk, cgrid);
    } else if (o.eps1 > 0) {
      const double eta = o.eta > 0 ? o.eta : 0.1;
      const double cb = o.cbound > 0 ? o.cbound : 20.0;
      const int mx = o.max_patch > 0 ? o.max_patch : 32;
      P = eps_patches(Ak, prev.coords, prev.cdim, o.eps1 / std::pow(eta, k - 1), cb,
                      Energy::Split, mx);
    } else {
      const int tgt = targets[std::min<size_t>(k - 1, targets.size() - 1)];
      P = greedy_patches(Ak, prev.coords, prev.cdim, tgt);
    }
    const int np = static_cast<int>(P.size());
    if (np >= prev.n || np < min_coarse) break;
    if (k == 1) renumber_level0(h, P);

    LevelHost L;
    L.n = np;
    L.patch_ptr.assign(np + 1, 0);
    for (int j = 0; j < np; ++j) L.patch_ptr[j + 1] = L.patch_ptr[j] + static_cast<int>(P[j].size());
    L.members.resize(L.patch_ptr[np]);
    for (int j = 0; j < np; ++j) std::copy(P[j].begin(), P[j].end(), L.members.begin() + L.patch_ptr[j]);
    L.phi.assign(L.members.size(), 0.0);
    L.hh_u.assign(L.members.size(), 0.0);
    L.hh_scale.assign(np, 0.0);
    L.eps_patch.assign(np, 0.0);
    const Energy ekind = o.eps1 > 0 ? Energy::Split : k >= 2 ? Energy::Closed : Energy::Interior;
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < np; ++j) {
      const int p = static_cast<int>(P[j].size());
      const int off = L.patch_ptr[j];
      if (p == 1) {
        L.phi[off] = 1.0;
        L.eps_patch[j] = 0.0;
      } else {
        std::vector<double> E = patch_energy(Ak, P[j], ekind);
        std::vector<double> w, Z;
        dense::sym_eig(p, E.data(), w, &Z);
        double sum = 0.0;
        for (int i = 0; i < p; ++i) sum += Z[(size_t)i * p];
        double sg = 1.0;
        if (sum < 0) sg = -1.0;
        else if (sum == 0) {
          for (int i = 0; i < p; ++i)
            if (Z[(size_t)i * p] != 0) {
              sg = Z[(size_t)i * p] < 0 ? -1.0 : 1.0;
              break;
            }
        }
        for (int i = 0; i < p; ++i) L.phi[off + i] = sg * Z[(size_t)i * p];
        L.eps_patch[j] = w[1] > 0 ? 1.0 / w[1] : std::numeric_limits<double>::infinity();
      }
      // Householder pivot: the first i with |phi_i| >= (1 - 1e-8) max |phi|,
      // so the sign choice never rests on an entry that is zero up to
      // rounding, and maxima that symmetry makes equal do not let rounding
      // pick among them.  Slot order of the transfer: the pivot first, then
      // the other members ascending; phi keeps the ascending member order.
      double amax = 0.0;
      for (int i = 0; i < p; ++i) amax = std::max(amax, std::fabs(L.phi[off + i]));
      int t = 0;
      while (t < p - 1 && !(std::fabs(L.phi[off + t]) >= (1.0 - 1e-8) * amax)) ++t;
      const double s_piv = L.phi[off + t] >= 0 ? 1.0 : -1.0;
      double uu = 0.0;
      for (int i = 0; i < p; ++i) {
        const double u = L.phi[off + i] + (i == t ? s_piv : 0.0);
        uu += u * u;
      }
      L.members[off] = P[j][t];
      L.hh_u[off] = L.phi[off + t] + s_piv;
      for (int i = 0, q = 1; i < p; ++i) {
        if (i == t) continue;
        L.members[off + q] = P[j][i];
        L.hh_u[off + q] = L.phi[off + i];
        ++q;
      }
      L.hh_scale[j] = 2.0 / uu;
    }
    L.eps_level = 0.0;
    for (double e : L.eps_patch) L.eps_level = std::max(L.eps_level, e);
    if (prev.n <= o.exact_max_n)
      L.Psi = psi_exact(Ak, P, L.phi, L.patch_ptr);
    else
      L.Psi = psi_localized(Ak, P, L.phi, L.patch_ptr,
                            k >= 2 && o.r_hops_coarse > 0 ? o.r_hops_coarse : r_hops);
    drop_zeros(L.Psi);
    L.A = galerkin(L.Psi, &Ak);
    L.M = galerkin(L.Psi, k == 1 ? nullptr : &prev.M);
    L.lam_max_M = gershgorin(L.M);
    if (prev.cdim > 0) {
      L.cdim = prev.cdim;
      L.coords.assign((size_t)np * prev.cdim, 0.0);
      for (int j = 0; j < np; ++j) {
        for (int a = 0; a < prev.cdim; ++a) {
          double s = 0.0;
          for (int v : P[j]) s += prev.coords[(size_t)v * prev.cdim + a];
          L.coords[(size_t)j * prev.cdim + a] = s / static_cast<double>(P[j].size());
        }
      }
    }
    L.grid = cgrid;
    if (const char* e = std::getenv("MMDEIG_LOG"))
      if (std::atoi(e) != 0)
        std::fprintf(stderr, "[mmd_build] level %d: %d -> %d dofs, nnz(A) %lld, eps %.4g, %.2f s\n",
                     k, prev.n, np, static_cast<long long>(L.A.nnz()), L.eps_level,
                     omp_get_wtime() - t_level);
    h.host.push_back(std::move(L));
    h.eps.push_back(h.eps.back() + h.host.back().eps_level);
  }
  h.K = static_cast<int>(h.host.size()) - 1;
}

namespace {
void upload_csr(const HostCSR& X, DBuf<int>& ptr, DBuf<int>& col, DBuf<double>& val,
                CsrView& v, hipStream_t s) {
  MMD_REQUIRE(X.nnz() < (int64_t(1) << 31), MMD_EINVAL, "level operator exceeds 2^31 entries");
  std::vector<int> p32(X.ptr.begin(), X.ptr.end());
  ptr.upload(p32, s);
  col.upload(X.col, s);
  val.upload(X.val, s);
  v.n_rows = X.n_rows;
  v.n_cols = X.n_cols;
  v.nnz = X.nnz();
  v.rowptr = ptr.p;
  v.col = col.p;
  v.val = val.p;
  v.diag = nullptr;
  v.avg_row = X.n_rows ? static_cast<double>(X.nnz()) / X.n_rows : 1.0;
}
}  // namespace

// Row-block tiling of the level-0 edge form for the LDS-staged block SpMM:
// per block of consecutive rows, the distinct rows of X its entries gather
// (own rows first) and each entry's position in that list.  Rows are grouped
// greedily, a block closing before the row that would take it past the
// shape's rows, distinct touched rows (own rows and columns) or entries.  A
// row that alone exceeds a cap leaves the level untiled for that shape.
struct TileSet {
  std::vector<int> trow, uptr, urow;
  std::vector<unsigned short> lcol;
  int nblk = 0;
  bool ok = false;
};

TileSet make_tiles(const HostCSR& W, const TileShape& sh) {
  TileSet T;
  const int n = W.n_rows;
  std::vector<int> trow{0}, stamp(n, -1);
  {
    int r0 = 0, touched = 0, tile = 0;
    int64_t ents = 0;
    auto count_new = [&](int r) {  // distinct rows row r adds to the current tile
      int c = stamp[r] != tile ? 1 : 0;
      for (int64_t q = W.ptr[r]; q < W.ptr[r + 1]; ++q)
        if (stamp[W.col[q]] != tile) ++c;
      return c;
    };
    for (int r = 0; r < n; ++r) {
      int c = count_new(r);
      const int64_t e = W.ptr[r + 1] - W.ptr[r];
      if (r > r0 && (r - r0 >= sh.rows || touched + c > sh.cols || ents + e > sh.nnz)) {
        trow.push_back(r);
        ++tile;
        r0 = r;
        touched = 0;
        ents = 0;
        c = count_new(r);
      }
      if (c > sh.cols || e > sh.nnz) return T;  // one row alone exceeds a cap
      stamp[r] = tile;
      for (int64_t q = W.ptr[r]; q < W.ptr[r + 1]; ++q) stamp[W.col[q]] = tile;
      touched += c;
      ents += e;
    }
    trow.push_back(n);
  }
  const int nblk = static_cast<int>(trow.size()) - 1;
  std::vector<std::vector<int>> urows(nblk);
  std::vector<unsigned short> lcol(W.nnz());
#pragma omp parallel for schedule(dynamic, 64)
  for (int t = 0; t < nblk; ++t) {
    const int r0 = trow[t], r1 = trow[t + 1];
    std::vector<int> halo;
    for (int64_t q = W.ptr[r0]; q < W.ptr[r1]; ++q)
      if (W.col[q] < r0 || W.col[q] >= r1) halo.push_back(W.col[q]);
    std::sort(halo.begin(), halo.end());
    halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
    const int own = r1 - r0;
    std::vector<int>& u = urows[t];
    for (int i = r0; i < r1; ++i) u.push_back(i);
    u.insert(u.end(), halo.begin(), halo.end());
    for (int64_t q = W.ptr[r0]; q < W.ptr[r1]; ++q) {
      const int c = W.col[q];
      const int pos = (c >= r0 && c < r1)
                          ? c - r0
                          : own + static_cast<int>(std::lower_bound(halo.begin(), halo.end(), c) -
                                                   halo.begin());
      lcol[q] = static_cast<unsigned short>(pos);
    }
  }
  std::vector<int> uptr(nblk + 1, 0), urow;
  for (int t = 0; t < nblk; ++t) {
    // the grouping above guarantees the caps; a block that broke one would
    // overrun the kernel's LDS arrays, so the shape would not be used
    if (static_cast<int>(urows[t].size()) > sh.cols ||
        W.ptr[trow[t + 1]] - W.ptr[trow[t]] > sh.nnz || trow[t + 1] - trow[t] > sh.rows)
      return T;
    uptr[t + 1] = uptr[t] + static_cast<int>(urows[t].size());
  }
  urow.reserve(uptr[nblk]);
  for (auto& u : urows) urow.insert(urow.end(), u.begin(), u.end());
  T.trow = std::move(trow);
  T.uptr = std::move(uptr);
  T.urow = std::move(urow);
  T.lcol = std::move(lcol);
  T.nblk = nblk;
  T.ok = true;
  return T;
}

void install_tiles(const TileSet& T, int kind, LevelDev& D, hipStream_t s) {
  D.t_row.upload(T.trow, s);
  D.t_uptr.upload(T.uptr, s);
  D.t_urow.upload(T.urow, s);
  D.t_lcol.upload(T.lcol, s);
  D.A.t_kind = kind;
  D.A.t_row = D.t_row.p;
  D.A.t_uptr = D.t_uptr.p;
  D.A.t_urow = D.t_urow.p;
  D.A.t_lcol = D.t_lcol.p;
  D.A.t_nblk = T.nblk;
  MMD_HIP(hipStreamSynchronize(s));  // the host lists must outlive their copies
}

// Build-time autotuning of the tile shape: every shape whose tiling exists is
// installed in turn and timed with HIP events on the level-0 block-CG step
// with the folded update (k_cg_tile) at 256 columns (one warm-up and three
// timed launches on zero data; the kernels' time does not depend on the
// values), and the fastest is kept.
// MMDEIG_TILE=<k> forces shape k.
void build_tiles(const HostCSR& W, LevelDev& D, hipStream_t s) {
  const int n = W.n_rows;
  int forced = -1;
  if (const char* e = std::getenv("MMDEIG_TILE")) {
    if (e[0]) forced = std::atoi(e);
  }
  std::vector<TileSet> sets(kNumTileShapes);
  std::vector<int> cand;
  for (int k = 0; k < kNumTileShapes; ++k) {
    if (forced >= 0 && k != forced) continue;
    sets[k] = make_tiles(W, kTileShapes[k]);
    if (sets[k].ok) cand.push_back(k);
  }
  if (cand.empty()) return;
  std::vector<double> us(kNumTileShapes, -1.0);
  int best = cand[0];
  if (cand.size() > 1) {
    // the kernel timed is the one the level-0 block CG spends its time in:
    // the step with the previous update folded in (the plain fused SpMM when
    // tiles are switched off for it)
    const int b = 256;
    const size_t nb = (size_t)n * b;
    DBuf<double> X(nb), R(nb), Q(nb), Ra(nb), Qa(nb), P(nb), alpha(b), beta(b),
        part((size_t)4 * kRedBlocks * b);
    for (DBuf<double>* v : {&X, &R, &Q, &Ra, &Qa, &P})
      MMD_HIP(hipMemsetAsync(v->p, 0, sizeof(double) * nb, s));
    MMD_HIP(hipMemsetAsync(alpha.p, 0, sizeof(double) * b, s));
    MMD_HIP(hipMemsetAsync(beta.p, 0, sizeof(double) * b, s));
    auto step = [&]() {
      if (cg_tile_ok(D.A))
        cg_tile_step(D.A, X.p, b, R.p, Q.p, Ra.p, Qa.p, P.p, b, b, true, false, alpha.p, beta.p,
                     part.p, (size_t)kRedBlocks * b, s);
      else
        spmm(D.A, R.p, b, Q.p, b, b, s, true, false, beta.p, P.p, b, part.p);
    };
    hipEvent_t e0, e1;
    MMD_HIP(hipEventCreate(&e0));
    MMD_HIP(hipEventCreate(&e1));
    for (int k : cand) {
      install_tiles(sets[k], k, D, s);
      step();
      MMD_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) step();
      MMD_HIP(hipEventRecord(e1, s));
      MMD_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      MMD_HIP(hipEventElapsedTime(&ms, e0, e1));
      us[k] = 1000.0 * ms / 3.0;
    }
    best = cand[0];
    for (int k : cand)
      if (us[k] < us[best]) best = k;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  install_tiles(sets[best], best, D, s);
  const char* e = std::getenv("MMDEIG_LOG");
  if (e && std::atoi(e) != 0) {
    std::fprintf(stderr, "[mmd_build] level-0 tile shapes (rows x staged rows, us per 256-column step):");
    for (int k = 0; k < kNumTileShapes; ++k)
      if (us[k] >= 0) std::fprintf(stderr, " %dx%d %.1f", kTileShapes[k].rows, kTileShapes[k].cols, us[k]);
    const TileSet& T = sets[best];
    std::fprintf(stderr, "; using %dx%d: %d blocks, %.1f rows and %.1f staged rows per block\n",
                 kTileShapes[best].rows, kTileShapes[best].cols, T.nblk,
                 static_cast<double>(n) / T.nblk, static_cast<double>(T.uptr[T.nblk]) / T.nblk);
  }
}

void upload_hierarchy(mmd_handle& h, hipStream_t s) {
  h.dev.clear();
  h.dev.resize(h.host.size());
  if (!h.perm.empty()) h.d_perm.upload(h.perm, s);
  // level 0: edge form (off-diagonal weights w = -a_ij and self-loops s)
  {
    const LevelHost& L0 = h.host[0];
    LevelDev& D0 = h.dev[0];
    HostCSR W;
    W.n_rows = W.n_cols = L0.n;
    W.ptr.assign(L0.n + 1, 0);
    for (int i = 0; i < L0.n; ++i) {
      int64_t c = 0;
      for (int64_t k = L0.A.ptr[i]; k < L0.A.ptr[i + 1]; ++k)
        if (L0.A.col[k] != i) ++c;
      W.ptr[i + 1] = W.ptr[i] + c;
    }
    W.col.reserve(W.ptr[L0.n]);
    W.val.reserve(W.ptr[L0.n]);
    for (int i = 0; i < L0.n; ++i)
      for (int64_t k = L0.A.ptr[i]; k < L0.A.ptr[i + 1]; ++k)
        if (L0.A.col[k] != i) {
          W.col.push_back(L0.A.col[k]);
          W.val.push_back(-L0.A.val[k]);
        }
    upload_csr(W, D0.a_ptr, D0.a_col, D0.a_val, D0.A, s);
    D0.a_diag.upload(L0.s, s);
    D0.A.diag = D0.a_diag.p;
    D0.A.avg_row = static_cast<double>(L0.A.nnz()) / L0.n;
    build_tiles(W, D0, s);
  }
  for (size_t k = 1; k < h.host.size(); ++k) {
    const LevelHost& L = h.host[k];
    LevelDev& D = h.dev[k];
    upload_csr(L.A, D.a_ptr, D.a_col, D.a_val, D.A, s);
    upload_csr(L.M, D.m_ptr, D.m_col, D.m_val, D.M, s);
    upload_csr(L.Psi, D.p_ptr, D.p_col, D.p_val, D.Psi, s);
    D.h_ptr.upload(L.patch_ptr, s);
    D.h_mem.upload(L.members, s);
    D.h_u.upload(L.hh_u, s);
    D.h_scale.upload(L.hh_scale, s);
    D.H.npatch = L.n;
    D.H.nfine = h.host[k - 1].n;
    D.H.nred = h.host[k - 1].n - L.n;
    D.H.ptr = D.h_ptr.p;
    D.H.members = D.h_mem.p;
    D.H.u = D.h_u.p;
    D.H.scale = D.h_scale.p;
  }
  MMD_HIP(hipStreamSynchronize(s));
}

}  // namespace mmd
