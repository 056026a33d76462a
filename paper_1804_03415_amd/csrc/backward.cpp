// Eigen-backward: gradient of a loss of the nev leftmost eigenpairs with
// respect to the stored entries of A (first-order perturbation of a symmetric
// matrix; the paper gives no derivative).
//
//   S = sum_k g_lambda_k v_k v_k^T - sum_k (x_k v_k^T + v_k x_k^T) / 2
//   x_k = sum_{j != k} v_j (v_j^T g_k) / (lambda_j - lambda_k)
//         + [(A - lambda_k I) on V-perp]^-1 (I - V V^T) g_k
//
// The first part of x_k is a small dense product with V; the second is a
// block CG on the complement of the computed eigenvectors (SPD there since
// lambda_k < lambda_{nev+1}), shifted per column.  S is evaluated only on the
// caller's stored pattern (sampled dense-dense product).
#include <algorithm>
#include <cmath>
#include <vector>

#include "solver.h"

namespace mmd {

void Solver::cg_shift_defl(const double* Rhs, double* Y, int b, const double* shift_neg,
                           const double* V, int nev, double tol) {
  const int n = nlev(0);
  ColScalars sc = make_scalars(pool_, "bw", b);
  double* R = pool_.d("bw:R", (size_t)n * b);
  double* P = pool_.d("bw:P", (size_t)n * b);
  double* Q = pool_.d("bw:Q", (size_t)n * b);
  double* p1 = pool_.d("bw:p1", (size_t)kRedBlocks * b);
  double* p2 = pool_.d("bw:p2", (size_t)kRedBlocks * b);
  double* W = pool_.d("bw:W", (size_t)nev * b);
  double* gw = pool_.d("bw:gw", gram_work_size(n, nev, b));
  copy_block(Rhs, b, R, b, n, b, s_);
  zero_block(Y, b, n, b, s_);
  const int nb = col_dot(R, b, R, b, n, b, p1, s_);
  cg_init(sc, p1, nullptr, nb, b, tol, nullptr, s_);
  MMD_HIP(hipMemsetAsync(sc.notspd, 0, sizeof(int), s_));
  auto project = [&](double* Z) {  // Z -= V (V^T Z)
    gram(V, nev, Z, b, n, nev, b, W, b, gw, s_);
    gemm_nn(V, nev, W, b, Z, b, n, nev, b, -1.0, 1.0, s_);
  };
  auto iterate = [&](bool first) {
    xpay(R, b, P, b, n, b, sc.beta, first, s_);
    applyA(0, P, b, Q, b, b);
    scale_cols(P, b, shift_neg, Q, b, n, b, true, s_);  // Q = (A - shift) P
    project(Q);
    const int np = col_dot(P, b, Q, b, n, b, p1, s_);
    cg_alpha(sc, p1, np, b, s_);
    const int nu = cg_update(Y, b, R, P, Q, b, n, b, sc.alpha, p2, s_);
    cg_beta(sc, p2, nu, b, s_);
  };
  const int maxit = 100000;
  int done = 0, chunk = 4;
  bool first = true;
  while (true) {
    for (int t = 0; t < chunk; ++t) {
      iterate(first);
      first = false;
    }
    done += chunk;
    hi_.ensure(b + 1);
    d2h(hi_.p, sc.active, b);
    d2h(hi_.p + b, sc.notspd, 1);
    sync();
    MMD_REQUIRE(hi_.p[b] == 0, MMD_ENOTSPD,
                "eigen-backward: the shifted operator is not positive on the complement "
                "(eigenpairs not the leftmost ones, or not converged)");
    bool any = false;
    for (int c = 0; c < b; ++c) any |= hi_.p[c] != 0;
    if (!any) break;
    MMD_REQUIRE(done < maxit, MMD_ENOCONV, "eigen-backward CG reached the iteration cap");
    chunk = std::min(chunk * 2, 64);
  }
  project(Y);
}

void Solver::backward(int nev, const double* evals, const double* evecs, const double* g_evals,
                      const double* g_evecs, double tol, double* g_vals) {
  const int n = nlev(0);
  MMD_REQUIRE(nev >= 1 && nev < n, MMD_EINVAL, "nev must be in [1, n)");
  MMD_REQUIRE(tol > 0 && tol < 1, MMD_EINVAL, "tol must be in (0, 1)");
  for (int k = 0; k < nev; ++k)
    MMD_REQUIRE(std::isfinite(evals[k]), MMD_EINVAL, "non-finite eigenvalue");
  const int* perm = h_.perm.empty() ? nullptr : h_.d_perm.p;
  // V, G in the internal (renumbered) row-major layout, ld = nev
  double* V = pool_.d("bw:V", (size_t)n * nev);
  from_colmajor(evecs, n, nev, perm, V, nev, s_);
  double* X = nullptr;
  if (g_evecs) {
    double* G = pool_.d("bw:G", (size_t)n * nev);
    from_colmajor(g_evecs, n, nev, perm, G, nev, s_);
    // C = V^T G (C[j, k] = v_j^T g_k) and the column norms of G
    double* C = pool_.d("bw:C", (size_t)nev * nev);
    double* gw = pool_.d("bw:gwc", gram_work_size(n, nev, nev));
    gram(V, nev, G, nev, n, nev, nev, C, nev, gw, s_);
    double* part = pool_.d("bw:part", (size_t)kRedBlocks * nev);
    double* gn = pool_.d("bw:gn", nev);
    const int g = col_dot(G, nev, G, nev, n, nev, part, s_);
    reduce_partials(part, g, nev, gn, s_);
    std::vector<double> Ch((size_t)nev * nev), gn2(nev);
    d2h(Ch.data(), C, Ch.size());
    d2h(gn2.data(), gn, nev);
    sync();
    // in-span coefficients D[j, k] = C[j, k] / (lambda_j - lambda_k), j != k
    std::vector<double> Dh((size_t)nev * nev, 0.0);
    for (int k = 0; k < nev; ++k) {
      if (!(gn2[k] > 0.0)) continue;
      for (int j = 0; j < nev; ++j) {
        if (j == k) continue;
        const double c = Ch[(size_t)j * nev + k];
        const double gap = evals[j] - evals[k];
        if (std::fabs(gap) <= 1e-10 * std::fabs(evals[k])) {
          MMD_REQUIRE(std::fabs(c) <= 1e-12 * std::sqrt(gn2[k]), MMD_EINVAL,
                      "eigen-backward: repeated eigenvalue with a coupled eigenvector "
                      "adjoint (the gradient is undefined)");
          continue;
        }
        Dh[(size_t)j * nev + k] = c / gap;
      }
    }
    X = pool_.d("bw:X", (size_t)n * nev);
    double* Dd = pool_.d("bw:D", (size_t)nev * nev);
    h2d(Dd, Dh.data(), Dh.size());
    gemm_nn(V, nev, Dd, nev, X, nev, n, nev, nev, 1.0, 0.0, s_);
    // complement right-hand sides G - V C, solved on V-perp
    gemm_nn(V, nev, C, nev, G, nev, n, nev, nev, -1.0, 1.0, s_);
    std::vector<double> sh(nev);
    for (int k = 0; k < nev; ++k) sh[k] = -evals[k];
    double* shd = pool_.d("bw:sh", nev);
    h2d(shd, sh.data(), nev);
    double* Yc = pool_.d("bw:Y", (size_t)n * nev);
    sync();  // host arrays above must outlive their copies
    cg_shift_defl(G, Yc, nev, shd, V, nev, tol);
    axpby(1.0, Yc, nev, 1.0, X, nev, n, nev, s_);
  }
  // factors back to the caller's numbering for the sampled product
  const double* Vu = V;
  const double* Xu = X;
  if (perm) {
    double* V2 = pool_.d("bw:Vu", (size_t)n * nev);
    permute_rows(V, nev, V2, nev, n, nev, perm, true, s_);
    Vu = V2;
    if (X) {
      double* X2 = pool_.d("bw:Xu", (size_t)n * nev);
      permute_rows(X, nev, X2, nev, n, nev, perm, true, s_);
      Xu = X2;
    }
  }
  const HostCSR& U = h_.perm.empty() ? h_.host[0].A : h_.A_user;
  if (!h_.has_upat) {
    std::vector<int> ptr(U.ptr.begin(), U.ptr.end());
    h_.u_ptr.ensure(ptr.size());
    h_.u_col.ensure(std::max<size_t>(1, U.col.size()));
    MMD_HIP(hipMemcpy(h_.u_ptr.p, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice));
    if (!U.col.empty())
      MMD_HIP(hipMemcpy(h_.u_col.p, U.col.data(), sizeof(int) * U.col.size(),
                        hipMemcpyHostToDevice));
    h_.has_upat = true;
  }
  const double* gl = nullptr;
  if (g_evals) {
    double* gld = pool_.d("bw:gl", nev);
    h2d(gld, g_evals, nev);
    gl = gld;
  }
  sddmm_eig(n, h_.u_ptr.p, h_.u_col.p, Vu, Xu, nev, nev, gl, g_vals, s_);
  sync();
}

}  // namespace mmd
