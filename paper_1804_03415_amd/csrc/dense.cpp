// Host dense FP64 linear algebra (see dense.h).
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace mmd {
namespace dense {

namespace {

// Householder reduction a = Q T Q^T of a symmetric matrix; returns the
// diagonal d, sub-diagonal e and qt = Q^T (row-major) so that rotations of the
// QL iteration act on contiguous rows.
void tridiagonalize(int n, std::vector<double>& a, std::vector<double>& d,
                    std::vector<double>& e, std::vector<double>* qt) {
  d.assign(n, 0.0);
  e.assign(n > 0 ? n - 1 : 0, 0.0);
  std::vector<std::vector<double>> vs;  // Householder vectors (length n-k-1)
  std::vector<double> p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* col = nullptr;
    std::vector<double> v(m);
    for (int i = 0; i < m; ++i) v[i] = a[(size_t)(k + 1 + i) * n + k];
    double sig = 0.0;
    for (int i = 1; i < m; ++i) sig += v[i] * v[i];
    (void)col;
    if (sig == 0.0) {
      vs.emplace_back();  // identity reflector
      continue;
    }
    const double x0 = v[0];
    const double nrm = std::sqrt(x0 * x0 + sig);
    const double alpha = x0 >= 0 ? -nrm : nrm;
    v[0] = x0 - alpha;
    const double vn = std::sqrt(v[0] * v[0] + sig);
    for (int i = 0; i < m; ++i) v[i] /= vn;
    // sub-block B = a[k+1:, k+1:]; p = B v; K = v^T p; q = p - K v; B -= 2 (v q^T + q v^T)
    for (int i = 0; i < m; ++i) {
      const double* row = &a[(size_t)(k + 1 + i) * n + (k + 1)];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
    }
    double K = 0.0;
    for (int i = 0; i < m; ++i) K += v[i] * p[i];
    for (int i = 0; i < m; ++i) q[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = &a[(size_t)(k + 1 + i) * n + (k + 1)];
      const double vi = 2.0 * v[i], qi = 2.0 * q[i];
      for (int j = 0; j < m; ++j) row[j] -= vi * q[j] + qi * v[j];
    }
    a[(size_t)(k + 1) * n + k] = alpha;
    a[(size_t)k * n + (k + 1)] = alpha;
    for (int i = 1; i < m; ++i) {
      a[(size_t)(k + 1 + i) * n + k] = 0.0;
      a[(size_t)k * n + (k + 1 + i)] = 0.0;
    }
    vs.push_back(std::move(v));
  }
  for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)(i + 1) * n + i];
  if (!qt) return;
  // Q = H_0 H_1 ... ; build Q^T = ... H_1 H_0 by applying reflectors to rows of I
  std::vector<double>& Q = *qt;
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  // Q^T x = H_last ... H_0 x ; rows of Q^T: Q^T = (H_0 ... H_last)^T = H_last ... H_0.
  // Apply H_k from the right to Q (Q <- Q H_k) for k ascending, acting on
  // columns k+1.. ; then transpose.  Work on Q directly then transpose.
  std::vector<double> Qm((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Qm[(size_t)i * n + i] = 1.0;
  for (int k = static_cast<int>(vs.size()) - 1; k >= 0; --k) {
    const std::vector<double>& v = vs[k];
    if (v.empty()) continue;
    const int m = n - k - 1;
    // Qm <- H_k Qm on rows k+1.. (backward accumulation: Q = H_0 (H_1 (... )))
    std::vector<double> t(n, 0.0);
    for (int i = 0; i < m; ++i) {
      const double* row = &Qm[(size_t)(k + 1 + i) * n];
      const double vi = v[i];
      for (int j = 0; j < n; ++j) t[j] += vi * row[j];
    }
    for (int i = 0; i < m; ++i) {
      double* row = &Qm[(size_t)(k + 1 + i) * n];
      const double vi = 2.0 * v[i];
      for (int j = 0; j < n; ++j) row[j] -= vi * t[j];
    }
  }
  // Qm = Q ; Q^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[(size_t)j * n + i] = Qm[(size_t)i * n + j];
}

}  // namespace

void tridiag_eig(int n, const double* din, const double* ein, std::vector<double>& w,
                 double* track, int ntrack) {
  // Implicit QL with shifts on the tridiagonal; track rows are rotated like
  // the columns of the eigenvector matrix (stored transposed: track[j*ntrack+r]
  // would be column-major; here track holds rows r of Z: track[r*n + j]).
  std::vector<double> d(din, din + n);
  std::vector<double> e(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) e[i] = ein[i];
  const double eps = std::numeric_limits<double>::epsilon();
  // rotations act on pairs of columns (i, i+1) of the tracked rows; they are
  // applied to a transposed copy, where each column is a contiguous row
  std::vector<double> zt;
  if (track) {
    zt.resize((size_t)n * ntrack);
    for (int r = 0; r < ntrack; ++r)
      for (int j = 0; j < n; ++j) zt[(size_t)j * ntrack + r] = track[(size_t)r * n + j];
  }
  auto rot = [&](int i, double c, double s) {
    if (!track) return;
    double* zi = zt.data() + (size_t)i * ntrack;
    double* zj = zi + ntrack;
    for (int r = 0; r < ntrack; ++r) {
      const double h = zj[r];
      zj[r] = s * zi[r] + c * h;
      zi[r] = c * zi[r] - s * h;
    }
  };
  double f = 0.0, tst = 0.0;
  for (int l = 0; l < n; ++l) {
    tst = std::max(tst, std::fabs(d[l]) + std::fabs(e[l]));
    int m = l;
    while (m < n - 1 && std::fabs(e[m]) > eps * tst) ++m;
    if (m > l) {
      int guard = 0;
      do {
        if (++guard > 200) break;
        double g = d[l];
        double p = (d[l + 1] - g) / (2.0 * e[l]);
        double r = std::hypot(p, 1.0);
        if (p < 0) r = -r;
        d[l] = e[l] / (p + r);
        d[l + 1] = e[l] * (p + r);
        const double dl1 = d[l + 1];
        double h = g - d[l];
        for (int i = l + 2; i < n; ++i) d[i] -= h;
        f += h;
        p = d[m];
        double c = 1.0, c2 = 1.0, c3 = 1.0, s = 0.0, s2 = 0.0;
        const double el1 = e[l + 1];
        for (int i = m - 1; i >= l; --i) {
          c3 = c2;
          c2 = c;
          s2 = s;
          g = c * e[i];
          h = c * p;
          r = std::hypot(p, e[i]);
          e[i + 1] = s * r;
          s = e[i] / r;
          c = p / r;
          p = c * d[i] - s * g;
          d[i + 1] = h + s * (c * g + s * d[i]);
          rot(i, c, s);
        }
        p = -s * s2 * c3 * el1 * e[l] / dl1;
        e[l] = s * p;
        d[l] = c * p;
      } while (std::fabs(e[l]) > eps * tst);
    }
    d[l] += f;
    e[l] = 0.0;
  }
  // sort ascending (stable), permuting tracked columns
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  w.resize(n);
  for (int j = 0; j < n; ++j) w[j] = d[idx[j]];
  if (track)
    for (int j = 0; j < n; ++j) {
      const double* src = zt.data() + (size_t)idx[j] * ntrack;
      for (int r = 0; r < ntrack; ++r) track[(size_t)r * n + j] = src[r];
    }
}

void sym_eig(int n, const double* a_in, std::vector<double>& w, std::vector<double>* z) {
  w.clear();
  if (n == 0) {
    if (z) z->clear();
    return;
  }
  std::vector<double> a(a_in, a_in + (size_t)n * n);
  for (int i = 0; i < n; ++i)  // symmetrise
    for (int j = i + 1; j < n; ++j) {
      const double v = 0.5 * (a[(size_t)i * n + j] + a[(size_t)j * n + i]);
      a[(size_t)i * n + j] = v;
      a[(size_t)j * n + i] = v;
    }
  std::vector<double> d, e;
  if (!z) {
    tridiagonalize(n, a, d, e, nullptr);
    tridiag_eig(n, d.data(), e.data(), w, nullptr, 0);
    return;
  }
  std::vector<double> qt;
  tridiagonalize(n, a, d, e, &qt);
  // rows of Z = Q * Y : track all rows of Q (Q = qt^T)
  std::vector<double> Z((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Z[(size_t)i * n + j] = qt[(size_t)j * n + i];
  tridiag_eig(n, d.data(), e.data(), w, Z.data(), n);
  *z = std::move(Z);
}

bool cholesky_upper(int n, const double* g, std::vector<double>& r) {
  // right-looking, row-major: after step j, row j holds R(j, j..n-1) and the
  // trailing rows hold the Schur complement (contiguous row updates)
  r.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = i; k < n; ++k) r[(size_t)i * n + k] = 0.5 * (g[(size_t)i * n + k] + g[(size_t)k * n + i]);
  for (int j = 0; j < n; ++j) {
    double* rj = r.data() + (size_t)j * n;
    const double d = rj[j];
    if (!(d > 0.0)) return false;
    const double rjj = std::sqrt(d);
    const double inv = 1.0 / rjj;
    rj[j] = rjj;
    for (int k = j + 1; k < n; ++k) rj[k] *= inv;
    for (int i = j + 1; i < n; ++i) {
      const double f = rj[i];
      if (f == 0.0) continue;
      double* ri = r.data() + (size_t)i * n;
      for (int k = i; k < n; ++k) ri[k] -= f * rj[k];
    }
  }
  return true;
}

void upper_inverse(int n, const double* r, std::vector<double>& ri) {
  ri.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    ri[(size_t)j * n + j] = 1.0 / r[(size_t)j * n + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += r[(size_t)i * n + k] * ri[(size_t)k * n + j];
      ri[(size_t)i * n + j] = -s / r[(size_t)i * n + i];
    }
  }
}

bool gen_eig(int n, const double* a, const double* m, std::vector<double>& lam,
             std::vector<double>& z) {
  std::vector<double> r;
  if (!cholesky_upper(n, m, r)) return false;  // m = r^T r
  std::vector<double> ri;
  upper_inverse(n, r.data(), ri);
  // c = r^-T a r^-1
  std::vector<double> t((size_t)n * n, 0.0), c((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double aik = a[(size_t)i * n + k];
      if (aik == 0.0) continue;
      for (int j = k; j < n; ++j) t[(size_t)i * n + j] += aik * ri[(size_t)k * n + j];
    }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k <= i; ++k) {
      const double rki = ri[(size_t)k * n + i];
      if (rki == 0.0) continue;
      for (int j = 0; j < n; ++j) c[(size_t)i * n + j] += rki * t[(size_t)k * n + j];
    }
  std::vector<double> y;
  sym_eig(n, c.data(), lam, &y);
  z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = i; k < n; ++k) {
      const double rik = ri[(size_t)i * n + k];
      if (rik == 0.0) continue;
      for (int j = 0; j < n; ++j) z[(size_t)i * n + j] += rik * y[(size_t)k * n + j];
    }
  return true;
}

void shifted_qr_step(int m, double* t, double sigma, double* q) {
  std::vector<double> r(t, t + (size_t)m * m);
  for (int i = 0; i < m; ++i) r[(size_t)i * m + i] -= sigma;
  std::vector<double> cs(m > 0 ? m - 1 : 0), sn(m > 0 ? m - 1 : 0);
  for (int k = 0; k + 1 < m; ++k) {
    const double a = r[(size_t)k * m + k], b = r[(size_t)(k + 1) * m + k];
    const double h = std::hypot(a, b);
    double c = 1.0, s = 0.0;
    if (h > 0.0) {
      c = a / h;
      s = b / h;
    }
    cs[k] = c;
    sn[k] = s;
    double* rk = &r[(size_t)k * m];
    double* rk1 = &r[(size_t)(k + 1) * m];
    for (int j = 0; j < m; ++j) {
      const double x = rk[j], y = rk1[j];
      rk[j] = c * x + s * y;
      rk1[j] = -s * x + c * y;
    }
  }
  // t = R Q + sigma I with Q = G_0^T G_1^T ... : rotate column pairs of R and q
  for (int k = 0; k + 1 < m; ++k) {
    const double c = cs[k], s = sn[k];
    for (int i = 0; i < m; ++i) {
      double* ri = &r[(size_t)i * m];
      const double x = ri[k], y = ri[k + 1];
      ri[k] = c * x + s * y;
      ri[k + 1] = -s * x + c * y;
      double* qi = &q[(size_t)i * m];
      const double u = qi[k], v = qi[k + 1];
      qi[k] = c * u + s * v;
      qi[k + 1] = -s * u + c * v;
    }
  }
  for (int i = 0; i < m; ++i) r[(size_t)i * m + i] += sigma;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) {
      const double v = 0.5 * (r[(size_t)i * m + j] + r[(size_t)j * m + i]);
      t[(size_t)i * m + j] = v;
      t[(size_t)j * m + i] = v;
    }
}

}  // namespace dense
}  // namespace mmd
