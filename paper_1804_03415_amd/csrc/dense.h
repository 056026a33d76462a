// Small dense FP64 linear algebra on the host: the tridiagonal and Ritz
// eigenproblems of Alg. 2/4/5, the coarsest-level generalised eigenproblem of
// Alg. 6 and the Cholesky factors of CholQR.  Matrices are row-major.
#pragma once

#include <vector>

namespace mmd {
namespace dense {

// Symmetric eigendecomposition of the n x n matrix a (row-major, only read).
// w: eigenvalues ascending; z (if non-null): z[i*n + j] = component i of
// eigenvector j.  Householder tridiagonalisation followed by the implicit QL
// iteration (Bowdler, Martin, Reinsch & Wilkinson 1968).
void sym_eig(int n, const double* a, std::vector<double>& w, std::vector<double>* z);

// Eigen-decomposition of the symmetric tridiagonal matrix (d[0..n-1],
// e[0..n-2] sub-diagonal).  w ascending; if track != null it must hold
// ntrack*n entries with track[r*n + j] = row r of the accumulating
// orthogonal matrix on input, and on output holds the same rows of Z*Q where
// Z holds the eigenvectors as columns (for Ritz residuals only the last row
// is tracked).
void tridiag_eig(int n, const double* d, const double* e, std::vector<double>& w,
                 double* track, int ntrack);

// Upper Cholesky factor: g = r^T r.  Returns false if g is not positive
// definite.  r is n x n row-major with zeros below the diagonal.
bool cholesky_upper(int n, const double* g, std::vector<double>& r);

// Inverse of an upper-triangular n x n matrix.
void upper_inverse(int n, const double* r, std::vector<double>& rinv);

// Generalised problem a z = lambda m z (m SPD): lambda ascending, z with
// z^T m z = I (column j of the row-major n x n z).  Returns false if m is
// not positive definite.
bool gen_eig(int n, const double* a, const double* m, std::vector<double>& lam,
             std::vector<double>& z);

// One explicit shifted QR step on the symmetric m x m matrix t (row-major,
// updated in place): t - sigma I = Q R, t <- R Q + sigma I; q (m x m) is
// multiplied on the right by Q.
void shifted_qr_step(int m, double* t, double sigma, double* q);

}  // namespace dense
}  // namespace mmd
