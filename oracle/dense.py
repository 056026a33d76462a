"""Plain definition of the result and per-eigenpair error measures.

eig_leftmost(A, nev) returns the nev smallest eigenvalues of the SPD matrix A
(ascending) and orthonormal eigenvectors.  For small n this is a dense
symmetric eigensolve; that is the brute-force pin of the hierarchical method.
"""
import numpy as np
import scipy.sparse as sp


def smallest_dense(A, nev):
    """Brute force: all eigenpairs of the dense matrix, keep the nev smallest."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    w, V = np.linalg.eigh(0.5 * (Ad + Ad.T))
    return w[:nev], V[:, :nev]


def rel_residuals(A, lam, V):
    """rho_i = ||A v_i - lambda_i v_i||_2 / (lambda_i ||v_i||_2), all in float64."""
    R = A @ V - V * lam[None, :]
    return np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(V, axis=0))


def clusters(lam, rel_gap=1e-6):
    """Maximal runs with (lam[i+1] - lam[i]) / lam[i] < rel_gap, as index lists."""
    out = [[0]] if len(lam) else []
    for i in range(1, len(lam)):
        if (lam[i] - lam[i - 1]) / abs(lam[i - 1]) < rel_gap:
            out[-1].append(i)
        else:
            out.append([i])
    return out


def cluster_angles(lam_ref, V_ref, V, rel_gap=1e-6):
    """Largest principal angle (sin) between matching cluster subspaces.

    Only clusters that end strictly before the last index are compared
    unless the reference holds the whole cluster; returns (angles, clusters).
    """
    cl = clusters(lam_ref, rel_gap)
    ang = []
    for idx in cl:
        Qr, _ = np.linalg.qr(V_ref[:, idx])
        Q, _ = np.linalg.qr(V[:, idx])
        # sin of the largest principal angle, without the cancellation of 1 - cos^2
        R = Q - Qr @ (Qr.T @ Q)
        ang.append(float(np.linalg.norm(R, 2)))
    return np.array(ang), cl


def component_count(A):
    """Connected components of the graph of A's off-diagonal pattern."""
    from scipy.sparse.csgraph import connected_components
    G = sp.csr_matrix(A).copy()
    G.setdiag(0)
    G.eliminate_zeros()
    return connected_components(G, directed=False)[0]


def shift_cluster(A):
    """Smallest eigenvalue of each connected component of a stored graph
    operator A = L + diag(s) (Section 2.1 energy form), ascending.

    On a component C the indicator vector 1_C is an exact eigenvector of the
    exact-arithmetic matrix when every row sum s_i equals the same shift; the
    stored FP64 diagonal a_ii = sum_j w_ij + s_i is rounded, so the stored
    matrix's row sums deviate by up to u ||A||_inf.  Its eigenvalue nearest the
    shift is then the Rayleigh quotient of 1_C, the mean row sum over C (each
    row summed exactly with math.fsum), up to a second-order term (spread of
    the row sums over C)^2 / (spectral gap of C).  This is the reference value
    of the shift cluster of a graph Laplacian plus a shift.
    """
    import math
    from scipy.sparse.csgraph import connected_components
    A = sp.csr_matrix(A)
    G = A.copy()
    G.setdiag(0)
    G.eliminate_zeros()
    nc, lab = connected_components(G, directed=False)
    rs = np.array([math.fsum(A.data[A.indptr[i]:A.indptr[i + 1]]) for i in range(A.shape[0])])
    out = np.empty(nc)
    for c in range(nc):
        out[c] = math.fsum(rs[lab == c]) / np.count_nonzero(lab == c)
    return np.sort(out)
