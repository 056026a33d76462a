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
