"""Pins of the eigen-backward oracle (CPU): dense reference gradient from the
full eigendecomposition and central finite differences of the forward map."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import backward as bw
from oracle import dense


def _edges(A):
    """Upper-triangle off-diagonal entries: edge list and weights w = -a_ij."""
    T = sp.triu(sp.csr_matrix(A), k=1).tocoo()
    return T.row.astype(np.int64), T.col.astype(np.int64), -T.data


def _rebuild(n, ei, ej, w, shift):
    rp, ci, v = wl.generators.laplacian_from_edges(n, ei, ej, w, shift)
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


@pytest.fixture(scope="module")
def knn_small():
    p = wl.knn_gmm(300, 10, 1)
    A = p.scipy()
    nev = 8
    lam_all, V_all = np.linalg.eigh(A.toarray())
    gaps = np.diff(lam_all[:nev + 1]) / lam_all[1:nev + 1]
    assert gaps.min() > 1e-3          # simple eigenvalues: the gradient exists
    assert dense.component_count(A) == 1
    return p, A, nev, lam_all, V_all


def test_sampled_matches_dense_reference(knn_small):
    """Deflated-CG adjoints agree with the full-spectrum formula (no solve)."""
    p, A, nev, lam_all, V_all = knn_small
    rng = np.random.default_rng(3)
    g_lam = rng.standard_normal(nev)
    g_V = rng.standard_normal((p.n, nev))
    lam, V = lam_all[:nev], V_all[:, :nev]
    s = bw.sampled_gradient(A, lam, V, g_lam, g_V, tol=1e-13)
    S = bw.dense_gradient(A, lam_all, V_all, nev, g_lam, g_V)
    Acoo = A.tocoo()
    ref = S[Acoo.row, Acoo.col]
    assert np.max(np.abs(s - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_eigenvalue_gradient_closed_form(knn_small):
    """g_V = 0: S = sum g_k v_k v_k^T exactly (no adjoint solve)."""
    p, A, nev, lam_all, V_all = knn_small
    g_lam = np.arange(1.0, nev + 1)
    s = bw.sampled_gradient(A, lam_all[:nev], V_all[:, :nev], g_lam, None)
    Acoo = A.tocoo()
    ref = np.einsum("k,ik,ik->i", g_lam, V_all[Acoo.row, :nev], V_all[Acoo.col, :nev])
    assert np.allclose(s, ref, rtol=0, atol=1e-14)


def test_edge_gradient_finite_differences(knn_small):
    """f = sum_k lambda_k + sum_i x_i v_2[i]^2 (sign-invariant Fiedler quadratic):
    edge-weight gradient against central differences with h = 1e-4 w_e.  (At
    h = 1e-6 w_e the rounding of the dense forward solves, ~1e-15 absolute in f,
    already gives 1e-4 relative noise in the differences; at 1e-4 the central
    truncation error O(h^2) and the noise are both below 1e-5.)"""
    p, A, nev, lam_all, V_all = knn_small
    n = p.n
    ei, ej, w = _edges(A)
    shift = 1e-6
    x = p.coords[:, 0]

    def f(wv):
        lam, V = np.linalg.eigh(_rebuild(n, ei, ej, wv, shift).toarray())
        return lam[:nev].sum() + np.sum(x * V[:, 1] ** 2)

    lam, V = lam_all[:nev], V_all[:, :nev]
    g_lam = np.ones(nev)
    g_V = np.zeros((n, nev))
    g_V[:, 1] = 2.0 * x * V[:, 1]
    s = bw.sampled_gradient(A, lam, V, g_lam, g_V, tol=1e-13)
    ge = bw.edge_gradient(s, A, ei, ej)
    rng = np.random.default_rng(7)
    pick = rng.choice(ei.size, size=20, replace=False)
    for e in pick:
        h = 1e-4 * w[e]
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (f(wp) - f(wm)) / (2 * h)
        assert abs(fd - ge[e]) <= 1e-5 * abs(fd)


def test_repeated_eigenvalue_with_coupled_adjoint_raises():
    """A 2-D constant grid has exact pairs: an adjoint coupling the two copies
    has no gradient."""
    p = wl.grid2d(8)
    A = p.scipy()
    lam_all, V_all = np.linalg.eigh(A.toarray())
    nev = 3                          # lambda_2 = lambda_3 on the square grid
    assert abs(lam_all[1] - lam_all[2]) <= 1e-12 * lam_all[1]
    g_V = np.zeros((p.n, nev))
    g_V[:, 1] = V_all[:, 2]
    with pytest.raises(bw.UndefinedGradient):
        bw.sampled_gradient(A, lam_all[:nev], V_all[:, :nev], None, g_V)
