"""Eigen-backward through the C ABI against the oracle (oracle/backward.py).

The eigenpairs fed to both sides come from the dense oracle solve, so the
comparison isolates the backward computation; the autograd test runs the GPU
forward and checks edge-weight gradients against the oracle gradient and
against central differences of the dense forward map.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import backward as bw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _eig_dense(A, nev):
    lam_all, V_all = np.linalg.eigh(A.toarray())
    return lam_all, V_all, lam_all[:nev], V_all[:, :nev]


@pytest.mark.parametrize("case", ["knn_300", "rgg_2000", "knn_1500"])
def test_backward_matches_oracle(torch_cuda, case):
    torch = torch_cuda
    from paper_1804_03415_amd import Decomposition
    if case == "knn_300":
        p, nev, kw = wl.knn_gmm(300, 10, 1), 8, dict(levels=2)
    elif case == "rgg_2000":
        p, nev, kw = wl.rgg(2000, 0), 12, dict(levels=3)
    else:
        p, nev, kw = wl.knn_gmm(1500, 10, 1), 20, dict(levels=2)
    A = p.scipy()
    lam_all, V_all, lam, V = _eig_dense(A, nev)
    rng = np.random.default_rng(11)
    g_lam = rng.standard_normal(nev)
    g_V = rng.standard_normal((p.n, nev))
    # degenerate clusters (the RGG's null space) carry no coupled adjoint
    null = np.abs(lam - 1e-6) < 1e-9
    if null.sum() > 1:
        g_V[:, null] = 0.0
    dec = Decomposition.from_problem(p, **kw)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).cuda()
    Gt = torch.from_numpy(np.ascontiguousarray(g_V.T)).cuda()
    g = dec.eig_backward(lam, Vt, g_lam, Gt, tol=1e-12).cpu().numpy()
    ref = bw.sampled_gradient(A, lam, V, g_lam, g_V, tol=1e-13)
    assert np.max(np.abs(g - ref)) <= 1e-9 * np.max(np.abs(ref))
    # eigenvalue term alone (closed form, no solve)
    g0 = dec.eig_backward(lam, Vt, g_lam, None).cpu().numpy()
    ref0 = bw.sampled_gradient(A, lam, V, g_lam, None)
    assert np.max(np.abs(g0 - ref0)) <= 1e-13 * np.max(np.abs(ref0))


def test_backward_dense_reference(torch_cuda):
    """Against the full-spectrum formula (no CG anywhere)."""
    torch = torch_cuda
    from paper_1804_03415_amd import Decomposition
    p = wl.knn_gmm(300, 10, 1)
    A = p.scipy()
    nev = 8
    lam_all, V_all, lam, V = _eig_dense(A, nev)
    rng = np.random.default_rng(5)
    g_lam, g_V = rng.standard_normal(nev), rng.standard_normal((p.n, nev))
    dec = Decomposition.from_problem(p, levels=2)
    g = dec.eig_backward(lam, torch.from_numpy(np.ascontiguousarray(V.T)).cuda(), g_lam,
                         torch.from_numpy(np.ascontiguousarray(g_V.T)).cuda(),
                         tol=1e-12).cpu().numpy()
    S = bw.dense_gradient(A, lam_all, V_all, nev, g_lam, g_V)
    Acoo = A.tocoo()
    ref = S[Acoo.row, Acoo.col]
    assert np.max(np.abs(g - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_backward_repeated_eigenvalue_raises(torch_cuda):
    torch = torch_cuda
    from paper_1804_03415_amd import Decomposition, MMDError
    p = wl.grid2d(8)
    A = p.scipy()
    lam_all, V_all, lam, V = _eig_dense(A, 3)
    g_V = np.zeros((p.n, 3))
    g_V[:, 1] = V_all[:, 2]
    dec = Decomposition.from_problem(p, levels=1, exact_max_n=4096)
    with pytest.raises(MMDError):
        dec.eig_backward(lam, torch.from_numpy(np.ascontiguousarray(V.T)).cuda(), None,
                         torch.from_numpy(np.ascontiguousarray(g_V.T)).cuda())


def _laplacian_values(torch, A, shift):
    """values(w) of A = L(w) + shift I as torch ops over the edge weights, so
    autograd carries dL/dvalues to dL/dw."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    up = rows < cols
    ei, ej = rows[up], cols[up]
    w0 = -A.data[up]
    key = {(int(i), int(j)): e for e, (i, j) in enumerate(zip(ei, ej))}
    off = np.array([key[(min(r, c), max(r, c))] if r != c else -1
                    for r, c in zip(rows, cols)], dtype=np.int64)
    diag_pos = np.full(n, -1, dtype=np.int64)
    diag_pos[rows[rows == cols]] = np.nonzero(rows == cols)[0]

    def values(w):
        v = torch.zeros(A.nnz, dtype=torch.float64)
        offp = np.nonzero(off >= 0)[0]
        v = v.index_add(0, torch.from_numpy(offp), -w[torch.from_numpy(off[offp])])
        v = v.index_add(0, torch.from_numpy(diag_pos[ei]), w)
        v = v.index_add(0, torch.from_numpy(diag_pos[ej]), w)
        v = v + torch.from_numpy(np.where(rows == cols, shift, 0.0))
        return v

    return ei.astype(np.int64), ej.astype(np.int64), w0, values


def test_autograd_edge_weights(torch_cuda):
    """Sum of eigenvalues plus the Fiedler quadratic through EigLeftmost: the
    edge-weight gradient matches the oracle gradient and central differences of
    the dense forward map."""
    torch = torch_cuda
    from paper_1804_03415_amd import EigLeftmost
    p = wl.knn_gmm(300, 10, 1)
    A = p.scipy()
    nev = 8
    ei, ej, w0, values = _laplacian_values(torch, A, 1e-6)
    w = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
    x = torch.from_numpy(p.coords[:, 0]).cuda()
    vals = values(w)
    assert np.allclose(vals.detach().numpy(), A.data, rtol=0, atol=1e-15)
    lam, V = EigLeftmost.apply(vals, p.rowptr, p.col, nev, 1e-12,
                               dict(levels=2, coords=p.coords))
    loss = lam.sum() + (x * V[1] ** 2).sum()
    loss.backward()
    gw = w.grad.numpy()
    # oracle gradient on the dense eigenpairs
    lam_all, V_all, lam_d, V_d = _eig_dense(A, nev)
    g_V = np.zeros((p.n, nev))
    g_V[:, 1] = 2.0 * p.coords[:, 0] * V_d[:, 1]
    s = bw.sampled_gradient(A, lam_d, V_d, np.ones(nev), g_V, tol=1e-13)
    ge = bw.edge_gradient(s, A, ei, ej)
    assert np.max(np.abs(gw - ge)) <= 1e-7 * np.max(np.abs(ge))

    def f(wv):
        rp, ci, v = wl.generators.laplacian_from_edges(p.n, ei, ej, wv, 1e-6)
        lm, Vm = np.linalg.eigh(sp.csr_matrix((v, ci, rp), shape=A.shape).toarray())
        return lm[:nev].sum() + np.sum(p.coords[:, 0] * Vm[:, 1] ** 2)

    rng = np.random.default_rng(9)
    for e in rng.choice(ei.size, size=10, replace=False):
        h = 1e-4 * w0[e]
        wp, wm = w0.copy(), w0.copy()
        wp[e] += h
        wm[e] -= h
        fd = (f(wp) - f(wm)) / (2 * h)
        # relative 1e-5, plus the rounding floor of the differences
        # (~1e-15 in f over h ~ 1e-5)
        assert abs(fd - gw[e]) <= 1e-5 * abs(fd) + 1e-9
