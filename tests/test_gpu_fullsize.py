"""Full-size workloads through the C ABI, in the configuration bench.py times.

The oracle cannot solve these sizes element by element, so the checks are
properties that hold at any size plus sampled comparisons the CPU can do:
every returned pair meets the residual target, the vectors are orthonormal,
the multiplicity of the shift eigenvalue equals the connected-component
count, the 30 smallest eigenvalues of the RGG agree with a shift-invert
Lanczos (sparse LU, scipy), the mixed-precision form agrees pair by pair with
FP64, and the eigen-backward satisfies <S_lambda, A> = sum(lambda) with an
eigenvector term orthogonal to A.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as wl
from oracle import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _check_pairs(A, lam, Vh, ortho=1e-10):
    assert np.all(np.diff(lam) >= 0)
    assert dense.rel_residuals(A, lam, Vh).max() <= 1e-8
    G = Vh.T @ Vh
    assert np.abs(G - np.eye(G.shape[0])).max() < ortho


def test_rgg_1e5_300_fp64_and_mixed(torch_cuda):
    from paper_1804_03415_amd import Decomposition
    p = wl.rgg(100000, 0)
    A = p.scipy()
    dec = Decomposition.from_problem(p, levels=3, targets=(4, 8))
    lam, V, st = dec.eig_leftmost(300, tol=1e-9)
    Vh = V.cpu().numpy().T
    _check_pairs(A, lam, Vh)
    ncomp = dense.component_count(A)
    assert ncomp == 8
    null = np.abs(lam - 1e-6) < 1e-12
    assert null.sum() == ncomp
    w = np.sort(sla.eigsh(A.tocsc(), k=30, sigma=0, which="LM", return_eigenvectors=False))
    nn = np.abs(w - 1e-6) >= 1e-12
    assert np.max(np.abs(lam[:30][nn] - w[nn]) / w[nn]) < 1e-10
    lm, Vm, _ = dec.eig_leftmost(300, tol=1e-9, precision="fp32-refine")
    Vmh = Vm.cpu().numpy().T
    _check_pairs(A, lm, Vmh)
    assert np.sum(np.abs(lm - 1e-6) < 1e-12) == ncomp
    assert np.max(np.abs(lm[~null] - lam[~null]) / lam[~null]) < 1e-10
    ang, cl = dense.cluster_angles(lam, Vh, Vmh)
    full = [i for i, c in enumerate(cl) if c[-1] < 299]
    assert ang[full].max() < 1e-8


def test_diffusion_64cubed_500(torch_cuda):
    """3-D 7-point lognormal diffusion, n = 262144, 500 pairs (FP64)."""
    from paper_1804_03415_amd import Decomposition
    p = wl.grid3d_lognormal(64, 0)
    A = p.scipy()
    dec = Decomposition.from_problem(p, levels=3)
    lam, V, st = dec.eig_leftmost(500, tol=1e-9)
    _check_pairs(A, lam, V.cpu().numpy().T)
    assert st["nconv"] == 500


def test_knn_2e5_forward_backward(torch_cuda):
    """kNN-GMM n = 2e5: 20 pairs, eigen-backward of sum(lambda) + the Fiedler
    quadratic; properties of the gradient that hold at any size."""
    torch = torch_cuda
    from paper_1804_03415_amd import Decomposition
    p = wl.knn_gmm(200000, 10, 1)
    A = p.scipy()
    dec = Decomposition.from_problem(p, levels=3, targets=(4, 8), exact_max_n=8000)
    lam, V, st = dec.eig_leftmost(20, tol=1e-9)
    Vh = V.cpu().numpy().T
    _check_pairs(A, lam, Vh)
    assert np.sum(np.abs(lam - 1e-6) < 1e-12) == dense.component_count(A)
    x = torch.from_numpy(p.coords[:, 0]).cuda()
    gV = torch.zeros_like(V)
    gV[1] = 2.0 * x * V[1]
    g = dec.eig_backward(lam, V, np.ones(20), gV, tol=1e-10).cpu().numpy()
    gl = dec.eig_backward(lam, V, np.ones(20), None).cpu().numpy()
    # <S_lambda, A> = sum_k v_k^T A v_k = sum(lambda)
    assert abs(np.dot(gl, A.data) - lam.sum()) <= 1e-9 * lam.sum()
    # eigenvector term: <x_k v_k^T, A> = lambda_k x_k^T v_k = 0
    gv = g - gl
    assert abs(np.dot(gv, A.data)) <= 1e-8 * np.abs(gv).max() * np.sqrt(A.nnz)
    assert np.abs(gv).max() > 0


def test_rgg_batch_members(torch_cuda):
    """The first four members of the 64-problem batch (sizes 5000-50000,
    mean degree 8), 100 pairs each, through eig_leftmost_batched."""
    from paper_1804_03415_amd import Decomposition, eig_leftmost_batched
    probs = wl.rgg_batch(64, seed=0)[:4]
    decs = [Decomposition.from_problem(q, levels=3, targets=(4, 8)) for q in probs]
    out = eig_leftmost_batched(decs, [100] * 4, tol=1e-9, streams=4)
    for q, (lam, V, st) in zip(probs, out):
        A = q.scipy()
        _check_pairs(A, lam, V.cpu().numpy().T)
        assert np.sum(np.abs(lam - 1e-6) < 1e-12) == dense.component_count(A)
