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
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import workloads as wl
from oracle import dense

pytestmark = pytest.mark.gpu

SHIFT = 1e-6


def rr_floor(lam):
    """Rounding of the final Rayleigh-Ritz step on the m x m projection
    (absolute u lambda_max per entry, accumulated over m): 4 sqrt(m) u lambda_max."""
    return 4.0 * np.sqrt(lam.size) * 2.0 ** -52 * float(np.max(lam))


def check_shift_cluster(A, lam):
    """The smallest values of a graph Laplacian + shift against the stored
    matrix's shift cluster (oracle dense.shift_cluster: per connected
    component the mean exactly-summed row sum), element by element at the
    1e-10 relative eigenvalue bar or the Rayleigh-Ritz rounding floor; the
    next value must lie clearly above the cluster.  Returns the cluster mask."""
    ref = dense.shift_cluster(A)
    k = min(ref.size, lam.size)
    bar = np.maximum(1e-10 * ref[:k], rr_floor(lam))
    assert np.all(np.abs(lam[:k] - ref[:k]) <= bar)
    if lam.size > ref.size:
        assert lam[ref.size] > 2.0 * ref.max()
    mask = np.zeros(lam.size, bool)
    mask[:k] = True
    return mask


def per_pair(A, lam, Vh, lam_ref, Vh_ref):
    """rho_i, e_i and the cluster angle of each pair against a reference run."""
    rho = dense.rel_residuals(A, lam, Vh)
    e = np.abs(lam - lam_ref) / np.abs(lam_ref)
    ang, cl = dense.cluster_angles(lam_ref, Vh_ref, Vh)
    angle = np.zeros(lam.size)
    full = np.zeros(lam.size, bool)
    for a, c in zip(ang, cl):
        angle[c] = a
        full[c] = c[-1] < lam.size - 1
    return rho, e, angle, full


def angle_bound(A, lam, Vh, lam_ref, Vh_ref):
    """Davis-Kahan sin-theta bound per pair for two approximations of the same
    eigenvector cluster: sin angle <= (||r|| + ||r_ref||) / gap, with r the
    cluster's residual block and gap the distance of the cluster's
    eigenvalues to the rest of the computed spectrum (both runs' residuals
    are at most about 1e-9 lambda, so close clusters allow angles above 1e-8)."""
    cl = dense.clusters(lam_ref)
    out = np.zeros(lam.size)
    for c in cl:
        lo_gap = lam_ref[c[0]] - lam_ref[c[0] - 1] if c[0] > 0 else np.inf
        hi_gap = lam_ref[c[-1] + 1] - lam_ref[c[-1]] if c[-1] + 1 < lam.size else np.inf
        gap = min(lo_gap, hi_gap)
        R = A @ Vh[:, c] - Vh[:, c] * lam[c][None, :]
        Rr = A @ Vh_ref[:, c] - Vh_ref[:, c] * lam_ref[c][None, :]
        out[c] = (np.linalg.norm(R, 2) + np.linalg.norm(Rr, 2)) / gap
    return out


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
    null = check_shift_cluster(A, lam)
    assert null.sum() == ncomp
    w = np.sort(sla.eigsh(A.tocsc(), k=30, sigma=0, which="LM", return_eigenvectors=False))
    nn = np.abs(w - 1e-6) >= 1e-12
    assert np.max(np.abs(lam[:30][nn] - w[nn]) / w[nn]) < 1e-10
    lm, Vm, _ = dec.eig_leftmost(300, tol=1e-9, precision="fp32-refine")
    Vmh = Vm.cpu().numpy().T
    _check_pairs(A, lm, Vmh)
    check_shift_cluster(A, lm)
    assert np.max(np.abs(lm[~null] - lam[~null]) / lam[~null]) < 1e-10
    ang, cl = dense.cluster_angles(lam, Vh, Vmh)
    full = [i for i, c in enumerate(cl) if c[-1] < 299]
    assert ang[full].max() < 1e-8


@pytest.mark.timeout(900)
def test_diffusion_64cubed_500_fp64_and_mixed(torch_cuda):
    """3-D 7-point lognormal diffusion, n = 262144, 500 pairs, FP64 and the
    mixed form (FP32 CG inside FP64 refinement): every pair of both runs meets
    the residual target, and per eigenpair the mixed run's relative eigenvalue
    difference (1e-10) and cluster angle against the FP64 run: 1e-8, or the
    Davis-Kahan bound of the two runs' residuals where a neighbouring
    eigenvalue is close."""
    from paper_1804_03415_amd import Decomposition
    p = wl.grid3d_lognormal(64, 0)
    A = p.scipy()
    dec = Decomposition.from_problem(p, levels=3)
    lam, V, st = dec.eig_leftmost(500, tol=1e-9)
    Vh = V.cpu().numpy().T
    _check_pairs(A, lam, Vh)
    assert st["nconv"] == 500
    lm, Vm, _ = dec.eig_leftmost(500, tol=1e-9, precision="fp32-refine")
    Vmh = Vm.cpu().numpy().T
    _check_pairs(A, lm, Vmh)
    rho, e, angle, full = per_pair(A, lm, Vmh, lam, Vh)
    assert rho.max() <= 1e-8
    assert e.max() <= 1e-10
    # 1e-8 where the clusters are well separated, else the sin-theta bound
    bar = np.maximum(1e-8, angle_bound(A, lm, Vmh, lam, Vh))
    assert np.all(angle[full] <= bar[full])
    assert np.median(angle[full]) <= 1e-9


@pytest.mark.timeout(900)
def test_grid3d_64_constant_closed_form(torch_cuda):
    """The same 64^3 operator at sigma = 0 (all face coefficients 1): the 501
    smallest eigenvalues are sums over the three axes of 4 sin^2(j pi / 130)
    (112 distinct values, 59 six-fold and 47 three-fold clusters; nev = 501
    ends with the cluster 496-501), the eigenvectors products of sines.
    Eigenvalues to 1e-10 relative, cluster angles to 1e-8: this also proves
    that no eigenvalue below lambda_501 was skipped."""
    from paper_1804_03415_amd import Decomposition
    m, nev = 64, 501
    p = wl.grid3d_lognormal(m, 0, sigma=0.0)
    A = p.scipy()
    dec = Decomposition.from_problem(p, levels=3)
    lam, V, st = dec.eig_leftmost(nev, tol=1e-10)
    j = np.arange(1, m + 1)
    s1 = 4 * np.sin(j * np.pi / (2 * (m + 1))) ** 2
    tot = (s1[:, None, None] + s1[None, :, None] + s1[None, None, :]).ravel()
    order = np.argsort(tot, kind="stable")[:nev]
    ref = tot[order]
    assert np.max(np.abs(lam - ref) / ref) < 1e-10
    # closed-form eigenvectors: index (z*m + y)*m + x, mode (c, b, a) over (z, y, x)
    S = np.sin(np.outer(j, j) * np.pi / (m + 1))  # S[a-1, x-1] = sin(a pi x / (m+1))
    S /= np.linalg.norm(S, axis=1)[:, None]
    Vref = np.empty((m ** 3, nev))
    for q, idx in enumerate(order):
        c, b, a = np.unravel_index(idx, (m, m, m))
        Vref[:, q] = np.einsum("z,y,x->zyx", S[a], S[b], S[c]).ravel()
    Vh = V.cpu().numpy().T
    ang, cl = dense.cluster_angles(ref, Vref, Vh)
    assert len(cl) == 112
    assert ang.max() < 1e-8
    assert dense.rel_residuals(A, lam, Vh).max() <= 1e-8


@pytest.mark.timeout(600)
def test_diffusion_32cubed_completeness(torch_cuda):
    """No eigenvalue below the returned ones is missed, by Sylvester's law of
    inertia: sigma just above lambda_300 of the 32^3 lognormal diffusion, the
    symmetric LDL^T-form factorisation of A - sigma I (sparse LU restricted to
    diagonal pivots and a symmetric ordering) has exactly 300 negative pivots."""
    from paper_1804_03415_amd import Decomposition
    p = wl.grid3d_lognormal(32, 0)
    A = p.scipy()
    dec = Decomposition.from_problem(p, levels=3)
    lam, V, st = dec.eig_leftmost(300, tol=1e-9)
    _check_pairs(A, lam, V.cpu().numpy().T)
    sigma = lam[-1] * (1 + 1e-7)
    lu = sla.splu((A - sigma * sp.eye(p.n)).tocsc(), permc_spec="MMD_AT_PLUS_A",
                  diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    assert np.array_equal(lu.perm_r, lu.perm_c)
    assert int(np.sum(lu.U.diagonal() < 0)) == 300


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
    assert check_shift_cluster(A, lam).sum() == dense.component_count(A)
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
    mean degree 8), 100 pairs each, through eig_leftmost_batched, in FP64 and
    in the mixed form; per member the residuals, the null cluster and, for the
    mixed run, each pair against the FP64 run (1e-10 eigenvalues, 1e-8
    cluster angles)."""
    from paper_1804_03415_amd import Decomposition, eig_leftmost_batched
    probs = wl.rgg_batch(64, seed=0)[:4]
    decs = [Decomposition.from_problem(q, levels=3, targets=(4, 8)) for q in probs]
    out = eig_leftmost_batched(decs, [100] * 4, tol=1e-9, streams=4)
    outm = eig_leftmost_batched(decs, [100] * 4, tol=1e-9, streams=4, precision="fp32-refine")
    for q, (lam, V, st), (lm, Vm, _) in zip(probs, out, outm):
        A = q.scipy()
        Vh, Vmh = V.cpu().numpy().T, Vm.cpu().numpy().T
        _check_pairs(A, lam, Vh)
        _check_pairs(A, lm, Vmh)
        nc = dense.component_count(A)
        null = check_shift_cluster(A, lam)
        assert null.sum() == nc
        check_shift_cluster(A, lm)
        rho, e, angle, full = per_pair(A, lm, Vmh, lam, Vh)
        assert e[~null].max() <= 1e-10
        assert angle[full].max() <= 1e-8
