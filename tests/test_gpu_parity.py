"""GPU path (through the C ABI) against the CPU oracle, element by element.

Inputs are seeded and synthetic (workloads package); expected values come only
from the oracle package or from closed forms.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as wl
from oracle import dense, krylov, mmd as mm

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


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------------------------------- SpMM kernel
@pytest.mark.parametrize("shape", [(1, 1, 1), (37, 50, (0, 6)), (1000, 1000, (3, 14)),
                                   (3001, 2000, (40, 120)), (513, 700, (0, 250))])
@pytest.mark.parametrize("b", [1, 3, 7, 32, 64, 130])
def test_spmm_random(torch_cuda, shape, b):
    torch = torch_cuda
    from paper_1804_03415_amd import spmm
    nr, nc, per = shape
    rp, ci, v = wl.random_csr(nr, nc, per, seed=nr + b, empty_frac=0.1)
    X = wl.random_block(nc, b, seed=b)
    A = sp.csr_matrix((v, ci, rp), shape=(nr, nc))
    ref = A @ X
    Y = spmm(_t(torch, rp), _t(torch, ci), _t(torch, v), _t(torch, X), n_cols=nc).cpu().numpy()
    bound = 1e-14 * (abs(A) @ np.abs(X)) + 1e-300
    assert np.all(np.abs(Y - ref) <= 8 * bound)


# ------------------------------------------------------------------- decomposition parity
CASES = {
    "grid2d_32": (lambda: wl.grid2d(32), dict(levels=3, exact_max_n=4096)),
    "rgg_2000": (lambda: wl.rgg(2000, 0), dict(levels=3)),
    "knn_1500": (lambda: wl.knn_gmm(1500, 10, 1), dict(levels=2)),
    "grid3d_8": (lambda: wl.grid3d_lognormal(8, 0), dict(levels=2, grid_blocks=(2, 2))),
    # partition to prescribed accuracy (eps_1, eta, c) on the SwissRoll graph
    "swissroll_3000": (lambda: wl.swissroll(3000, seed=2), dict(levels=2, eps1=1e-5, eta=0.1,
                                                                cbound=20.0, r_hops=5)),
}


def _oracle_build(p, kw):
    return mm.build_mmd(p.scipy(), coords=None if p.grid else p.coords, grid=p.grid, **kw)


@pytest.fixture(scope="module", params=sorted(CASES))
def built(request, torch_cuda):
    from paper_1804_03415_amd import Decomposition
    make, kw = CASES[request.param]
    p = make()
    dec = Decomposition.from_problem(p, **kw)
    return p, kw, dec, _oracle_build(p, kw)


def test_build_parity(built):
    p, kw, dec, M = built
    info = dec.info()
    assert info["sizes"] == [l.n for l in M.levels]
    assert np.allclose(info["eps"], M.eps, rtol=1e-10)
    for k in range(1, M.K + 1):
        for which, ref in ((0, M.levels[k].A), (1, M.levels[k].M), (2, M.levels[k].Psi)):
            rp, ci, v, shape = dec.export(k, which)
            X = sp.csr_matrix((v, ci, rp), shape=shape)
            assert X.shape == ref.shape
            # same stored pattern, except entries that are zero in exact
            # arithmetic and come out as rounding noise on one side only (the
            # coarse SwissRoll basis has 27 such in 17413); the value check
            # below holds every one-sided entry to 1e-11 max|ref|
            Xs = sp.csr_matrix((np.ones(X.nnz), X.indices, X.indptr), shape=shape)
            Rs = sp.csr_matrix((np.ones(ref.nnz), ref.indices, ref.indptr), shape=shape)
            only = (Xs - Rs).tocsr()
            only.eliminate_zeros()
            assert only.nnz <= 1e-2 * ref.nnz
            assert abs(X - ref).max() <= 1e-11 * abs(ref).max()


def _export(dec, k, which):
    rp, ci, v, shape = dec.export(k, which)
    return sp.csr_matrix((v, ci, rp), shape=shape)


def spmv_bar(A, X, ref):
    """1e-12 max|ref|, or the rounding bound of length-m dot products,
    gamma_m |A| |X| with m the longest stored row (Higham's gamma_m = m u /
    (1 - m u), doubled for two summation orders), whichever is larger: dense
    coarse rows (hundreds of entries) sum with cancellation."""
    A = sp.csr_matrix(A)
    m = int(np.diff(A.indptr).max()) if A.nnz else 1
    u = 2.0 ** -53
    return np.maximum(1e-12 * np.abs(ref).max(), 2 * m * u / (1 - m * u) * (abs(A) @ np.abs(X)))


def solve_floor(A, X, B):
    """Attainable accuracy of a recursive-residual Krylov solve, relative to
    ||b||: c u ||A|| ||x|| with c = 50, or 5 m for rows of m entries (each
    product's rounding grows with the row length)."""
    A = sp.csr_matrix(A)
    m = int(np.diff(A.indptr).max()) if A.nnz else 1
    c = max(50.0, 5.0 * m)
    return c * 2.2e-16 * sla.norm(A.toarray(), 2) * np.linalg.norm(X, axis=0) / np.linalg.norm(
        B, axis=0)


def test_level_operators(built, torch_cuda):
    torch = torch_cuda
    p, kw, dec, M = built
    b = 5
    for k in range(0, M.K + 1):
        lev = M.levels[k]
        X = wl.random_block(lev.n, b, seed=k)
        refA = krylov.EdgeForm(p.scipy()) @ X if k == 0 else lev.A @ X
        Y = dec.apply(k, "A", _t(torch, X)).cpu().numpy()
        # the kernel against the library's own matrix (rounding bound), and
        # against the oracle's matrix at the build-parity bar (coarse entries
        # agree to 1e-11 of the largest: their local solves are ill conditioned)
        Alib = p.scipy() if k == 0 else _export(dec, k, 0)
        assert np.all(np.abs(Y - Alib @ X) <= spmv_bar(Alib, X, Alib @ X))
        assert np.abs(Y - refA).max() <= 1e-11 * np.abs(refA).max()
        if k >= 1:
            Y = dec.apply(k, "M", _t(torch, X)).cpu().numpy()
            Mlib = _export(dec, k, 1)
            assert np.all(np.abs(Y - Mlib @ X) <= spmv_bar(Mlib, X, Mlib @ X))
            refM = lev.M @ X
            assert np.abs(Y - refM).max() <= 1e-11 * np.abs(refM).max()
        if k < M.K:
            up = M.levels[k + 1]
            Y = dec.apply(k, "Ut", _t(torch, X)).cpu().numpy()
            ref = up.Ut_apply(X)
            assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
            Xr = wl.random_block(up.nb(), b, seed=10 + k)
            Y = dec.apply(k, "U", _t(torch, Xr)).cpu().numpy()
            ref = up.U_apply(Xr)
            assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
            Aop = krylov.EdgeForm(p.scipy()) if k == 0 else lev.A
            ref = up.Ut_apply(Aop @ up.U_apply(Xr))
            Y = dec.apply(k, "B", _t(torch, Xr)).cpu().numpy()
            assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()
            Xc = wl.random_block(up.n, b, seed=20 + k)
            Y = dec.apply(k, "Psi", _t(torch, Xc)).cpu().numpy()
            Plib = _export(dec, k + 1, 2)
            assert np.all(np.abs(Y - Plib @ Xc) <= spmv_bar(Plib, Xc, Plib @ Xc))
            ref = up.Psi @ Xc
            assert np.abs(Y - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("b", [33, 64, 130, 300])
def test_level0_wide_apply_and_solve(built, torch_cuda, b):
    """Level-0 block products wider than 32 columns: the LDS-tiled SpMM on the
    graphs with coordinates (Morton row order), the row-per-wavefront kernel
    on the grids; plain product and the fused CG form inside a block solve,
    1, 2 and 5 column tiles with ragged last tiles."""
    torch = torch_cuda
    p, kw, dec, M = built
    X = wl.random_block(p.n, b, seed=40 + b)
    ref = krylov.EdgeForm(p.scipy()) @ X
    Y = dec.apply(0, "A", _t(torch, X)).cpu().numpy()
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()
    tol = 1e-10
    Ad = p.scipy()
    rhs = wl.random_block(p.n, b, seed=60 + b)
    Xs, it = dec.solve(0, 0, _t(torch, rhs), tol=tol)
    Xs = Xs.cpu().numpy()
    nb = np.linalg.norm(rhs, axis=0)
    floor = 50 * 2.2e-16 * float(abs(Ad).sum(axis=1).max()) * np.linalg.norm(Xs, axis=0) / nb
    res = np.linalg.norm(rhs - Ad @ Xs, axis=0) / nb
    assert np.all(res <= 1.5 * tol + floor)


def test_deferred_cg_step_matches_separate_update(torch_cuda, monkeypatch):
    """Level-0 block CG with each step's X and R update folded into the next
    step's tiled SpMM (the default) against the form with a separate update
    pass (MMDEIG_CG_DEFER=0).  The two are the same CG in exact arithmetic;
    in rounding they differ in the order of the dot products and in beta,
    whose residual norm is expanded from r.r, r.q and q.q of the previous
    step instead of summed after the update.  Over hundreds of steps at
    condition ~1e7 that moves a column's stopping step by a few (a float64
    model of both forms on a 5000-point RGG: 0 to 2 of ~600), so the
    comparison is of the work (total column-steps within 1%, each column
    within 5% + 2 steps) and of the result (both meet the tolerance).  The
    right-hand sides A^m g (m = 0, 1, 2) converge at different steps, so the
    working set is compacted several times while steps are pending; 150
    columns leave a ragged third 64-column slice."""
    torch = torch_cuda
    from paper_1804_03415_amd import Decomposition
    p = wl.rgg(20000, 3)
    Ad = p.scipy()
    dec = Decomposition.from_problem(p, levels=2, targets=(4, 8))
    b = 150
    g = wl.random_block(p.n, b, seed=77)
    rhs = g.copy()
    rhs[:, 50:100] = Ad @ g[:, 50:100]
    rhs[:, 100:] = Ad @ (Ad @ g[:, 100:])
    tol = 1e-9
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("MMDEIG_CG_DEFER", mode)
        X, it = dec.solve(0, 0, _t(torch, rhs), tol=tol)
        out[mode] = (X.cpu().numpy(), it.copy())
    dec.close()
    (Xd, itd), (Xp, itp) = out["1"], out["0"]
    assert len(set(itp.tolist())) > 10  # the columns stop at many different steps
    itd, itp = itd.astype(int), itp.astype(int)
    assert itd.sum() <= 1.01 * itp.sum() and itp.sum() <= 1.01 * itd.sum()
    assert np.all(np.abs(itd - itp) <= 0.05 * itp + 2)
    nb = np.linalg.norm(rhs, axis=0)
    for Xs in (Xd, Xp):
        floor = 50 * 2.2e-16 * float(abs(Ad).sum(axis=1).max()) * np.linalg.norm(Xs, axis=0) / nb
        res = np.linalg.norm(rhs - Ad @ Xs, axis=0) / nb
        assert np.all(res <= 1.5 * tol + floor)


def test_level0_tiling_engaged(torch_cuda, capfd, monkeypatch):
    """The tiled SpMM is what runs on a graph with coordinates (the build log
    reports the timed tile shapes and the one in use)."""
    from paper_1804_03415_amd import Decomposition
    monkeypatch.setenv("MMDEIG_LOG", "1")
    p = wl.rgg(3000, 2)
    dec = Decomposition.from_problem(p, levels=2)
    err = capfd.readouterr().err
    assert "level-0 tile shapes" in err and "; using " in err
    X = wl.random_block(p.n, 96, seed=5)
    Y = dec.apply(0, "A", _t(torch_cuda, X)).cpu().numpy()
    ref = krylov.EdgeForm(p.scipy()) @ X
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("b", [1, 4])
def test_level_solves(built, torch_cuda, b):
    """b = 1 runs the persistent single-vector kernel (from zero and from a
    caller's start), b = 4 the block kernels."""
    torch = torch_cuda
    p, kw, dec, M = built
    tol = 1e-10
    for k in range(0, M.K + 1):
        lev = M.levels[k]
        Ad = p.scipy().toarray() if k == 0 else lev.A.toarray()
        rhs = wl.random_block(lev.n, b, seed=30 + k)
        X, it = dec.solve(k, 0, _t(torch, rhs), tol=tol)
        X = X.cpu().numpy()
        # true residual within the solver's stop rule plus the attainable FP64
        # accuracy of a recursive-residual Krylov method, c u ||A|| ||x|| / ||b||
        nb = np.linalg.norm(rhs, axis=0)
        floor = solve_floor(p.scipy() if k == 0 else lev.A, X, rhs)
        res = np.linalg.norm(rhs - Ad @ X, axis=0) / nb
        assert np.all(res <= 1.5 * tol + floor)
        Aop = krylov.EdgeForm(p.scipy()) if k == 0 else lev.A
        for c in range(b):
            xo = krylov.pcg(lambda v: Aop @ v, rhs[:, c], lev.M, None, tol)
            # same system, same stop rule: the two solutions agree to the solve accuracy
            err = np.linalg.norm(X[:, c] - xo) / np.linalg.norm(xo)
            cond = np.linalg.cond(Ad) if lev.n <= 4096 else 1e8
            assert err <= 3 * tol * cond
        if b == 1:
            # warm start (x0 from the caller, as in the refinement): from the
            # solution scaled by 1 + 1e-6 the start residual is ~1e-6 ||b||, so
            # the solve meets the same tolerance in no more iterations, and in
            # fewer unless the cold solve itself needs only a handful
            Xw, itw = dec.solve(k, 0, _t(torch, rhs), x0=_t(torch, X * (1.0 + 1e-6)), tol=tol)
            Xw = Xw.cpu().numpy()
            floor = solve_floor(p.scipy() if k == 0 else lev.A, Xw, rhs)
            res = np.linalg.norm(rhs - Ad @ Xw, axis=0) / nb
            assert np.all(res <= 1.5 * tol + floor)
            assert itw[0] <= it[0] and (it[0] <= 10 or itw[0] < it[0])
        if k < M.K:
            up = M.levels[k + 1]
            U = up.U_apply(np.eye(up.nb()))
            B = U.T @ Ad @ U
            r2 = wl.random_block(up.nb(), max(b, 2), seed=40 + k)
            G, it = dec.solve(k, 1, _t(torch, r2), tol=tol)
            G = G.cpu().numpy()
            nb2 = np.linalg.norm(r2, axis=0)
            floor = solve_floor(sp.csr_matrix(B), G, r2)
            res = np.linalg.norm(r2 - B @ G, axis=0) / nb2
            assert np.all(res <= 1.5 * tol + floor)


@pytest.mark.parametrize("b", [3, 70])
def test_level0_mixed_solve(built, torch_cuda, b):
    """FP32 CG inside FP64 iterative refinement (solve kind 2): the FP64 true
    residual meets the same stop rule as the FP64 solve, and the FP32 inner
    iterations stay within a bounded multiple of the FP64 CG iterations (a
    wrong FP32 operator would still converge through the FP64 loop, only
    slowly).  Without a deflation basis, random right-hand sides of the
    near-singular graph Laplacians (shift 1e-6) cost FP32 CG several times the
    FP64 iterations: rounding at the FP32 level keeps re-exciting the
    near-null components.
    b = 3 runs the narrow FP32 SpMM, b = 70 the 128-column form and column
    compaction."""
    torch = torch_cuda
    p, kw, dec, M = built
    tol = 1e-10
    Ad = p.scipy()
    rhs = wl.random_block(p.n, b, seed=50 + b)
    X, it = dec.solve(0, 2, _t(torch, rhs), tol=tol)
    X = X.cpu().numpy()
    nb = np.linalg.norm(rhs, axis=0)
    floor = 50 * 2.2e-16 * sla.norm(Ad.toarray(), 2) * np.linalg.norm(X, axis=0) / nb
    res = np.linalg.norm(rhs - Ad @ X, axis=0) / nb
    assert np.all(res <= 1.5 * tol + floor)
    X64, it64 = dec.solve(0, 0, _t(torch, rhs), tol=tol)
    X64 = X64.cpu().numpy()
    cond = np.linalg.cond(Ad.toarray()) if p.n <= 4096 else 1e8
    err = np.linalg.norm(X - X64, axis=0) / np.linalg.norm(X64, axis=0)
    assert np.all(err <= 3 * tol * cond)
    assert np.all(it <= 8 * it64 + 100)


# ------------------------------------------------------------------- eigensolver
def _run_both(p, nev, tol, kw, precision="fp64"):
    from paper_1804_03415_amd import Decomposition
    dec = Decomposition.from_problem(p, **kw)
    lam, V, st = dec.eig_leftmost(nev, tol=tol, precision=precision)
    okw = dict(kw)
    okw["coords"] = None if p.grid else p.coords
    okw["grid"] = p.grid
    lo, Vo = krylov.eig_leftmost(p.scipy(), nev, tol, mmd_kwargs=okw)
    return lam, V.cpu().numpy().T, st, lo, Vo


def _closed_2d(n, count):
    j = np.arange(1, n + 1)
    s = 4 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())[:count]


def test_eig_c1_grid(torch_cuda):
    p = wl.grid2d(32)
    lam, V, st, lo, Vo = _run_both(p, 50, 1e-10, dict(levels=3, exact_max_n=4096))
    ref = _closed_2d(32, 50)
    assert np.max(np.abs(lam - ref) / ref) < 1e-10
    assert np.max(np.abs(lam - lo) / lo) < 1e-10
    ang, cl = dense.cluster_angles(lo, Vo, V)
    assert ang.max() < 1e-8
    assert dense.rel_residuals(p.scipy(), lam, V).max() < 1e-8
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-13)


@pytest.mark.parametrize("case", ["rgg", "knn", "grid3d_const"])
def test_eig_small(torch_cuda, case):
    if case == "rgg":
        p, nev, kw = wl.rgg(400, 11, mean_degree=5), 30, dict(levels=2)
    elif case == "knn":
        p, nev, kw = wl.knn_gmm(300, 10, 1), 15, dict(levels=2)
    else:
        p, nev, kw = wl.grid3d_lognormal(8, 0, sigma=0.0), 20, dict(levels=1, grid_blocks=(2,))
    lam, V, st, lo, Vo = _run_both(p, nev, 1e-11, kw)
    A = p.scipy()
    if case == "grid3d_const":
        null = np.zeros(nev, bool)
    else:
        null = check_shift_cluster(A, lo)
        check_shift_cluster(A, lam)
    assert np.max(np.abs(lam[~null] - lo[~null]) / lo[~null]) < 1e-10
    ang, cl = dense.cluster_angles(lo, Vo, V)
    full = [i for i, c in enumerate(cl) if c[-1] < nev - 1]
    assert ang[full].max() < 1e-8
    assert dense.rel_residuals(A, lam, V).max() < 1e-8


@pytest.mark.parametrize("case", ["c1_grid", "rgg"])
def test_eig_mixed(torch_cuda, case):
    """precision fp32-refine: the same bars against the oracle as the FP64 mode,
    and per-eigenpair agreement with the FP64 GPU run."""
    if case == "c1_grid":
        p, nev, tol, kw = wl.grid2d(32), 50, 1e-10, dict(levels=3, exact_max_n=4096)
    else:
        p, nev, tol, kw = wl.rgg(400, 11, mean_degree=5), 30, 1e-11, dict(levels=2)
    lam, V, st, lo, Vo = _run_both(p, nev, tol, kw, precision="fp32-refine")
    A = p.scipy()
    if case == "c1_grid":
        null = np.zeros(nev, bool)
    else:
        null = check_shift_cluster(A, lo)
        check_shift_cluster(A, lam)
    assert np.max(np.abs(lam[~null] - lo[~null]) / lo[~null]) < 1e-10
    if case == "c1_grid":
        ref = _closed_2d(32, 50)
        assert np.max(np.abs(lam - ref) / ref) < 1e-10
    ang, cl = dense.cluster_angles(lo, Vo, V)
    full = [i for i, c in enumerate(cl) if c[-1] < nev - 1]
    assert ang[full].max() < 1e-8
    assert dense.rel_residuals(A, lam, V).max() < 1e-8
    from paper_1804_03415_amd import Decomposition
    dec = Decomposition.from_problem(p, **kw)
    l64, V64, _ = dec.eig_leftmost(nev, tol=tol)
    assert np.max(np.abs(lam - l64) / l64) < 1e-10
    a64, _ = dense.cluster_angles(l64, V64.cpu().numpy().T, V)
    assert a64[full].max() < 1e-8


def test_eig_knn_coarse_tolerance(torch_cuda):
    """kNN graph whose coarse-level eps^(k) = 0.1 eps_k exceeds 1 (no rescaling):
    the capped relative PCG tolerance keeps OP nonzero on those levels; GPU and
    oracle agree with dense eigenpairs."""
    p = wl.knn_gmm(3000, 10, 1)
    kw = dict(levels=3, exact_max_n=8000)
    lam, V, st, lo, Vo = _run_both(p, 12, 1e-10, kw)
    A = p.scipy()
    w, Z = dense.smallest_dense(A, 12)
    # the shift eigenvalue of the stored matrix against its reference; dense
    # eigvalsh knows it to absolute u ||A|| only, so it is left out there
    null = check_shift_cluster(A, lo)
    check_shift_cluster(A, lam)
    assert np.max(np.abs(lo[~null] - w[~null]) / w[~null]) < 1e-10
    assert np.max(np.abs(lam[~null] - w[~null]) / w[~null]) < 1e-10
    ang, cl = dense.cluster_angles(w, Z, V)
    assert ang.max() < 1e-8
    assert dense.rel_residuals(A, lam, V).max() < 1e-8


# ------------------------------------------------------------------- FP32 operator (a4)
@pytest.mark.parametrize("b", [1, 3, 64, 70, 129])
def test_fp32_level0_operator_elementwise(built, torch_cuda, b):
    """The FP32 kernel of the mixed-precision solves (mmd_apply op "A32"),
    entry by entry.  Reference: the same edge form y_i = s_i x_i +
    sum_j w_ij (x_i - x_j) evaluated in FP64 on the FP32-rounded x, w and s,
    so the only difference is FP32 arithmetic: |y - ref| <= (deg_i + 3) u32
    (|s_i x_i| + sum_j w_ij (|x_i| + |x_j|)).  b = 1, 3: the narrow kernel;
    64: its widest form; 70, 129: the 128-column float2 kernel with ragged
    last column tiles."""
    torch = torch_cuda
    p, kw, dec, M = built
    E = krylov.EdgeForm(p.scipy())
    E.w = E.w.astype(np.float32).astype(np.float64)
    E.s = E.s.astype(np.float32).astype(np.float64)
    X = wl.random_block(p.n, b, seed=70 + b).astype(np.float32).astype(np.float64)
    ref = E @ X
    ax = np.abs(X)
    mag = E.s[:, None] * ax + np.stack(
        [np.bincount(E.rows, weights=E.w * (ax[E.rows, c] + ax[E.cols, c]), minlength=p.n)
         for c in range(b)], axis=1)
    deg = np.bincount(E.rows, minlength=p.n)
    bound = (deg + 3)[:, None] * 2.0 ** -24 * mag
    Y = dec.apply(0, "A32", _t(torch, X)).cpu().numpy()
    assert np.all(np.abs(Y - ref) <= bound + 1e-300)
    # not the FP64 kernel: FP32 rounding is visible somewhere
    Y64 = dec.apply(0, "A", _t(torch, X)).cpu().numpy()
    assert np.abs(Y - Y64).max() > 0


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_level0_tile_shapes(torch_cuda, shape, monkeypatch):
    """Every tile shape of the LDS-staged level-0 SpMMs, forced instead of
    chosen by the build-time timing (MMDEIG_TILE): the FP64 product (plain
    and inside the fused block CG of a solve) and the FP32 product of the
    edge form, with ragged column slices."""
    from paper_1804_03415_amd import Decomposition
    torch = torch_cuda
    monkeypatch.setenv("MMDEIG_TILE", str(shape))
    p = wl.rgg(6000, 7)
    dec = Decomposition.from_problem(p, levels=1)
    E = krylov.EdgeForm(p.scipy())
    for b in (33, 70, 257):
        X = wl.random_block(p.n, b, seed=90 + b)
        ref = E @ X
        Y = dec.apply(0, "A", _t(torch, X)).cpu().numpy()
        assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()
    rhs = wl.random_block(p.n, 70, seed=97)
    Xs, it = dec.solve(0, 0, _t(torch, rhs), tol=1e-10)
    Xs = Xs.cpu().numpy()
    res = np.linalg.norm(rhs - p.scipy() @ Xs, axis=0) / np.linalg.norm(rhs, axis=0)
    assert np.all(res <= 1.5e-10 + solve_floor(p.scipy(), Xs, rhs))
    E32 = krylov.EdgeForm(p.scipy())
    E32.w = E32.w.astype(np.float32).astype(np.float64)
    E32.s = E32.s.astype(np.float32).astype(np.float64)
    for b in (70, 129):
        X = wl.random_block(p.n, b, seed=80 + b).astype(np.float32).astype(np.float64)
        ref = E32 @ X
        ax = np.abs(X)
        mag = E32.s[:, None] * ax + np.stack(
            [np.bincount(E32.rows, weights=E32.w * (ax[E32.rows, c] + ax[E32.cols, c]),
                         minlength=p.n) for c in range(b)], axis=1)
        deg = np.bincount(E32.rows, minlength=p.n)
        Y = dec.apply(0, "A32", _t(torch, X)).cpu().numpy()
        assert np.all(np.abs(Y - ref) <= (deg + 3)[:, None] * 2.0 ** -24 * mag + 1e-300)
    dec.close()


def test_graph_replay_matches_eager(torch_cuda, monkeypatch):
    """Block-CG chunks replayed as HIP graphs run the same kernels with the
    same arguments as the eager launches: a narrow level-0 block solve, the CG
    on B^(1) and a whole eigensolve give bit-identical results with graphs on and
    off, over many replays (each chunk of a stage replays one graph, with the
    host's convergence checks and compactions between the replays)."""
    from paper_1804_03415_amd import Decomposition
    torch = torch_cuda
    p = wl.rgg(3000, 5)
    dec = Decomposition.from_problem(p, levels=2)
    info = dec.info()
    out = {}
    side = torch.cuda.Stream()   # graphs are captured on non-default streams only
    for g in ("0", "1"):
        monkeypatch.setenv("MMDEIG_GRAPHS", g)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            r1 = wl.random_block(info["sizes"][0], 4, seed=11)
            X1, it1 = dec.solve(0, 0, _t(torch, r1), tol=1e-10)
            nb = info["sizes"][0] - info["sizes"][1]
            rb = wl.random_block(nb, 6, seed=12)
            XB, itB = dec.solve(0, 1, _t(torch, rb), tol=1e-10)
            lam, V, st = dec.eig_leftmost(25, tol=1e-10)
        side.synchronize()
        out[g] = (X1.cpu().numpy(), it1, XB.cpu().numpy(), itB, lam, V.cpu().numpy())
    a, b = out["0"], out["1"]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
    assert max(a[1]) > 32 and max(a[3]) > 32      # several chunks, so several replays
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    dec.close()


# ------------------------------------------------------------------- sign rule, element-wise
@pytest.mark.parametrize("case", ["rgg", "knn"])
def test_eigenvectors_elementwise_after_sign_rule(torch_cuda, case):
    """Simple, well separated eigenvalues have a unique unit eigenvector up to
    sign; both sides return the canonical sign (largest-magnitude entry
    positive), so the vectors agree entry by entry within the 1e-8 angle bar.
    Columns whose two largest magnitudes nearly tie with opposite signs are
    skipped (rounding may decide that tie either way)."""
    if case == "rgg":
        p, nev, kw = wl.rgg(400, 11, mean_degree=5), 30, dict(levels=2)
    else:
        p, nev, kw = wl.knn_gmm(300, 10, 1), 15, dict(levels=2)
    lam, V, st, lo, Vo = _run_both(p, nev, 1e-11, kw)
    checked = 0
    for i in range(nev):
        lo_gap = (lo[i] - lo[i - 1]) / lo[i] if i > 0 else np.inf
        hi_gap = (lo[i + 1] - lo[i]) / lo[i] if i + 1 < nev else 0.0
        if min(lo_gap, hi_gap) < 1e-3:
            continue
        a = np.sort(np.abs(Vo[:, i]))[::-1]
        top = np.argsort(-np.abs(Vo[:, i]))[:2]
        if a[0] - a[1] < 1e-6 * a[0] and np.sign(Vo[top[0], i]) != np.sign(Vo[top[1], i]):
            continue
        assert np.abs(V[:, i] - Vo[:, i]).max() <= 1.5e-8
        assert V[np.argmax(np.abs(V[:, i])), i] > 0
        checked += 1
    assert checked >= 5


# ------------------------------------------------------------------- K = 0 (IRLM-CG) path
@pytest.mark.parametrize("case", ["grid2d_32", "rgg", "knn"])
def test_no_hierarchy_matches_oracle(torch_cuda, case):
    """levels = 0: no decomposition, restarted Lanczos on A^-1 with the
    level-0 CG as the operator (the paper's IRLM-CG comparison solver, Section
    8).  Against the oracle's K = 0 run (itself pinned equal to the MMD run and
    to dense eigenpairs) and, for the grid, the closed form."""
    if case == "grid2d_32":
        p, nev, tol = wl.grid2d(32), 50, 1e-10
    elif case == "rgg":
        # connected: single-vector Lanczos without the hierarchy cannot
        # resolve a repeated shift eigenvalue (a many-component graph ends in
        # the restart cap, in the oracle as here; at tol 1e-11 the oracle also
        # stalls there on the connected rgg(500, 2))
        p, nev, tol = wl.rgg(500, 3), 30, 1e-11
    else:
        p, nev, tol = wl.knn_gmm(300, 10, 1), 15, 1e-11
    lam, V, st, lo, Vo = _run_both(p, nev, tol, dict(levels=0))
    assert st["K"] == 0
    A = p.scipy()
    if case == "grid2d_32":
        null = np.zeros(nev, bool)
    else:
        null = check_shift_cluster(A, lo)
        check_shift_cluster(A, lam)
    assert np.max(np.abs(lam[~null] - lo[~null]) / lo[~null]) < 1e-10
    if case == "grid2d_32":
        assert np.max(np.abs(lam - _closed_2d(32, 50)) / _closed_2d(32, 50)) < 1e-10
    ang, cl = dense.cluster_angles(lo, Vo, V)
    full = [i for i, c in enumerate(cl) if c[-1] < nev - 1]
    assert ang[full].max() < 1e-8
    assert dense.rel_residuals(A, lam, V).max() < 1e-8


# ------------------------------------------------------------------- Lanczos breakdown
def _paths(n3, n2):
    """Disjoint 3-vertex and 2-vertex paths (unit weights) + 1e-6 I: the
    Laplacian spectrum {0, 1, 3} and {0, 2} repeated, so every Krylov space
    from one start vector has dimension <= 4 and Lanczos breaks down."""
    blocks = [sp.csr_matrix([[1., -1, 0], [-1, 2, -1], [0, -1, 1]])] * n3 + \
             [sp.csr_matrix([[1., -1], [-1, 1]])] * n2
    A = sp.csr_matrix(sp.block_diag(blocks, format="csr") + SHIFT * sp.eye(3 * n3 + 2 * n2))
    A.sort_indices()
    return A


@pytest.mark.parametrize("levels", [0, 1])
def test_lanczos_breakdown_multiplicity(torch_cuda, levels):
    """Breakdown handling of Alg. 3 (fresh random direction, deflated) and the
    level-0 multiplicity check: 60 three-vertex and 60 two-vertex paths, the
    130 smallest pairs are the 120-fold shift eigenvalue and 10 of the 60-fold
    eigenvalue 1 + 1e-6.  Any orthonormal basis of the cut cluster is valid:
    the values, the residuals, orthonormality and the invariant subspace are
    checked (the oracle gives the same values on this input)."""
    from paper_1804_03415_amd import Decomposition
    A = _paths(60, 60)
    dec = Decomposition(A.indptr, A.indices, A.data, levels=levels, targets=(4,))
    lam, V, st = dec.eig_leftmost(130, tol=1e-10)
    Vh = V.cpu().numpy().T
    check_shift_cluster(A, lam)
    assert np.all(np.abs(lam[120:] - (1 + SHIFT)) <= 1e-10 * (1 + SHIFT))
    assert np.abs(Vh.T @ Vh - np.eye(130)).max() < 1e-10
    assert dense.rel_residuals(A, lam, Vh).max() < 1e-8
    # the first 120 span exactly the component indicators
    C = sp.csr_matrix(A - SHIFT * sp.eye(A.shape[0]))
    assert np.linalg.norm(C @ Vh[:, :120]) < 1e-8
    lo, Vo = krylov.eig_leftmost(A, 130, 1e-10, mmd_kwargs=dict(levels=levels, targets=(4,)))
    check_shift_cluster(A, lo)
    assert np.max(np.abs(lam[120:] - lo[120:]) / lo[120:]) < 1e-10


# ------------------------------------------------------------------- solver error paths
def test_solver_error_paths(torch_cuda):
    """Status codes of eig_leftmost through the ABI: EINVAL for nev or tol out
    of range, ENOCONV when the refinement or restart caps are too small (the
    outputs are not written)."""
    from paper_1804_03415_amd import Decomposition, MMDError
    p = wl.grid2d(16)
    dec = Decomposition.from_problem(p, levels=2, grid_blocks=(2, 2), exact_max_n=4096)
    for nev, tol in ((0, 1e-10), (p.n + 1, 1e-10), (5, 0.0), (5, 1.5)):
        with pytest.raises(MMDError) as e:
            dec.eig_leftmost(nev, tol=tol)
        assert e.value.code == 1
    with pytest.raises(MMDError) as e:
        dec.eig_leftmost(20, tol=1e-10, max_refine=1)
    assert e.value.code == 4 and "refinement" in str(e.value)
    dec0 = Decomposition.from_problem(p, levels=0)
    with pytest.raises(MMDError) as e:
        dec0.eig_leftmost(20, tol=1e-10, max_restarts=1)
    assert e.value.code == 4
    # the handle stays usable after an error
    lam, V, st = dec.eig_leftmost(10, tol=1e-10)
    assert np.max(np.abs(lam - _closed_2d(16, 10)) / _closed_2d(16, 10)) < 1e-10


# ------------------------------------------------------------------- coarse-level approximation
@pytest.mark.parametrize("case", ["grid2d_32", "rgg"])
def test_coarse_level_approximation(torch_cuda, case):
    """stop_level = k (Section 7.3): the level-k pairs lifted by Psi^(1) ...
    Psi^(k), against the oracle's coarse mode and the dense generalized
    eigenproblem of the exported A^(k), M^(k); on the exact-Psi grid also the
    Lemma 3.3 bounds |mu_i - mu_i(A^-1)| <= eps_k, ||A^-1 v - mu v|| <= 2 eps_k."""
    from paper_1804_03415_amd import Decomposition
    if case == "grid2d_32":
        p, kw, runs = wl.grid2d(32), dict(levels=3, exact_max_n=4096), ((3, 4), (2, 10), (1, 20))
    else:
        p, kw, runs = wl.rgg(900, 5), dict(levels=2), ((2, 8), (1, 12))
    A = p.scipy()
    dec = Decomposition.from_problem(p, **kw)
    info = dec.info()
    okw = dict(kw)
    okw["coords"] = None if p.grid else p.coords
    okw["grid"] = p.grid
    Mo = mm.build_mmd(A, **okw)
    Ad = A.toarray()
    w = np.linalg.eigvalsh(Ad)
    Ainv = np.linalg.inv(Ad) if case == "grid2d_32" else None
    for k, nev in runs:
        lam, V, st = dec.eig_leftmost(nev, tol=1e-10, stop_level=k)
        Vh = V.cpu().numpy().T
        eps_k = info["eps"][k]
        lo, Vo = krylov.eig_leftmost(A, nev, 1e-10, mmd=Mo, stop_level=k)
        mu, muo = 1.0 / lam, 1.0 / lo
        assert np.all(np.diff(lam) >= 0)
        assert np.abs(Vh.T @ Vh - np.eye(nev)).max() < 1e-10
        rp, ci, v, shape = dec.export(k, 0)
        Ak = sp.csr_matrix((v, ci, rp), shape=shape).toarray()
        rp, ci, v, shape = dec.export(k, 1)
        Mk = sp.csr_matrix((v, ci, rp), shape=shape).toarray()
        mu_k = 1.0 / sla.eigh(Ak, Mk, eigvals_only=True)[:nev]
        bar = 1e-10 * mu_k.max() if k == info["K"] else 0.25 * eps_k
        assert np.max(np.abs(mu - mu_k)) <= bar
        assert np.max(np.abs(mu - muo)) <= 2 * bar
        assert np.all(lam >= w[:nev] * (1 - 1e-10))
        if Ainv is not None:
            assert np.max(np.abs(mu - 1.0 / w[:nev])) <= 1.1 * eps_k
            R = Ainv @ Vh - Vh / w[None, :nev]
            assert np.max(np.linalg.norm(R, axis=0)) <= 2.2 * eps_k


def test_swissroll_prescribed_accuracy(torch_cuda):
    """SwissRoll graph (Section 7.1, 2000 points at the full roll's density)
    decomposed with the paper's (eps_1, eta, c) = (1e-5, 0.1, 20): the level
    sizes match the oracle's, the full solve (Alg. 6 continued to level 0)
    matches the oracle pair by pair, and the paper's own output (stop at
    level 1) meets Lemma 3.3, |mu_i - mu_i(A^-1)| <= eps_1, against the dense
    spectrum, and matches the oracle's coarse mode."""
    from paper_1804_03415_amd import Decomposition
    p = wl.swissroll(2000, seed=2)
    kw = dict(levels=2, eps1=1e-5, eta=0.1, cbound=20.0, r_hops=5)
    A = p.scipy()
    dec = Decomposition.from_problem(p, **kw)
    info = dec.info()
    Mo = mm.build_mmd(A, coords=p.coords, **kw)
    assert info["sizes"] == [lev.n for lev in Mo.levels]
    w = np.linalg.eigvalsh(A.toarray())
    nev = 20
    lam, V, st = dec.eig_leftmost(nev, tol=1e-10)
    lo, Vo = krylov.eig_leftmost(A, nev, 1e-10, mmd=Mo)
    assert np.max(np.abs(lam - lo) / lo) < 1e-10
    assert np.max(np.abs(lam - w[:nev]) / w[:nev]) < 1e-9
    Vh = V.cpu().numpy().T
    ang, cl = dense.cluster_angles(lo, Vo, Vh)
    assert ang.max() < 1e-7
    assert dense.rel_residuals(A, lam, Vh).max() < 1e-8
    lam1, V1, _ = dec.eig_leftmost(nev, tol=1e-10, stop_level=1)
    lo1, _ = krylov.eig_leftmost(A, nev, 1e-10, mmd=Mo, stop_level=1)
    eps1 = info["eps"][1]
    assert eps1 <= 1e-5
    assert np.max(np.abs(1.0 / lam1 - 1.0 / w[:nev])) <= eps1
    assert np.max(np.abs(1.0 / lam1 - 1.0 / lo1)) <= 0.5 * eps1
    dec.close()


# ------------------------------------------------------------------- FP64 MFMA products (a8)
@pytest.mark.parametrize("n,m,p", [(1, 1, 1), (5, 7, 3), (1000, 16, 16), (4099, 65, 33),
                                   (100003, 300, 300), (20000, 301, 17)])
def test_mfma_gram_and_gemm(torch_cuda, n, m, p):
    """C = X^T Y and Z = alpha X C + beta Z on the FP64 matrix cores, entry by
    entry against numpy FP64, within the worst-case rounding of a length-k
    FP64 dot product, (k + 16) u (|X|^T |Y|) (k = n or m): a wrong lane layout
    or tile index gives O(1) errors.  Shapes cover single elements, partial
    16 x 16 MFMA tiles, partial 64 x 64 workgroup tiles and the refinement's
    300-column blocks over 1e5 rows."""
    torch = torch_cuda
    from paper_1804_03415_amd import gemm, gram
    u = 2.0 ** -52
    X = wl.random_block(n, m, seed=n + m)
    Y = wl.random_block(n, p, seed=n + p + 1)
    C = gram(_t(torch, X), _t(torch, Y)).cpu().numpy()
    ref = X.T @ Y
    bound = (n + 16) * u * (np.abs(X).T @ np.abs(Y))
    assert np.all(np.abs(C - ref) <= bound)
    Cm = wl.random_block(m, p, seed=m * p)
    Z0 = wl.random_block(n, p, seed=7)
    Z = gemm(_t(torch, X), _t(torch, Cm), _t(torch, Z0), alpha=-0.5, beta=2.0).cpu().numpy()
    ref = -0.5 * (X @ Cm) + 2.0 * Z0
    bound = (m + 16) * u * (0.5 * np.abs(X) @ np.abs(Cm) + 2.0 * np.abs(Z0))
    assert np.all(np.abs(Z - ref) <= bound)
