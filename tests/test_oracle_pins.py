"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed-form spectra, theorems of the paper stated as
invariants, brute-force dense linear algebra, or graph facts.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as wl
from oracle import dense, energy, krylov, mmd as mm
from oracle.philox import philox4x32_10, uniform_vector


# --------------------------------------------------------------------------- philox
def test_philox_known_answers():
    # Random123 known-answer vectors for philox4x32_10
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, out in kat:
        assert [int(x) for x in philox4x32_10(ctr, key)] == out


def test_uniform_vector_range_and_determinism():
    v = uniform_vector(1001, 7, 2, 3)
    assert v.shape == (1001,)
    assert np.all(v >= -0.5) and np.all(v < 0.5)
    assert np.array_equal(v, uniform_vector(1001, 7, 2, 3))
    assert not np.array_equal(v, uniform_vector(1001, 7, 2, 4))
    assert abs(v.mean()) < 0.05


# --------------------------------------------------------------------------- inputs
def test_workload_shapes():
    p = wl.grid2d(32)
    assert (p.n, p.nnz) == (1024, 4992)
    A = p.scipy()
    assert abs(A - A.T).max() == 0
    p3 = wl.grid3d_lognormal(16, 0)
    assert p3.nnz == 16 ** 3 + 6 * 16 * 16 * 15


def test_rgg_components_and_shift():
    p = wl.rgg(100000, 0)
    assert p.nnz == 1096918
    assert dense.component_count(p.scipy()) == 8


# --------------------------------------------------------------------------- energy
def test_interior_energy_level0_is_internal_laplacian_plus_selfloops():
    p = wl.rgg(500, 3)
    A = p.scipy()
    ei, ej, w, s = energy.energy_elements(A)
    mem = np.sort(np.random.default_rng(0).choice(500, 12, replace=False))
    # independent construction from the element list
    pos = {int(v): a for a, v in enumerate(mem)}
    E = np.diag(s[mem]).astype(float)
    for i, j, wij in zip(ei, ej, w):
        if int(i) in pos and int(j) in pos:
            a, b = pos[int(i)], pos[int(j)]
            E[a, a] += wij; E[b, b] += wij; E[a, b] -= wij; E[b, a] -= wij
    assert np.allclose(energy.interior_energy(A, mem), E, atol=1e-14)


def test_energy_rejects_positive_offdiagonal():
    A = sp.csr_matrix(np.array([[2.0, 0.5], [0.5, 2.0]]))
    with pytest.raises(energy.UnsupportedMatrix):
        energy.energy_elements(A)


# --------------------------------------------------------------------------- partition / Householder
def test_partitions_cover_exactly_once():
    p = wl.rgg(3000, 1)
    pt = mm.greedy_partition(p.scipy(), p.coords, 6)
    allv = np.concatenate(pt)
    assert np.array_equal(np.sort(allv), np.arange(3000))
    g, cg = mm.grid_partition((32, 32), 4)
    assert len(g) == 64 and cg == (8, 8) and all(len(m) == 16 for m in g)
    assert list(g[1][:4]) == [4, 5, 6, 7]
    g3, c3 = mm.grid_partition((8, 8, 8), 2)
    assert len(g3) == 64 and all(len(m) == 8 for m in g3)


def test_householder_complement():
    """H_j is orthogonal, its pivot column is +-phi, the other columns span
    phi's complement; the pivot is the largest-magnitude entry, also when the
    first entry is zero or at rounding level."""
    rng = np.random.default_rng(0)
    for case in range(4):
        phi = rng.standard_normal(9)
        if case == 2:
            phi[0] = 0.0
        if case == 3:
            phi[0] = 1e-300
        phi /= np.linalg.norm(phi)
        if case == 1:
            phi = -phi
        u, t = mm.householder_vector(phi)
        assert t == int(np.argmax(np.abs(phi)))  # distinct magnitudes here
        H = np.eye(9) - 2 * np.outer(u, u) / (u @ u)
        assert np.allclose(H @ H.T, np.eye(9), atol=1e-14)
        assert np.allclose(H[:, t], -np.sign(phi[t]) * phi, atol=1e-14)
        rest = [i for i in range(9) if i != t]
        assert np.allclose(H[:, rest].T @ phi, 0, atol=1e-14)
    # maxima equal in exact arithmetic but not after rounding: the first one
    phi = np.array([0.1, 0.5, 0.5 * (1 + 1e-15), 0.5 * (1 - 1e-15), 0.2])
    phi /= np.linalg.norm(phi)
    assert mm.householder_vector(phi)[1] == 1
    assert mm.householder_vector(phi[::-1].copy())[1] == 1


# --------------------------------------------------------------------------- MMD invariants
@pytest.fixture(scope="module")
def c1_exact():
    p = wl.grid2d(32)
    return p, mm.build_mmd(p.scipy(), coords=p.coords, grid=p.grid, levels=3, exact_max_n=4096)


def _phi_matrix(lev, nfine):
    Phi = np.zeros((nfine, len(lev.patches)))
    for j, (m, ph) in enumerate(zip(lev.patches, lev.phis)):
        Phi[m, j] = ph
    return Phi


def _U_matrix(lev):
    nb = lev.nb()
    return lev.U_apply(np.eye(nb))


def test_mmd_exact_invariants(c1_exact):
    p, M = c1_exact
    A = p.scipy().toarray()
    l1 = M.levels[1]
    Psi = l1.Psi.toarray()
    Phi = _phi_matrix(l1, 1024)
    U = _U_matrix(l1)
    assert np.allclose(Phi.T @ Psi, np.eye(64), atol=1e-12)           # Phi^T Psi = I
    assert np.allclose(Phi.T @ Phi, np.eye(64), atol=1e-13)
    assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)       # QR completion
    assert np.allclose(U.T @ Phi, 0, atol=1e-13)
    assert np.abs(U.T @ A @ Psi).max() < 1e-11                         # U^T A Psi = 0
    B = U.T @ A @ U
    Ast = l1.A.toarray()
    Ainv = np.linalg.inv(A)
    rec = U @ np.linalg.solve(B, U.T) + Psi @ np.linalg.solve(Ast, Psi.T)
    assert np.abs(rec - Ainv).max() < 1e-10 * np.abs(Ainv).max()       # eq. Ainv_representation
    # Theorem 2.1: ||A^-1 - Theta|| <= eps(P)
    Theta = Psi @ np.linalg.solve(Ast, Psi.T)
    assert np.linalg.norm(Ainv - Theta, 2) <= M.levels[1].eps_level
    # Lemma 4.3: lambda_min(Psi^T Psi) >= 1
    assert np.linalg.eigvalsh(l1.M.toarray()).min() >= 1 - 1e-12
    # Theorem 2.2: lambda_min(A_st) >= lambda_min(A)
    assert np.linalg.eigvalsh(Ast).min() >= np.linalg.eigvalsh(A).min() * (1 - 1e-12)


def test_mmd_multilevel_ordering(c1_exact):
    """A^-1 = Theta^(0) >= Theta^(1) >= ... (Lemma 3.3): mu_i^(k) <= mu_i^(k-1)."""
    p, M = c1_exact
    prev = np.sort(1.0 / np.linalg.eigvalsh(p.scipy().toarray()))[::-1]
    for k in range(1, M.K + 1):
        lev = M.levels[k]
        lam = sla.eigh(lev.A.toarray(), lev.M.toarray(), eigvals_only=True)
        mu = np.sort(1.0 / lam)[::-1]
        assert np.all(mu <= prev[:mu.size] * (1 + 1e-10))
        # |mu_i - mu_i^(k)| <= eps_k for the essential pairs (Lemma 3.3, exact Psi)
        assert np.max(np.abs(prev[:mu.size] - mu)) <= M.eps[k] + 1e-9
        prev = mu


def test_mmd_localized_invariants():
    p = wl.rgg(1500, 2)
    A = p.scipy()
    M = mm.build_mmd(A, coords=p.coords, levels=2, targets=(4, 8), r_hops=1)
    lam0 = np.linalg.eigvalsh(A.toarray())
    for k in range(1, M.K + 1):
        lev, prev = M.levels[k], M.levels[k - 1]
        Phi = _phi_matrix(lev, prev.n)
        # KKT solves on patch neighbourhoods with condition ~1e7 (the 1e-6 shift)
        assert np.allclose(Phi.T @ lev.Psi.toarray(), np.eye(lev.n), atol=1e-8)
        Mk = lev.M.toarray()
        assert np.linalg.eigvalsh(Mk).min() >= 1 - 1e-10
        assert lev.lam_max_M >= np.linalg.eigvalsh(Mk).max() * (1 - 1e-12)
        lamk = sla.eigh(lev.A.toarray(), Mk, eigvals_only=True)
        # Rayleigh-Ritz on the nested subspace span(Psi-composite): interlacing
        assert np.all(lamk >= lam0[:lamk.size] * (1 - 1e-8))
        assert abs(lev.A - lev.A.T).max() == 0


# --------------------------------------------------------------------------- CG / PCG
def test_cg_and_pcg_match_dense_solve():
    p = wl.grid3d_lognormal(6, 1)
    A = p.scipy()
    b = np.random.default_rng(1).standard_normal(p.n)
    xs = np.linalg.solve(A.toarray(), b)
    x, it = krylov.cg(lambda v: A @ v, b, None, 1e-12)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    Mp = sp.csr_matrix(np.diag(np.linspace(1, 3, p.n)) + 0.0)
    xp = krylov.pcg(lambda v: A @ v, b, Mp, None, 1e-12)
    assert np.linalg.norm(xp - xs) <= 1e-9 * np.linalg.norm(xs)
    # warm start at the solution: zero iterations
    st = dict(pcg_A_calls=0, pcg_A_iters=0, pcg_A_max=0, cg_M_calls=0, cg_M_iters=0)
    krylov.pcg(lambda v: A @ v, b, Mp, xs, 1e-8, st)
    assert st["pcg_A_iters"] == 0


def test_cg_iteration_bound():
    """Theorem 4.2: iterations <= ceil(sqrt(kappa)/2 * ln(2 sqrt(kappa)/eps)) (l2 form)."""
    p = wl.grid2d(20)
    A = p.scipy()
    w = np.linalg.eigvalsh(A.toarray())
    kappa = w[-1] / w[0]
    b = np.random.default_rng(2).standard_normal(p.n)
    _, it = krylov.cg(lambda v: A @ v, b, None, 1e-10)
    bound = np.ceil(np.sqrt(kappa) / 2 * np.log(2 * np.sqrt(kappa) / 1e-10))
    assert it <= bound


def test_edge_form_equals_csr_and_keeps_null_vectors():
    p = wl.rgg(800, 4)
    A = p.scipy()
    E = krylov.EdgeForm(A)
    x = np.random.default_rng(3).standard_normal(p.n)
    assert np.allclose(E @ x, A @ x, rtol=0, atol=1e-13 * np.abs(A).max())
    ones = np.ones(p.n)
    assert np.array_equal(E @ ones, E.s)


# --------------------------------------------------------------------------- Lanczos / restart / refine
@pytest.fixture(scope="module")
def small_level():
    p = wl.grid2d(12)
    M = mm.build_mmd(p.scipy(), coords=p.coords, grid=p.grid, levels=1, grid_blocks=(2,), exact_max_n=10000)
    return p, M


def test_lanczos_relation_and_restart(small_level):
    p, M = small_level
    st = krylov.Stats()
    ops = krylov.LevelOps(M, 1, 1e-12, st)
    Mk = M.levels[1].M.toarray()
    Vini = np.zeros((ops.n, 0))
    L = krylov.Lanczos(ops, Vini, seed=5)
    L.steps(10)
    V, T = L.V, L.T
    assert np.allclose(V.T @ Mk @ V, np.eye(10), atol=1e-12)
    assert np.allclose(T, T.T) and np.allclose(np.triu(T, 2), 0, atol=1e-12)
    OPV = np.stack([ops.op(V[:, j]) for j in range(10)], axis=1)
    e = np.zeros(10); e[-1] = 1
    assert np.linalg.norm(OPV - V @ T - np.outer(L.f, e)) < 1e-9 * np.linalg.norm(OPV)
    theta_before = np.sort(np.linalg.eigvalsh(T))
    L.restart(6, 4)
    V, T = L.V, L.T
    assert V.shape[1] == 6
    assert np.allclose(V.T @ Mk @ V, np.eye(6), atol=1e-10)
    OPV = np.stack([ops.op(V[:, j]) for j in range(6)], axis=1)
    e = np.zeros(6); e[-1] = 1
    assert np.linalg.norm(OPV - V @ T - np.outer(L.f, e)) < 1e-8 * np.linalg.norm(OPV)
    # the shifts removed the 4 smallest Ritz values: remaining are the 6 largest
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), theta_before[4:], rtol=1e-10)


def test_refinement_converges_to_level_eigenpairs():
    p = wl.grid2d(16)
    A = p.scipy()
    M = mm.build_mmd(A, coords=p.coords, grid=p.grid, levels=2, grid_blocks=(2, 2), exact_max_n=10000)
    st = krylov.Stats()
    lev1, lev2 = M.levels[1], M.levels[2]
    lam2, Z2 = sla.eigh(lev2.A.toarray(), lev2.M.toarray())
    m = 12
    V = lev2.Psi @ Z2[:, :m]
    D = 1.0 / lam2[:m]
    ops = krylov.LevelOps(M, 1, 1e-10, st)
    Q, Dh = krylov.refine(ops, V, D, 1e-10, 0.0, lev1.lam_max_M)
    Mk = lev1.M.toarray()
    assert np.allclose(Q.T @ Mk @ Q, np.eye(Q.shape[1]), atol=1e-10)
    lam1 = sla.eigh(lev1.A.toarray(), Mk, eigvals_only=True)
    mu_true = 1.0 / lam1[:Q.shape[1]]
    assert np.max(np.abs(Dh[:8] - mu_true[:8]) / mu_true[:8]) < 1e-8


# --------------------------------------------------------------------------- end to end
def _closed_form_2d(n, count):
    j = np.arange(1, n + 1)
    s = 4 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())[:count]


@pytest.fixture(scope="module")
def c1_solution(c1_exact):
    p, M = c1_exact
    lam, V, st = krylov.eig_leftmost(p.scipy(), 50, 1e-10, mmd=M, return_stats=True)
    return p, lam, V, st


def test_c1_closed_form_eigenvalues(c1_solution):
    p, lam, V, st = c1_solution
    ref = _closed_form_2d(32, 50)
    assert np.max(np.abs(lam - ref) / ref) < 1e-10
    assert abs(ref[0] - 0.0181123) < 1e-7 and abs(ref[49] - 0.6349859) < 1e-7


def test_c1_closed_form_eigenvectors(c1_solution):
    p, lam, V, st = c1_solution
    n = 32
    x = np.arange(1, n + 1)
    modes = []
    for j in range(1, n + 1):
        for k in range(1, n + 1):
            s = 4 * np.sin(j * np.pi / 66) ** 2 + 4 * np.sin(k * np.pi / 66) ** 2
            modes.append((s, j, k))
    modes.sort()
    Vref = np.zeros((n * n, 50))
    for c, (s, j, k) in enumerate(modes[:50]):
        u = np.outer(np.sin(k * np.pi * x / 33), np.sin(j * np.pi * x / 33)).ravel()
        Vref[:, c] = u / np.linalg.norm(u)
    ang, cl = dense.cluster_angles(np.array([m[0] for m in modes[:50]]), Vref, V)
    assert ang.max() < 1e-8
    assert len(cl) == 28
    assert dense.rel_residuals(p.scipy(), lam, V).max() < 1e-9


def test_c1_stats_schema(c1_solution):
    st = c1_solution[3]
    assert set(st.levels) == {0, 1, 2, 3}
    assert st.levels[0]["ext_out"] == 50


def test_rgg_small_vs_dense_and_components():
    p = wl.rgg(400, 11, mean_degree=5)
    A = p.scipy()
    ncomp = dense.component_count(A)
    assert ncomp > 1
    lam, V = krylov.eig_leftmost(A, 30, 1e-11, mmd_kwargs=dict(coords=p.coords, levels=2, targets=(4, 8)))
    lr, Vr = dense.smallest_dense(A, 30)
    # the shifted null cluster: multiplicity = number of components, value exactly 1e-6
    # the shift cluster: multiplicity = number of components, each value the
    # stored matrix's eigenvalue at its component indicator (1e-10 relative,
    # or the rounding of the final m x m Rayleigh-Ritz step, 4 sqrt(m) u lambda_max)
    ref = dense.shift_cluster(A)
    assert ref.size == ncomp
    bar = np.maximum(1e-10 * ref, 4 * np.sqrt(lam.size) * 2.0 ** -52 * lam.max())
    assert np.all(np.abs(lam[:ncomp] - ref) <= bar) and lam[ncomp] > 2 * ref.max()
    big = lr > 2e-6
    assert np.max(np.abs(lam[big] - lr[big]) / lr[big]) < 1e-10
    ang, cl = dense.cluster_angles(lr, Vr, V)
    assert ang.max() < 1e-8


def test_no_hierarchy_is_plain_irlm_and_agrees():
    p = wl.knn_gmm(300, 10, 1)
    A = p.scipy()
    lam0, V0 = krylov.eig_leftmost(A, 15, 1e-11, mmd_kwargs=dict(levels=0))
    lam2, V2 = krylov.eig_leftmost(A, 15, 1e-11, mmd_kwargs=dict(coords=p.coords, levels=2, targets=(4, 8)))
    assert np.max(np.abs(lam0 - lam2) / lam0) < 1e-10
    lr, _ = dense.smallest_dense(A, 15)
    ref = dense.shift_cluster(A)
    assert abs(lam0[0] - ref[0]) <= max(1e-10 * ref[0], 4 * np.sqrt(lam0.size) * 2.0 ** -52 * lam0.max())
    assert np.max(np.abs(lam0[1:] - lr[1:]) / lr[1:]) < 1e-10


def test_grid3d_constant_coefficient_closed_form():
    m = 8
    p = wl.grid3d_lognormal(m, 0, sigma=0.0)
    lam, V = krylov.eig_leftmost(p.scipy(), 20, 1e-11, mmd_kwargs=dict(
        coords=p.coords, grid=p.grid, levels=1, grid_blocks=(2,), r_hops=1))
    j = np.arange(1, m + 1)
    s = 4 * np.sin(j * np.pi / (2 * (m + 1))) ** 2
    ref = np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())[:20]
    assert np.max(np.abs(lam - ref) / ref) < 1e-10


def test_oracle_grid2d_32_golden():
    """The oracle's 50 smallest pairs of the 32 x 32 grid (3 levels, exact Psi)
    against the stored closed-form values (tests/golden/grid2d_32_nev50.txt);
    lambda_50 < lambda_51 with a 2.4% gap, so the set is well defined."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "grid2d_32_nev50.txt")
    ref = np.loadtxt(path)
    assert ref.size == 51 and (ref[50] - ref[49]) / ref[49] > 0.02
    p = wl.grid2d(32)
    lam, V = krylov.eig_leftmost(p.scipy(), 50, 1e-10, mmd_kwargs=dict(
        grid=p.grid, levels=3, exact_max_n=4096))
    assert np.max(np.abs(lam - ref[:50]) / ref[:50]) < 1e-10


# --------------------------------------------------------------------------- coarsest level, Psi, sign rule
def test_coarsest_matches_generalized_eigh():
    """Alg. 6 first step against LAPACK's generalized symmetric eigensolver
    (scipy.linalg.eigh(A, M)): the mu = 1/lambda >= mu_ex filter, the m_tar
    cap, M-orthonormal vectors and the vectors themselves up to sign."""
    p = wl.rgg(900, 5)
    M = mm.build_mmd(p.scipy(), coords=p.coords, levels=2, targets=(4, 8), r_hops=1)
    lev = M.levels[M.K]
    Ad, Md = lev.A.toarray(), lev.M.toarray()
    lam, Zr = sla.eigh(Ad, Md)
    mu_ref = 1.0 / lam                       # descending
    assert lev.n >= 12 and np.all(np.diff(lam) > 1e-8 * lam[1:])
    # a threshold between two reference values: the count is known exactly
    cut = 7
    mu_ex = 0.5 * (mu_ref[cut - 1] + mu_ref[cut])
    Z, mu = krylov.coarsest(M, mu_ex, m_tar=100)
    assert mu.size == cut
    assert np.allclose(mu, mu_ref[:cut], rtol=1e-12, atol=0)
    assert np.allclose(Z.T @ Md @ Z, np.eye(cut), atol=1e-12)
    for j in range(cut):
        s = np.sign(Z[:, j] @ Md @ Zr[:, j])
        assert np.abs(s * Z[:, j] - Zr[:, j]).max() < 1e-9 * np.abs(Zr[:, j]).max()
    # m_tar caps the count; a threshold below every value keeps min(n, m_tar)
    Z2, mu2 = krylov.coarsest(M, 0.0, m_tar=5)
    assert mu2.size == 5 and np.allclose(mu2, mu_ref[:5], rtol=1e-12)
    Z3, mu3 = krylov.coarsest(M, 0.0, m_tar=10 ** 6)
    assert mu3.size == lev.n


def test_psi_localized_kkt_and_energy_minimal():
    """Appendix A form of the localized Psi (reading R4): column j minimises
    psi^T A psi over vectors supported on the patches within r hops of P_j
    subject to phi_i^T psi = delta_ij on those patches.  Checked through the
    optimality conditions, not the oracle's own solve: the support is the
    union of the r-hop patches (adjacency rebuilt here from A's pattern), the
    constraints hold, A_SS psi_S lies in span(Phi_C) (Lagrange condition), and
    feasible perturbations never lower the energy."""
    p = wl.rgg(700, 9)
    A = p.scipy()
    A.sort_indices()
    patches = mm.greedy_partition(A, p.coords, 4)
    phis = [mm.local_basis(A, m)[0] for m in patches]
    npch = len(patches)
    owner = np.empty(A.shape[0], np.int64)
    for j, m in enumerate(patches):
        owner[m] = j
    coo = A.tocoo()
    adj = sp.csr_matrix((np.ones(coo.nnz), (owner[coo.row], owner[coo.col])), shape=(npch, npch))
    adj = ((adj + sp.eye(npch)) > 0).astype(float)
    rng = np.random.default_rng(4)
    for r in (1, 2):
        Psi = mm.psi_localized(A, patches, phis, r).tocsc()
        reach = adj.copy()
        for _ in range(r - 1):
            reach = ((reach @ adj) > 0).astype(float)
        reach = reach.tocsr()
        for j in rng.choice(npch, 12, replace=False):
            C = np.sort(reach.indices[reach.indptr[j]:reach.indptr[j + 1]])
            S = np.sort(np.concatenate([patches[i] for i in C]))
            col = Psi[:, j].toarray().ravel()
            assert np.all(col[np.setdiff1d(np.arange(A.shape[0]), S)] == 0)
            psi = col[S]
            pos = {int(v): a for a, v in enumerate(S)}
            PhiC = np.zeros((S.size, C.size))
            for b, i in enumerate(C):
                PhiC[[pos[int(v)] for v in patches[i]], b] = phis[i]
            e = (C == j).astype(float)
            assert np.abs(PhiC.T @ psi - e).max() < 1e-10
            g = A[S][:, S] @ psi
            lag, *_ = np.linalg.lstsq(PhiC, g, rcond=None)
            assert np.linalg.norm(g - PhiC @ lag) <= 1e-8 * np.linalg.norm(g)
            # feasible directions: orthogonal to span(Phi_C)
            Qc, _ = np.linalg.qr(PhiC)
            ASS = A[S][:, S].toarray()
            E0 = psi @ ASS @ psi
            for _ in range(5):
                d = rng.standard_normal(S.size)
                d -= Qc @ (Qc.T @ d)
                d *= 1e-3 * np.linalg.norm(psi) / np.linalg.norm(d)
                assert (psi + d) @ ASS @ (psi + d) >= E0 * (1 - 1e-12)


def test_canonical_sign_rule():
    """Output sign rule (section 8(b) of the interface): the entry of largest
    magnitude is made positive, the lowest index wins an exact tie."""
    V = np.array([[0.1, -0.5, 0.0, 0.2],
                  [-0.7, 0.5, 0.0, -0.2],
                  [0.2, 0.1, -1.0, 0.1]])
    W = krylov.canonical_sign(V)
    ref = np.array([[-0.1, 0.5, 0.0, 0.2],
                    [0.7, -0.5, 0.0, -0.2],
                    [-0.2, -0.1, 1.0, 0.1]])
    assert np.array_equal(W, ref)
    assert np.array_equal(V[:, 3], W[:, 3])       # already canonical: unchanged
    assert np.array_equal(krylov.canonical_sign(W), W)  # idempotent


# --------------------------------------------------------------------------- coarse-level approximation
def test_coarse_level_approximation(c1_exact):
    """Section 7.3 / Lemma 3.3 with the exact Psi of the 32 x 32 grid: the
    level-k approximation returned with stop_level = k satisfies
    |mu_i - mu_i(A^-1)| <= eps_k and ||A^-1 v_i - mu_i v_i|| <= 2 eps_k
    (slack 0.1 eps_k for the level's own solve accuracy), its values match the
    dense generalized eigenproblem A^(k) z = lambda M^(k) z (exactly on the
    coarsest level), and the lifted vectors are orthonormal."""
    p, M = c1_exact
    A = p.scipy()
    Ad = A.toarray()
    w, Vd = np.linalg.eigh(Ad)
    mu_true = 1.0 / w
    Ainv = np.linalg.inv(Ad)
    for k, nev in ((3, 4), (2, 10), (1, 20)):
        lam, V = krylov.eig_leftmost(A, nev, 1e-10, mmd=M, stop_level=k)
        mu = 1.0 / lam
        eps_k = M.eps[k]
        assert np.all(np.diff(lam) >= 0)
        assert np.max(np.abs(mu - mu_true[:nev])) <= 1.1 * eps_k
        R = Ainv @ V - V * mu_true[None, :nev]
        assert np.max(np.linalg.norm(R, axis=0)) <= 2.2 * eps_k
        assert np.allclose(V.T @ V, np.eye(nev), atol=1e-10)
        lev = M.levels[k]
        lk = sla.eigh(lev.A.toarray(), lev.M.toarray(), eigvals_only=True)[:nev]
        tol_k = 1e-12 * lk.max() if k == M.K else 0.25 * eps_k
        assert np.max(np.abs(mu - 1.0 / lk)) <= tol_k
        # Theta^(k) <= A^-1: the approximations never exceed the true mu
        assert np.all(1.0 / lk <= mu_true[:nev] * (1 + 1e-12))


def test_coarse_level_approximation_localized():
    """Localized Psi on a random geometric graph: the stop_level = 1 output
    matches the dense level-1 generalized eigenpairs (values within
    0.1 eps_1, vectors Psi z up to sign) and interlaces the true values."""
    p = wl.rgg(900, 5)
    A = p.scipy()
    M = mm.build_mmd(A, coords=p.coords, levels=2, targets=(4, 8), r_hops=1)
    nev = 12
    lam, V = krylov.eig_leftmost(A, nev, 1e-10, mmd=M, stop_level=1)
    lev = M.levels[1]
    lk, Zk = sla.eigh(lev.A.toarray(), lev.M.toarray())
    assert np.max(np.abs(1.0 / lam - 1.0 / lk[:nev])) <= 0.1 * M.eps[1]
    w = np.linalg.eigvalsh(A.toarray())[:nev]
    assert np.all(lam >= w * (1 - 1e-10))
    # vectors: sin(angle) <= residual / gap in mu, residual <= 0.2 eps_1
    Vd = lev.Psi @ Zk[:, :nev]
    mu_k = 1.0 / lk[:nev + 1]
    for i in range(nev):
        gap = min(mu_k[i - 1] - mu_k[i] if i > 0 else np.inf, mu_k[i] - mu_k[i + 1])
        if gap < 1e-3 * mu_k[i]:
            continue
        c = abs(V[:, i] @ Vd[:, i]) / np.linalg.norm(Vd[:, i])
        assert np.sqrt(max(0.0, 1 - c * c)) <= 0.2 * M.eps[1] / gap


def test_shift_cluster_reference():
    """The component-wise mean row sum is the eigenvalue of the stored matrix
    at each component indicator: exact when every row sum is representable
    (integer weights, shift 2^-20), and against dense eigvalsh (absolute
    accuracy u ||A||) on an RGG with several components."""
    rng = np.random.default_rng(0)
    n, shift = 60, 2.0 ** -20
    rows, cols = [], []
    for c in range(3):                      # three path components of 20 vertices
        for i in range(20 * c, 20 * c + 19):
            rows.append(i); cols.append(i + 1)
    w = rng.integers(1, 5, size=len(rows)).astype(float)
    W = sp.csr_matrix((w, (rows, cols)), shape=(n, n))
    W = W + W.T
    A = sp.csr_matrix(sp.diags(np.asarray(W.sum(axis=1)).ravel() + shift) - W)
    ref = dense.shift_cluster(A)
    assert ref.size == 3 and np.all(ref == shift)
    assert np.allclose(np.linalg.eigvalsh(A.toarray())[:3], shift, rtol=0, atol=1e-14)
    p = wl.rgg(400, 11, mean_degree=5)
    A = p.scipy()
    ref = dense.shift_cluster(A)
    wd = np.linalg.eigvalsh(A.toarray())[:ref.size]
    assert ref.size == dense.component_count(A) == 19
    assert np.max(np.abs(wd - ref)) <= 4 * 2.0 ** -52 * float(abs(A).sum(axis=1).max())


# --------------------------------------------------------------------------- prescribed-accuracy partition
def test_split_energy_sums_below_the_matrix():
    """Section 2.2 patch bound: the split energies of any partition sum to at
    most the level matrix (A - sum_P E_P is positive semidefinite), also for a
    dense coarse Galerkin matrix with positive off-diagonals; on a Laplacian
    plus a nonnegative diagonal they equal the interior energies."""
    p = wl.rgg(600, 4)
    A0 = p.scipy()
    M = mm.build_mmd(A0, coords=p.coords, levels=1, exact_max_n=10 ** 6)
    A1 = M.levels[1].A.tocsr()
    assert (A1 - sp.diags(A1.diagonal())).max() > 0      # not an M-matrix
    rng = np.random.default_rng(3)
    for A in (A0, A1):
        n = A.shape[0]
        perm = rng.permutation(n)
        cuts = np.sort(rng.choice(np.arange(1, n), size=n // 5, replace=False))
        patches = [np.sort(c) for c in np.split(perm, cuts)]
        S = np.zeros((n, n))
        for mem in patches:
            S[np.ix_(mem, mem)] += energy.split_energy(A, mem)
        w = np.linalg.eigvalsh(A.toarray() - S)
        assert w.min() >= -1e-12 * abs(A).max()
    for mem in [np.sort(rng.choice(600, 7, replace=False)) for _ in range(20)]:
        assert np.allclose(energy.split_energy(A0, mem), energy.interior_energy(A0, mem),
                           rtol=0, atol=1e-14 * abs(A0).max())



def test_eps_partition_meets_its_bounds():
    """SwissRoll graph (Section 7.1, a 1500-point sample at the full roll's
    point density) partitioned to prescribed accuracy with the paper's
    (eps_1, eta, c) = (1e-5, 0.1, 20): every patch of every level satisfies
    eps(P) <= eps_k and eps(P) delta(P) <= c, recomputed here from the
    definitions (Section 2.2: eps = 1 / lambda_2 of the patch energy,
    delta = 1 / (phi^T Abar^-1 phi)), the patches cover each level exactly
    once, the levels coarsen, and M^(k) >= I (Lemma 4.3; the localized Psi
    keeps Phi^T Psi = I)."""
    p = wl.swissroll(1500, seed=2)
    A = p.scipy()
    # unit self-loops: A 1 = 1 on a connected graph, lambda_1 = 1
    assert np.allclose(A @ np.ones(p.n), 1.0, rtol=0, atol=1e-6 * abs(A).max())
    M = mm.build_mmd(A, coords=p.coords, levels=2, eps1=1e-5, eta=0.1, cbound=20.0, r_hops=2)
    assert M.K == 2
    for k in (1, 2):
        lev, prev = M.levels[k], M.levels[k - 1]
        eps_k = 1e-5 / 0.1 ** (k - 1)
        allv = np.sort(np.concatenate(lev.patches))
        assert np.array_equal(allv, np.arange(prev.n))
        assert lev.n < 0.8 * prev.n
        for mem in lev.patches:
            if len(mem) < 2:
                continue
            E = energy.split_energy(prev.A, mem)
            w, V = np.linalg.eigh(E)
            eps = 1.0 / w[1]
            Abar = prev.A[mem][:, mem].toarray()
            delta = 1.0 / (V[:, 0] @ np.linalg.solve(Abar, V[:, 0]))
            assert eps <= eps_k * (1 + 1e-12)
            assert eps * delta <= 20.0 * (1 + 1e-12)
        assert np.linalg.eigvalsh(lev.M.toarray()).min() >= 1 - 1e-10


def test_eps_partition_coarse_spectrum_within_eps1():
    """Theorem 2.6 / Lemma 3.3 on the prescribed-accuracy partition: with the
    exact Psi = A^-1 Phi (Phi^T A^-1 Phi)^-1 the level-1 pencil (A^(1), M^(1))
    reproduces mu_i = 1 / lambda_i(A) within eps_1 = 1e-5 (the interior patch
    energies on level 1 make eps(P) a valid bound); the localized Psi needs
    support radius 5 patch hops on this graph to keep that accuracy, while
    radius 1 loses the low spectrum entirely (mu_1 error near 1)."""
    p = wl.swissroll(1500, seed=2)
    A = p.scipy()
    mu0 = 1.0 / np.linalg.eigvalsh(A.toarray())[:12]
    errs = {}
    for name, kw in (("exact", dict(exact_max_n=10 ** 9)), ("r5", dict(r_hops=5)),
                     ("r1", dict(r_hops=1))):
        M = mm.build_mmd(A, coords=p.coords, levels=1, eps1=1e-5, eta=0.1, cbound=20.0, **kw)
        lev = M.levels[1]
        mu = 1.0 / sla.eigh(lev.A.toarray(), lev.M.toarray(), eigvals_only=True)[:12]
        # Galerkin: mu^(1) <= mu (Courant-Fischer), up to the rounding of the
        # formed Psi and A^(1), a modest multiple of u kappa(A) = 2.6e-10
        assert np.all(mu <= mu0 * (1 + 2e-8))
        errs[name] = np.max(np.abs(mu - mu0))
        assert M.eps[1] <= 1e-5
    assert errs["exact"] <= 1e-5
    assert errs["r5"] <= 1e-5
    assert errs["r1"] > 0.5


def test_eps_partition_full_roll_level1_size():
    """The paper's 20000-point SwissRoll with eps_1 = 1e-5, c = 20 has 5528
    level-1 dofs (decomposition table of Section 7.2); this partition reading
    gives a level-1 size within 2% of it."""
    p = wl.swissroll(20000, seed=0)
    P = mm.eps_partition(p.scipy(), p.coords, 1e-5, 20.0, "split", 32)
    assert abs(len(P) - 5528) <= 0.02 * 5528
