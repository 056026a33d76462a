"""Krylov parts of the hierarchical eigensolver (Sections 2.4, 4, 5, 6 of the paper).

Everything is float64 and unblocked; block operations are loops over columns
so each step can be read against the paper.  Notation: mu = 1/lambda, the
wanted values are the largest mu of (A^(k))^-1 M^(k) on level k; V_hat are
coefficient vectors, M-orthonormal (Section 4, end).

Readings of silent or ambiguous points (each listed with its reason in the
design notes):
  * pcg(A, b, M, x0, eps) stops when ||r||_2 <= eps ||b||_2; the
    preconditioner M^-1 is itself an inner CG to eps_hat = 0.1 eps, so the
    outer iteration is flexible CG with beta = r_new^T (z_new - z_old) / r^T z.
  * Alg. 3 on breakdown (||f||_M tiny) draws a fresh random direction; the
    coupling entry of T is the true (tiny) beta, set to 0.
  * Re-orthogonalisation is a second classical Gram-Schmidt pass in the
    M inner product against [V_ini, V_hat], always performed.
  * Alg. 2 uses the p smallest Ritz values as exact shifts; f is updated
    with the basis from before the truncation.
  * Ritz residual test: ||f||_M |e_k^T y| <= eps (absolute in mu on coarse
    levels; eps * theta on level 0).
  * Alg. 5 "QR with respect to M" is CholQR2 in the M inner product; "Schur
    decomposition" of S is the symmetric eigendecomposition of (S + S^T)/2.
  * Alg. 5 stop: ||Q_mh - Q'_mh Q'_mh^T M Q_mh||_F < eps / sqrt(lambda_max(M))
    with lambda_max(M) bounded by the Gershgorin row sum.  m_h also obeys the
    efficiency condition (ii) of Section 5 with the current Ritz values:
    mu_ml <= gamma mu_mh, gamma = (1 + beta) / alpha, so guard columns remain.
  * Alg. 6 is continued down to level 0 (A^(0) = A, M^(0) = I), then a final
    inverse-iteration + Rayleigh-Ritz step with A gives the output pairs; it
    is repeated while a returned pair's relative residual exceeds 10 tol
    (until that residual stagnates).
  * Single-vector Lanczos cannot see a second copy of an exactly degenerate
    eigenvalue; level 0 ends with a multiplicity check (fresh random start
    deflated against the accepted pairs) that swaps in any missed pair.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .mmd import MMD, build_mmd, schedule
from .philox import uniform_vector


class NotConverged(RuntimeError):
    pass


class NotSPD(RuntimeError):
    pass


@dataclass
class Stats:
    """Per-level counters in the paper's statistics schema (Section 7.3)."""
    levels: dict = field(default_factory=dict)

    def lev(self, k):
        return self.levels.setdefault(k, dict(
            ref_in=0, ref_out=0, ref_iter=0, cg_B_calls=0, cg_B_iters=0,
            pcg_A_calls=0, pcg_A_iters=0, pcg_A_max=0, cg_M_calls=0, cg_M_iters=0,
            ext_in=0, ext_out=0, lanczos_steps=0, restarts=0))


# ----------------------------------------------------------------------------
# CG and flexible PCG
# ----------------------------------------------------------------------------

def cg(apply: Callable, b: np.ndarray, x0: Optional[np.ndarray], tol: float,
       maxit: int = 100000):
    """Plain conjugate gradients; stop when ||r|| <= tol ||b||.  Returns (x, iters)."""
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - apply(x)
    if np.linalg.norm(r) <= tol * bn:
        return x, 0
    p = r.copy()
    rr = r @ r
    for it in range(1, maxit + 1):
        q = apply(p)
        pq = p @ q
        if not pq > 0:
            raise NotSPD("CG curvature p^T A p <= 0")
        a = rr / pq
        x += a * p
        r -= a * q
        rr_new = r @ r
        if np.sqrt(rr_new) <= tol * bn:
            return x, it
        p = r + (rr_new / rr) * p
        rr = rr_new
    raise NotConverged("CG reached the iteration cap")


def pcg(applyA: Callable, b: np.ndarray, M: Optional[sp.csr_matrix], x0, tol: float,
        stats: Optional[dict] = None, maxit: int = 100000):
    """pcg(A, b, M, x0, tol) of Section 4 with the inner CG preconditioner (flexible)."""
    if M is None:
        x, it = cg(applyA, b, x0, tol, maxit)
        if stats is not None:
            stats["pcg_A_calls"] += 1
            stats["pcg_A_iters"] += it
            stats["pcg_A_max"] = max(stats["pcg_A_max"], it)
        return x
    tol_in = 0.1 * tol
    applyM = lambda v: M @ v

    def minv(r):
        z, it = cg(applyM, r, None, tol_in, maxit)
        if stats is not None:
            stats["cg_M_calls"] += 1
            stats["cg_M_iters"] += it
        return z

    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b)
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - applyA(x)
    it = 0
    if np.linalg.norm(r) > tol * bn:
        z = minv(r)
        p = z.copy()
        rz = r @ z
        while True:
            it += 1
            if it > maxit:
                raise NotConverged("PCG reached the iteration cap")
            q = applyA(p)
            pq = p @ q
            if not pq > 0:
                raise NotSPD("PCG curvature p^T A p <= 0")
            a = rz / pq
            x += a * p
            r -= a * q
            if np.linalg.norm(r) <= tol * bn:
                break
            z_new = minv(r)
            beta = (r @ z_new - r @ z) / rz
            rz = r @ z_new
            z = z_new
            p = z + beta * p
    if stats is not None:
        stats["pcg_A_calls"] += 1
        stats["pcg_A_iters"] += it
        stats["pcg_A_max"] = max(stats["pcg_A_max"], it)
    return x


# ----------------------------------------------------------------------------
# small dense helpers
# ----------------------------------------------------------------------------

def mnorm(M, x):
    return float(np.sqrt(x @ (x if M is None else M @ x)))


def mqr(F: np.ndarray, M: Optional[sp.csr_matrix]) -> np.ndarray:
    """QR with respect to the M inner product: CholQR applied twice (Q^T M Q = I)."""
    Q = F.copy()
    for _ in range(2):
        MQ = Q if M is None else M @ Q
        G = Q.T @ MQ
        G = 0.5 * (G + G.T)
        R = np.linalg.cholesky(G).T          # upper, positive diagonal
        Q = sla.solve_triangular(R, Q.T, trans="T", lower=False).T
    return Q


def eig_desc(S: np.ndarray):
    """Symmetric eigendecomposition of (S + S^T)/2 with descending eigenvalues."""
    w, P = np.linalg.eigh(0.5 * (S + S.T))
    return w[::-1].copy(), P[:, ::-1].copy()


# ----------------------------------------------------------------------------
# level operators
# ----------------------------------------------------------------------------

class EdgeForm:
    """Level-0 product in edge form: y_i = s_i x_i + sum_j w_ij (x_i - x_j).

    Same operator as the CSR product with A = L + diag(s); each edge term is
    a difference, so vectors constant on a connected component give exactly
    s_i x_i (Laplacian null vectors stay exact in floating point).
    """

    def __init__(self, A: sp.csr_matrix):
        from .energy import energy_elements
        A = sp.csr_matrix(A)
        C = A.tocoo()
        off = C.row != C.col
        self.rows = C.row[off].astype(np.int64)
        self.cols = C.col[off].astype(np.int64)
        self.w = -C.data[off]
        self.s = energy_elements(A)[3]
        self.n = A.shape[0]

    def __matmul__(self, x):
        x = np.asarray(x)
        if x.ndim == 2:
            return np.stack([self @ x[:, j] for j in range(x.shape[1])], axis=1)
        d = self.w * (x[self.rows] - x[self.cols])
        return self.s * x + np.bincount(self.rows, weights=d, minlength=self.n)


class LevelOps:
    """Operators on level k: A^(k), M^(k), B^(k+1) = U^T A^(k) U and OP."""

    def __init__(self, mmd: MMD, k: int, eps_op: float, stats: Stats, edge0=None):
        self.mmd = mmd
        self.k = k
        self.lev = mmd.levels[k]
        self.up = mmd.levels[k + 1] if k + 1 <= mmd.K else None
        self.A = edge0 if (k == 0 and edge0 is not None) else self.lev.A
        self.M = self.lev.M
        self.n = self.lev.n
        self.eps = eps_op
        self.st = stats.lev(k)
        self.draws = 0          # random-vector draw counter of this level

    def applyA(self, x):
        return self.A @ x

    def applyM(self, x):
        return x if self.M is None else self.M @ x

    def applyB(self, y):
        return self.up.Ut_apply(self.A @ self.up.U_apply(y))

    def op(self, x):
        """Operator OP(x; A, M, eps): w = M x, y = pcg(A, w, M, 0, eps)."""
        return pcg(self.applyA, self.applyM(x), self.M, None, self.eps, self.st)


# ----------------------------------------------------------------------------
# Lanczos with the M inner product (Alg. 3) and implicit restart (Alg. 2)
# ----------------------------------------------------------------------------

class Lanczos:
    """State (V_hat, T, f_hat) with OP V = V T + f e^T, V^T M V = I, V^T M V_ini = 0."""

    def __init__(self, ops: LevelOps, Vini: np.ndarray, seed: int):
        self.ops = ops
        self.M = ops.M
        self.Vini = Vini
        self.V = np.zeros((ops.n, 0))
        self.T = np.zeros((0, 0))
        self.seed = seed
        self.wnorm = 1.0
        self.f = self.random_direction()

    def basis(self):
        return np.hstack([self.Vini, self.V])

    def orth(self, w):
        """Two classical Gram-Schmidt passes in the M inner product against [V_ini, V]."""
        B = self.basis()
        h = np.zeros(B.shape[1])
        for _ in range(2):
            c = B.T @ self.ops.applyM(w)
            w = w - B @ c
            h += c
        return w, h

    def random_direction(self):
        v = uniform_vector(self.ops.n, self.seed, self.ops.k, self.ops.draws)
        self.ops.draws += 1
        v, _ = self.orth(v)
        return v

    def steps(self, nsteps):
        st = self.ops.st
        for _ in range(nsteps):
            j = self.V.shape[1]
            beta = mnorm(self.M, self.f)
            if j > 0 and beta <= 1e-12 * self.wnorm:
                f = self.random_direction()
                v = f / mnorm(self.M, f)
                coupling = 0.0
            else:
                v = self.f / beta
                coupling = beta
            self.V = np.hstack([self.V, v[:, None]])
            T = np.zeros((j + 1, j + 1))
            T[:j, :j] = self.T
            if j > 0:
                T[j, j - 1] = T[j - 1, j] = coupling
            w = self.ops.op(v)
            self.wnorm = mnorm(self.M, w)
            f, h = self.orth(w)
            T[j, j] = h[self.Vini.shape[1] + j]
            self.T = T
            self.f = f
            st["lanczos_steps"] += 1

    def ritz(self):
        """Ritz values (descending), vectors of T, residual norms ||f||_M |e_k^T y|."""
        theta, Y = eig_desc(self.T)
        res = mnorm(self.M, self.f) * np.abs(Y[-1, :])
        return theta, Y, res

    def converged(self, nwant, eps, relative):
        theta, Y, res = self.ritz()
        lim = eps * np.abs(theta[:nwant]) if relative else eps
        return bool(np.all(res[:nwant] <= lim))

    def restart(self, k, p):
        """Alg. 2: apply the p smallest Ritz values as exact shifts, keep k vectors."""
        m = self.T.shape[0]
        assert m == k + p
        theta = np.linalg.eigvalsh(0.5 * (self.T + self.T.T))
        T = self.T.copy()
        Q = np.eye(m)
        for sigma in theta[:p]:
            Qj, _ = np.linalg.qr(T - sigma * np.eye(m))
            T = Qj.T @ T @ Qj
            T = 0.5 * (T + T.T)
            Q = Q @ Qj
        f = self.V @ Q[:, k] * T[k, k - 1] + self.f * Q[m - 1, k - 1]
        self.V = self.V @ Q[:, :k]
        self.T = T[:k, :k].copy()
        self.f = f
        self.ops.st["restarts"] += 1


def extend(ops: LevelOps, Vini, Dini, m_tar, eps, mu_ex, d, c=1, relative=False,
           seed=0, max_restarts=2000):
    """Eigenpair Extension (Alg. 4) on one level."""
    mi = Vini.shape[1]
    st = ops.st
    st["ext_in"] += mi
    want_total = m_tar - mi
    cap = ops.n - mi
    if want_total <= 0 or cap <= 0:
        st["ext_out"] += mi
        return Vini, Dini
    L = Lanczos(ops, Vini, seed)
    k = 0
    restarts = 0

    def converge(kk, p):
        nonlocal restarts
        while not L.converged(kk, eps, relative):
            if p <= 0:
                break
            L.steps(p)
            L.restart(kk, p)
            restarts += 1
            if restarts > max_restarts:
                raise NotConverged("extension: restart cap reached")

    while True:
        kk = min(k + d, want_total, cap)
        p = min(c * d, cap - kk)
        L.steps(kk - L.V.shape[1])
        converge(kk, p)
        k = kk
        theta = np.sort(np.linalg.eigvalsh(0.5 * (L.T + L.T.T)))
        mu_hat = theta[min(d, k) - 1]
        if mu_hat < mu_ex or k >= want_total or k >= cap:
            break
    m_new = k
    converge(m_new, min(c * m_new, cap - m_new))
    theta, Y = eig_desc(L.T)
    Vex = np.hstack([Vini, L.V @ Y])
    Dex = np.concatenate([Dini, theta])
    order = np.argsort(-Dex, kind="stable")
    st["ext_out"] += Vex.shape[1]
    return Vex[:, order], Dex[order]


def multiplicity_check(ops: LevelOps, V, D, eps, d, c=1, relative=True, seed=0, max_swaps=64):
    """Look for a pair that single-vector Lanczos missed (a further copy of a
    degenerate eigenvalue).  A short Lanczos run from a fresh random vector,
    M-orthogonal to the accepted pairs, must not produce a Ritz value above the
    smallest accepted mu; when it does, that direction is converged (one wanted
    pair, restarts as in Alg. 2), swapped in for the smallest pair, and the
    check repeats."""
    cap = ops.n - V.shape[1]
    if cap <= 0 or V.shape[1] == 0:
        return V, D
    for _ in range(max_swaps):
        L = Lanczos(ops, V, seed)
        s = min(d + 10, cap)
        L.steps(s)
        theta, Y, res = L.ritz()
        lim = D[-1] * (1.0 + eps) if relative else D[-1] + eps
        if theta[0] <= lim:
            return V, D
        p = min(c * d, cap - 1)
        while p > 0 and not L.converged(1, eps, relative):
            L.restart(1, L.T.shape[0] - 1)
            L.steps(p)
        theta, Y, res = L.ritz()
        u = L.V @ Y[:, 0]
        V = np.hstack([V[:, :-1], u[:, None]])
        D = np.concatenate([D[:-1], theta[:1]])
        order = np.argsort(-D, kind="stable")
        V, D = V[:, order], D[order]
        ops.st["missed_swaps"] = ops.st.get("missed_swaps", 0) + 1
    raise NotConverged("multiplicity check: too many swaps")


# ----------------------------------------------------------------------------
# refinement (Alg. 5)
# ----------------------------------------------------------------------------

def keep_count(D, mu_h, gamma):
    """m_h of Alg. 5: mu_mh >= mu_h, and at most the count that keeps the Ritz
    estimate of the convergence ratio mu_ml / mu_mh <= gamma (condition (ii)
    of Section 5, so the remaining m_l - m_h columns act as guard vectors)."""
    ml = D.size
    mh = int(np.sum(D >= mu_h))
    while mh > 0 and D[ml - 1] > gamma * D[mh - 1]:
        mh -= 1
    return mh


def refine(ops: LevelOps, Vl, Dl, eps, mu_h, lam_max_M, gamma=2.0 / 3.0, max_iter=200,
           eps_solve=None):
    """Eigenpair Refinement (Alg. 5): level-(k+1) pairs reformed to level k -> level-k pairs.

    eps_solve (default eps) is the PCG tolerance; on level 0 the driver passes
    0.1 eps so the stop test at eps lies above the noise of the solves.  The
    loop also stops when the distance has stagnated below 10 eps (no 10%
    decrease over 5 iterations): the attainable floor of inexact solves.
    """
    if eps_solve is None:
        eps_solve = eps
    st = ops.st
    ml = Vl.shape[1]
    st["ref_in"] += ml
    if ml == 0:
        return Vl, Dl
    up = ops.up
    # start block: F = Q D + U G, g_i = cg(B, U^T M q_i, 0, eps)
    MQ = ops.applyM(Vl)
    G = np.zeros((up.nb(), ml))
    for i in range(ml):
        rhs = up.Ut_apply(MQ[:, i])
        G[:, i], it = cg(ops.applyB, rhs, None, eps_solve)
        st["cg_B_calls"] += 1
        st["cg_B_iters"] += it
    F = Vl * Dl[None, :] + up.U_apply(G)
    mu_prev = Dl.copy()
    Qprev = None
    thresh = eps / np.sqrt(lam_max_M)
    hist = []
    for it in range(1, max_iter + 1):
        Q = mqr(F, ops.M)
        W = ops.applyM(Q)
        F = np.zeros_like(Q)
        for i in range(ml):
            F[:, i] = pcg(ops.applyA, W[:, i], ops.M, mu_prev[i] * Q[:, i], eps_solve, st)
        S = W.T @ F
        D, P = eig_desc(S)
        mh = keep_count(D, mu_h, gamma)
        Q = Q @ P
        F = F @ P
        st["ref_iter"] += 1
        done = False
        if Qprev is not None:
            X = Qprev[:, :mh].T @ ops.applyM(Q[:, :mh])
            E = Q[:, :mh] - Qprev[:, :mh] @ X
            dist = np.linalg.norm(E)
            hist.append(dist)
            done = dist < thresh or (len(hist) > 5 and dist < 10 * thresh
                                     and dist > 0.9 * hist[-6])
        Qprev = Q
        mu_prev = D
        if done:
            break
    else:
        raise NotConverged("refinement: iteration cap reached")
    st["ref_out"] += mh
    return Q[:, :mh], D[:mh]


# ----------------------------------------------------------------------------
# level driver (Alg. 6 continued to level 0) and output step
# ----------------------------------------------------------------------------

def coarsest(mmd: MMD, mu_ex, m_tar):
    """Alg. 6 first step: eigenpairs of A^(K) z = lambda M^(K) z (dense, Cholesky of M)."""
    lev = mmd.levels[mmd.K]
    A = lev.A.toarray()
    M = np.eye(lev.n) if lev.M is None else lev.M.toarray()
    L = np.linalg.cholesky(0.5 * (M + M.T))
    Linv_A = sla.solve_triangular(L, A, lower=True)
    C = sla.solve_triangular(L, Linv_A.T, lower=True)
    lam, Y = np.linalg.eigh(0.5 * (C + C.T))
    Z = sla.solve_triangular(L.T, Y, lower=False)
    mu = 1.0 / lam
    keep = min(int(np.sum(mu >= mu_ex)), m_tar)
    return Z[:, :keep], mu[:keep]


def canonical_sign(V):
    """Flip each column so its largest-magnitude entry (lowest index on ties) is positive."""
    V = V.copy()
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def final_pairs(A, V, D, nev, tol, st, max_passes=30):
    """Output step on level 0: F = A^-1 V (CG from mu_i v_i), orthonormalise, Rayleigh-Ritz with A.

    A is the level-0 operator in edge form.  The step is repeated (block
    inverse iteration on the Ritz block) while a returned pair misses the
    relative residual ||A v - lambda v|| / (lambda ||v||) <= 10 tol, until the
    largest such residual stops falling by 10% per pass or max_passes is
    reached (reading of the output accuracy, see the module notes).
    """
    prev = np.inf
    for _ in range(max_passes):
        F = np.zeros_like(V)
        for i in range(V.shape[1]):
            F[:, i] = pcg(lambda x: A @ x, V[:, i], None, D[i] * V[:, i], tol, st)
        Q = mqr(F, None)
        H = Q.T @ (A @ Q)
        lam, Y = np.linalg.eigh(0.5 * (H + H.T))
        Vall = Q @ Y
        R = A @ Vall[:, :nev] - Vall[:, :nev] * lam[None, :nev]
        rho = np.linalg.norm(R, axis=0) / (np.abs(lam[:nev]) * np.linalg.norm(Vall[:, :nev], axis=0))
        worst = float(rho.max())
        if worst <= 10.0 * tol or worst > 0.9 * prev:
            break
        prev = worst
        V, D = Vall, 1.0 / lam
    Vout = Vall[:, :nev]
    Vout /= np.linalg.norm(Vout, axis=0)[None, :]
    return lam[:nev], canonical_sign(Vout)


def coarse_pairs(mmd: MMD, k: int, V, D, nev):
    """Coarse-level approximation (Section 7.3): the level-k pairs z_i with
    mu_i = 1 / lambda_i, lifted as v_i = Psi^(1) ... Psi^(k) z_i.  With z
    M^(k)-orthonormal the v_i are orthonormal (M^(k) is the Gram matrix of the
    composite basis); |mu_i - mu_i(A^-1)| <= eps_k by Lemma 3.3."""
    if V.shape[1] < nev:
        raise NotConverged("coarse-level approximation: fewer pairs than nev on level %d" % k)
    Z = V[:, :nev]
    for j in range(k, 0, -1):
        Z = mmd.levels[j].Psi @ Z
    Z = Z / np.linalg.norm(Z, axis=0)[None, :]
    return 1.0 / D[:nev], canonical_sign(Z)


def eig_leftmost(A, nev, tol, mmd: Optional[MMD] = None, alpha=3.0, beta=1.0, c=1,
                 seed=0, mmd_kwargs=None, return_stats=False, stop_level=0):
    """The nev smallest eigenpairs of the SPD matrix A by Alg. 6 (continued to level 0).

    stop_level k >= 1 stops Alg. 6 after level k (the printed algorithm stops
    at level 1) and returns the coarse-level approximation of that level.
    Returns (lambda ascending [nev], V [n, nev]) and, optionally, Stats.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    if not (0 < nev <= n):
        raise ValueError("nev out of range")
    if mmd is None:
        mmd = build_mmd(A, **(mmd_kwargs or {}))
    sch = schedule(mmd, nev, tol, alpha, beta)
    stats = Stats()
    E0 = EdgeForm(A)
    K = mmd.K
    if not 0 <= stop_level <= K:
        raise ValueError("stop_level must lie between 0 and K")
    if K == 0:
        V = np.zeros((n, 0))
        D = np.zeros(0)
    else:
        # on the coarsest level itself the approximation keeps the nev leading
        # pairs of the dense problem, without the exploration threshold
        V, D = coarsest(mmd, sch.mu_ex[K] if stop_level < K else 0.0, nev)
        stats.lev(K)["ext_out"] = V.shape[1]
    for k in range(K - 1, stop_level - 1, -1):
        # the PCG of OP and of the refinement stops at a relative residual
        # eps^(k); without the paper's scaling (lambda_1 = 1) eps^(k) = 0.1 eps_k
        # can exceed 1, where x = 0 already passes and OP vanishes: the
        # relative tolerance on levels k >= 1 is min(eps^(k), 0.1)
        t_pcg = 0.1 * sch.eps_op[k] if k == 0 else min(0.1, sch.eps_op[k])
        if k == stop_level and k > 0 and D.size:
            # the returned level: OP accurate to eps^(k) in mu units, i.e.
            # relative eps^(k) / mu_1 (mu_1 = 1 under the paper's scaling)
            t_pcg = min(0.1, sch.eps_op[k] / float(D[0]))
        ops = LevelOps(mmd, k, sch.eps_op[k] if k == 0 else t_pcg, stats, E0)
        V = mmd.levels[k + 1].Psi @ V
        V, D = refine(ops, V, D, sch.eps_op[k], sch.mu_re[k], mmd.levels[k].lam_max_M,
                      gamma=(1.0 + beta) / alpha, eps_solve=t_pcg)
        V, D = extend(ops, V, D, nev, sch.eps_op[k], sch.mu_ex[k], sch.d[k], c,
                      relative=(k == 0), seed=seed)
    if stop_level > 0:
        if stop_level < K:
            # missed copies of repeated eigenvalues, as on level 0 (absolute test in mu)
            V, D = multiplicity_check(ops, V, D, sch.eps_op[stop_level], sch.d[stop_level], c,
                                      relative=False, seed=seed)
        lam, Vout = coarse_pairs(mmd, stop_level, V, D, nev)
        if return_stats:
            return lam, Vout, stats
        return lam, Vout
    if K == 0:
        ops = LevelOps(mmd, 0, tol, stats, E0)
        V, D = extend(ops, V, D, nev, tol, 0.0, sch.d[0], c, relative=True, seed=seed)
    V, D = multiplicity_check(ops, V, D, tol, sch.d[0], c, relative=True, seed=seed)
    lam, Vout = final_pairs(E0, V, D, nev, tol, stats.lev(0))
    if return_stats:
        return lam, Vout, stats
    return lam, Vout
