"""Multiresolution matrix decomposition (Sections 2.2-2.3 of the paper).

Per level k >= 1, from the level-(k-1) matrix A^(k-1) (A^(0) = A, M^(0) = I):
  1. partition the level-(k-1) dofs into patches P_j            (reading: see
     partition functions below; the paper defers its partitioner to its
     companion work);
  2. phi_j = unit eigenvector of the smallest eigenvalue of the patch's
     energy (q = 1, Section 2.2), sign: sum(phi_j) > 0; the patch error
     factor is 1 / lambda_2(patch energy) (Section 2.2).  Patch energy:
     interior energy on level 1, closed energy on levels >= 2; the split
     energy on every level of a partition to prescribed accuracy (energy.py);
  3. U_j = the complement of phi_j inside the patch, realised as columns
     2..|P_j| of one Householder reflector H_j with H_j e_1 = +-phi_j
     (Lemma 2.3 remark: QR completion gives kappa(U^T U) = 1);
  4. Psi = A^-1 Phi (Phi^T A^-1 Phi)^-1 (eq. psi_closedform with the missing
     transpose restored), either exactly or localised: psi_j minimises
     psi^T A psi over vectors supported on the patches within r hops of P_j
     subject to phi_i^T psi = delta_ij for those patches (the constrained
     energy form of Appendix A);
  5. A^(k) = Psi^T A^(k-1) Psi, M^(k) = Psi^T M^(k-1) Psi (eq. MMD and the
     recursion above it); B^(k) = U^T A^(k-1) U stays implicit.
Accuracy schedule (Section 2.3 Thm 2.6 and Section 5):
  eps_k = sum_{k' <= k} eps(P^(k')),  eps^(k) = 0.1 eps_k,
  mu_re^(k) = alpha eps_{k+1},  mu_ex^(k) = beta eps_k.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .energy import closed_energy, energy_elements, interior_energy, split_energy


# ----------------------------------------------------------------------------
# partitions
# ----------------------------------------------------------------------------

def grid_partition(shape, block):
    """Tensor-grid patches of block^d vertices (smaller at the far edges).

    Vertex (x, y[, z]) has index (z*ny + y)*nx + x; patch (px, py[, pz]) has
    id (pz*npy + py)*npx + px; members are listed in ascending vertex order.
    Returns (patches, coarse_shape).
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    nb = tuple((s + block - 1) // block for s in shape)
    if d == 2:
        nx, ny = shape
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        pid = (y // block) * nb[0] + (x // block)
    else:
        nx, ny, nz = shape
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        pid = ((z // block) * nb[1] + (y // block)) * nb[0] + (x // block)
    pid = pid.ravel()
    npatch = int(np.prod(nb))
    order = np.argsort(pid, kind="stable")
    counts = np.bincount(pid, minlength=npatch)
    splits = np.cumsum(counts)[:-1]
    patches = [np.sort(p) for p in np.split(order, splits)]
    return patches, nb


def morton_order(coords: np.ndarray) -> np.ndarray:
    """Vertex order by interleaved-bit (Morton) code of the quantised coordinates.

    Coordinates are scaled to the bounding box and quantised to 16 bits (2-D)
    or 10 bits (3-D) per axis: q = floor((x - lo) / (hi - lo) * 2^B), clamped.
    Ties keep ascending vertex order.
    """
    coords = np.asarray(coords, dtype=np.float64)
    n, d = coords.shape
    bits = 16 if d == 2 else 10
    scale = float(1 << bits)
    q = np.zeros((n, d), dtype=np.int64)
    for a in range(d):
        lo = coords[:, a].min()
        hi = coords[:, a].max()
        if hi > lo:
            t = np.floor((coords[:, a] - lo) / (hi - lo) * scale)
            q[:, a] = np.clip(t, 0, (1 << bits) - 1).astype(np.int64)
    code = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        for a in range(d):
            code |= ((q[:, a] >> b) & 1) << (d * b + a)
    return np.lexsort((np.arange(n), code))


def greedy_partition(A: sp.csr_matrix, coords: Optional[np.ndarray], target: int):
    """Greedy breadth-first aggregation (reading of the deferred partitioner).

    Seeds are visited in Morton order of the coordinates (vertex order when
    there are none).  An unassigned seed opens a patch that grows breadth
    first over unassigned neighbours (CSR order, ascending index) up to
    ``target`` vertices.  Afterwards, in ascending patch order, every patch
    with fewer than target/2 vertices is merged into the adjacent patch it
    shares the most matrix entries with (ties: lowest patch id).  Empty
    patches are dropped, ids are compacted in ascending order, and members
    are sorted.
    """
    n = A.shape[0]
    order = morton_order(coords) if coords is not None else np.arange(n)
    indptr, indices = A.indptr, A.indices
    pid = np.full(n, -1, dtype=np.int64)
    patches: List[list] = []
    for s in order:
        s = int(s)
        if pid[s] >= 0:
            continue
        cur = len(patches)
        members = [s]
        pid[s] = cur
        head = 0
        while head < len(members) and len(members) < target:
            v = members[head]
            head += 1
            for u in indices[indptr[v]:indptr[v + 1]]:
                u = int(u)
                if pid[u] < 0:
                    pid[u] = cur
                    members.append(u)
                    if len(members) >= target:
                        break
        patches.append(members)
    for p in range(len(patches)):
        mem = patches[p]
        if not mem or 2 * len(mem) >= target:
            continue
        cnt = {}
        for v in mem:
            for u in indices[indptr[v]:indptr[v + 1]]:
                q = int(pid[u])
                if q != p:
                    cnt[q] = cnt.get(q, 0) + 1
        if not cnt:
            continue
        best = min(cnt.items(), key=lambda kv: (-kv[1], kv[0]))[0]
        for v in mem:
            pid[v] = best
        patches[best].extend(mem)
        patches[p] = []
    out = [np.sort(np.asarray(m, dtype=np.int64)) for m in patches if m]
    return out


def patch_energy(A: sp.csr_matrix, members, energy: str) -> np.ndarray:
    """The patch energy named by `energy`: "interior", "closed" or "split"."""
    if energy == "closed":
        return closed_energy(A, members)
    if energy == "split":
        return split_energy(A, members)
    return interior_energy(A, members)


def eps_partition(A: sp.csr_matrix, coords: Optional[np.ndarray], eps_k: float, cbound: float,
                  energy: str = "split", max_size: int = 32):
    """Partition with prescribed accuracy (Section 2.3: the partition must give
    error factor eps(P) <= eps_k and eps(P) delta(P) <= c; reading of the
    deferred partitioner).

    Seeds in Morton order (vertex order without coordinates).  A seed opens a
    patch that grows greedily: among the unassigned vertices adjacent to the
    patch and not yet refused by it, the one with the largest total coupling
    sum_{p in P} |a_vp| to the patch is tried next (ties: smaller vertex id).
    It joins when the enlarged patch still has eps(P) = 1 / lambda_2(E_P) <=
    eps_k (E_P the patch energy named by `energy`, the split energy in the
    decomposition) and
    eps(P) delta(P) <= c with delta(P) = 1 / (phi^T Abar_P^-1 phi), phi the
    unit eigenvector of lambda_1(E_P) and Abar_P the closed energy (principal
    submatrix); otherwise the patch refuses it.  The patch closes when no
    candidate is left or it holds max_size vertices.  Members sorted; patches
    in creation order.
    """
    n = A.shape[0]
    order = morton_order(coords) if coords is not None else np.arange(n)
    indptr, indices, data = A.indptr, A.indices, A.data
    pid = np.full(n, -1, dtype=np.int64)
    patches = []
    for s0 in order:
        s0 = int(s0)
        if pid[s0] >= 0:
            continue
        cur = len(patches)
        members = [s0]
        pid[s0] = cur
        coupling = {}           # candidate -> total coupling to the patch
        refused = set()

        def add_couplings(v):
            for a in range(indptr[v], indptr[v + 1]):
                u = int(indices[a])
                if u != v and pid[u] < 0:
                    coupling[u] = coupling.get(u, 0.0) + abs(float(data[a]))

        add_couplings(s0)
        while len(members) < max_size:
            cands = [(-w, u) for u, w in coupling.items() if u not in refused and pid[u] < 0]
            if not cands:
                break
            u = min(cands)[1]
            cand = np.sort(np.asarray(members + [u], dtype=np.int64))
            Abar = A[cand][:, cand].toarray()  # closed energy: principal submatrix
            E = patch_energy(A, cand, energy)
            w, V = np.linalg.eigh(0.5 * (E + E.T))
            ok = False
            if w[1] > 0:
                eps = 1.0 / w[1]
                phi = V[:, 0]
                delta = 1.0 / float(phi @ np.linalg.solve(Abar, phi))
                ok = eps <= eps_k and eps * delta <= cbound
            if ok:
                members.append(u)
                pid[u] = cur
                del coupling[u]
                add_couplings(u)
            else:
                refused.add(u)
        patches.append(np.sort(np.asarray(members, dtype=np.int64)))
    return patches


def patch_id_of(patches, n):
    pid = np.empty(n, dtype=np.int64)
    for j, m in enumerate(patches):
        pid[m] = j
    return pid


def patch_neighbours(A: sp.csr_matrix, patches, pid):
    """Sorted neighbour patch ids (structural adjacency through A)."""
    nb = []
    for j, mem in enumerate(patches):
        s = set()
        for v in mem:
            for u in A.indices[A.indptr[v]:A.indptr[v + 1]]:
                q = int(pid[u])
                if q != j:
                    s.add(q)
        nb.append(sorted(s))
    return nb


def hop_set(nbrs, j, r):
    """Patches within r hops of patch j (sorted)."""
    seen = {j}
    frontier = [j]
    for _ in range(r):
        nxt = []
        for a in frontier:
            for b in nbrs[a]:
                if b not in seen:
                    seen.add(b)
                    nxt.append(b)
        frontier = nxt
    return sorted(seen)


# ----------------------------------------------------------------------------
# per-patch basis, Householder complement, Psi
# ----------------------------------------------------------------------------

def local_basis(A: sp.csr_matrix, members, closed=False, energy=None):
    """phi (unit, sum > 0; first nonzero > 0 if the sum vanishes), lambda_1, lambda_2.

    The patch energy is the interior energy on the first level and the closed
    energy (principal submatrix) on later levels, or the split energy on every
    level of a partition to prescribed accuracy (`energy` names it).
    """
    if energy is None:
        energy = "closed" if closed else "interior"
    E = patch_energy(A, members, energy)
    E = 0.5 * (E + E.T)
    w, V = np.linalg.eigh(E)
    phi = V[:, 0].copy()
    s = phi.sum()
    if s < 0 or (s == 0 and phi[np.nonzero(phi)[0][0]] < 0):
        phi = -phi
    lam2 = w[1] if w.size > 1 else np.inf
    return phi, w[0], lam2


def householder_vector(phi):
    """(u, t): H = I - 2 u u^T / u^T u maps e_t to -sign(phi_t) phi, with the
    pivot slot t the first i with |phi_i| >= (1 - 1e-8) max_j |phi_j|.

    u = phi + s e_t, s = +1 if phi_t >= 0 else -1 (no cancellation).  The
    complement U of phi in the patch is the columns H e_i, i != t, in
    ascending slot order (Lemma 2.3 remark: any orthonormal completion).  A
    pivot of near-maximal magnitude keeps the sign choice, and with it U, away
    from entries that rounding alone decides (an eigenvector entry that is
    zero in exact arithmetic); taking the first of the near-maximal entries
    keeps the choice stable when symmetry makes several maxima equal in exact
    arithmetic.
    """
    a = np.abs(phi)
    t = int(np.nonzero(a >= (1.0 - 1e-8) * a.max())[0][0])
    u = phi.copy()
    s = 1.0 if phi[t] >= 0 else -1.0
    u[t] += s
    return u, t


def psi_exact(A: sp.csr_matrix, patches, phis):
    n = A.shape[0]
    m = len(patches)
    Phi = np.zeros((n, m))
    for j, (mem, ph) in enumerate(zip(patches, phis)):
        Phi[mem, j] = ph
    Ad = A.toarray()
    c = sla.cho_factor(Ad)
    Y = sla.cho_solve(c, Phi)
    G = Phi.T @ Y
    G = 0.5 * (G + G.T)
    Psi = sla.cho_solve(sla.cho_factor(G), Y.T).T
    rows = np.repeat(np.arange(n, dtype=np.int64), m)
    cols = np.tile(np.arange(m, dtype=np.int64), n)
    return sp.csr_matrix((Psi.ravel(), (rows, cols)), shape=(n, m))


def psi_localized(A: sp.csr_matrix, patches, phis, r_hops):
    """Column j: argmin psi^T A psi, supp psi in S_j, phi_i^T psi = delta_ij (i in S_j)."""
    n = A.shape[0]
    pid = patch_id_of(patches, n)
    nbrs = patch_neighbours(A, patches, pid)
    rows, cols, vals = [], [], []
    for j in range(len(patches)):
        C = hop_set(nbrs, j, r_hops)
        S = np.sort(np.concatenate([patches[i] for i in C]))
        pos = {int(v): a for a, v in enumerate(S)}
        ASS = A[S][:, S].toarray()
        PhiC = np.zeros((S.size, len(C)))
        for b, i in enumerate(C):
            PhiC[[pos[int(v)] for v in patches[i]], b] = phis[i]
        c = sla.cho_factor(ASS)
        Y = sla.cho_solve(c, PhiC)
        G = PhiC.T @ Y
        G = 0.5 * (G + G.T)
        e = np.zeros(len(C))
        e[C.index(j)] = 1.0
        coef = sla.cho_solve(sla.cho_factor(G), e)
        psi = Y @ coef
        rows.append(S)
        cols.append(np.full(S.size, j, dtype=np.int64))
        vals.append(psi)
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, len(patches)))


def galerkin(Psi: sp.csr_matrix, X: Optional[sp.csr_matrix]):
    """Psi^T X Psi (X = None means identity), symmetrised, on the structural pattern.

    The pattern is that of |Psi|^T |X| |Psi| (no entry dropped for exact
    cancellation); values are 0.5 (C + C^T) with C = Psi^T (X Psi).
    """
    Psi = sp.csr_matrix(Psi)
    aPsi = abs(Psi)
    if X is None:
        C = (Psi.T @ Psi).tocsr()
        P = (aPsi.T @ aPsi).tocsr()
    else:
        C = (Psi.T @ (X @ Psi)).tocsr()
        P = (aPsi.T @ (abs(X) @ aPsi)).tocsr()
    C = 0.5 * (C + C.T)
    C = sp.csr_matrix(C)
    C.sort_indices()
    P.sort_indices()
    P = sp.csr_matrix(P)
    coo = P.tocoo()
    v = np.asarray(C[coo.row, coo.col]).ravel()
    out = sp.csr_matrix((v, P.indices.copy(), P.indptr.copy()), shape=P.shape)
    return out


# ----------------------------------------------------------------------------
# the decomposition
# ----------------------------------------------------------------------------

@dataclass
class Level:
    k: int
    A: sp.csr_matrix
    M: Optional[sp.csr_matrix]            # None on level 0 (identity)
    coords: Optional[np.ndarray] = None
    grid: Optional[tuple] = None
    # transfer from level k-1 (k >= 1):
    Psi: Optional[sp.csr_matrix] = None    # N_{k-1} x N_k
    patches: list = field(default_factory=list)
    phis: list = field(default_factory=list)
    hh: list = field(default_factory=list)   # (u, pivot slot) per patch
    eps_patch: Optional[np.ndarray] = None
    eps_level: float = 0.0                 # eps(P^(k))
    lam_max_M: float = 1.0                 # Gershgorin bound on lambda_max(M^(k))

    @property
    def n(self):
        return self.A.shape[0]

    # U^(k) maps the reduced space (one dof fewer per patch) to level k-1
    def nb(self):
        return sum(len(m) - 1 for m in self.patches)

    def U_apply(self, y: np.ndarray) -> np.ndarray:
        """x = U y: per patch place y's slots in the non-pivot slots (ascending),
        0 in the pivot slot, and apply H_j."""
        y = np.asarray(y)
        nfine = sum(len(m) for m in self.patches)
        x = np.zeros((nfine,) + y.shape[1:])
        off = 0
        for mem, (u, t) in zip(self.patches, self.hh):
            p = len(mem)
            rest = [i for i in range(p) if i != t]
            z = np.zeros((p,) + y.shape[1:])
            z[rest] = y[off:off + p - 1]
            off += p - 1
            z = z - (2.0 / (u @ u)) * np.multiply.outer(u, u @ z)
            x[mem] = z
        return x

    def Ut_apply(self, x: np.ndarray) -> np.ndarray:
        """y = U^T x: per patch apply H_j to x_P and keep the non-pivot slots."""
        x = np.asarray(x)
        out = []
        for mem, (u, t) in zip(self.patches, self.hh):
            z = x[mem]
            z = z - (2.0 / (u @ u)) * np.multiply.outer(u, u @ z)
            out.append(np.delete(z, t, axis=0))
        return np.concatenate(out) if out else np.zeros((0,) + x.shape[1:])


@dataclass
class MMD:
    levels: List[Level]
    eps: List[float]          # eps_k cumulative, eps[0] = 0

    @property
    def K(self):
        return len(self.levels) - 1


def gershgorin_max(M: Optional[sp.csr_matrix]) -> float:
    if M is None:
        return 1.0
    return float(np.max(np.asarray(abs(M).sum(axis=1)).ravel()))


def build_mmd(A, coords=None, grid=None, levels=3, targets=(4, 8), grid_blocks=(4, 2),
              r_hops=1, exact_max_n=0, min_coarse=4, eps1=0.0, eta=0.1, cbound=20.0,
              r_hops_coarse=0,
              max_patch=32):
    """Build the K-level decomposition.

    levels      number of coarse levels K (stops early when a level would not
                shrink or would drop below ``min_coarse`` dofs)
    targets     greedy patch size per level for graphs (last entry repeats)
    grid_blocks tensor block edge per level for structured grids (last repeats)
    r_hops      localisation radius of Psi in patch hops
    r_hops_coarse  radius of Psi^(k) for k >= 2 (0: r_hops)
    exact_max_n levels with N_{k-1} <= exact_max_n use the exact Psi
    eps1, eta, cbound, max_patch
                eps1 > 0: graphs are partitioned to prescribed accuracy,
                eps(P^(k)) <= eps1 / eta^(k-1) and eps delta <= cbound
                (Section 2.3), patches of at most max_patch vertices
    """
    A = sp.csr_matrix(A)
    A.sort_indices()
    energy_elements(A)  # validates the edge-type decomposition of level 0
    lev0 = Level(0, A, None, None if coords is None else np.asarray(coords, float),
                 None if grid is None else tuple(grid))
    out = [lev0]
    eps = [0.0]
    for k in range(1, levels + 1):
        prev = out[-1]
        Ak = prev.A
        if prev.grid is not None:
            blk = grid_blocks[min(k - 1, len(grid_blocks) - 1)]
            patches, cgrid = grid_partition(prev.grid, blk)
        elif eps1 > 0:
            patches = eps_partition(Ak, prev.coords, eps1 / eta ** (k - 1), cbound, "split",
                                    max_patch)
            cgrid = None
        else:
            tgt = targets[min(k - 1, len(targets) - 1)]
            patches = greedy_partition(Ak, prev.coords, tgt)
            cgrid = None
        if len(patches) >= prev.n or len(patches) < min_coarse:
            break
        phis, hh, epsp = [], [], []
        for mem in patches:
            phi, l1, l2 = local_basis(Ak, mem, energy=("split" if eps1 > 0 else
                                                       "closed" if k >= 2 else "interior"))
            phis.append(phi)
            hh.append(householder_vector(phi))
            epsp.append(0.0 if len(mem) < 2 else (1.0 / l2 if l2 > 0 else np.inf))
        if prev.n <= exact_max_n:
            Psi = psi_exact(Ak, patches, phis)
        else:
            Psi = psi_localized(Ak, patches, phis,
                                r_hops_coarse if (k >= 2 and r_hops_coarse > 0) else r_hops)
        # the support of psi_j is the set of its nonzero entries: a stored exact
        # zero carries no coupling into the Galerkin patterns
        Psi.eliminate_zeros()
        Anew = galerkin(Psi, Ak)
        Mnew = galerkin(Psi, prev.M)
        ccoords = None
        if prev.coords is not None:
            ccoords = np.stack([prev.coords[m].mean(axis=0) for m in patches])
        lev = Level(k, Anew, Mnew, ccoords, cgrid, Psi, patches, phis, hh,
                    np.asarray(epsp), float(np.max(epsp)), gershgorin_max(Mnew))
        out.append(lev)
        eps.append(eps[-1] + lev.eps_level)
    return MMD(out, eps)


@dataclass
class Schedule:
    """Per-level accuracies and thresholds (Section 5, eq. parameter_choice)."""
    eps_op: List[float]
    mu_re: List[float]
    mu_ex: List[float]
    d: List[int]


def schedule(mmd: MMD, m_tar: int, tol: float, alpha=3.0, beta=1.0):
    K = mmd.K
    eps_op, mu_re, mu_ex, d = [], [], [], []
    for k in range(K + 1):
        eps_op.append(tol if k == 0 else 0.1 * mmd.eps[k])
        mu_re.append(alpha * mmd.eps[k + 1] if k + 1 <= K else 0.0)
        mu_ex.append(beta * mmd.eps[k])
        n_k = mmd.levels[k].n
        d.append(max(1, min(n_k // 10, m_tar // 10)))
    return Schedule(eps_op, mu_re, mu_ex, d)
