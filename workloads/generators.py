"""Seeded generators for the sparse SPD test and benchmark matrices.

Every matrix is returned in CSR form with int64 row pointers, int32 column
indices sorted within each row, and float64 values.  The matrices are graph
Laplacians plus a nonnegative diagonal (off-diagonals <= 0), which is the
energy-decomposable class the hierarchical solver works on (Section 2.1 of the
paper: edge elements plus self-loop elements).

Workloads (sizes as used by the benchmark and tests):
  * grid2d(32)          2-D 5-point Dirichlet Laplacian, n = 1024
  * rgg(100000, 0)      random geometric graph in the unit square, mean degree
                        about 10, weights exp(-d^2/r^2), plus 1e-6 I
  * grid3d_lognormal(64) 3-D 7-point diffusion with lognormal face
                        coefficients (Dirichlet ghosts included), n = 262144
  * rgg_batch(64)       64 RGG Laplacians, sizes uniform in [5000, 50000]
  * knn_gmm(200000, 10) kNN graph of a 3-component Gaussian mixture in R^3,
                        weights exp(-d^2), plus 1e-6 I
  * swissroll(20000)    the paper's SwissRoll point cloud, kNN (k = 10) graph,
                        weights exp(-r^2/0.1), rescaled Laplacian plus I
The paper's own data sets (bunny, brain point clouds) are external; these
synthetic graphs stand in for them with the same structure (kNN / radius
graphs of point clouds, Laplacian plus a small diagonal).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class Problem:
    name: str
    n: int
    rowptr: np.ndarray          # int64 [n+1]
    col: np.ndarray             # int32 [nnz]
    val: np.ndarray             # float64 [nnz]
    coords: Optional[np.ndarray] = None   # float64 [n, d] or None
    grid: Optional[Tuple[int, ...]] = None  # (nx, ny[, nz]) for structured grids
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col.astype(np.int64), self.rowptr),
                             shape=(self.n, self.n))


def _csr_from_coo(n, rows, cols, vals):
    """Sum duplicates and return sorted CSR arrays."""
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    vals = vals[order]
    if rows.size:
        key = rows.astype(np.int64) * n + cols
        uniq, start = np.unique(key, return_index=True)
        sums = np.add.reduceat(vals, start) if vals.size else vals
        rows = (uniq // n).astype(np.int64)
        cols = (uniq % n).astype(np.int64)
        vals = sums
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), vals.astype(np.float64)


def laplacian_from_edges(n, ei, ej, w, diag_extra):
    """L + diag(diag_extra) for undirected edges (ei < ej) with weights w."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    deg = np.zeros(n)
    np.add.at(deg, ei, w)
    np.add.at(deg, ej, w)
    diag = deg + np.broadcast_to(np.asarray(diag_extra, dtype=np.float64), (n,))
    idx = np.arange(n, dtype=np.int64)
    rows = np.concatenate([ei, ej, idx])
    cols = np.concatenate([ej, ei, idx])
    vals = np.concatenate([-w, -w, diag])
    return _csr_from_coo(n, rows, cols, vals)


def grid2d(nx: int, ny: Optional[int] = None) -> Problem:
    """A = I (x) T + T (x) I, T = tridiag(-1, 2, -1); vertex (x, y) -> y*nx + x."""
    ny = nx if ny is None else ny
    n = nx * ny
    ei, ej = [], []
    ids = np.arange(n).reshape(ny, nx)
    ei.append(ids[:, :-1].ravel()); ej.append(ids[:, 1:].ravel())
    ei.append(ids[:-1, :].ravel()); ej.append(ids[1:, :].ravel())
    ei = np.concatenate(ei); ej = np.concatenate(ej)
    w = np.ones(ei.size)
    # Dirichlet ghosts: each missing neighbour contributes 1 to the diagonal.
    deg_missing = np.zeros((ny, nx))
    deg_missing[:, 0] += 1; deg_missing[:, -1] += 1
    deg_missing[0, :] += 1; deg_missing[-1, :] += 1
    rowptr, col, val = laplacian_from_edges(n, ei, ej, w, deg_missing.ravel())
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([xx.ravel(), yy.ravel()], axis=1).astype(np.float64)
    return Problem(f"grid2d_{nx}x{ny}", n, rowptr, col, val, coords, (nx, ny))


def grid3d_lognormal(m: int, seed: int = 0, sigma: float = 1.0) -> Problem:
    """7-point diffusion on an m^3 grid, one coefficient exp(sigma Z) per face.

    Faces to the Dirichlet ghost layer carry coefficients too; they only add
    to the diagonal.  Vertex (x, y, z) -> (z*m + y)*m + x.
    """
    rng = np.random.default_rng(seed)
    n = m ** 3
    ids = np.arange(n).reshape(m, m, m)  # [z, y, x]
    ax = rng.standard_normal((m, m, m + 1))   # faces normal to x
    ay = rng.standard_normal((m, m + 1, m))
    az = rng.standard_normal((m + 1, m, m))
    cx = np.exp(sigma * ax); cy = np.exp(sigma * ay); cz = np.exp(sigma * az)
    extra = np.zeros((m, m, m))
    extra[:, :, 0] += cx[:, :, 0]; extra[:, :, -1] += cx[:, :, -1]
    extra[:, 0, :] += cy[:, 0, :]; extra[:, -1, :] += cy[:, -1, :]
    extra[0, :, :] += cz[0, :, :]; extra[-1, :, :] += cz[-1, :, :]
    ei = np.concatenate([ids[:, :, :-1].ravel(), ids[:, :-1, :].ravel(), ids[:-1, :, :].ravel()])
    ej = np.concatenate([ids[:, :, 1:].ravel(), ids[:, 1:, :].ravel(), ids[1:, :, :].ravel()])
    w = np.concatenate([cx[:, :, 1:-1].ravel(), cy[:, 1:-1, :].ravel(), cz[1:-1, :, :].ravel()])
    rowptr, col, val = laplacian_from_edges(n, ei, ej, w, extra.ravel())
    zz, yy, xx = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.float64)
    return Problem(f"grid3d_lognormal_{m}", n, rowptr, col, val, coords, (m, m, m),
                   {"seed": seed, "sigma": sigma})


def rgg(n: int, seed: int = 0, mean_degree: float = 10.0, shift: float = 1e-6) -> Problem:
    """Random geometric graph Laplacian + shift*I in the unit square.

    r = sqrt(mean_degree / (pi (n-1))); an edge joins points closer than r,
    with weight exp(-d^2 / r^2).
    """
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = float(np.sqrt(mean_degree / (np.pi * (n - 1))))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray").astype(np.int64)
    if pairs.size:
        pairs.sort(axis=1)
        order = np.lexsort((pairs[:, 1], pairs[:, 0]))
        pairs = pairs[order]
    else:
        pairs = np.zeros((0, 2), dtype=np.int64)
    d2 = np.sum((pts[pairs[:, 0]] - pts[pairs[:, 1]]) ** 2, axis=1)
    w = np.exp(-d2 / (r * r))
    rowptr, col, val = laplacian_from_edges(n, pairs[:, 0], pairs[:, 1], w, shift)
    return Problem(f"rgg_{n}_s{seed}", n, rowptr, col, val, pts, None,
                   {"seed": seed, "radius": r, "shift": shift})


def rgg_batch(count: int = 64, seed: int = 0, lo: int = 5000, hi: int = 50000,
              mean_degree: float = 8.0, shift: float = 1e-6):
    """A list of RGG Laplacians with sizes uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=count)
    return [rgg(int(nb), seed=seed * 1000 + 1 + b, mean_degree=mean_degree, shift=shift)
            for b, nb in enumerate(sizes)]


def knn_gmm(n: int, k: int = 10, seed: int = 1, shift: float = 1e-6) -> Problem:
    """kNN graph (union-symmetrised) of a 3-component Gaussian mixture in R^3.

    Mixture weights (0.5, 0.3, 0.2), means (0,0,0), (3,0,0), (7,0,0),
    identity covariance, edge weight exp(-d^2).
    """
    rng = np.random.default_rng(seed)
    comp = rng.choice(3, size=n, p=[0.5, 0.3, 0.2])
    means = np.array([[0.0, 0, 0], [3.0, 0, 0], [7.0, 0, 0]])
    pts = means[comp] + rng.standard_normal((n, 3))
    dist, nbr = cKDTree(pts).query(pts, k=k + 1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = nbr[:, 1:].ravel().astype(np.int64)
    a = np.minimum(src, dst); b = np.maximum(src, dst)
    keep = a != b
    a = a[keep]; b = b[keep]
    key = np.unique(a * n + b)
    ei = key // n; ej = key % n
    d2 = np.sum((pts[ei] - pts[ej]) ** 2, axis=1)
    w = np.exp(-d2)
    rowptr, col, val = laplacian_from_edges(n, ei, ej, w, shift)
    return Problem(f"knn_gmm_{n}_k{k}_s{seed}", n, rowptr, col, val, pts, None,
                   {"seed": seed, "k": k, "shift": shift})


def swissroll(n: int = 20000, k: int = 10, seed: int = 0, sigma: float = 0.1,
              noise_std: float = 0.05, kappa: float = 1.15e6,
              y_max: Optional[float] = None) -> Problem:
    """The SwissRoll data set of the paper's experiments (Section 7.1).

    Points (t cos t, y, t sin t) + eta with t ~ U[1.5 pi, 4.5 pi],
    y ~ U[0, 20], eta ~ N(0, s^2 I_3) with s = noise_std = 0.05: the paper's
    covariance parameter 0.05 is read as the standard deviation, because with
    it the graph has the stored-entry count the paper reports for this data set
    (248010; seeds 0 and 1 give 248072 and 247968, against 255650 and 255602
    when 0.05 is taken as the variance);
    union-symmetrised kNN graph, edge weight exp(-r^2 / sigma).  The
    Laplacian is rescaled and given unit self-loops, A = c L + I, so that
    lambda_1 = 1; c is fixed by the condition number the paper reports for
    this data set, kappa(A) = c lambda_max(L) + 1 = kappa (lambda_max(L) from
    Lanczos with a fixed start vector, so the input is deterministic).

    The paper's roll has n = 20000 points over y in [0, 20].  A smaller n keeps
    that point density (y_max = 20 n / 20000 unless given), so neighbour
    distances, edge weights and the low spectrum (lambda_2 = O(1)) keep the
    structure of the full-size graph; a small n over the full y range would
    leave a sparse cloud with near-disconnected pieces and a cluster of
    eigenvalues within 1e-6 of lambda_1.
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    rng = np.random.default_rng(seed)
    t = rng.uniform(1.5 * np.pi, 4.5 * np.pi, n)
    if y_max is None:
        y_max = 20.0 * n / 20000.0
    y = rng.uniform(0.0, y_max, n)
    pts = np.stack([t * np.cos(t), y, t * np.sin(t)], axis=1)
    pts = pts + rng.normal(0.0, noise_std, (n, 3))
    dist, nbr = cKDTree(pts).query(pts, k=k + 1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = nbr[:, 1:].ravel().astype(np.int64)
    a = np.minimum(src, dst); b = np.maximum(src, dst)
    keep = a != b
    a = a[keep]; b = b[keep]
    key = np.unique(a * n + b)
    ei = key // n; ej = key % n
    w = np.exp(-np.sum((pts[ei] - pts[ej]) ** 2, axis=1) / sigma)
    W = sp.csr_matrix((w, (ei, ej)), shape=(n, n))
    W = W + W.T
    L = sp.csr_matrix(sp.diags(np.asarray(W.sum(axis=1)).ravel()) - W)
    lmax = float(sla.eigsh(L, k=1, which="LA", v0=np.ones(n), tol=1e-12,
                           return_eigenvectors=False)[0])
    c = (kappa - 1.0) / lmax
    rowptr, col, val = laplacian_from_edges(n, ei, ej, c * w, 1.0)
    return Problem(f"swissroll_{n}_k{k}_s{seed}", n, rowptr, col, val, pts, None,
                   {"seed": seed, "k": k, "sigma": sigma, "scale": c, "lambda_max_L": lmax})


def random_csr(n_rows: int, n_cols: int, nnz_per_row, seed: int = 0,
               empty_frac: float = 0.0):
    """Random general CSR (rowptr int64, col int32, val float64) for kernel tests.

    nnz_per_row may be an int or a (lo, hi) range; a fraction of rows is empty.
    """
    rng = np.random.default_rng(seed)
    if isinstance(nnz_per_row, tuple):
        counts = rng.integers(nnz_per_row[0], nnz_per_row[1] + 1, size=n_rows)
    else:
        counts = np.full(n_rows, int(nnz_per_row))
    counts = np.minimum(counts, n_cols)
    if empty_frac > 0:
        counts[rng.random(n_rows) < empty_frac] = 0
    rowptr = np.zeros(n_rows + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(counts)
    col = np.empty(int(rowptr[-1]), dtype=np.int32)
    for i in range(n_rows):
        c = counts[i]
        if c:
            col[rowptr[i]:rowptr[i + 1]] = np.sort(rng.choice(n_cols, size=c, replace=False))
    val = rng.standard_normal(int(rowptr[-1]))
    return rowptr, col, val


def random_block(n: int, b: int, seed: int = 0) -> np.ndarray:
    """Dense float64 [n, b] block with standard normal entries."""
    return np.random.default_rng(seed).standard_normal((n, b))


def by_name(name: str) -> Problem:
    """Small and full-size named workloads."""
    table = {
        "grid2d_32": lambda: grid2d(32),
        "grid2d_8": lambda: grid2d(8),
        "grid2d_16": lambda: grid2d(16),
        "grid3d_8": lambda: grid3d_lognormal(8, 0),
        "grid3d_16": lambda: grid3d_lognormal(16, 0),
        "grid3d_64": lambda: grid3d_lognormal(64, 0),
        "rgg_500": lambda: rgg(500, 0),
        "rgg_2000": lambda: rgg(2000, 0),
        "rgg_20000": lambda: rgg(20000, 0),
        "rgg_100000": lambda: rgg(100000, 0),
        "knn_300": lambda: knn_gmm(300, 10, 1),
        "knn_200000": lambda: knn_gmm(200000, 10, 1),
    }
    return table[name]()


def rgg_window(p: Problem, frac: float, shift: float = 1e-6) -> Problem:
    """The RGG of the points of p inside the corner square of area `frac`.

    Same point density, radius and weights as p; the Laplacian is rebuilt from
    the kept edges (a spatial sample of the same workload).
    """
    w = float(np.sqrt(frac))
    keep = np.where((p.coords[:, 0] < w) & (p.coords[:, 1] < w))[0]
    A = p.scipy()[keep][:, keep].tocoo()
    off = A.row < A.col
    rowptr, col, val = laplacian_from_edges(keep.size, A.row[off], A.col[off], -A.data[off], shift)
    return Problem(f"{p.name}_window{frac:g}", keep.size, rowptr, col, val, p.coords[keep].copy(),
                   None, {"parent": p.name, "frac": frac, "shift": shift})
