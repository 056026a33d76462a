"""Energy elements and patch energies (Section 2.1 of the paper).

A matrix is energy decomposable when A = sum_k E_k with E_k >= 0.  For a
graph Laplacian plus a nonnegative diagonal the finest elements are the edge
elements w_ij (e_i - e_j)(e_i - e_j)^T, w_ij = -a_ij >= 0, and the self-loop
elements s_i e_i e_i^T with s_i = a_ii - sum_{j != i} w_ij >= 0.

The paper names the interior energy of a patch (the sum of the elements
supported inside the patch) but defines it in its companion work.  Reading
used here, on every level: the level matrix is split into generalised edge
elements |a_ij| (e_i - sgn(a_ij) e_j)(e_i - sgn(a_ij) e_j)^T plus the
diagonal remainder r_i = a_ii - sum_{j != i} |a_ij|, clamped at 0.  The
interior energy of patch P is the sum of the elements inside P:
    off-diagonal  a_ij                      (i, j in P, i != j)
    diagonal      sum_{j in P, j != i} |a_ij| + max(r_i, 0).
On level 0 (all a_ij <= 0, r_i = s_i >= 0) this is exactly "edges inside P
plus the self-loops"; that is what patches of the first level use.

Coarse matrices (levels >= 1) are far from diagonally dominant and their
inherited elements (Definition 2.4) are spread over several coarse patches by
the overlap of the localized Psi, so almost no element is interior to a small
coarse patch.  Patches of the second and later levels therefore use the
closed energy, the principal submatrix A^(k)[P, P] (always SPD).

The partition to prescribed accuracy uses the split energy instead, on
every level: E_P = A[P, P] - diag(sum_{j not in P} |a_ij|).  The rest,
A - sum_P E_P, is the off-patch part plus the diagonal of its absolute row
sums, which is diagonally dominant and so positive semidefinite; hence
sum_P E_P <= A, the property the patch error bound of Section 2.2 needs.  On
level 0 of a Laplacian plus a nonnegative diagonal it equals the interior
energy.
"""
import numpy as np
import scipy.sparse as sp


class UnsupportedMatrix(ValueError):
    """Off-diagonal > 0 or a negative self-loop: no edge-type decomposition."""


def energy_elements(A: sp.csr_matrix):
    """Edge list (i < j, w_ij) and self-loop weights s_i of a Laplacian + diagonal.

    Raises UnsupportedMatrix when an off-diagonal is positive or s_i is
    negative beyond 1e-14 * a_ii (values in that band are clamped to 0).
    """
    A = sp.csr_matrix(A)
    C = A.tocoo()
    off = C.row != C.col
    if np.any(C.data[off] > 0):
        raise UnsupportedMatrix("positive off-diagonal entry")
    diag = A.diagonal()
    offsum = np.zeros(A.shape[0])
    np.add.at(offsum, C.row[off], C.data[off])
    s = diag + offsum
    bad = s < -1e-14 * np.abs(diag)
    if np.any(bad):
        raise UnsupportedMatrix("negative self-loop weight (not diagonally dominant)")
    s = np.where(s < 0, 0.0, s)
    up = off & (C.row < C.col)
    return C.row[up].astype(np.int64), C.col[up].astype(np.int64), -C.data[up], s


def interior_energy(A: sp.csr_matrix, members: np.ndarray) -> np.ndarray:
    """Dense interior energy matrix of the patch with (sorted) vertex list members."""
    members = np.asarray(members, dtype=np.int64)
    pos = {int(v): a for a, v in enumerate(members)}
    p = members.size
    E = np.zeros((p, p))
    for a, i in enumerate(members):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        diag = 0.0
        offabs = 0.0
        inner = 0.0
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            c = int(c)
            if c == i:
                diag += v
                continue
            offabs += abs(v)
            b = pos.get(c)
            if b is not None:
                E[a, b] = v
                inner += abs(v)
        E[a, a] = inner + max(diag - offabs, 0.0)
    return E


def closed_energy(A: sp.csr_matrix, members: np.ndarray) -> np.ndarray:
    """Dense principal submatrix A[P, P] of the (sorted) vertex list members."""
    members = np.asarray(members, dtype=np.int64)
    pos = {int(v): a for a, v in enumerate(members)}
    p = members.size
    E = np.zeros((p, p))
    for a, i in enumerate(members):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            b = pos.get(int(c))
            if b is not None:
                E[a, b] = v
    return E


def split_energy(A: sp.csr_matrix, members: np.ndarray) -> np.ndarray:
    """E_P = A[P, P] - diag(sum_{j not in P} |a_ij|) for the (sorted) vertex
    list members: sum over patches of E_P is bounded by A (Section 2.2 patch
    energy; see the module docstring)."""
    members = np.asarray(members, dtype=np.int64)
    pos = {int(v): a for a, v in enumerate(members)}
    p = members.size
    E = np.zeros((p, p))
    for a, i in enumerate(members):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        outside = 0.0
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            b = pos.get(int(c))
            if b is None:
                outside += abs(v)
            else:
                E[a, b] = v
        E[a, a] -= outside
    return E
