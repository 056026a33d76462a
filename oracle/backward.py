"""Eigen-backward oracle (test infrastructure only; never imported by the library).

The paper computes eigenpairs only; the reverse-mode derivative is the
standard first-order perturbation theory of a symmetric matrix, written out
here for the nev leftmost pairs (A v_k = lambda_k v_k, V^T V = I):

  d lambda_k = v_k^T dA v_k
  d v_k      = -(A - lambda_k I)^+ dA v_k      (simple lambda_k, v_k^T d v_k = 0)

For a loss L(lambda, V) with adjoints g_lambda, g_V, and a symmetric
perturbation dA, dL = sum_ij S_ij dA_ij with

  S = sum_k g_lambda_k v_k v_k^T - sum_k sym(x_k v_k^T),
  x_k = (A - lambda_k I)^+ (I - v_k v_k^T) g_V_k
      = sum_{j != k, j <= nev} v_j (v_j^T g_V_k) / (lambda_j - lambda_k)
        + (A - lambda_k I)^-1 restricted to V-perp applied to (I - V V^T) g_V_k,

sym(Y) = (Y + Y^T) / 2.  The second part of x_k is a CG solve with A -
lambda_k I on the complement of the computed eigenvectors, which is SPD
there because lambda_k < lambda_{nev+1}.  Only S on the stored pattern of A
is returned (the sampled product of the low-rank factors).

A pair j != k with lambda_j == lambda_k (relative 1e-10) and
v_j^T g_V_k != 0 has no defined gradient: ValueError.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp

from .krylov import cg


class UndefinedGradient(ValueError):
    pass


def complement_solve(A: sp.csr_matrix, V: np.ndarray, lam_k: float, r: np.ndarray,
                     tol: float) -> np.ndarray:
    """y in V-perp with P (A - lam_k I) P y = r, P = I - V V^T, r in V-perp (plain CG
    with the projection applied to every operator product)."""
    def proj(y):
        return y - V @ (V.T @ y)

    def op(y):
        return proj(A @ y - lam_k * y)

    y, _ = cg(op, proj(r), None, tol)
    return proj(y)


def adjoint_vectors(A: sp.csr_matrix, lam: np.ndarray, V: np.ndarray,
                    g_V: Optional[np.ndarray], tol: float = 1e-12,
                    degen_rel: float = 1e-10) -> np.ndarray:
    """x_k for every column (zero where g_V_k = 0)."""
    n, nev = V.shape
    X = np.zeros((n, nev))
    if g_V is None:
        return X
    C = V.T @ g_V                      # C[j, k] = v_j^T g_V_k
    for k in range(nev):
        g = g_V[:, k]
        if not np.any(g):
            continue
        xk = np.zeros(n)
        for j in range(nev):
            if j == k:
                continue
            gap = lam[j] - lam[k]
            if abs(gap) <= degen_rel * abs(lam[k]):
                if abs(C[j, k]) > 1e-12 * np.linalg.norm(g):
                    raise UndefinedGradient("repeated eigenvalue with a coupled adjoint")
                continue
            xk += V[:, j] * (C[j, k] / gap)
        rk = g - V @ C[:, k]
        if np.linalg.norm(rk) > 0.0:
            xk += complement_solve(A, V, lam[k], rk, tol)
        X[:, k] = xk
    return X


def sampled_gradient(A: sp.csr_matrix, lam: np.ndarray, V: np.ndarray,
                     g_lam: Optional[np.ndarray], g_V: Optional[np.ndarray],
                     tol: float = 1e-12) -> np.ndarray:
    """S_ij for every stored entry of A, in A's CSR order."""
    A = sp.csr_matrix(A)
    X = adjoint_vectors(A, lam, V, g_V, tol)
    gl = np.zeros(V.shape[1]) if g_lam is None else np.asarray(g_lam, dtype=float)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    out = np.zeros(A.nnz)
    for k in range(V.shape[1]):
        vi, vj = V[rows, k], V[cols, k]
        out += gl[k] * vi * vj - 0.5 * (X[rows, k] * vj + vi * X[cols, k])
    return out


def dense_gradient(A, lam_all: np.ndarray, V_all: np.ndarray, nev: int,
                   g_lam: Optional[np.ndarray], g_V: Optional[np.ndarray]) -> np.ndarray:
    """Reference S from the full eigendecomposition (small dense inputs): x_k
    summed over every other eigenvector, no solve."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    n = Ad.shape[0]
    S = np.zeros((n, n))
    for k in range(nev):
        v = V_all[:, k]
        if g_lam is not None:
            S += g_lam[k] * np.outer(v, v)
        if g_V is not None and np.any(g_V[:, k]):
            c = V_all.T @ g_V[:, k]
            d = lam_all - lam_all[k]
            d[k] = 1.0
            c[k] = 0.0
            x = V_all @ (c / d)
            S -= 0.5 * (np.outer(x, v) + np.outer(v, x))
    return S


def edge_gradient(S_vals: np.ndarray, A: sp.csr_matrix, ei: np.ndarray,
                  ej: np.ndarray) -> np.ndarray:
    """dL/dw_e for A = L(w) + diag: A_ii and A_jj grow by w_e, A_ij and A_ji
    fall by w_e, so dL/dw_e = S_ii + S_jj - S_ij - S_ji."""
    A = sp.csr_matrix(A)
    S = sp.csr_matrix((S_vals, A.indices, A.indptr), shape=A.shape)
    Sd = S.diagonal()
    sij = np.asarray(S[ei, ej]).ravel()
    sji = np.asarray(S[ej, ei]).ravel()
    return Sd[ei] + Sd[ej] - sij - sji
