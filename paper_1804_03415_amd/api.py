"""Python face of the C ABI: decomposition handles and the eigensolver calls.

Device buffers are torch tensors on the current HIP device; all work is
enqueued on the current torch stream.  Functions mirror include/mmdeig.h.
"""
import atexit
import ctypes
import weakref

import numpy as np

from . import _lib
from ._lib import MMDError, check, eig_opts, eig_stats, lib, mmd_build_opts, mmd_csr

OPS = {"A": 0, "M": 1, "B": 2, "U": 3, "Ut": 4, "Psi": 5, "A32": 6}

# every open handle, so they can all be released while the HIP runtime is
# still fully alive (at interpreter exit, before native exit handlers run)
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for d in list(_LIVE):
        d.close()


def build_options(levels=3, targets=(4, 8), grid_blocks=(4, 2), r_hops=1, exact_max_n=0,
                  min_coarse=4, eps1=0.0, eta=0.1, cbound=20.0, max_patch=32,
                  r_hops_coarse=0):
    """mmd_build_opts; eps1 > 0 partitions graphs to prescribed accuracy
    (eps(P^(k)) <= eps1 / eta^(k-1), eps delta <= cbound) instead of the
    target patch sizes."""
    o = mmd_build_opts()
    o.eps1, o.eta, o.cbound, o.max_patch = eps1, eta, cbound, max_patch
    o.r_hops_coarse = r_hops_coarse
    o.levels = levels if levels > 0 else -1
    o.n_targets = len(targets)
    for i, t in enumerate(targets):
        o.targets[i] = t
    o.n_grid_blocks = len(grid_blocks)
    for i, t in enumerate(grid_blocks):
        o.grid_blocks[i] = t
    o.r_hops = r_hops
    o.exact_max_n = exact_max_n
    o.min_coarse = min_coarse
    return o


def solver_options(alpha=3.0, beta=1.0, restart_mult=1, seed=0, max_restarts=2000,
                   max_refine=200, precision="fp64", streams=8, stop_level=0, d=0):
    """eig_opts; precision "fp64" or "fp32-refine" (FP32 CG inside FP64
    iterative refinement for the level-0 block solves); stop_level k >= 1
    returns the coarse-level approximation of level k; d the extension block
    size (0: default)."""
    o = eig_opts()
    o.stop_level, o.d = stop_level, d
    o.alpha, o.beta, o.restart_mult, o.seed = alpha, beta, restart_mult, seed
    o.max_restarts, o.max_refine = max_restarts, max_refine
    if precision not in ("fp64", "fp32-refine"):
        raise ValueError("precision must be 'fp64' or 'fp32-refine'")
    o.precision = 0 if precision == "fp64" else 1
    o.streams = streams
    return o


class Decomposition:
    """Handle of a multiresolution decomposition (mmd_build ... mmd_free)."""

    def __init__(self, rowptr, col, val, coords=None, grid=None, stream=None, **opts):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        n = rowptr.size - 1
        c = mmd_csr()
        c.n, c.nnz = n, int(rowptr[-1])
        c.rowptr, c.colind, c.val = _lib._ptr(rowptr), _lib._ptr(col), _lib._ptr(val)
        c.mem = 0
        self._coords = None
        if coords is not None:
            self._coords = np.ascontiguousarray(coords, dtype=np.float64)
            c.coord_dim = self._coords.shape[1]
            c.coords = _lib._ptr(self._coords)
        if grid is not None:
            c.grid_dim = len(grid)
            for i, g in enumerate(grid):
                c.grid[i] = int(g)
        o = build_options(**opts)
        h = ctypes.c_void_p()
        check(lib().mmd_build(ctypes.byref(c), ctypes.byref(o), _lib._stream(stream), ctypes.byref(h)))
        self.h = h
        self._L = lib()
        self.n = n
        self.nnz = int(rowptr[-1])
        _LIVE.add(self)

    @classmethod
    def from_problem(cls, p, **opts):
        return cls(p.rowptr, p.col, p.val, coords=None if p.grid else p.coords, grid=p.grid, **opts)

    def close(self):
        """Release the handle and its device memory now (mmd_free); idempotent."""
        h = getattr(self, "h", None)
        L = getattr(self, "_L", None)
        if h is not None and h.value and L is not None:
            L.mmd_free(h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        self.close()

    def info(self):
        K = ctypes.c_int32()
        sizes = np.zeros(_lib.MMD_MAX_LEVELS, np.int64)
        nnzA = np.zeros_like(sizes)
        nnzM = np.zeros_like(sizes)
        eps = np.zeros(_lib.MMD_MAX_LEVELS)
        check(lib().mmd_info(self.h, ctypes.byref(K), _lib._ptr(sizes), _lib._ptr(nnzA),
                             _lib._ptr(nnzM), _lib._ptr(eps)))
        k = K.value
        return {"K": k, "sizes": sizes[:k + 1].tolist(), "nnzA": nnzA[:k + 1].tolist(),
                "nnzM": nnzM[:k + 1].tolist(), "eps": eps[:k + 1].tolist()}

    def export(self, level, which):
        """Host CSR (rowptr, col, val, shape) of A^(k) (0), M^(k) (1) or Psi^(k) (2)."""
        nr, nc, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().mmd_export(self.h, level, which, ctypes.byref(nr), ctypes.byref(nc),
                               ctypes.byref(nz), None, None, None))
        rp = np.zeros(nr.value + 1, np.int64)
        ci = np.zeros(nz.value, np.int32)
        v = np.zeros(nz.value)
        check(lib().mmd_export(self.h, level, which, None, None, None, _lib._ptr(rp),
                               _lib._ptr(ci), _lib._ptr(v)))
        return rp, ci, v, (nr.value, nc.value)

    def apply(self, level, op, X, stream=None):
        """Y = op X for a row-major [rows, b] float64 CUDA tensor X (returns a new tensor)."""
        import torch
        X = X.contiguous()
        b = X.shape[1] if X.dim() == 2 else 1
        out_rows = self._out_rows(level, OPS[op])
        Y = torch.empty((out_rows, b), dtype=torch.float64, device=X.device)
        check(lib().mmd_apply(self.h, level, OPS[op], _lib._ptr(X), _lib._ptr(Y), b,
                              _lib._stream(stream)))
        return Y

    def _out_rows(self, level, op):
        s = self.info()["sizes"]
        if op in (0, 1, 3, 5, 6):
            return s[level]
        return s[level] - s[level + 1]  # B and U^T map into the reduced space

    def solve(self, level, kind, rhs, x0=None, tol=1e-10, stream=None):
        """Column-wise PCG on A^(k) (kind 0), CG on B^(k+1) (kind 1) or the level-0
        solve by FP32 CG inside FP64 iterative refinement (kind 2); returns (X, iters)."""
        import torch
        rhs = rhs.contiguous()
        b = rhs.shape[1]
        X = torch.zeros_like(rhs) if x0 is None else x0.clone().contiguous()
        it = np.zeros(b, np.int32)
        check(lib().mmd_solve(self.h, level, kind, _lib._ptr(rhs), _lib._ptr(X), b,
                              0 if x0 is None else 1, tol, _lib._ptr(it), _lib._stream(stream)))
        return X, it

    def eig_leftmost(self, nev, tol=1e-10, stream=None, **opts):
        """(evals ascending numpy [nev], evecs CUDA tensor [nev, n], stats dict)."""
        import torch
        evals = np.zeros(nev)
        evecs = torch.empty((nev, self.n), dtype=torch.float64, device="cuda")
        st = eig_stats()
        o = solver_options(**opts)
        check(lib().eig_leftmost(self.h, nev, tol, ctypes.byref(o), _lib._ptr(evals),
                                 _lib._ptr(evecs), ctypes.byref(st), _lib._stream(stream)))
        return evals, evecs, st.as_dict()


    def eig_backward(self, evals, evecs, g_evals=None, g_evecs=None, tol=1e-10, stream=None):
        """Gradient per stored entry of A (CUDA float64 [nnz], the CSR order given
        to the constructor) of a loss with adjoints g_evals ([nev], host or
        device) and g_evecs ([nev, n] CUDA, row k = adjoint of eigenvector k)."""
        import torch
        evals = np.ascontiguousarray(np.asarray(
            evals.detach().cpu() if hasattr(evals, "detach") else evals, dtype=np.float64))
        nev = evals.size
        evecs = evecs.detach().contiguous()
        gl = None
        if g_evals is not None:
            gl = np.ascontiguousarray(np.asarray(
                g_evals.detach().cpu() if hasattr(g_evals, "detach") else g_evals,
                dtype=np.float64))
        gv = None if g_evecs is None else g_evecs.detach().to(torch.float64).contiguous()
        out = torch.empty(self.nnz, dtype=torch.float64, device=evecs.device)
        check(lib().eig_backward(self.h, nev, _lib._ptr(evals), _lib._ptr(evecs),
                                 None if gl is None else _lib._ptr(gl),
                                 None if gv is None else _lib._ptr(gv), tol, _lib._ptr(out),
                                 _lib._stream(stream)))
        return out


def eig_leftmost_batched(decs, nevs, tol=1e-10, stream=None, **opts):
    """eig_leftmost for many decompositions at once (opts["streams"] in flight).
    Returns a list of (evals, evecs, stats) in the order of decs."""
    import torch
    B = len(decs)
    nev = np.ascontiguousarray(nevs, dtype=np.int32)
    if nev.shape != (B,):
        raise ValueError("one nev per decomposition")
    evals = [np.zeros(int(k)) for k in nev]
    evecs = [torch.empty((int(k), d.n), dtype=torch.float64, device="cuda")
             for k, d in zip(nev, decs)]
    hs = (ctypes.c_void_p * B)(*[d.h.value for d in decs])
    ev_p = (ctypes.c_void_p * B)(*[_lib._ptr(e) for e in evals])
    vec_p = (ctypes.c_void_p * B)(*[_lib._ptr(v) for v in evecs])
    st = (eig_stats * B)()
    o = solver_options(**opts)
    check(lib().eig_leftmost_batched(B, hs, _lib._ptr(nev), tol, ctypes.byref(o), ev_p, vec_p,
                                     st, _lib._stream(stream)))
    return [(evals[b], evecs[b], st[b].as_dict()) for b in range(B)]


class EigLeftmost:
    """torch.autograd.Function over the stored values of a symmetric CSR matrix.

    ``evals, evecs = EigLeftmost.apply(values, rowptr, col, nev, tol, build)``
    builds the decomposition of A(values) (``build``: dict of
    Decomposition options, optionally ``coords`` / ``grid``), returns the nev
    smallest eigenvalues (CUDA float64 [nev]) and eigenvectors ([nev, n]), and
    in the backward pass returns dL/dvalues from eig_backward: the gradient for
    symmetric perturbations, so values built symmetrically from parameters (for
    example edge weights scattered into a Laplacian) receive the exact chain rule.
    """

    @staticmethod
    def _function():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, values, rowptr, col, nev, tol, build):
                b = dict(build or {})
                coords, grid = b.pop("coords", None), b.pop("grid", None)
                dec = Decomposition(np.asarray(rowptr), np.asarray(col),
                                    values.detach().cpu().numpy(), coords=coords, grid=grid,
                                    **b)
                lam, V, _ = dec.eig_leftmost(nev, tol=tol)
                lam_t = torch.from_numpy(lam).to(V.device)
                ctx.dec, ctx.tol = dec, tol
                ctx.save_for_backward(lam_t, V)
                ctx.dev = values.device
                return lam_t, V

            @staticmethod
            def backward(ctx, g_lam, g_V):
                lam_t, V = ctx.saved_tensors
                g = ctx.dec.eig_backward(lam_t.cpu().numpy(), V,
                                         None if g_lam is None else g_lam.detach().cpu().numpy(),
                                         g_V, tol=ctx.tol)
                return g.to(ctx.dev), None, None, None, None, None

        return _F

    @classmethod
    def apply(cls, values, rowptr, col, nev, tol=1e-10, build=None):
        if not hasattr(cls, "_F"):
            cls._F = cls._function()
        return cls._F.apply(values, rowptr, col, nev, tol, build)


def spmm(rowptr, col, val, X, n_cols=None, stream=None):
    """Y = A X for a CUDA CSR (int64 rowptr, int32 col, float64 val) and row-major X."""
    import torch
    n_rows = rowptr.numel() - 1
    n_cols = X.shape[0] if n_cols is None else n_cols
    X = X.contiguous()
    b = X.shape[1]
    Y = torch.empty((n_rows, b), dtype=torch.float64, device=X.device)
    check(lib().mmdk_spmm(n_rows, n_cols, _lib._ptr(rowptr), _lib._ptr(col), _lib._ptr(val),
                          _lib._ptr(X), _lib._ptr(Y), b, _lib._stream(stream)))
    return Y


def spmm_noalloc(rowptr, col, val, X, Y, n_cols=None, stream=None):
    """Y = A X through mmdk_spmm_noalloc: the caller provides Y (CUDA float64
    [n_rows, b]); the library allocates nothing (its row-pointer staging is a
    fixed device array, at most 4194304 rows).  Returns Y."""
    n_rows = rowptr.numel() - 1
    n_cols = X.shape[0] if n_cols is None else n_cols
    b = X.shape[1]
    check(lib().mmdk_spmm_noalloc(n_rows, n_cols, _lib._ptr(rowptr), _lib._ptr(col),
                                  _lib._ptr(val), _lib._ptr(X), _lib._ptr(Y), b,
                                  _lib._stream(stream)))
    return Y


def gram(X, Y, stream=None):
    """C = X^T Y for row-major CUDA float64 X [n, m] and Y [n, p] (FP64 MFMA)."""
    import torch
    X, Y = X.contiguous(), Y.contiguous()
    n, m = X.shape
    p = Y.shape[1]
    C = torch.empty((m, p), dtype=torch.float64, device=X.device)
    check(lib().mmdk_gram(n, m, p, _lib._ptr(X), m, _lib._ptr(Y), p, _lib._ptr(C), p,
                          _lib._stream(stream)))
    return C


def gemm(X, C, Z=None, alpha=1.0, beta=0.0, stream=None):
    """Z = alpha X C + beta Z for row-major CUDA float64 X [n, m], C [m, p]
    (FP64 MFMA); Z is created when not given (then beta must be 0)."""
    import torch
    X, C = X.contiguous(), C.contiguous()
    n, m = X.shape
    p = C.shape[1]
    if Z is None:
        Z = torch.empty((n, p), dtype=torch.float64, device=X.device)
    check(lib().mmdk_gemm(n, m, p, alpha, _lib._ptr(X), m, _lib._ptr(C), p, beta, _lib._ptr(Z),
                          p, _lib._stream(stream)))
    return Z
