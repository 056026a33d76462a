"""ctypes binding of libmmdeig.so (argument marshalling only).

Every numerical step runs inside the library's HIP kernels and host C++
driver; this module converts numpy / torch arguments into the pointers and
sizes of the C ABI declared in include/mmdeig.h.  It raises if the compiled
library is missing: there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmdeig.so")

MMD_MAX_LEVELS = 16
STATUS = {0: "MMD_OK", 1: "MMD_EINVAL", 2: "MMD_ENOTSPD", 3: "MMD_EUNSUPPORTED",
          4: "MMD_ENOCONV", 5: "MMD_ENOMEM", 6: "MMD_EHIP"}


class MMDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class mmd_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("mem", ctypes.c_int32), ("coord_dim", ctypes.c_int32),
                ("coords", ctypes.c_void_p), ("grid_dim", ctypes.c_int32),
                ("grid", ctypes.c_int32 * 3)]


class mmd_build_opts(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("n_targets", ctypes.c_int32),
                ("targets", ctypes.c_int32 * 8), ("n_grid_blocks", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32 * 8), ("r_hops", ctypes.c_int32),
                ("exact_max_n", ctypes.c_int64), ("min_coarse", ctypes.c_int32),
                ("max_patch", ctypes.c_int32), ("eps1", ctypes.c_double),
                ("eta", ctypes.c_double), ("cbound", ctypes.c_double),
                ("r_hops_coarse", ctypes.c_int32)]


class eig_opts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("restart_mult", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("max_restarts", ctypes.c_int32),
                ("max_refine", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("stop_level", ctypes.c_int32),
                ("d", ctypes.c_int32)]


_L = MMD_MAX_LEVELS


class eig_stats(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("nconv", ctypes.c_int32),
                ("ref_in", ctypes.c_int64 * _L), ("ref_out", ctypes.c_int64 * _L),
                ("ref_iter", ctypes.c_int64 * _L), ("cg_B_calls", ctypes.c_int64 * _L),
                ("cg_B_iters", ctypes.c_int64 * _L), ("pcg_A_calls", ctypes.c_int64 * _L),
                ("pcg_A_iters", ctypes.c_int64 * _L), ("cg_M_iters", ctypes.c_int64 * _L),
                ("ext_in", ctypes.c_int64 * _L), ("ext_out", ctypes.c_int64 * _L),
                ("lanczos_steps", ctypes.c_int64 * _L), ("restarts", ctypes.c_int64 * _L),
                ("missed_swaps", ctypes.c_int64), ("seconds_level", ctypes.c_double * _L),
                ("seconds_total", ctypes.c_double), ("seconds_phase", ctypes.c_double * 8),
                ("spmm0_launches", ctypes.c_int64), ("spmm0_ms", ctypes.c_double),
                ("spmm0_bytes", ctypes.c_double), ("spmm0_b", ctypes.c_int32),
                ("mixed_fallbacks", ctypes.c_int32)]

    PHASES = ("refine_pcg", "refine_bcg", "refine_host_dense", "refine_qr_gram", "extend_op",
              "extend_orth", "restart", "output")

    def as_dict(self):
        K = self.K
        out = {"K": K, "nconv": self.nconv, "missed_swaps": self.missed_swaps,
               "mixed_fallbacks": self.mixed_fallbacks,
               "seconds_total": self.seconds_total, "levels": {},
               "phases": {n: round(self.seconds_phase[i], 4) for i, n in enumerate(self.PHASES)},
               "spmm0": {"launches": self.spmm0_launches, "ms": self.spmm0_ms,
                         "bytes": self.spmm0_bytes, "b": self.spmm0_b}}
        for k in range(K + 1):
            out["levels"][k] = {f: getattr(self, f)[k] for f in (
                "ref_in", "ref_out", "ref_iter", "cg_B_calls", "cg_B_iters", "pcg_A_calls",
                "pcg_A_iters", "cg_M_iters", "ext_in", "ext_out", "lanczos_steps", "restarts",
                "seconds_level")}
        return out


_lib = None


def lib():
    """Load libmmdeig.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmmdeig.so is not built (run __graft_entry__.build() or "
                          "python paper_1804_03415_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.mmd_build.argtypes = [ctypes.POINTER(mmd_csr), ctypes.POINTER(mmd_build_opts), vp,
                            ctypes.POINTER(vp)]
    L.mmd_info.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mmd_export.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    L.eig_leftmost.argtypes = [vp, i32, dbl, ctypes.POINTER(eig_opts), vp, vp,
                               ctypes.POINTER(eig_stats), vp]
    L.mmd_apply.argtypes = [vp, i32, i32, vp, vp, i32, vp]
    L.mmd_solve.argtypes = [vp, i32, i32, vp, vp, i32, i32, dbl, vp, vp]
    L.mmdk_spmm.argtypes = [i64, i64, vp, vp, vp, vp, vp, i32, vp]
    L.mmdk_spmm_noalloc.argtypes = [i64, i64, vp, vp, vp, vp, vp, i32, vp]
    L.mmdk_gram.argtypes = [i64, i32, i32, vp, i32, vp, i32, vp, i32, vp]
    L.mmdk_gemm.argtypes = [i64, i32, i32, dbl, vp, i32, vp, i32, dbl, vp, i32, vp]
    L.eig_backward.argtypes = [vp, i32, vp, vp, vp, vp, dbl, vp, vp]
    L.eig_leftmost_batched.argtypes = [i32, vp, vp, dbl, ctypes.POINTER(eig_opts), vp, vp, vp,
                                       vp]
    L.mmd_free.argtypes = [vp]
    L.mmd_free.restype = None
    L.mmd_last_error.restype = ctypes.c_char_p
    for f in ("mmd_build", "mmd_info", "mmd_export", "eig_leftmost", "mmd_apply", "mmd_solve",
              "mmdk_spmm", "mmdk_spmm_noalloc", "mmdk_gram", "mmdk_gemm", "eig_backward", "eig_leftmost_batched"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def check(code):
    if code != 0:
        raise MMDError(code, lib().mmd_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    """The HIP stream handle of a torch stream (default: torch's current one).
    Without a visible device this is NULL, the HIP default stream: input
    checks that precede device work still report their status, and the first
    device call fails with MMD_EHIP."""
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return None
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)
