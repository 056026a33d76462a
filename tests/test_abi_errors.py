"""Error paths of the C ABI that are decided on the host before any device
work (mmd_build input validation, Section 2.1 energy decomposition): each
call returns its status code and leaves a message in mmd_last_error().  No
GPU is needed: the library rejects the input before touching the device."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1804_03415_amd import Decomposition, MMDError
from paper_1804_03415_amd._lib import lib

import workloads as wl


def _csr(dense):
    A = sp.csr_matrix(np.asarray(dense, dtype=float))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)


def _build(rp, ci, v, **kw):
    return Decomposition(rp, ci, v, levels=1, targets=(2,), **kw)


def _code(excinfo):
    return excinfo.value.code


def test_positive_offdiagonal_is_unsupported():
    # a_01 > 0: no edge-type energy element w_01 = -a_01 >= 0
    rp, ci, v = _csr([[2.0, 0.5, 0.0], [0.5, 2.0, -1.0], [0.0, -1.0, 2.0]])
    with pytest.raises(MMDError) as e:
        _build(rp, ci, v)
    assert _code(e) == 3  # MMD_EUNSUPPORTED
    assert b"off-diagonal" in lib().mmd_last_error() or b"positive" in lib().mmd_last_error()


def test_negative_self_loop_is_unsupported():
    # row sum < 0: the self-loop element s_0 = a_00 - sum_j w_0j is negative
    rp, ci, v = _csr([[1.0, -2.0], [-2.0, 3.0]])
    with pytest.raises(MMDError) as e:
        _build(rp, ci, v)
    assert _code(e) == 3


def test_nonpositive_diagonal_is_not_spd():
    rp, ci, v = _csr([[0.0, 0.0], [0.0, 1.0]])
    # the explicit zero must be stored for the diagonal check
    rp = np.array([0, 1, 2], np.int64)
    ci = np.array([0, 1], np.int32)
    v = np.array([0.0, 1.0])
    with pytest.raises(MMDError) as e:
        _build(rp, ci, v)
    assert _code(e) == 2  # MMD_ENOTSPD


@pytest.mark.parametrize("case", ["asymmetric_values", "asymmetric_pattern", "unsorted",
                                  "nan", "rowptr", "column_range"])
def test_malformed_input_is_invalid(case):
    p = wl.grid2d(4)
    rp, ci, v = p.rowptr.copy(), p.col.copy(), p.val.copy()
    if case == "asymmetric_values":
        v[1] = v[1] * 1.5
    elif case == "asymmetric_pattern":
        # drop one stored off-diagonal entry of row 0
        keep = np.ones(ci.size, bool)
        keep[1] = False
        ci, v = ci[keep], v[keep]
        rp = rp.copy()
        rp[1:] -= 1
    elif case == "unsorted":
        ci[0], ci[1] = ci[1], ci[0]
        v[0], v[1] = v[1], v[0]
    elif case == "nan":
        v[0] = np.nan
    elif case == "rowptr":
        rp = rp.copy()
        rp[-1] += 1
    elif case == "column_range":
        ci = ci.copy()
        ci[-1] = p.n
    with pytest.raises(MMDError) as e:
        Decomposition(rp, ci, v, levels=1)
    assert _code(e) == 1  # MMD_EINVAL
    assert len(lib().mmd_last_error()) > 0


def test_bad_build_options_are_invalid():
    p = wl.grid2d(4)
    with pytest.raises(MMDError) as e:
        Decomposition(p.rowptr, p.col, p.val, levels=1, targets=(1,))
    assert _code(e) == 1
    with pytest.raises(MMDError) as e:
        Decomposition(p.rowptr, p.col, p.val, grid=(5, 4), levels=1)
    assert _code(e) == 1
