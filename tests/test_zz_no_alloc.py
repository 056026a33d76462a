"""The allocation-free SpMM entry point (mmdk_spmm_noalloc) against the
allocating one (mmdk_spmm), through the C ABI: identical launches, so the
results agree bit for bit; two calls in a row, the second on a smaller input
(the shared scratch keeps the previous call's contents), and the size limit."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_matches_allocating_spmm_twice():
    import torch
    from paper_1804_03415_amd import spmm, spmm_noalloc
    assert torch.cuda.is_available()
    for nr, nc, per, b in ((30000, 25000, (2, 40), 70), (700, 900, (0, 12), 3)):
        rp, ci, v = wl.random_csr(nr, nc, per, seed=nr, empty_frac=0.1)
        X = wl.random_block(nc, b, seed=b)
        args = (_t(torch, rp), _t(torch, ci), _t(torch, v), _t(torch, X))
        ref = spmm(*args, n_cols=nc).cpu().numpy()
        Y = torch.full((nr, b), np.nan, dtype=torch.float64, device="cuda")
        out = spmm_noalloc(*args, Y, n_cols=nc).cpu().numpy()
        assert np.array_equal(out, ref)


def test_noalloc_rejects_oversize_before_device_work():
    import torch
    from paper_1804_03415_amd import MMDError, spmm_noalloc
    rp = torch.zeros(4194304 + 2, dtype=torch.int64, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = torch.zeros(1, dtype=torch.float64, device="cuda")
    X = torch.zeros((4, 1), dtype=torch.float64, device="cuda")
    Y = torch.zeros((4194304 + 1, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(MMDError) as e:
        spmm_noalloc(rp, ci, v, X, Y, n_cols=4)
    assert e.value.code == 1 and "scratch capacity" in str(e.value)
