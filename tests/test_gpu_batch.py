"""eig_leftmost_batched through the C ABI: every problem of a mixed batch
against the dense definition (oracle/dense.py) and against its own
eig_leftmost run; error reporting of a bad member."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import torch
    assert torch.cuda.is_available()
    from paper_1804_03415_amd import Decomposition
    probs = [
        (wl.rgg(2500, 3, mean_degree=8), 20, dict(levels=2)),
        (wl.rgg(900, 4, mean_degree=8), 12, dict(levels=2)),
        (wl.knn_gmm(800, 10, 2), 10, dict(levels=2)),
        (wl.grid2d(20), 15, dict(levels=2, exact_max_n=4096)),
        (wl.rgg(1600, 5, mean_degree=8), 16, dict(levels=2)),
        (wl.knn_gmm(1200, 10, 3), 8, dict(levels=2)),
    ]
    decs = [Decomposition.from_problem(p, **kw) for p, _, kw in probs]
    return probs, decs


@pytest.mark.parametrize("streams", [1, 4])
def test_batched_matches_dense_and_single(batch, streams):
    from paper_1804_03415_amd import eig_leftmost_batched
    probs, decs = batch
    tol = 1e-11
    out = eig_leftmost_batched(decs, [nev for _, nev, _ in probs], tol=tol, streams=streams)
    for (p, nev, kw), dec, (lam, V, st) in zip(probs, decs, out):
        A = p.scipy()
        w, Z = dense.smallest_dense(A, nev)
        Vh = V.cpu().numpy().T
        null = np.abs(w - 1e-6) < 1e-12
        assert np.sum(np.abs(lam - 1e-6) < 1e-12) == np.sum(null)
        assert np.max(np.abs(lam[~null] - w[~null]) / w[~null]) < 1e-10
        ang, cl = dense.cluster_angles(w, Z, Vh)
        full = [i for i, c in enumerate(cl) if c[-1] < nev - 1]
        assert ang[full].max() < 1e-8
        assert dense.rel_residuals(A, lam, Vh).max() < 1e-8
        assert st["nconv"] == nev
        l1, V1, _ = dec.eig_leftmost(nev, tol=tol)
        assert np.max(np.abs(lam - l1) / l1) < 1e-10


def test_batched_reports_bad_member(batch):
    from paper_1804_03415_amd import MMDError, eig_leftmost_batched
    probs, decs = batch
    nevs = [nev for _, nev, _ in probs]
    nevs[2] = 0
    with pytest.raises(MMDError) as e:
        eig_leftmost_batched(decs, nevs, tol=1e-10, streams=3)
    assert "problem 2" in str(e.value)
    with pytest.raises(MMDError):
        eig_leftmost_batched([decs[0], decs[0]], [5, 5], tol=1e-10)


def test_operator_solves_are_merged(batch, capfd, monkeypatch):
    """With several problems in flight, their single-vector operator solves
    share cooperative launches of the batched persistent kernel: fewer
    launches than solves (counts from the MMDEIG_LOG line of the batch)."""
    import re
    from paper_1804_03415_amd import eig_leftmost_batched
    probs, decs = batch
    monkeypatch.setenv("MMDEIG_LOG", "1")
    capfd.readouterr()
    out = eig_leftmost_batched(decs, [nev for _, nev, _ in probs], tol=1e-10, streams=6)
    err = capfd.readouterr().err
    m = re.search(r"batch: (\d+) operator solves in (\d+) batched launches", err)
    assert m, err[-2000:]
    solves, launches = int(m.group(1)), int(m.group(2))
    assert solves > 0 and launches < solves
    for (p, nev, kw), (lam, V, st) in zip(probs, out):
        assert dense.rel_residuals(p.scipy(), lam, V.cpu().numpy().T).max() < 1e-8
