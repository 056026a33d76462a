"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the
source-hash gate on the committed HBM counters, and the CPU-baseline sample
of the RGG point cloud."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_follows_the_committed_counters(tmp_path, monkeypatch):
    """The traffic figure is reported only while the dominant kernel's source
    text hashes to the value recorded with the counters; edits elsewhere in
    the file leave it valid."""
    import hashlib
    name = "cg_tile_rgg_n1e5_traffic.json"
    path = os.path.join(ROOT, "profiles", name)
    with open(path) as f:
        d = json.load(f)
    start, launcher = d["source_region"]
    fake = tmp_path / "profiles"
    fake.mkdir()
    src = tmp_path / d["source"]
    src.parent.mkdir(parents=True)
    region = start + " (stand-in)\n" + launcher + "int x) {\n  return x;\n}\n"
    body = "// other kernels\n" + region + "// more kernels\n"
    src.write_text(body)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d["source_sha256"] = hashlib.sha256(region.encode()).hexdigest()
    (fake / name).write_text(json.dumps(d))
    want = round(1024.0 * (d["fetch_size_kib_per_launch"] * d["fetch_scale"] +
                           d["write_size_kib_per_launch"] * d["write_scale"]))
    assert bench.measured_traffic() == want and want > 0
    # edits outside the kernel keep the figure
    src.write_text("// a new kernel\n" + body + "// another\n")
    assert bench.measured_traffic() == want
    # a summary taken on other kernel source gives no traffic figure
    src.write_text(body.replace("return x;", "return x + 1;"))
    assert bench.measured_traffic() is None
    # the committed summary matches the kernel source in the tree
    assert bench.kernel_source_sha(os.path.join(ROOT, d["source"]), (start, launcher)) == \
        json.load(open(path))["source_sha256"]
    assert (start, launcher) == bench.CG_TILE_REGION


def test_cpu_sample_is_a_window_of_the_same_cloud():
    p = workloads.rgg(20000, 0)
    q = workloads.rgg_window(p, 0.05)
    # about 5% of the points, same density, all inside the corner square
    assert 0.03 * p.n < q.n < 0.07 * p.n
    side = np.sqrt(0.05)
    assert np.all(q.coords <= side + 1e-12)
    # same mean degree up to the window's boundary loss, same shift
    deg_p = p.nnz / p.n - 1
    deg_q = q.nnz / q.n - 1
    assert 0.8 * deg_p < deg_q <= deg_p * 1.05
    A = q.scipy()
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), 1e-6)
