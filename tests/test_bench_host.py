"""Host-side parts of bench.py (no GPU): the one-GPU guard and the lookup of the
committed HBM counters, which must refuse figures taken on another kernel source or in
another sample layout."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        data = json.load(f)
    with open(bench.KERNEL_SRC, "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == data["kernel_source_sha256"]
    kernels = data["kernels"]
    layout = data.get("sample_layout", "grid")
    other_layout = "grid" if layout == "rows" else "rows"
    assert set(kernels) >= {"forward_fp32_mk", "adjoint_fp32_mk"}
    for name, entry in kernels.items():
        want = entry["fetch_bytes"] + entry["write_bytes"]
        # measured bytes sit near the algorithmic ones (within 30%): a summary of some
        # other workload would not
        assert 0.7 < want / 16318254696 < 1.3, name
        # taken on this kernel source: reported; else (kernels changed since): null
        assert bench.traffic_for(name, layout) == (pytest.approx(want) if current else None)
        # figures of one layout never stand for the other
        assert bench.traffic_for(name, other_layout) is None
    assert bench.traffic_for("no_such_kernel", layout) is None
    # the same summary against a different kernel source gives no figure at all
    other = tmp_path / "kernels.hip"
    other.write_text("// another kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(other))
    assert bench.traffic_for("forward_fp32_mk", layout) is None


def test_product_work_counts():
    """The multiply-adds per row the bench assigns to the blocked products, counted by
    hand for p = 3 and blocks of 4 x 4 x 16 rows on banded rows: the last direction over
    10 x 10 window pairs (100 pairs x 64 points x 4 entries over 256 rows = 100 per table),
    the second over 10 first-direction columns (4 nodes x 10 x 4 entries x 4 / 4 = 160 per
    table), the first direction (64 points x 4 = 256 per term) and the samples (64 per term)."""
    import bench
    assert bench.product_macs(3, 4, "M") == 100 + 160 + 256 + 64
    assert bench.product_macs(3, 4, "K") == 2 * 100 + 3 * 160 + 3 * (256 + 64)
    # p = 2: 8 x 8 pairs, 3 nodes per direction
    assert bench.product_macs(2, 4, "M") == 64 * 3 * 3 / 16 + 3 * 8 * 3 * 3 / 4 + 27 * 3 + 27
