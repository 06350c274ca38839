"""bench.py reports a kernel's HBM traffic from profiles/traffic.json only
while the record matches the kernel source, the shipped tuning table (which
fixes the block order) and the tile shape it was measured with."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

WORKLOAD = "batch64_480x640_f32depth_sobel_median"


def _records(tmp_path, entry):
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({WORKLOAD: entry}))
    return str(p)


def test_traffic_record_needs_kernel_table_and_tile(tmp_path, monkeypatch):
    good = {"bytes_per_launch": 123456789, "tile": "4,4,32",
            "kernel_sha": bench.kernel_hash(), "table_sha": bench.table_hash()}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _records(tmp_path, good))
    assert bench.measured_traffic(WORKLOAD, (4, 4, 32)) == 123456789
    assert bench.measured_traffic(WORKLOAD, (4, 8, 32)) is None      # another tile
    assert bench.measured_traffic(WORKLOAD, None) is None
    assert bench.measured_traffic("no_such_workload", (4, 4, 32)) is None
    for key in ("kernel_sha", "table_sha"):
        stale = dict(good, **{key: "0" * 16})
        monkeypatch.setattr(bench, "TRAFFIC_FILE", _records(tmp_path, stale))
        assert bench.measured_traffic(WORKLOAD, (4, 4, 32)) is None, key
    # a record written before the table hash was kept is not trusted either
    old = {k: v for k, v in good.items() if k != "table_sha"}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _records(tmp_path, old))
    assert bench.measured_traffic(WORKLOAD, (4, 4, 32)) is None


def test_table_hash_follows_the_table(tmp_path, monkeypatch):
    t = tmp_path / "tuning.txt"
    t.write_text(open(bench.TUNING_FILE).read())
    monkeypatch.setattr(bench, "TUNING_FILE", str(t))
    h0 = bench.table_hash()
    t.write_text(open(bench.TUNING_FILE).read().replace(" 16 1\n", " 0 1\n", 1))
    assert bench.table_hash() != h0


def test_kernel_hash_ignores_comments_and_spacing(tmp_path, monkeypatch):
    src = open(bench.KERNEL_SRC).read()
    k = tmp_path / "k.hip"
    k.write_text(src)
    monkeypatch.setattr(bench, "KERNEL_SRC", str(k))
    h0 = bench.kernel_hash()
    k.write_text("// a new comment\n" + src.replace("\n", "\n\n", 3))
    assert bench.kernel_hash() == h0
    k.write_text(src.replace("kWideRun = 16", "kWideRun = 8", 1))
    assert bench.kernel_hash() != h0
