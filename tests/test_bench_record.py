"""Host-side checks of the benchmark's roofline bookkeeping (no GPU): the HBM
traffic of the operator apply is taken from the committed counter record only
while that record was taken from the current apply2d.hip, and the record
covers the kernel name that bench.py builds for every 2D tile variant."""
import json
import os
import shutil

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REC = os.path.join("profiles", "apply2d_2d_128_dg1_pmc.json")
SRC = os.path.join("paper_1801_04984_amd", "csrc", "apply2d.hip")


def _tree(tmp_path, edit_source=False):
    for rel in (REC, SRC):
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    if edit_source:
        with open(tmp_path / SRC, "a") as f:
            f.write("\n// edited\n")
    return str(tmp_path)


def test_record_names_every_fp64_variant():
    rec = json.load(open(os.path.join(ROOT, REC)))
    for ts, lp in ((16, "false"), (8, "false"), (8, "true")):
        key = f"bt::apply2d_kernel<double, 2, false, {ts}, {lp}>"
        assert key in rec["kernels"], key
        assert rec["kernels"][key]["traffic_bytes_per_launch"] > 0


def test_traffic_only_for_matching_source(tmp_path, monkeypatch):
    key = "bt::apply2d_kernel<double, 2, false, 8, true>"
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path / "same"))
    t = bench.measured_traffic(key)
    assert t is not None and t > 0
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path / "edited", edit_source=True))
    assert bench.measured_traffic(key) is None
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path / "same2"))
    assert bench.measured_traffic("bt::apply2d_kernel<double, 2, false, 32, true>") is None
