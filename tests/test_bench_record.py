"""Host-side checks of the benchmark's roofline bookkeeping (no GPU): the HBM
traffic of a kernel is taken from the committed counter record only while
every source the record was taken from is unchanged, and the committed record
(once present) names the kernels bench.py reports."""
import hashlib
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record(tmp_path, src_text):
    src = tmp_path / "k.hip"
    src.write_text(src_text)
    rec = {"kernels": {"bt::k<double>": {
        "traffic_bytes_per_launch": 123.0,
        "sources_sha256": {"k.hip": hashlib.sha256(src_text.encode()).hexdigest()}}}}
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    return str(path)


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    rec = _record(tmp_path, "// kernel\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "PMC_RECORD", rec)
    assert bench.measured_traffic("bt::k<double>") == 123.0
    assert bench.measured_traffic("bt::other<double>") is None
    (tmp_path / "k.hip").write_text("// kernel, edited\n")
    assert bench.measured_traffic("bt::k<double>") is None
    monkeypatch.setattr(bench, "PMC_RECORD", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("bt::k<double>") is None


def test_committed_record_covers_the_reported_kernels():
    path = os.path.join(ROOT, "profiles", "counters_pmc.json")
    if not os.path.exists(path):
        return
    rec = json.load(open(path))
    assert "bt::uapply3d_kernel<double>" in rec["kernels"]
    for key, k in rec["kernels"].items():
        assert k["traffic_bytes_per_launch"] > 0, key
        assert k["sources_sha256"], key
        for rel in k["sources_sha256"]:
            assert os.path.exists(os.path.join(ROOT, rel)), (key, rel)
