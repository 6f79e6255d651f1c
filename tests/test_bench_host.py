"""Host-side contract of bench.py (no GPU): the one-GPU refusal and the rule
that a committed HBM counter record is used only while the kernel sources it
was taken from are unchanged (otherwise the bench line's traffic is null)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports no torch and touches no GPU at import)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def _record(tmp_path, sources, sha, traffic=1.5e10):
    p = tmp_path / "rec.json"
    p.write_text(json.dumps({"sources": sources, "sources_sha256": sha, "traffic_bytes": traffic}))
    return str(p)


def test_traffic_record_follows_its_sources(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel v1\n")
    files = [str(src)]
    rec = _record(tmp_path, files, bench.sources_sha256(tuple(files)))
    assert bench.measured_traffic(rec) == 1.5e10
    # any edit of a listed source voids the record
    src.write_text("kernel v2\n")
    assert bench.measured_traffic(rec) is None


def test_traffic_record_rejects_bad_records(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel\n")
    files = [str(src)]
    sha = bench.sources_sha256(tuple(files))
    wrong = ("0" if sha[0] != "0" else "1") + sha[1:]
    assert bench.measured_traffic(_record(tmp_path, files, wrong)) is None
    assert bench.measured_traffic(_record(tmp_path, [], sha)) is None  # no sources listed
    assert bench.measured_traffic(_record(tmp_path, [str(tmp_path / "missing.hip")], sha)) is None
    assert bench.measured_traffic(str(tmp_path / "no_record.json")) is None


def test_committed_record_is_consistent():
    """The committed deposit record names its sources and, while they are
    unchanged, gives a traffic figure of the deposit's size (28.5 GB per
    launch on the 537M-particle workload, above the 19.6 GB algorithmic)."""
    path = os.path.join(ROOT, "profiles", "c5_deposit_traffic.json")
    rec = json.load(open(path))
    assert rec["sources"] and all(os.path.exists(os.path.join(ROOT, f)) for f in rec["sources"])
    t = bench.measured_traffic(os.path.join("profiles", "c5_deposit_traffic.json"))
    if t is not None:
        assert t == float(rec["traffic_bytes"])
        assert 19.6e9 < t < 60e9
