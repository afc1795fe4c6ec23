"""Host side of the benchmark's contract, no GPU: more than one GPU is refused
with a message, and the counter traffic of the committed rocprofv3 summaries
is used only while they were taken on the current kernel sources (and on the
workload and size asked for); otherwise the line reports null."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2304_10078_amd.profiling import source_digest  # noqa: E402


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    kd = tmp_path / "profiles" / "traffic_k_distribute_zipf1.2_hashed_n1000.json"
    ps = tmp_path / "profiles" / "traffic_passes_semisort_equal_zipf1.2_hashed_n1000.json"
    rec = {"workload": "zipf1.2_hashed", "n": 1000, "source_digest": source_digest(), "bytes_per_launch": 123.0}
    passes = dict(rec, passes={"distribute": {"fetch_bytes": 1.0, "write_bytes": 2.0}})
    kd.write_text(json.dumps(rec))
    ps.write_text(json.dumps(passes))
    assert bench.load_traffic("zipf1.2_hashed", 1000) == 123.0
    assert bench.load_pass_traffic("semisort_=", "zipf1.2_hashed", 1000) == passes["passes"]
    # another size or workload than the summary's
    assert bench.load_traffic("zipf1.2_hashed", 2000) is None
    assert bench.load_traffic("uniform1e9", 1000) is None
    # kernels changed since the counters were taken
    kd.write_text(json.dumps(dict(rec, source_digest="0" * 16)))
    ps.write_text(json.dumps(dict(passes, source_digest="0" * 16)))
    assert bench.load_traffic("zipf1.2_hashed", 1000) is None
    assert bench.load_pass_traffic("semisort_=", "zipf1.2_hashed", 1000) is None
    # unreadable summary
    kd.write_text("{")
    assert bench.load_traffic("zipf1.2_hashed", 1000) is None


def test_committed_headline_summary_matches_the_sources():
    """The committed summary behind the headline's `traffic` was taken on the
    kernel sources in the tree, so the benchmark reports it (not null)."""
    assert bench.load_traffic("zipf1.2_hashed", 10 ** 9) is not None
