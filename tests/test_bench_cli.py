"""bench.py's command line on the host: one GPU per process, and a refusal
(exit status 2, one JSON line naming the error) for more."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_help_lists_the_serve_options():
    p = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 0
    for opt in ("--serve-mix", "--autotune-sample", "--serve-rates", "--workload",
                "--serve-ceiling", "--plain-slices", "--large"):
        assert opt in p.stdout


def test_roofline_record_flags_cache_served_fractions():
    sys.path.insert(0, str(ROOT))
    import bench
    r = bench.roofline_record(4000.0, None, None)
    assert r["frac"] == 0.5 and "note" not in r and r["traffic_source"] is None
    r = bench.roofline_record(10740.0, 1.2e13, "profiles/x.json")
    assert r["frac"] > 1 and "cache" in r["note"] and r["traffic_source"] == "profiles/x.json"


def test_byte_model_per_algorithm():
    sys.path.insert(0, str(ROOT))
    import bench
    assert bench.byte_model("node2vec", True, False) == dict(scan=8, emit=4)
    assert bench.byte_model("deepwalk", True, False)["scan"] == 4
    assert bench.byte_model("metapath", False, True)["scan"] == 1
    assert bench.byte_model("ppr", True, False)["moving_only"]
