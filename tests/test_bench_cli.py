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
    for opt in ("--serve-mix", "--autotune-sample", "--serve-rates", "--workload"):
        assert opt in p.stdout
