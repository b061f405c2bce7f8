"""The committed counter records (profiles/traffic_*.json) are consistent:
bytes = FETCH_SIZE KiB x 1024 x its copy-calibration factor + WRITE_SIZE KiB
x 1024 x its factor, each names a summary that exists and that quotes the
same walker-source hash and raw counter values."""
import json
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
RECORDS = sorted((ROOT / "profiles").glob("traffic_*.json"))


def test_records_exist():
    assert RECORDS


@pytest.mark.parametrize("path", RECORDS, ids=lambda p: p.stem)
def test_record_consistent(path):
    r = json.loads(path.read_text())
    total = r["fetch_kib"] * 1024 * r["fetch_scale"] + r["write_kib"] * 1024 * r["write_scale"]
    assert abs(total - r["hbm_bytes_per_launch"]) <= 1e-9 * total
    assert 1.9 < r["fetch_scale"] < 2.1 and r["write_scale"] == 1.0
    assert len(r["kernel_source"]) == 12 and int(r["kernel_source"], 16) >= 0
    assert path.stem == f"traffic_{r['workload']}_{r['mode']}"
    summary = (ROOT / r["summary"]).read_text()
    assert r["kernel_source"] in summary
    assert f"{r['fetch_kib']:.1f}" in summary and f"{r['write_kib']:.1f}" in summary
