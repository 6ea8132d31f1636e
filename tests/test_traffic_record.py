"""bench.py reports roofline.traffic only from a counter record taken on the
current stencil and solver sources: the record lapses when any of them
changes or when its file list is not the current one, and it applies only to
the workload it was taken on."""
import json
import os
import shutil

import pytest

import bench
from paper_1010_2592_amd import rocprof_summary as rs

KEY = "16x16x16x32 12 rhs fp64 pass 3"


@pytest.fixture
def record(tmp_path, monkeypatch):
    root = tmp_path / "repo"
    for p in rs.STENCIL_SOURCES:
        (root / os.path.dirname(p)).mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(rs.ROOT, p), root / p)
    (root / "profiles").mkdir()
    monkeypatch.setattr(rs, "ROOT", str(root))
    monkeypatch.setattr(bench, "ROOT", str(root))
    rec = {"sources": list(rs.STENCIL_SOURCES), "sources_sha256_16": rs.sources_hash(), "workload": KEY,
           "traffic_bytes_per_launch": 123}
    path = root / "profiles" / "dslash_traffic.json"
    path.write_text(json.dumps(rec))
    return root, path, rec


def test_record_applies_to_its_sources_and_workload(record):
    assert bench.measured_traffic(KEY) == 123
    assert bench.measured_traffic("another workload") is None


@pytest.mark.parametrize("which", range(len(rs.STENCIL_SOURCES)))
def test_record_lapses_when_a_source_changes(record, which):
    root, path, rec = record
    with open(root / rs.STENCIL_SOURCES[which], "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic(KEY) is None


def test_record_lapses_with_an_old_file_list(record):
    root, path, rec = record
    old = dict(rec, sources=rec["sources"][:2])
    old["sources_sha256_16"] = rs.sources_hash(old["sources"])
    path.write_text(json.dumps(old))
    assert bench.measured_traffic(KEY) is None


def test_missing_or_broken_record(record):
    root, path, rec = record
    path.write_text("{not json")
    assert bench.measured_traffic(KEY) is None
    path.unlink()
    assert bench.measured_traffic(KEY) is None
