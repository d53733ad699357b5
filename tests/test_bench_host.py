"""Host logic of bench.py: the HBM traffic table lookup (no GPU)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _table(tmp_path, digest):
    p = tmp_path / "t.md"
    p.write_text("| Workload | Kernel | F | W | Bytes | Sources |\n|---|---|---|---|---|---|\n"
                 f"| c2 | anneal_kernel | 1.0 | 2.0 | 4,096 | `{digest}` |\n"
                 f"| c4-dense | dense_step_kernel | 1.0 | 2.0 | 8,192 | `{digest}` |\n")
    return str(p)


def test_digest_is_stable_and_short():
    a, b = bench.source_digest(), bench.source_digest()
    assert a == b and len(a) == 16 and int(a, 16) >= 0


def test_traffic_row_matches_only_its_digest(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_TABLE", _table(tmp_path, bench.source_digest()))
    assert bench.measured_traffic("c2", "anneal_kernel") == 4096
    assert bench.measured_traffic("c4-dense", "dense_step_kernel") == 8192
    assert bench.measured_traffic("c2", "dense_step_kernel") is None
    assert bench.measured_traffic("c3", "anneal_kernel") is None
    # sources changed since the counters were taken: no traffic figure
    monkeypatch.setattr(bench, "TRAFFIC_TABLE", _table(tmp_path, "0123456789abcdef"))
    assert bench.measured_traffic("c2", "anneal_kernel") is None


def test_missing_table_gives_none(monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_TABLE", os.path.join(ROOT, "no_such_table.md"))
    assert bench.measured_traffic("c2", "anneal_kernel") is None


@pytest.mark.parametrize("w", ["c1", "c2", "c3"])
def test_committed_table_has_the_workloads(w):
    with open(os.path.join(ROOT, "profiles", "hbm_traffic_by_workload.md")) as fh:
        assert f"| {w} | anneal_kernel |" in fh.read()
