"""Host logic of bench.py: the HBM traffic table lookup (no GPU)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _table(tmp_path, da, dd=None):
    dd = dd or da
    p = tmp_path / "t.md"
    p.write_text("| Workload | Kernel | F | W | Bytes | Sources |\n|---|---|---|---|---|---|\n"
                 f"| c2 | anneal_kernel | 1.0 | 2.0 | 4,096 | `{da}` |\n"
                 f"| c4-dense | dense_step_kernel | 1.0 | 2.0 | 8,192 | `{dd}` |\n")
    return str(p)


def test_digest_is_stable_short_and_per_kernel():
    a, b = bench.source_digest("anneal_kernel"), bench.source_digest("anneal_kernel")
    assert a == b and len(a) == 16 and int(a, 16) >= 0
    digests = {bench.source_digest(k) for k in bench.KERNEL_SOURCES}
    assert len(digests) == len(bench.KERNEL_SOURCES)


def test_traffic_row_matches_only_its_digest(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_TABLE", _table(tmp_path, bench.source_digest("anneal_kernel"),
                                                      bench.source_digest("dense_step_kernel")))
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


def test_issue_row_matches_only_its_digest(tmp_path, monkeypatch):
    p = tmp_path / "i.md"
    d = bench.source_digest("anneal_kernel")
    p.write_text("| Workload | Kernel | I | W | Per update | Busy | Sources |\n|---|---|---|---|---|---|---|\n"
                 f"| c3 | anneal_kernel | 9.0e10 | 4,096 | 56.2 | 0.88 | `{d}` |\n")
    monkeypatch.setattr(bench, "ISSUE_TABLE", str(p))
    assert bench.measured_issue("c3", "anneal_kernel") == (56.2, 0.88)
    assert bench.measured_issue("c2", "anneal_kernel") is None
    p.write_text(p.read_text().replace(d, "0123456789abcdef"))
    assert bench.measured_issue("c3", "anneal_kernel") is None


def test_plan_op_count_reproduces_the_workload_table():
    """The workload table's estimates: 74 lane-operations per update on the
    torus (degree 4, timing on), 76 on the n = 2,000 graph (degree 6)."""
    assert bench.plan_ops_per_update(4.0, True) == 74.0
    assert bench.plan_ops_per_update(6.0, True) == 76.0
    # the gfx950 lower bound of the same updates
    assert bench.ops_per_update(4 * bench.OPS_EDGE_FOUR_TRIALS, True) == 41.25
    assert bench.ops_per_update(6 * bench.OPS_EDGE_ONE_TRIAL, True) == 43.25


def test_default_workload_is_the_torus():
    import argparse
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--workload", default="c3"' in src
