"""bench.py's byte accounting without a GPU: the algorithmic bytes of a pass follow the
per-unit figures (arc 4 B, counter m B, row_ptr 4 B per node, one flag bit read and one
written per node of a pass over every node, two row_ptr entries per node a systolic pass
visits), and measured HBM traffic is reported only for the kernel source it was taken
on."""
import hashlib
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_dense_pass_at_full_size(bench):
    # symmetric R-MAT scale 22, 64 registers: every arc scanned and gathered, every own
    # counter read and every new counter written
    n, e, m = 1 << 22, 1 << 26, 64
    rec = {"arcs_scanned": e, "arcs_gathered": e, "rows_read": n, "rows_written": n}
    want = 4 * (n + 1) + 4 * e + m * e + m * n + m * n + n // 4
    assert bench.algorithmic_bytes(rec, n, m) == want == 5_118_099_460


def test_each_unit_counts_once(bench):
    n, m = 1000, 128
    base = {"arcs_scanned": 10, "arcs_gathered": 7, "rows_read": 5, "rows_written": 3}
    b0 = bench.algorithmic_bytes(base, n, m)
    for key, per_unit in [("arcs_scanned", 4), ("arcs_gathered", m), ("rows_read", m), ("rows_written", m)]:
        rec = dict(base, **{key: base[key] + 1})
        assert bench.algorithmic_bytes(rec, n, m) - b0 == per_unit, key
    # nodes of a pass over every node: row_ptr (4 B) and a quarter byte of flags each
    assert bench.algorithmic_bytes(base, n + 4, m) - b0 == 4 * 4 + 1


def test_systolic_pass_counts_only_visited_nodes(bench):
    n, m = 1 << 20, 64
    rec = {"systolic": True, "arcs_scanned": 100, "arcs_gathered": 60, "rows_read": 9, "rows_written": 4}
    assert bench.algorithmic_bytes(rec, n, m) == 8 * 9 + 4 * 100 + m * (60 + 9 + 4)
    assert bench.algorithmic_bytes(rec, 2 * n, m) == bench.algorithmic_bytes(rec, n, m)


def test_traffic_only_for_the_profiled_kernel_source(bench, tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_1011_5599_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "hanf_kernels.hip"
    src.write_text("// kernels as profiled\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    rec = {"kernel_source_sha256": sha, "traffic_bytes_per_launch": 1234}
    (tmp_path / "profiles" / "k_union_w_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w") == 1234
    assert bench.measured_traffic("other") is None          # no counter run recorded
    src.write_text("// kernels changed since\n")
    assert bench.measured_traffic("w") is None


def test_sequential_fifo_baseline(bench):
    # worked by hand: an idle gap, a queue, and a request that arrives as the queue empties
    arrivals = [0.0, 1.0, 1.5, 2.0, 10.0, 12.0]
    service = [0.5, 2.0, 1.0, 0.5, 2.0, 1.0]
    fin = bench.fifo_finish(arrivals, service)
    assert list(fin) == [0.5, 3.0, 4.0, 4.5, 12.0, 13.0]
    assert list(fin - arrivals) == [0.5, 2.0, 2.5, 2.5, 2.0, 1.0]


def test_model_bytes_leave_out_staged_gathers(bench):
    # successor counters read from a light tile's counters staged in LDS are not device
    # memory traffic; everything else is counted as in the algorithmic bytes
    n, m = 1 << 24, 128
    rec = {"arcs_scanned": 1000, "arcs_gathered": 900, "rows_read": 50, "rows_written": 40, "arcs_local": 600}
    assert bench.model_bytes(rec, n, m) == bench.algorithmic_bytes(rec, n, m) - 600 * m
    rec0 = dict(rec, arcs_local=0)
    assert bench.model_bytes(rec0, n, m) == bench.algorithmic_bytes(rec0, n, m)
    sysrec = dict(rec, systolic=True)
    assert bench.model_bytes(sysrec, n, m) == 8 * 50 + 4 * 1000 + m * (900 - 600 + 50 + 40)


def test_cpu_threads_follow_affinity_and_share(bench, monkeypatch):
    monkeypatch.setattr(bench.os, "sched_getaffinity", lambda pid: set(range(96)))
    monkeypatch.setenv("OMP_NUM_THREADS", "16")
    assert bench.cpu_threads() == (96, 16)
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.cpu_threads() == (96, 96)
    monkeypatch.setattr(bench.os, "sched_getaffinity", lambda pid: set(range(8)))
    monkeypatch.setenv("OMP_NUM_THREADS", "16")
    assert bench.cpu_threads() == (8, 8)


def test_model_bytes_leave_out_near_gathers(bench):
    # with a near count from the instrumented kernels, those successor counters are left out
    # (and the LDS count is not subtracted again: staged reads are near ones)
    n, m = 1 << 24, 128
    rec = {"arcs_scanned": 1000, "arcs_gathered": 900, "rows_read": 50, "rows_written": 40, "arcs_local": 300}
    assert bench.model_bytes(rec, n, m, near=700) == bench.algorithmic_bytes(rec, n, m) - 700 * m
    assert bench.model_bytes(rec, n, m, near=-1) == bench.algorithmic_bytes(rec, n, m) - 300 * m
