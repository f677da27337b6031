"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function
declared in include/hanf.h, and its pure host functions and argument checks behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

hanf = pytest.importorskip("paper_1011_5599_amd")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hanf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hanf_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    lib = hanf.lib()
    for name in names:
        assert hasattr(lib, name), name
    # and the binding exposes each under the same name
    for name in names:
        assert callable(getattr(hanf, name)), name


def test_footprint_matches_memory_model():
    """Two register arrays of n*m bytes dominate (the O(n m) register memory of Section 3.4)."""
    n, arcs = 1 << 22, 1 << 26
    for b in range(4, 9):
        fb = hanf.hanf_footprint(n, arcs, b, copy_graph=False)
        # plus flags, estimates, tiles, the schedule scan, the N_hat history (8 B per pass
        # allowed, n + 1 passes) and at most 65536 pass records of 64 bytes
        assert 2 * n * (1 << b) <= fb <= 2 * n * (1 << b) + 48 * n + (1 << 23)
        fg = hanf.hanf_footprint(n, arcs, b, copy_graph=True)
        assert fg - fb == 4 * (n + 1) + 4 * arcs


@pytest.mark.parametrize("args", [(0, 10, 6, 1), (10, -1, 6, 1), (10, 1 << 31, 6, 1), (10, 10, 3, 1),
                                  (10, 10, 9, 1), (hanf.HANF_MAX_NODES + 1, 10, 6, 1),
                                  (10, hanf.HANF_MAX_ARCS + 1, 6, 1)])
def test_footprint_rejects_bad_arguments(args):
    with pytest.raises(hanf.HanfError) as e:
        hanf.hanf_footprint(*args)
    assert e.value.code == hanf.HANF_EINVAL
    assert "out of range" in hanf.hanf_last_error(None)


def test_size_limits_match_the_header():
    """The binding's size limits are the header's, 2^31 - 2^20, and a graph at both limits is
    accepted by the footprint (whose arithmetic is 64-bit)."""
    text = open(os.path.join(ROOT, "include", "hanf.h")).read()
    for name in ("HANF_MAX_NODES", "HANF_MAX_ARCS"):
        value = int(re.search(rf"#define {name} (\d+)", text).group(1))
        assert value == getattr(hanf, name) == (1 << 31) - (1 << 20)
    assert hanf.hanf_footprint(hanf.HANF_MAX_NODES, hanf.HANF_MAX_ARCS, 4, 0) > 16 * hanf.HANF_MAX_NODES


def test_null_context_calls_fail_cleanly():
    lib = hanf.lib()
    i32 = ctypes.c_int32()
    i64 = ctypes.c_int64()
    assert lib.hanf_set_option(None, hanf.HANF_OPT_FRONTIER, 1) == hanf.HANF_EINVAL
    assert lib.hanf_load_csr(None, 1, 0, None, None, 0) == hanf.HANF_EINVAL
    assert lib.hanf_init_counters(None, 6, 1) == hanf.HANF_EINVAL
    assert lib.hanf_iterate(None, 0, ctypes.byref(i32), ctypes.byref(i64)) == hanf.HANF_EINVAL
    assert lib.hanf_read_nt(None, None, 0, ctypes.byref(i32)) == hanf.HANF_EINVAL
    assert lib.hanf_read_registers(None, None, 0, 0) == hanf.HANF_EINVAL
    assert lib.hanf_stats(None, 0.9, 0.0, 0, None) == hanf.HANF_EINVAL
    lib.hanf_destroy(None)  # safe on NULL
    assert "NULL" in hanf.hanf_last_error(None)


def test_create_without_device_reports_error():
    """In a process with no GPU, hanf_create fails with HANF_EDEVICE (never aborts)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(hanf.HanfError) as e:
        hanf.hanf_create(0)
    assert e.value.code in (hanf.HANF_EDEVICE, hanf.HANF_EINVAL)


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(hanf, "_lib", None)
    monkeypatch.setattr(hanf, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        hanf.lib()


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_single_hip_runtime_in_process():
    """Loading the library and torch leaves exactly one HIP runtime mapped in the process."""
    import subprocess
    import sys
    code = ("import paper_1011_5599_amd as h; h.lib(); import torch; "
            "rts = h._hip_runtimes(); assert len(rts) == 1, rts; print('ok')")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr


def test_host_stats_match_the_oracle():
    """hanf_stats_nt (the statistics code the device kernels run, here on the host) against
    the oracle's Sections 4-5 and Algorithm 3 on the N_hat sequences of small oracle runs
    and on crafted sequences (one value; a plateau; a cycle's closed-form moments)."""
    import math

    import numpy as np

    import graphgen
    import oracle
    from oracle import stats as ostats
    seqs = []
    for g in (graphgen.rmat(9, 3000, seed=2), graphgen.clique_path_clique(10, 5),
              graphgen.directed_cycle(50), graphgen.erdos_renyi(400, 1600, seed=3)):
        nt, _, _ = oracle.run(*g, 6, 11)
        seqs.append(list(nt))
    n = 40  # exact N(t) of a directed cycle: n (t + 1) pairs at distance <= t
    seqs += [[5.0], [3.0, 3.0, 3.0], [float(n * (t + 1)) for t in range(n)]]
    for nt in seqs:
        for alpha, eps, distinct in ((0.9, 0.0, False), (0.5, 0.05, False), (0.9, 0.1, True)):
            got = hanf.hanf_stats_nt(nt, alpha, eps, distinct)
            want = ostats.stats(nt, alpha, distinct)
            for k in ("ed", "ied", "avg_dist", "var", "spid", "n_max"):
                if isinstance(want[k], float) and math.isnan(want[k]):
                    assert math.isnan(got[k]), (k, nt[:3])
                else:
                    assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-12), (k, nt[:3])
            assert got["T"] == want["T"] == len(nt) - 1
            lo, hi = ostats.diameter_interval(nt, eps, alpha)
            assert got["d_lo"] == (-1 if lo is None else lo) and got["d_hi"] == (-1 if hi is None else hi)
    cyc = hanf.hanf_stats_nt([float(n * (t + 1)) for t in range(n)], 0.9, 0.0, True)
    assert cyc["avg_dist"] == pytest.approx(n / 2) and cyc["var"] == pytest.approx(n * (n - 2) / 12)
    for bad in (([], 0.9, 0.0), ([1.0], 0.0, 0.0), ([1.0], 0.9, -1.0)):
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_stats_nt(*bad)
        assert e.value.code == hanf.HANF_EINVAL


def test_footprint_counts_the_reordered_graph():
    """HANF_FP_ORDER adds the graph rewritten in the library's node order (row_ptr, col_idx)
    and the two order tables; with HANF_FP_TRANSPOSE a reordered transpose as well."""
    n, arcs = 1 << 20, 1 << 24
    graph = (n + 1) * 4 + arcs * 4
    base = hanf.hanf_footprint(n, arcs, 6, copy_graph=False)
    assert hanf.hanf_footprint(n, arcs, 6, copy_graph=False, order=True) - base == graph + 8 * n
    t = hanf.hanf_footprint(n, arcs, 6, copy_graph=False, transpose=True)
    assert hanf.hanf_footprint(n, arcs, 6, copy_graph=False, transpose=True, order=True) - t == 2 * graph + 8 * n
