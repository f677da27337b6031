"""GPU parity at the full workload sizes, in the benchmark's launch configuration.

* symmetric R-MAT scale 22 (2^26 arcs), 64 registers, hash seed 7: registers byte-equal to
  the oracle's at every iteration, N_hat(t) within 1e-12, same T (also with 5-bit packed
  registers);
* web-like graph of 2^24 nodes (3.4e8 arcs, 80% intra-host), 128 registers, hash seed 1:
  registers byte-equal to the oracle's at every iteration in three runs side by side
  (flag-frontier passes, the benchmark's configuration; systolic passes marked by a forward
  scan; systolic passes over a transposed graph built on the device), N_hat(t) within
  1e-12, same T; N_hat(0) against its closed form and, for sampled nodes, c_t[v]
  against the counter of the ball B(v, t) built by BFS (the identity of Section 3.2) at
  t = 1, 2, 3.
* a graph with the largest arc count the library takes (2^31 - 2^20 arcs: 2^21 nodes of
  1023 successors, then 2^20 nodes of one successor whose rows end at that count), 16
  registers: registers byte-equal to the oracle's at every iteration, N_hat(t) within
  1e-12, same T.
* 2^28 nodes of 256 registers (2^32 row lanes, more threads than one launch holds):
  initialisation and the estimates of a resumed run sweep the lanes in steps; and the
  largest node count the library takes, 2^31 - 2^20 nodes of 16 registers: every node's
  estimate, N_hat(0) and sampled counters against closed forms and the oracle.
* directed R-MAT scale 14 at every iteration is in test_gpu_parity.py.
"""
import math
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")

THREADS = max(1, min(16, os.cpu_count() or 1))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("systolic,packed", [(False, False), (True, False), (True, True), ("forward", False)])
def test_rmat22sym_every_iteration(systolic, packed):
    """With systolic=True in the benchmark's configuration: the symmetric graph's own
    device arrays serve as its transpose; "forward": no transpose, systolic passes marked by
    a forward scan; False: no transpose and flag-frontier passes. packed: 5-bit registers
    (read back unpacked)."""
    import torch
    spec = graphgen.WORKLOADS["rmat22sym"]
    rp, ci = graphgen.workload_graph(spec)
    b, seed = spec["log2m"], spec["seed"]
    _say(f"[fullsize] rmat22sym n={len(rp) - 1} arcs={len(ci)} b={b} seed={seed} systolic={systolic} "
         f"packed={packed}")
    with hanf.HyperANF(0, packed5=int(packed), forward=int(systolic == "forward")) as h:  # (forward: option)
        if systolic is True:
            drp, dci = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
            h.load(drp, dci).load_transpose(drp, dci)
        else:
            h.load(rp, ci)
        h.init(b, seed)
        want = []
        T = None
        for t, c, s in oracle.run_steps(rp, ci, b, seed, nthreads=THREADS):
            want.append(s)
            got = h.registers()
            assert np.array_equal(got, c), f"registers differ at t={t}"
            st, _, _ = h.step(1)
            T = t
            _say(f"[fullsize] rmat22sym t={t} ok")
        assert st == hanf.HANF_DONE
        nt = h.nt()
        assert len(nt) == T + 1
        np.testing.assert_allclose(nt, np.array(want), rtol=1e-12, atol=0)
        kinds = {r["systolic"] for r in h.pass_log()}
        assert kinds == ({0, 1} if systolic is True else {0, 2} if systolic == "forward" else {0}), kinds


@pytest.mark.timeout(1200)
def test_web24_every_iteration():
    """The web-like workload at full size (2^24 nodes, 80% of the arcs intra-host), run
    three times side by side: no transposed graph with flag-frontier passes (the benchmark's
    configuration), the same with systolic passes marked by a forward scan, and systolic
    passes through a transposed graph built on the device. At every t every run's registers
    equal the oracle's c_t byte for byte; N_hat(t) within 1e-12; same
    T. Also N_hat(0) against its closed form and, for sampled nodes, c_t[v] against the
    counter of the ball B(v, t) (Section 3.2) at t = 1, 2, 3."""
    spec = graphgen.WORKLOADS["web24"]
    rp, ci = graphgen.workload_graph(spec)
    n = len(rp) - 1
    b, seed = spec["log2m"], spec["seed"]
    m = 1 << b
    _say(f"[fullsize] web24 n={n} arcs={len(ci)} b={b} seed={seed} threads={THREADS}")
    rng = np.random.default_rng(2024)
    sample = rng.choice(n, 8, replace=False)
    with hanf.HyperANF(0, forward=1) as hf, hanf.HyperANF(0) as h, hanf.HyperANF(0) as hs:
        hf.load(rp, ci).init(b, seed)
        h.load(rp, ci).init(b, seed)
        hs.load(rp, ci).build_transpose().init(b, seed)
        want = []
        T = None
        for t, c, s in oracle.run_steps(rp, ci, b, seed, nthreads=THREADS):
            want.append(s)
            for name, ctx in (("forward", hf), ("frontier", h), ("systolic", hs)):
                got = ctx.registers()
                assert np.array_equal(got, c), f"{name}: registers differ at t={t}"
                del got
            if 1 <= t <= 3:
                for v in sample:
                    M, _ = oracle.ball_counter(rp, ci, b, seed, int(v), t)
                    assert np.array_equal(c[v], M), (t, int(v))
            st, _, _ = h.step(1)
            st_s, _, _ = hs.step(1)
            st_f, _, _ = hf.step(1)
            T = t
            _say(f"[fullsize] web24 t={t} ok")
        assert st == hanf.HANF_DONE and st_s == hanf.HANF_DONE and st_f == hanf.HANF_DONE
        assert T >= 10  # a long diameter: many passes, frontier skipping exercised
        for ctx in (hf, h, hs):
            nt = ctx.nt()
            assert len(nt) == T + 1
            np.testing.assert_allclose(nt, np.array(want), rtol=1e-12, atol=0)
        assert want[0] == pytest.approx(n * m * math.log(m / (m - 1)), rel=1e-12)
        assert {r["systolic"] for r in hs.pass_log()} == {0, 1}
        assert {r["systolic"] for r in hf.pass_log()} == {0, 2}
        assert not any(r["systolic"] for r in h.pass_log())
        assert any(not r["gather_all"] for r in h.pass_log())  # flag-frontier passes ran


@pytest.mark.timeout(900)
def test_arc_limit_every_iteration():
    """Arc positions up to 2^31 - 2^20 (int32 throughout the kernels): the heavy rows are
    split into chunks, the light rows at the end of col_idx go through the light rounds."""
    rp, ci = graphgen.limit_graph()
    n, arcs = len(rp) - 1, len(ci)
    assert arcs == hanf.HANF_MAX_ARCS and int(rp[-1]) == arcs
    b, seed = 4, 11
    _say(f"[fullsize] arc limit n={n} arcs={arcs} b={b} seed={seed}")
    with hanf.HyperANF(0) as h:
        h.load(rp, ci).init(b, seed)
        _say("[fullsize] arc limit: loaded")
        want = []
        T = None
        for t, c, s in oracle.run_steps(rp, ci, b, seed, nthreads=THREADS):
            want.append(s)
            assert np.array_equal(h.registers(), c), f"registers differ at t={t}"
            st, steps, _ = h.step(1)
            assert steps == 1
            _say(f"[fullsize] arc limit t={t} ok")
            T = t
        assert st == hanf.HANF_DONE
        kinds = "".join("D" if r["gather_all"] else "F" for r in h.pass_log())
        assert kinds.startswith("D") and "F" in kinds, kinds
        got = h.nt()
        assert len(got) == len(want) == T + 1
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)


def _one_register_counters(h, n, b, seed, label):
    """Checks a run on a graph without arcs, where each counter holds the one register its
    node's hash sets (Algorithm 1, add): V = m - 1 registers are zero, the raw estimate
    (under 0.8 m) is below 5m/2, so every estimate is the linear-counting value
    m ln(m / (m - 1)) and N_hat(0) is n times it; an all-zero counter (a node never
    initialised) would estimate 0. Also checks sampled counters, the last node's included,
    against the oracle's initialisation. Returns the registers (a device tensor)."""
    import torch
    m = 1 << b
    e1 = m * math.log(m / (m - 1))
    est = h.estimates()
    assert np.all(est == e1), (label, np.unique(est)[:4])
    del est
    nt = h.nt()
    assert len(nt) == 1
    np.testing.assert_allclose(nt[0], n * e1, rtol=1e-12, atol=0)
    regs = torch.empty(n * m, dtype=torch.uint8, device="cuda")
    h.registers(out=regs)
    sample = [0, 1, 12_345, n // 2 + 7, n - 2, n - 1]
    rows = regs.view(n, m)[torch.tensor(sample, device="cuda")].cpu().numpy()
    for v, row in zip(sample, rows):
        want = np.zeros(m, np.uint8)
        oracle.add(want, b, seed, v)
        assert np.array_equal(row, want), (label, v)
    _say(f"[fullsize] {label} ok")
    return regs


@pytest.mark.timeout(600)
def test_row_lanes_beyond_one_launch():
    """2^28 nodes without arcs, 256 registers each: n * 16 = 2^32 row lanes, more threads
    than one launch holds, so initialisation and the estimates of a resumed run sweep the
    lanes in steps. Checked after the run and after a checkpoint round trip through device
    memory (whose estimates come from the other sweep)."""
    n, b, seed = 1 << 28, 8, 5
    _say(f"[fullsize] row lanes n={n} m={1 << b} lanes={n * ((1 << b) // 16)}")
    with hanf.HyperANF(0) as h:
        h.load(np.zeros(n + 1, np.int32), np.zeros(0, np.int32)).init(b, seed)
        assert len(h.run()) == 1
        regs = _one_register_counters(h, n, b, seed, "row lanes: run")
        hanf.hanf_write_registers(h.ctx, regs, 0, h.nt())
        del regs
        _one_register_counters(h, n, b, seed, "row lanes: resumed")
        assert len(h.run()) == 1
    import torch
    torch.cuda.empty_cache()  # (the 64 GiB register copies stay out of later tests' way)


@pytest.mark.timeout(600)
def test_node_limit():
    """The largest node count the library takes, HANF_MAX_NODES = 2^31 - 2^20 nodes (no
    arcs, 16 registers): node ids up to 2^31 - 2^20 - 1 in every kernel of a run."""
    n, b, seed = hanf.HANF_MAX_NODES, 4, 3
    _say(f"[fullsize] node limit n={n} m={1 << b}")
    with hanf.HyperANF(0) as h:
        h.load(np.zeros(n + 1, np.int32), np.zeros(0, np.int32)).init(b, seed)
        assert len(h.run()) == 1
        _one_register_counters(h, n, b, seed, "node limit")
    import torch
    torch.cuda.empty_cache()


def test_schedule_beyond_one_launch_is_refused():
    """A schedule whose union launch would need 2^32 threads or more (one wavefront per
    chunk of one arc: node 0 holds all 2^26 arcs) is refused at initialisation, not
    launched."""
    n, arcs = 1 << 16, 1 << 26
    rp = np.full(n + 1, arcs, np.int32)
    rp[0] = 0
    ci = (np.arange(arcs, dtype=np.int64) % n).astype(np.int32)
    with hanf.HyperANF(0, chunk_arcs=1) as h:
        h.load(rp, ci)
        with pytest.raises(hanf.HanfError) as e:
            h.init(4, 1)
        assert e.value.code == hanf.HANF_EINVAL
        assert "one launch" in hanf.hanf_last_error(h.ctx)
