"""GPU parity at the full workload sizes, in the benchmark's launch configuration.

* symmetric R-MAT scale 22 (2^26 arcs), 64 registers, hash seed 7: registers byte-equal to
  the oracle's at every iteration, N_hat(t) within 1e-12, same T (also with 5-bit packed
  registers);
* web-like graph of 2^24 nodes (3.4e8 arcs), 128 registers, hash seed 1: N_hat(0) against
  its closed form, the final counters and T against a full (multi-threaded) oracle run
  (with and without systolic passes, the transposed graph built on the device),
  N_hat(T) against the oracle's sum on its own final counters, and, for sampled nodes,
  c_t[v] against the counter of the ball B(v, t) built by BFS (the identity of Section
  3.2) at t = 1, 2, 3.
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
@pytest.mark.parametrize("systolic,packed", [(False, False), (True, False), (True, True)])
def test_rmat22sym_every_iteration(systolic, packed):
    """With systolic=True in the benchmark's configuration: the symmetric graph's own
    device arrays serve as its transpose. packed: 5-bit registers (read back unpacked)."""
    import torch
    spec = graphgen.WORKLOADS["rmat22sym"]
    rp, ci = graphgen.workload_graph(spec)
    b, seed = spec["log2m"], spec["seed"]
    _say(f"[fullsize] rmat22sym n={len(rp) - 1} arcs={len(ci)} b={b} seed={seed} systolic={systolic} "
         f"packed={packed}")
    with hanf.HyperANF(0, packed5=int(packed)) as h:
        if systolic:
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
        assert any(r["systolic"] for r in h.pass_log()) == systolic


@pytest.mark.timeout(900)
def test_web24_final_counters_and_samples():
    spec = graphgen.WORKLOADS["web24"]
    rp, ci = graphgen.workload_graph(spec)
    n = len(rp) - 1
    b, seed = spec["log2m"], spec["seed"]
    m = 1 << b
    _say(f"[fullsize] web24 n={n} arcs={len(ci)} b={b} seed={seed}")
    rng = np.random.default_rng(2024)
    sample = rng.choice(n, 24, replace=False)
    with hanf.HyperANF(0) as h:
        h.load(rp, ci).init(b, seed)
        early = {}
        for t in range(4):
            regs = h.registers()
            early[t] = regs[sample].copy()
            del regs
            h.step(1)
        h.run()
        nt = h.nt()
        final = h.registers()
    with hanf.HyperANF(0) as h:  # systolic passes, transposed graph built on the device
        h.load(rp, ci).build_transpose().init(b, seed)
        nt_sys = h.run()
        assert any(r["systolic"] for r in h.pass_log())
        final_sys = h.registers()
    assert np.array_equal(final_sys, final)
    del final_sys
    np.testing.assert_allclose(nt_sys, nt, rtol=1e-12, atol=0)
    assert nt[0] == pytest.approx(n * m * math.log(m / (m - 1)), rel=1e-12)
    for t in (1, 2, 3):
        for i, v in enumerate(sample[:8]):
            M, _ = oracle.ball_counter(rp, ci, b, seed, int(v), t)
            assert np.array_equal(early[t][i], M), (t, int(v))
    _say("[fullsize] web24 samples ok; oracle run")
    _, T, regs = oracle.run(rp, ci, b, seed, nthreads=THREADS, want_regs=True, want_nt=False)
    assert len(nt) == T + 1
    assert np.array_equal(final, regs)
    del final
    nT = oracle.sum_sizes(regs, b)
    assert nt[-1] == pytest.approx(nT, rel=1e-12)
