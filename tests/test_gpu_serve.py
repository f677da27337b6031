"""Serving loop: requests admitted while others run, batched across graphs, overlapping on
the device. Every served result must equal the CPU oracle's run of the same request
(Algorithm 2: registers byte for byte, N_hat(t) within 1e-12, same T) and the same request
run alone through the plain path."""
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")
from paper_1011_5599_amd import serve  # noqa: E402

THREADS = max(1, min(16, os.cpu_count() or 1))


def _requests(count, seed, hi=1 << 13):
    reqs = graphgen.serve_requests(count, trace_seed=seed, hi=hi, median=1 << 11, sigma=1.0)
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(0.002, count))
    return [serve.Request(r["rid"], r["graph"][0], r["graph"][1], r["log2m"], r["seed"], float(a))
            for r, a in zip(reqs, arrivals)]


def _mix():
    """36 small requests (2^10..2^13 nodes, R-MAT or web-like, log2m in {4, 6, 8}) and two
    R-MAT graphs of 2^16 and 2^17 nodes (16 arcs per node; their largest rows have thousands
    of arcs and are split into chunks), arriving third and sixth."""
    reqs = _requests(36, 11)
    big = []
    for k, (scale, b) in enumerate(((16, 6), (17, 8))):
        rp, ci = graphgen.rmat(scale, 16 << scale, seed=900 + k)
        big.append(serve.Request(1000 + k, rp, ci, b, 77 + k, 0.0))
    reqs.insert(2, big[0])
    reqs.insert(5, big[1])
    rng = np.random.default_rng(5)
    for r, a in zip(reqs, np.cumsum(rng.exponential(0.002, len(reqs)))):
        r.arrival = float(a)
    return reqs


@pytest.mark.timeout(900)
def test_served_results_equal_oracle_and_alone():
    reqs = _mix()
    assert max(np.diff(r.row_ptr).max() for r in reqs) > 1024  # heavy rows in the mix
    srv = serve.Server(0, keep_registers=True, max_batches=4, passes_per_poll=1)
    srv.serve_trace(reqs)
    assert all(r.finish is not None and r.error is None for r in reqs)
    assert max(srv.batch_sizes) > 1, srv.batch_sizes  # iterations of several graphs batched
    # continuous batching: several batches were on the device at once, and some batch was
    # admitted while an earlier one was still running
    assert srv.max_flights >= 2, srv.max_flights
    batches = {}
    for r in reqs:
        lo, hi = batches.get(r.batch_id, (r.admitted, r.finish))
        batches[r.batch_id] = (min(lo, r.admitted), max(hi, r.finish))
    overlap = any(a0 < b0 < a1 for i, (a0, a1) in batches.items()
                  for j, (b0, _) in batches.items() if i != j)
    assert overlap, batches
    with hanf.HyperANF(0) as h:
        for r in reqs:
            print(f"[serve] request {r.rid} n={r.n} arcs={len(r.col_idx)} log2m={r.log2m} seed={r.seed} "
                  f"batch={r.batch_id} T={r.T}", flush=True)
            nt_o, T_o, regs_o = oracle.run(r.row_ptr, r.col_idx, r.log2m, r.seed, nthreads=THREADS,
                                           want_regs=True)
            assert r.T == T_o, r.rid
            np.testing.assert_allclose(r.nt, nt_o, rtol=1e-12, atol=0)
            assert np.array_equal(r.registers, regs_o), r.rid
            # the same request alone through the plain path
            h.load(r.row_ptr, r.col_idx).init(r.log2m, r.seed)
            nt = h.run()
            assert len(nt) == r.T + 1, r.rid
            np.testing.assert_allclose(r.nt, nt, rtol=1e-12, atol=0)
            assert np.array_equal(r.registers, h.registers()), r.rid
            st = h.stats()
            for k in ("ed", "avg_dist", "spid"):
                assert r.stats[k] == pytest.approx(st[k], rel=1e-9, abs=1e-12), (r.rid, k)


def test_admission_respects_budget():
    reqs = _requests(12, 3)
    probe = serve.Server(0)
    budget = max(probe._need(serve.footprint(r)) for r in reqs) + 1
    probe.close()
    srv = serve.Server(0, hbm_budget=budget, max_batches=8)
    for r in reqs:
        r.arrival = 0.0
    srv.serve_trace(reqs)
    assert all(r.finish is not None and r.error is None for r in reqs)
    assert max(srv.batch_sizes) >= 1
    assert srv.held() <= budget
    srv.close()
    with pytest.raises(ValueError):
        serve.Server(0, hbm_budget=10).submit(reqs[0])
