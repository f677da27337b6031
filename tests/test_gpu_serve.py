"""Serving loop: requests admitted while others run, batched across graphs, overlapping on
the device; each result must equal the same request run alone (registers exact, N_hat within
1e-12, same T)."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")
from paper_1011_5599_amd import serve  # noqa: E402


def _requests(count, seed, hi=1 << 13):
    reqs = graphgen.serve_requests(count, trace_seed=seed, hi=hi, median=1 << 11, sigma=1.0)
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(0.002, count))
    return [serve.Request(r["rid"], r["graph"][0], r["graph"][1], r["log2m"], r["seed"], float(a))
            for r, a in zip(reqs, arrivals)]


@pytest.mark.timeout(600)
def test_served_results_equal_alone():
    reqs = _requests(40, 11)
    srv = serve.Server(0, keep_registers=True, max_batches=4, passes_per_poll=1)
    srv.serve_trace(reqs)
    assert all(r.finish is not None for r in reqs)
    assert max(srv.batch_sizes) > 1, srv.batch_sizes  # iterations of several graphs batched
    with hanf.HyperANF(0) as h:
        for r in reqs:
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
    fps = [serve.footprint(r) for r in reqs]
    budget = max(fps) + 1
    srv = serve.Server(0, hbm_budget=budget, max_batches=8)
    for r in reqs:
        r.arrival = 0.0
    srv.serve_trace(reqs)
    assert all(r.finish is not None for r in reqs)
    assert max(srv.batch_sizes) >= 1
    with pytest.raises(ValueError):
        serve.Server(0, hbm_budget=10).submit(reqs[0])
