"""hanf_batch_stats_all_noalloc (the statistics of every batch component, staged in the
library's fixed device array instead of an allocation) against hanf_batch_stats_all, the
entry point it is a variant of: every field of every record equal, on two calls in a row,
the second on a smaller batch; and the component limit refused with HANF_ERANGE."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")

FIELDS = [f for f, _ in hanf.hanf_stats_t._fields_]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _graphs(k, base):
    gs = [graphgen.erdos_renyi(150 + 29 * i, 6 * (150 + 29 * i), seed=base + i) for i in range(k)]
    gs += [graphgen.rmat(8 + (i % 3), 2000 + 300 * i, seed=base + 50 + i) for i in range(k)]
    gs += [graphgen.empty(1), graphgen.directed_path(40), graphgen.directed_cycle(17)]
    return gs


def _records_equal(a, b, n):
    for f in FIELDS:
        x, y = a[f][:n], b[f][:n]
        if x.dtype.kind == "f":
            assert np.array_equal(x, y, equal_nan=True), f
        else:
            assert np.array_equal(x, y), f


@pytest.mark.timeout(300)
def test_noalloc_stats_match_allocating_entry_point():
    with hanf.Batch(0) as big, hanf.Batch(0) as small:
        cases = []
        for bt, k, S, b, base in ((big, 8, 4, 6, 300), (small, 3, 2, 4, 700)):
            gs = _graphs(k, base)
            seeds = [31 * g + s + 1 for g in range(len(gs)) for s in range(S)]
            _say(f"[noalloc] batch of {len(gs)} graphs x {S} seeds, b={b}")
            bt.load_graphs(gs, S).init(b, seeds)
            bt.run()
            cases.append((bt, len(gs) * S))
        assert cases[1][1] < cases[0][1]
        for distinct in (False, True):
            for bt, n in cases:  # two calls in a row, the second with fewer components
                want = np.zeros(n, hanf.STATS_DTYPE)
                assert hanf.lib().hanf_batch_stats_all(bt.ctx, 0.9, 0.05, int(distinct), want.ctypes.data) == 0
                got = np.full(n + 1, -7, hanf.STATS_DTYPE)  # one guard record past the end
                hanf.hanf_batch_stats_all_noalloc(bt.ctx, got, 0.9, 0.05, distinct)
                _records_equal(got, want, n)
                assert got["T"][n] == -7 and got["ed"][n] == -7.0  # nothing written past n
                assert (got["distinct"][:n] == int(distinct)).all()
                assert (got["T"][:n] == bt.fixpoints()).all()


@pytest.mark.timeout(300)
def test_noalloc_refuses_more_components_than_its_array():
    cap = 65536
    k = cap + 1  # one-node graphs, one seed each
    goff = np.arange(k + 1, dtype=np.int32)
    aoff = np.zeros(k + 1, np.int32)
    rp = np.zeros(k + 1, np.int32)
    ci = np.zeros(0, np.int32)
    with hanf.Batch(0) as bt:
        bt.load_union(goff, aoff, rp, ci, 1).init(4, list(range(1, k + 1)))
        bt.run()
        out = np.zeros(k, hanf.STATS_DTYPE)
        rc = hanf.lib().hanf_batch_stats_all_noalloc(bt.ctx, 0.9, 0.0, 0, out.ctypes.data)
        assert rc == hanf.HANF_ERANGE
        assert "HANF_NOALLOC_MAX_COMPONENTS" in hanf.hanf_last_error(bt.ctx)
        # the allocating entry point still serves it
        assert hanf.lib().hanf_batch_stats_all(bt.ctx, 0.9, 0.0, 0, out.ctypes.data) == 0
        assert (out["T"] == 0).all()
