"""The serving loop's host policy without a GPU: admission by device footprint, batches of
one register count, first-come order, per-request completion inside a batch, memory
returned when a batch ends, and contexts kept for later batches. The device calls are
replaced by a stand-in batch whose fixpoints the test sets by hand; the footprints are
the library's own (`hanf_footprint` is a host function)."""
import numpy as np
import pytest

from paper_1011_5599_amd import HANF_BUSY, HANF_DONE, HANF_OK
from paper_1011_5599_amd import serve


class FakeBatch:
    """Stands in for a library batch context. Like the library, it keeps the device memory
    of its largest batch until it is destroyed (`held`)."""
    made = []

    def __init__(self, device, **options):
        self.ctx = self
        self.enqueued = 0
        self.loads = []
        self.held = 0
        self.closed = False
        FakeBatch.made.append(self)

    def load_graphs(self, graphs, seeds_per_graph):
        assert seeds_per_graph == 1
        self.graphs = graphs
        self.loads.append(len(graphs))

    def init(self, log2m, seeds):
        self.log2m, self.seeds = log2m, list(seeds)
        self.T = [-1] * len(seeds)
        self.status = HANF_BUSY
        fp = sum(serve.footprint_of(len(rp) - 1, len(ci), log2m) for rp, ci in self.graphs)
        self.held = max(self.held, fp)

    def close(self):
        self.closed = True
        self.held = 0


@pytest.fixture
def fake(monkeypatch):
    FakeBatch.made = []
    monkeypatch.setattr(serve, "Batch", FakeBatch)

    def enqueue(ctx, passes):
        ctx.enqueued += passes
        ctx.status = HANF_BUSY

    monkeypatch.setattr(serve, "hanf_enqueue", enqueue)
    monkeypatch.setattr(serve, "hanf_poll", lambda ctx: (ctx.status, 0))
    monkeypatch.setattr(serve, "hanf_batch_info", lambda ctx: (None, np.array(ctx.T)))
    monkeypatch.setattr(serve, "hanf_batch_stats_all",
                        lambda ctx: {"spid": np.arange(len(ctx.seeds), dtype=np.float64)})
    monkeypatch.setattr(serve, "hanf_batch_read_nt",
                        lambda ctx, c: np.arange(max(ctx.T[c], 0) + 1, dtype=np.float64))
    monkeypatch.setattr(serve, "hanf_device_bytes", lambda ctx: (ctx.held, 0))
    return FakeBatch


def ring(n):
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = ((np.arange(n) + 1) % n).astype(np.int32)
    return row_ptr, col_idx


def req(rid, n=1000, log2m=6):
    rp, ci = ring(n)
    return serve.Request(rid, rp, ci, log2m, seed=rid + 1)


def finish(bt, comps, T=3, done=False):
    for c in comps:
        bt.T[c] = T
    bt.status = HANF_DONE if done else HANF_OK


def test_footprint_is_the_library_figure_plus_the_graph_copy():
    r = req(0, n=1000)
    assert serve.footprint(r) > 2 * 1024 * 64       # two register arrays at least
    assert serve.footprint(req(1, n=1000, log2m=8)) > serve.footprint(r)
    assert serve.footprint(req(2, n=4000)) > serve.footprint(r)


def test_admits_within_the_budget_and_keeps_the_rest_waiting(fake):
    fp = serve.footprint(req(0))
    srv = serve.Server(hbm_budget=3 * fp + fp // 2, alloc_slack=1.0)
    for i in range(5):
        srv.submit(req(i))
    srv.pump()
    assert len(srv.flights) == 1
    assert [r.rid for r in srv.flights[0].requests] == [0, 1, 2]
    assert srv.used == 3 * fp <= srv.budget
    assert [r.rid for r in srv.waiting] == [3, 4]
    assert all(r.admitted is not None for r in srv.flights[0].requests)


def test_a_batch_holds_one_register_count(fake):
    srv = serve.Server(hbm_budget=1 << 30)
    for i, b in enumerate([6, 4, 6, 8, 4]):
        srv.submit(req(i, log2m=b))
    srv.pump()
    groups = [[r.rid for r in fl.requests] for fl in srv.flights]
    assert groups == [[0, 2], [1, 4], [3]]
    assert [fl.batch.log2m for fl in srv.flights] == [6, 4, 8]
    assert [fl.batch.seeds for fl in srv.flights] == [[1, 3], [2, 5], [4]]


def test_batch_caps(fake):
    srv = serve.Server(hbm_budget=1 << 30, max_batches=2, max_batch_requests=2)
    for i in range(7):
        srv.submit(req(i))
    srv.pump()
    assert [[r.rid for r in fl.requests] for fl in srv.flights] == [[0, 1], [2, 3]]
    assert [r.rid for r in srv.waiting] == [4, 5, 6]


def test_the_oldest_request_is_not_passed_by_smaller_ones(fake):
    big, small = req(0, n=20000), req(1, n=100)
    fp_big, fp_small = serve.footprint(big), serve.footprint(small)
    srv = serve.Server(hbm_budget=fp_big + fp_small // 2, alloc_slack=1.0)
    first = req(9, n=100)
    srv.submit(first)
    srv.pump()                                     # the first small one takes some memory
    assert srv.used == fp_small
    srv.submit(big)
    srv.submit(small)
    srv.pump()                                     # the big one does not fit yet: nothing else enters
    assert len(srv.flights) == 1 and [r.rid for r in srv.waiting] == [0, 1]
    small_ctx = srv.flights[0].batch
    finish(small_ctx, [0], done=True)
    srv.pump()                                     # the poll (before admission) retires the batch;
    assert [r.rid for r in srv.done] == [9]        # its idle context still held its memory, and is
    assert small_ctx.closed and srv.idle_batches == []   # destroyed so that the big one enters first
    assert [[r.rid for r in fl.requests] for fl in srv.flights] == [[0]]
    assert [r.rid for r in srv.waiting] == [1]
    assert srv.held() <= srv.budget


def test_requests_finish_one_by_one_and_memory_returns_with_the_batch(fake):
    fp = serve.footprint(req(0))
    srv = serve.Server(hbm_budget=1 << 30, passes_per_poll=3)
    for i in range(3):
        srv.submit(req(i))
    srv.pump()
    (fl,) = srv.flights
    bt = fl.batch
    assert bt.enqueued == 3
    assert srv.pump() == []                        # passes still in flight
    finish(bt, [1], T=4)                           # one component at its fixpoint
    out = srv.pump()
    assert [r.rid for r in out] == [1]
    assert out[0].T == 4 and list(out[0].nt) == [0, 1, 2, 3, 4] and out[0].stats == {"spid": 1.0}
    assert out[0].finish is not None and out[0].latency is not None
    assert fl.open == {0, 2} and srv.used == 3 * fp
    assert bt.enqueued == 6                        # the rest keep going
    finish(bt, [0, 2], T=2, done=True)
    out = srv.pump()
    assert sorted(r.rid for r in out) == [0, 2]
    assert srv.used == 0 and srv.flights == [] and srv.idle()
    assert srv.idle_batches == [bt] and srv.held() == 3 * fp
    srv.submit(req(3))
    srv.pump()                                     # the context is reused, not made again
    assert srv.flights[0].batch is bt and len(FakeBatch.made) == 1
    assert bt.loads == [3, 1]


def test_a_request_larger_than_the_budget_is_refused(fake):
    r = req(0, n=5000)
    srv = serve.Server(hbm_budget=serve.footprint(r) - 1, alloc_slack=1.0)
    with pytest.raises(ValueError):
        srv.submit(r)
    assert srv.idle()


def test_size_classes_keep_small_requests_apart_from_large_ones(fake):
    srv = serve.Server(hbm_budget=1 << 30, size_classes=True)
    sizes = [1000, 64000, 1100, 900, 70000]
    for i, n in enumerate(sizes):
        srv.submit(req(i, n=n))
    srv.pump()
    assert [[r.rid for r in fl.requests] for fl in srv.flights] == [[0, 2, 3], [1, 4]]
    plain = serve.Server(hbm_budget=1 << 30, size_classes=False)
    for i, n in enumerate(sizes):
        plain.submit(req(i, n=n))
    plain.pump()
    assert [[r.rid for r in fl.requests] for fl in plain.flights] == [[0, 1, 2, 3, 4]]


def test_memory_held_by_idle_contexts_counts_against_the_budget(fake):
    """A context keeps the buffers of its largest batch; a later small batch on it does not
    give them back, and the server counts what is held, not only what it admitted."""
    big, fp_big = req(0, n=20000), serve.footprint(req(0, n=20000))
    fp_small = serve.footprint(req(1, n=100))
    srv = serve.Server(hbm_budget=fp_big + 2 * fp_small, alloc_slack=1.0, max_batches=1)
    srv.submit(big)
    srv.pump()
    finish(srv.flights[0].batch, [0], done=True)
    srv.pump()
    (ctx,) = srv.idle_batches
    srv.submit(req(2, n=100))
    srv.pump()                                    # reuses the context: it still holds fp_big
    assert srv.flights[0].batch is ctx and srv.used == fp_small
    assert srv.held() == fp_big
    srv.submit(req(3, n=100))
    srv.submit(req(4, n=100))
    finish(ctx, [0], done=True)
    srv.pump()
    srv.pump()
    assert srv.held() <= srv.budget


def test_slack_for_size_classes(fake):
    fp = serve.footprint(req(0))
    srv = serve.Server(hbm_budget=2 * fp)         # default slack 1.5: one request, not two
    for i in range(2):
        srv.submit(req(i))
    srv.pump()
    assert [len(fl.requests) for fl in srv.flights] == [1]


def test_a_batch_at_its_pass_cap_finishes_its_requests_alone(fake, monkeypatch):
    """HANF_EMAXITER from a batch: finished components are collected, the others are run
    alone through the plain path (cap n + 1); serving goes on."""
    from paper_1011_5599_amd import HANF_EMAXITER, HanfError

    ran = []

    class FakePlain:
        def __init__(self, device):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

        def load(self, rp, ci):
            self.n = len(rp) - 1
            return self

        def init(self, b, seed):
            ran.append(seed)
            return self

        def run(self):
            return np.arange(7, dtype=np.float64)

        def stats(self):
            return {"spid": -1.0}

    monkeypatch.setattr(serve, "HyperANF", FakePlain)
    srv = serve.Server(hbm_budget=1 << 30)
    for i in range(3):
        srv.submit(req(i))
    srv.pump()
    bt = srv.flights[0].batch
    bt.T[1] = 2

    def poll(ctx):
        raise HanfError(HANF_EMAXITER, "pass cap reached before the fixpoint")

    monkeypatch.setattr(serve, "hanf_poll", poll)
    out = srv.pump()
    assert sorted(r.rid for r in out) == [0, 1, 2]
    by = {r.rid: r for r in out}
    assert by[1].T == 2 and not by[1].alone
    assert by[0].alone and by[2].alone and by[0].T == 6 and ran == [1, 3]
    assert srv.flights == [] and srv.idle_batches == [bt]
    srv.submit(req(5))
    monkeypatch.setattr(serve, "hanf_poll", lambda ctx: (ctx.status, 0))
    srv.pump()
    assert len(srv.flights) == 1


def test_out_of_device_memory_at_admission_retries_then_fails_alone(fake, monkeypatch):
    from paper_1011_5599_amd import HANF_ENOMEM, HanfError

    def boom(self, log2m, seeds):
        raise HanfError(HANF_ENOMEM, "hipMalloc failed")

    monkeypatch.setattr(FakeBatch, "init", boom)
    srv = serve.Server(hbm_budget=1 << 30)
    srv.submit(req(0))
    srv.pump()                                    # nothing in flight to wait for: it fails
    assert srv.idle() and len(srv.done) == 1 and srv.done[0].error
    assert all(b.closed for b in FakeBatch.made)
