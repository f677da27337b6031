"""GPU: the node order a single graph runs in (HANF_OPT_HUBS: hubs, the nodes of largest
in-degree, first). The order is a layout choice: counters are hashed from the caller's ids
and every read maps back to them, so registers and per-node estimates equal the oracle's
bit for bit at every pass, N_hat(t) within 1e-12 relative, and T and the work counters
are equal. The order itself is checked against its definition, computed here with numpy.
"""
import numpy as np
import pytest

import graphgen
import oracle
from test_gpu_parity import RTOL, _flush, step_parity, transpose_csr

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")


def degree_levels(d):
    """Class level of each in-degree: d below 8, then 8 levels per octave (the leading bit's
    position and the three bits below it); 0 for no arcs in."""
    d = np.asarray(d, np.int64)
    e = np.zeros_like(d)
    nz = d > 0
    e[nz] = np.array([int(x).bit_length() - 1 for x in d[nz]], np.int64)  # leading bit
    lv = d.copy()
    big = e >= 3
    lv[big] = 8 * (e[big] - 2) + ((d[big] >> (e[big] - 3)) & 7)
    return lv


def expected_order(indeg, K):
    """Hubs first: the highest levels whose nodes number at most K (whole levels), larger
    levels first, by id within a level; then every other node by id."""
    lv = degree_levels(indeg)
    hist = np.bincount(lv, minlength=240)
    cum, lstar = 0, 240
    for level in range(239, 0, -1):
        cum += hist[level]
        if cum > K:
            break
        lstar = level
    cls = np.where((np.asarray(indeg) > 0) & (lv >= lstar), 239 - lv, 240)
    return np.argsort(cls, kind="stable").astype(np.int32), int((cls < 240).sum())


def test_degree_levels_are_monotone_classes():
    d = np.arange(1, 5000)
    lv = degree_levels(d)
    assert np.all(np.diff(lv) >= 0) and lv[0] == 1 and lv[7] == 8 and lv[15] == 16
    for e in range(3, 30):  # 8 levels per octave
        assert len(set(degree_levels(np.arange(1 << e, 1 << (e + 1), max(1, (1 << e) // 64))).tolist())) == 8


@pytest.mark.parametrize("transpose", ["self", "build", "host", None])
@pytest.mark.parametrize("K", [1, 50, 1000, 1 << 30])
def test_order_matches_its_definition(transpose, K):
    """The chosen order against its definition, with in-degrees from the transposed graph
    (self, built, loaded) or counted from col_idx (no transpose); the identity before the
    first initialisation and with K = 0."""
    sym = transpose == "self"
    rp, ci = graphgen.rmat(12, 40_000, symmetric=sym, seed=61)
    n = len(rp) - 1
    indeg = np.bincount(ci, minlength=n)
    want, hubs = expected_order(indeg, K)
    _flush(f"[order] transpose={transpose} K={K} hubs={hubs}")
    assert hubs <= min(K, n) and (K < 50 or hubs > 0)
    with hanf.HyperANF(0, hubs=K) as h:
        h.load(rp, ci)
        if transpose == "self":
            h.transpose_self()
        elif transpose == "build":
            h.build_transpose()
        elif transpose == "host":
            h.load_transpose(*transpose_csr(rp, ci))
        assert np.array_equal(h.order(), np.arange(n))
        h.init(5, 3)
        got = h.order()
        assert np.array_equal(got, want)
        if K >= 50:  # the order moves nodes (R-MAT's largest hub is node 0 anyway)
            assert not np.array_equal(got, np.arange(n))
    for opts in (dict(hubs=0), {}, dict(hubs=-1)):  # the caller's order: off, by default, auto on a small graph
        with hanf.HyperANF(0, **opts) as h:
            h.load(rp, ci).build_transpose().init(5, 3)
            assert np.array_equal(h.order(), np.arange(n))


@pytest.mark.parametrize("case", ["plain", "build", "host", "self", "packed", "frontier0", "persistent",
                                  "chunks"])
def test_order_parity_every_pass(case):
    """A forced order in every kind of pass: registers and estimates at every t, work
    counters, N_hat and T against the oracle."""
    if case == "self":
        rp, ci = graphgen.rmat(13, 60_000, symmetric=True, seed=62)
        step_parity(rp, ci, 6, 21, transpose="self", hubs=700)
        step_parity(rp, ci, 6, 22, transpose="declared", systolic=1, hubs=60)
        return
    rp, ci = graphgen.rmat(14, 262_144, seed=14)
    if case == "plain":
        step_parity(rp, ci, 4, 1, hubs=300)
    elif case == "build":
        step_parity(rp, ci, 4, 1, transpose="build", hubs=300)
    elif case == "host":
        step_parity(rp, ci, 4, 1, transpose="host", hubs=5000)
    elif case == "packed":
        step_parity(rp, ci, 6, 2, transpose="build", packed5=1, hubs=300)
    elif case == "frontier0":
        step_parity(rp, ci, 5, 3, frontier=0, hubs=2000)
    elif case == "persistent":
        step_parity(rp, ci, 5, 4, transpose="build", systolic=1, union_policy=2, hubs=2000)
    else:
        step_parity(rp, ci, 7, 5, transpose="build", chunk_arcs=150, light_max=8, hubs=900)


@pytest.mark.parametrize("name", ["empty100", "star_in", "star_out", "cycle", "complete", "loops_dups"])
def test_order_edge_graphs(name):
    """No arcs (the order stays the identity), one hub with every arc in, one node with
    every arc out, all in-degrees equal (every node one class, or none when K is smaller
    than the class), a complete graph, duplicate arcs and self-loops."""
    if name == "empty100":
        g = graphgen.empty(100)
    elif name == "star_in":
        g = graphgen.star_in(30_000)
    elif name == "star_out":
        g = graphgen.star_out(20_001)
    elif name == "cycle":
        g = graphgen.directed_cycle(300)
    elif name == "complete":
        g = graphgen.complete(120)
    else:
        rp, ci = graphgen.erdos_renyi(3000, 20_000, seed=8)
        n = len(rp) - 1
        arcs = [(u, int(w)) for u in range(n) for w in ci[rp[u]:rp[u + 1]]]
        arcs += arcs[::7] + [(u, u) for u in range(0, n, 5)]
        g = graphgen.from_arcs(n, arcs)
    rp, ci = g
    n = len(rp) - 1
    for K in (1, 50, n):
        step_parity(rp, ci, 4, 99, hubs=K)
        step_parity(rp, ci, 7, 98, transpose="build", systolic=1, hubs=K)
        with hanf.HyperANF(0, hubs=K) as h:
            h.load(rp, ci).init(4, 1)
            want, _ = expected_order(np.bincount(ci, minlength=n), K)
            if len(ci) == 0:
                want = np.arange(n, dtype=np.int32)
            assert np.array_equal(h.order(), want), K


def test_order_checkpoint_and_device_io():
    """Counters taken from a run in the caller's order resume in a reordered context (and
    the other way round) to the same fixpoint; device reads return the caller's order."""
    import torch
    rp, ci = graphgen.rmat(12, 50_000, seed=12)
    n = len(rp) - 1
    with hanf.HyperANF(0, hubs=0) as h:
        h.load(rp, ci).init(6, 77)
        full = h.run()
        final = h.registers()
        est_final = h.estimates()
    for src_hubs, dst_hubs in ((0, 400), (400, 0), (400, 50)):
        with hanf.HyperANF(0, hubs=src_hubs) as h:
            h.load(rp, ci).init(6, 77)
            h.step(3)
            regs = h.registers()
            prefix = h.nt()
        with hanf.HyperANF(0, hubs=dst_hubs) as h2:
            h2.load(rp, ci).init(6, 1)  # fixes m and the order; counters are replaced
            hanf.hanf_write_registers(h2.ctx, regs, 3, prefix)
            assert np.array_equal(h2.registers(), regs)
            nt = h2.run()
            assert np.array_equal(h2.registers(), final)
            assert np.array_equal(h2.estimates(), est_final)
            np.testing.assert_allclose(nt, full, rtol=RTOL, atol=0)
            assert len(nt) == len(full)
            out = torch.empty(n * 64, dtype=torch.uint8, device="cuda")
            h2.registers(out)
            assert np.array_equal(out.cpu().numpy().reshape(n, 64), final)
            order = torch.empty(n, dtype=torch.int32, device="cuda")
            h2.order(order)
            assert np.array_equal(order.cpu().numpy(), h2.order())
            # device counters in the caller's order resume too
            dregs = torch.from_numpy(regs.reshape(-1).copy()).cuda()
            hanf.hanf_write_registers(h2.ctx, dregs, 3, prefix)
            h2.run()
            assert np.array_equal(h2.registers(), final)


def test_transpose_loaded_after_the_order():
    """The order is chosen at the first initialisation (in-degrees counted from col_idx);
    a transposed graph loaded afterwards, in the caller's ids, is rewritten in that order
    and drives systolic passes to the oracle's fixpoint."""
    rp, ci = graphgen.rmat(13, 100_000, seed=63)
    b, seed = 5, 8
    nt_ref, T_ref, regs_ref = oracle.run(rp, ci, b, seed, want_regs=True)
    with hanf.HyperANF(0, hubs=500, systolic=1) as h:
        h.load(rp, ci).init(b, seed)
        order = h.order()
        h.load_transpose(*transpose_csr(rp, ci)).init(b, seed)
        assert np.array_equal(h.order(), order)
        nt = h.run()
        assert any(r["systolic"] for r in h.pass_log())
        assert np.array_equal(h.registers(), regs_ref)
        np.testing.assert_allclose(nt, nt_ref, rtol=RTOL, atol=0)
        assert len(nt) == T_ref + 1
        h.build_transpose().init(b, seed)  # built from the reordered graph
        nt2 = h.run()
        assert np.array_equal(h.registers(), regs_ref)
        np.testing.assert_allclose(nt2, nt_ref, rtol=RTOL, atol=0)


def test_auto_order_on_a_large_graph():
    """The default order (auto) on a symmetric R-MAT of 2^20 nodes at m = 64: the first run
    on an ingest keeps the caller's order (bit for bit the run with the order off); the
    second initialisation chooses 65536 hubs by definition, with the same registers,
    estimates, N_hat and T as the caller's order; a new ingest starts over. At m = 128 (a
    row per 128-byte line) auto keeps the caller's order."""
    import torch
    rp, ci = graphgen.rmat(20, 1 << 23, symmetric=True, seed=64)
    n = len(rp) - 1
    drp, dci = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    want, hubs = expected_order(np.diff(rp), 65536)
    _flush(f"[order] auto n={n} arcs={len(ci)} hubs={hubs}")
    with hanf.HyperANF(0) as a, hanf.HyperANF(0, hubs=0) as p:
        p.load(drp, dci).transpose_self().init(6, 5)
        npl = p.run()
        regs_p, est_p = p.registers(), p.estimates()
        a.load(drp, dci).transpose_self().init(6, 5)
        assert np.array_equal(a.order(), np.arange(n))
        assert np.array_equal(a.run(), npl)
        a.init(6, 5)  # the second run on this ingest: the order is chosen now
        assert np.array_equal(a.order(), want)
        na = a.run()
        assert len(na) == len(npl)
        np.testing.assert_allclose(na, npl, rtol=RTOL, atol=0)
        assert np.array_equal(a.registers(), regs_p)
        assert np.array_equal(a.estimates(), est_p)
        a.init(6, 6)  # kept for later runs
        assert np.array_equal(a.order(), want)
        a.load(drp, dci).transpose_self().init(6, 5)  # a new ingest
        assert np.array_equal(a.order(), np.arange(n))
        a.load(drp, dci).transpose_self().init(7, 5)
        a.init(7, 5)  # m = 128: rows fill a line, no order
        assert np.array_equal(a.order(), np.arange(n))


def test_order_errors():
    import ctypes

    import torch
    rp, ci = graphgen.erdos_renyi(100, 300, seed=1)
    with hanf.HyperANF(0) as h:
        for bad in (-2, 1 << 31):
            with pytest.raises(hanf.HanfError) as e:
                hanf.hanf_set_option(h.ctx, hanf.HANF_OPT_HUBS, bad)
            assert e.value.code == hanf.HANF_EINVAL
        with pytest.raises(hanf.HanfError) as e:
            h.order()
        assert e.value.code == hanf.HANF_ESTATE
        h.load(rp, ci).init(4, 1)
        lib = hanf.lib()
        buf = np.empty(100, np.int32)
        assert lib.hanf_read_order(h.ctx, buf.ctypes.data, 99, hanf.HANF_HOST_PTRS) == hanf.HANF_EINVAL
        assert lib.hanf_read_order(h.ctx, None, 100, hanf.HANF_HOST_PTRS) == hanf.HANF_EINVAL
        # a host buffer passed as device memory is refused before any kernel touches it
        assert lib.hanf_read_order(h.ctx, buf.ctypes.data, 100, hanf.HANF_DEVICE_PTRS) == hanf.HANF_EINVAL
        est = np.empty(100, np.float64)
        assert lib.hanf_read_estimates(h.ctx, est.ctypes.data, 100, hanf.HANF_DEVICE_PTRS) == hanf.HANF_EINVAL
        regs = np.empty(100 * 16, np.uint8)
        assert lib.hanf_read_registers(h.ctx, regs.ctypes.data, regs.size, hanf.HANF_DEVICE_PTRS) == hanf.HANF_EINVAL
        assert lib.hanf_read_registers(h.ctx, regs.ctypes.data, regs.size, 7) == hanf.HANF_EINVAL
        out = torch.empty(100, dtype=torch.int32, device="cuda")
        assert lib.hanf_read_order(h.ctx, ctypes.c_void_p(out.data_ptr()), 100, hanf.HANF_DEVICE_PTRS) == hanf.HANF_OK
        assert np.array_equal(out.cpu().numpy(), np.arange(100))
    with hanf.Batch(0) as bt:
        bt.load_graphs([(rp, ci)], 2).init(4, [1, 2])
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_read_order(bt.ctx, 100)
        assert e.value.code == hanf.HANF_EINVAL
        # batch reads refuse host buffers passed as device memory, too
        lib = hanf.lib()
        regs = np.empty(100 * 16, np.uint8)
        assert lib.hanf_batch_read_registers(bt.ctx, 0, regs.ctypes.data, regs.size,
                                             hanf.HANF_DEVICE_PTRS) == hanf.HANF_EINVAL
        est = np.empty(100, np.float64)
        assert lib.hanf_batch_read_estimates(bt.ctx, 0, est.ctypes.data, 100, hanf.HANF_DEVICE_PTRS) == hanf.HANF_EINVAL
        assert bt.registers(0).shape == (100, 16) and bt.estimates(0).shape == (100,)  # still usable
