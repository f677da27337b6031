"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Registers must be byte-identical at every iteration checked, N_hat(t) within 1e-12
relative (FP64 sums in a different order), the fixpoint iteration T equal, and the
per-pass work counters (counters changed, successor unions) exactly the oracle's.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
from oracle import stats as ostats

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")

RTOL = 1e-12


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def transpose_csr(rp, ci):
    """Predecessor lists (CSR) of a CSR graph, by a stable sort on the target."""
    n = len(rp) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    order = np.argsort(ci, kind="stable")
    trp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(ci, minlength=n), out=trp[1:])
    return trp.astype(np.int32), src[order].astype(np.int32)


def _load(h, rp, ci, transpose):
    """Loads the graph and, for systolic passes, its transpose: 'build' on the device,
    'host' from numpy, 'self' (symmetric graph: its own device arrays)."""
    if transpose == "self":
        import torch
        drp, dci = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
        h.load(drp, dci).load_transpose(drp, dci)
    elif transpose == "declared":
        h.load(rp, ci).transpose_self()
    else:
        h.load(rp, ci)
        if transpose == "build":
            h.build_transpose()
        elif transpose == "host":
            h.load_transpose(*transpose_csr(rp, ci))
    return h


def near_window(b, packed=False):
    """W of the pass records' arcs_near: the rows 4 MiB holds, halved (one counter per row)."""
    m = 1 << b
    row = (m // 64) * 40 if packed else m
    return (2 << 20) // row


def step_parity(rp, ci, b, seed, check_every=1, transpose=None, **opts):
    """Runs GPU and oracle side by side one pass at a time; checks everything."""
    n = len(rp) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    W = near_window(b, opts.get("packed5", 0) == 1 and b >= 6)
    near_arc = np.abs(np.asarray(ci, np.int64) - src) < W  # in the caller's ids
    check_near = opts.get("hubs", 0) <= 0  # (a chosen node order renumbers the ids)
    _flush(f"[parity] n={n} arcs={len(ci)} b={b} seed={seed} transpose={transpose} opts={opts}")
    ref = oracle.run_steps(rp, ci, b, seed, skip_unmodified=True)
    mod = np.ones(n, np.uint8)
    prev_changed = 0
    # without a transposed graph, systolic passes can take their marks from a forward scan of
    # the successor lists (HANF_OPT_FORWARD, off by default)
    forward = not transpose and opts.get("forward", 0)
    sys_div = opts.get("systolic", 4) if (transpose or forward) else 0
    with hanf.HyperANF(0, **opts) as h:
        _load(h, rp, ci, transpose).init(b, seed)
        nts = []
        T = None
        for t, c, s in ref:
            nts.append(s)
            if t % check_every == 0:
                got = h.registers()
                assert np.array_equal(got, c), f"registers differ at t={t}"
                # every node's estimate bit for bit (the per-node arithmetic of the reduction)
                assert np.array_equal(h.estimates(), oracle.sizes(c, b)), f"estimates differ at t={t}"
            # the oracle's next pass, for the exact work counters
            _, mod_out, changed, maxed = oracle.step(rp, ci, b, c, mod)
            st, steps, ch_last = h.step(1)
            assert steps == 1
            log = h.pass_log()[-1]
            assert log["changed"] == changed, (t, log, changed)
            if log["gather_all"]:
                assert log["arcs_gathered"] == log["arcs_scanned"], (t, log)
            else:
                assert log["arcs_gathered"] == maxed, (t, log, maxed)
            if check_near and log["arcs_near"] >= 0:  # (counted by the instrumented kernels)
                # gathered successors within W ids of their node
                gathered = near_arc if log["gather_all"] else near_arc & (mod[ci] != 0)
                assert log["arcs_near"] == int(np.count_nonzero(gathered)), (t, log)
            elif not (opts.get("stage") or opts.get("count_near")):
                assert log["arcs_near"] == -1, (t, log)
            if log["flag_summary"]:  # read only by frontier passes
                assert not log["gather_all"] and not log["systolic"], (t, log)
            assert log["gather_all"] == (t == 0 or not opts.get("frontier", 1)
                                         or (opts.get("dense_switch", 4) > 0
                                             and prev_changed >= max(1, n // opts.get("dense_switch", 4))))
            # systolic after a pass that changed < n / sys_div counters, unless signals through
            # the transpose would follow more than arcs / 16 arcs (a forward scan has no such
            # fallback: it has read every arc already)
            want_sys = (not log["gather_all"] and opts.get("frontier", 1) and sys_div > 0
                        and prev_changed * sys_div < n and (forward or maxed * 16 <= len(ci)))
            assert log["systolic"] == (0 if not want_sys else 2 if forward else 1), (t, log)
            if log["systolic"]:
                # every arc into a counter modified by the previous pass is signalled once:
                # the same arcs the frontier gathers (counted from the other end through the
                # transpose)
                assert log["arcs_signalled"] == maxed, (t, log, maxed)
                # and the union step reads exactly those arcs (each node's list of signalled
                # successors), not the whole successor lists of the signalled nodes
                assert log["arcs_scanned"] == log["arcs_gathered"] == maxed, (t, log, maxed)
            prev_changed = changed
            assert ch_last == changed
            mod = mod_out
            T = t
            if changed == 0:
                assert st == hanf.HANF_DONE
            else:
                assert st == hanf.HANF_OK
        got_nt = h.nt()
        want = np.array(nts)
        assert len(got_nt) == len(want) == T + 1
        np.testing.assert_allclose(got_nt, want, rtol=RTOL, atol=0)
        return h.stats(), want


def test_bytemax_exhaustive():
    """The packed register max equals np.maximum for every pair of byte values < 128 in
    every byte position."""
    import torch
    vals = np.arange(128, dtype=np.uint32)
    X, Y = np.meshgrid(vals, vals, indexing="ij")
    X = X.ravel()
    Y = Y.ravel()
    rng = np.random.default_rng(0)
    for pos in range(4):
        ox = rng.integers(0, 128, (X.size, 4)).astype(np.uint32)
        oy = rng.integers(0, 128, (X.size, 4)).astype(np.uint32)
        ox[:, pos] = X
        oy[:, pos] = Y
        wx = (ox[:, 0] | (ox[:, 1] << 8) | (ox[:, 2] << 16) | (ox[:, 3] << 24)).astype(np.uint32)
        wy = (oy[:, 0] | (oy[:, 1] << 8) | (oy[:, 2] << 16) | (oy[:, 3] << 24)).astype(np.uint32)
        want = np.maximum(ox, oy)
        want_w = (want[:, 0] | (want[:, 1] << 8) | (want[:, 2] << 16) | (want[:, 3] << 24)).astype(np.uint32)
        tx = torch.from_numpy(wx.view(np.int32)).cuda()
        ty = torch.from_numpy(wy.view(np.int32)).cuda()
        to = torch.empty_like(tx)
        hanf.hanf_bytemax_words(0, tx, ty, to)
        assert np.array_equal(to.cpu().numpy().view(np.uint32), want_w)


@pytest.mark.parametrize("from_first", [0, 1])
def test_gather_accumulator_exhaustive(from_first):
    """The union step's gather accumulator (packed 16-bit maxima of the words and of the
    words shifted up a byte, put together by a byte permute) equals np.maximum for every
    pair of byte values 0..255 in every byte position of a 16-byte lane, the other bytes
    random; and over random groups of 2..9 lanes."""
    import torch
    vals = np.arange(256, dtype=np.uint8)
    X, Y = np.meshgrid(vals, vals, indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    rng = np.random.default_rng(1 + from_first)
    for pos in range(16):
        a = rng.integers(0, 256, (X.size, 16), dtype=np.uint8)
        b = rng.integers(0, 256, (X.size, 16), dtype=np.uint8)
        a[:, pos], b[:, pos] = X, Y
        x = np.stack([a, b], axis=1)  # groups of k = 2 lanes
        out = torch.empty(X.size * 4, dtype=torch.int32, device="cuda")
        hanf.hanf_gathermax_lanes(0, torch.from_numpy(x.reshape(-1).view(np.int32).copy()).cuda(), 2, from_first, out)
        assert np.array_equal(out.cpu().numpy().view(np.uint8).reshape(-1, 16), np.maximum(a, b)), pos
    for k in range(2, 10):
        x = rng.integers(0, 256, (4096, k, 16), dtype=np.uint8)
        out = torch.empty(4096 * 4, dtype=torch.int32, device="cuda")
        hanf.hanf_gathermax_lanes(0, torch.from_numpy(x.reshape(-1).view(np.int32).copy()).cuda(), k, from_first, out)
        assert np.array_equal(out.cpu().numpy().view(np.uint8).reshape(-1, 16), x.max(axis=1)), k


def test_rmat14_every_iteration():
    """Directed R-MAT scale 14, 262,144 arcs, 16 registers, hash seed 1: registers at every
    t, N_hat, T, work counters; statistics against the oracle's."""
    rp, ci = graphgen.rmat(14, 262_144, seed=14)
    s, want = step_parity(rp, ci, 4, 1)
    ref = ostats.stats(list(want))
    for k in ("ed", "ied", "avg_dist", "var", "spid", "n_max"):
        assert s[k] == pytest.approx(ref[k], rel=1e-10), k
    assert s["T"] == ref["T"]


@pytest.mark.parametrize("b", [4, 5, 6, 7, 8])
def test_register_counts_with_heavy_rows(b):
    """Every m, on a graph whose high-degree rows are split over several wavefront chunks."""
    rp, ci = graphgen.rmat(12, 60_000, seed=40 + b)
    deg = np.diff(rp)
    assert deg.max() > 4 * 150
    step_parity(rp, ci, b, 1000 + b, chunk_arcs=150)
    step_parity(rp, ci, b, 2000 + b)


def test_frontier_off_identical():
    """Dense passes (no modified-counter skipping) give identical counters at every t."""
    rp, ci = graphgen.rmat(11, 20_000, seed=5)
    step_parity(rp, ci, 6, 3, frontier=0)


@pytest.mark.parametrize("opts", [dict(light_max=4, chunk_arcs=16), dict(light_max=1000, chunk_arcs=4096),
                                  dict(tile_nodes=16, unroll=2), dict(unroll=8, tile_nodes=256),
                                  dict(batch=1), dict(dense_switch=0), dict(dense_switch=1000000)])
def test_schedules_identical(opts):
    """Any work schedule gives the same counters (max is order-free)."""
    rp, ci = graphgen.rmat(12, 40_000, seed=6)
    step_parity(rp, ci, 6, 17, **opts)


@pytest.mark.parametrize("transpose,opts", [("build", {}), ("host", {}), ("build", dict(transpose_counting=1))])
def test_systolic_rmat14_every_iteration(transpose, opts):
    """Systolic passes (Section 3.3): same registers, N_hat and work counters at every t;
    the arcs signalled in a systolic pass are exactly the arcs into modified counters. The
    transposed graph comes from the bucket sort, the host, or the per-node counting build
    that graphs of more than 2^26 nodes use."""
    rp, ci = graphgen.rmat(14, 262_144, seed=14)
    step_parity(rp, ci, 4, 1, transpose=transpose, **opts)


@pytest.mark.parametrize("opts", [dict(systolic=1), dict(systolic=1, dense_switch=0),
                                  dict(systolic=2, chunk_arcs=150, light_max=8), dict(systolic=1000000),
                                  dict(systolic=0), dict(systolic=1, unroll=8, tile_nodes=256),
                                  dict(systolic=1, frontier=0), dict(systolic=1, batch=1),
                                  dict(systolic=1, union_policy=1), dict(systolic=1, union_policy=2),
                                  dict(systolic=0, union_policy=2), dict(frontier=0, union_policy=2),
                                  dict(systolic=1, union_policy=2, chunk_arcs=150, light_max=8, unroll=2),
                                  dict(systolic=1, union_policy=2, dense_switch=0, tile_nodes=16)])
def test_systolic_schedules_identical(opts):
    """Every schedule and either union kernel (one wavefront per work unit, or the
    persistent kernel that skips idle units) in every kind of pass."""
    rp, ci = graphgen.rmat(12, 40_000, seed=6)
    step_parity(rp, ci, 6, 17, transpose="build", **opts)


@pytest.mark.parametrize("b", [4, 6, 8])
def test_systolic_symmetric_self_transpose(b):
    """A symmetric graph is its own transpose: its device arrays serve both roles."""
    rp, ci = graphgen.rmat(13, 60_000, symmetric=True, seed=30 + b)
    step_parity(rp, ci, b, 7, transpose="self")
    step_parity(rp, ci, b, 8, transpose="self", dense_switch=0, systolic=1)
    step_parity(rp, ci, b, 9, transpose="declared", systolic=2)


@pytest.mark.parametrize("name,b", [("web", 6), ("rmat", 4), ("web15", 8)])
def test_flag_summary_passes(name, b):
    """Frontier passes after one that modified counters in few groups of 1024 nodes read the
    flag summary first; those runs still equal the oracle's at every t (registers, the
    gathered-arc counts, N_hat), and the summary is used in at least one pass."""
    graphs = {"web": lambda: graphgen.web(1 << 16, seed=61, keep_kind=True),
              "rmat": lambda: graphgen.rmat(15, 1 << 19, seed=62),
              "web15": lambda: graphgen.web(1 << 15, host_mean=300.0, seed=63, keep_kind=True)}
    rp, ci = graphs[name]()
    step_parity(rp, ci, b, 13)
    with hanf.HyperANF(0) as h:
        h.load(rp, ci).init(b, 13)
        h.run()
        log = h.pass_log()
    used = [t for t, r in enumerate(log) if r["flag_summary"]]
    _flush(f"[summary] {name}: passes {len(log)}, summary read in passes {used}")
    assert used, [(r["gather_all"], r["changed"]) for r in log]


def test_transpose_errors():
    rp, ci = graphgen.erdos_renyi(100, 300, seed=1)
    trp, tci = transpose_csr(rp, ci)
    with hanf.HyperANF(0) as h:
        with pytest.raises(hanf.HanfError) as e:
            h.build_transpose()
        assert e.value.code == hanf.HANF_ESTATE
        h.load(rp, ci)
        with pytest.raises(hanf.HanfError) as e:  # not the graph's arc count
            h.load_transpose(trp, tci[:-1])
        assert e.value.code == hanf.HANF_EINVAL
        bad = tci.copy()
        bad[3] = 100
        with pytest.raises(hanf.HanfError) as e:
            h.load_transpose(trp, bad)
        assert e.value.code == hanf.HANF_EINVAL
        badr = trp.copy()
        badr[5] = badr[6] + 1
        with pytest.raises(hanf.HanfError) as e:
            h.load_transpose(badr, tci)
        assert e.value.code == hanf.HANF_EINVAL
        # loading a transpose discards the run in progress
        h.init(6, 1)
        h.load_transpose(trp, tci)
        with pytest.raises(hanf.HanfError) as e:
            h.step(1)
        assert e.value.code == hanf.HANF_ESTATE
        h.init(6, 1)
        nt = h.run()
        assert any(r["systolic"] for r in h.pass_log())
    want, _, _ = oracle.run(rp, ci, 6, 1)
    np.testing.assert_allclose(nt, want, rtol=RTOL, atol=0)
    with hanf.Batch(0) as bt:
        bt.load_graphs([(rp, ci)], 2)
        with pytest.raises(hanf.HanfError) as e:
            bt.load_transpose(trp, tci)
        assert e.value.code == hanf.HANF_EINVAL


@pytest.mark.parametrize("kind", ["loaded", "declared", "declared_batch"])
def test_mismatched_transpose_stays_in_bounds(kind):
    """A transposed graph that is not the graph's transpose has the right shape, so it is
    accepted; its results are undefined, but the run must end normally. Here nodes with one
    successor (or none) are named as predecessors of thousands of nodes: a systolic pass
    signals them far more often than they have arcs, and the surplus must be dropped, not
    read. 'declared' calls a non-symmetric graph symmetric, which does the same to nodes
    whose in-degree is above their out-degree. Afterwards the same context runs the graph
    with its true transpose, and that run equals the oracle's."""
    rp, ci = graphgen.rmat(12, 40_000, seed=6)
    n = len(rp) - 1
    deg = np.diff(rp)
    trp, tci = transpose_csr(rp, ci)
    few = np.flatnonzero(deg <= 1)[:4]  # out-degree 0 or 1
    assert len(few) == 4 and (deg[few] == 0).any() and (deg[few] == 1).any()
    bad = tci.copy()
    bad[: len(bad) // 2] = np.resize(few, len(bad) // 2)
    assert np.bincount(bad, minlength=n)[few].min() > 1000
    b, seed = 6, 17
    nt_o, T_o, regs_o = oracle.run(rp, ci, b, seed, want_regs=True)
    _flush(f"[mismatched transpose] kind={kind} n={n} arcs={len(ci)} b={b} seed={seed}")
    if kind == "declared_batch":
        with hanf.Batch(0, systolic=1) as bt:
            bt.load_graphs([(rp, ci)], 1).transpose_self().init(b, [seed])
            bt.run()
            assert any(r["systolic"] for r in bt.pass_log())
            assert bt.registers(0).max() <= 31
            assert np.isfinite(bt.nt(0)).all()
        return
    with hanf.HyperANF(0, systolic=1) as h:
        h.load(rp, ci)
        if kind == "loaded":
            h.load_transpose(trp, bad)
        else:
            h.transpose_self()
        h.init(b, seed)
        st = h.step(0)[0]
        assert st == hanf.HANF_DONE
        log = h.pass_log()
        assert any(r["systolic"] and r["arcs_signalled"] > 0 for r in log), log
        assert h.registers().max() <= 31 and np.isfinite(h.nt()).all()
        h.load(rp, ci).load_transpose(trp, tci).init(b, seed)
        nt = h.run()
        assert any(r["systolic"] for r in h.pass_log())
        assert len(nt) == T_o + 1
        np.testing.assert_allclose(nt, nt_o, rtol=RTOL, atol=0)
        assert np.array_equal(h.registers(), regs_o)


@pytest.mark.parametrize("name", ["single", "empty100", "star_out", "star_in", "cycle", "path",
                                  "complete", "cpc", "loops_dups"])
def test_edge_graphs(name):
    if name == "single":
        g = graphgen.empty(1)
    elif name == "empty100":
        g = graphgen.empty(100)
    elif name == "star_out":
        g = graphgen.star_out(100_001)
    elif name == "star_in":
        g = graphgen.star_in(30_000)
    elif name == "cycle":
        g = graphgen.directed_cycle(300)
    elif name == "path":
        g = graphgen.directed_path(700)
    elif name == "complete":
        g = graphgen.complete(120)
    elif name == "cpc":
        g = graphgen.clique_path_clique(40, 7)
    else:
        rp, ci = graphgen.erdos_renyi(3000, 20_000, seed=8)
        n = len(rp) - 1
        arcs = [(u, int(w)) for u in range(n) for w in ci[rp[u]:rp[u + 1]]]
        arcs += arcs[::7] + [(u, u) for u in range(0, n, 5)]
        g = graphgen.from_arcs(n, arcs)
    for b in (4, 7):
        step_parity(*g, b, 99)
        step_parity(*g, b, 98, transpose="build", systolic=1)
        step_parity(*g, b, 97, transpose="build", systolic=1, union_policy=2, chunk_arcs=256)


def test_device_pointers_match_host():
    import torch
    rp, ci = graphgen.rmat(13, 100_000, seed=9)
    trp = torch.from_numpy(rp).cuda()
    tci = torch.from_numpy(ci).cuda()
    with hanf.HyperANF(0) as a, hanf.HyperANF(0) as d:
        a.load(rp, ci).init(6, 5)
        d.load(trp, tci).init(6, 5)
        na = a.run()
        nd = d.run()
        assert np.array_equal(na, nd)
        assert np.array_equal(a.registers(), d.registers())
        out = torch.empty(d.n * 64, dtype=torch.uint8, device="cuda")
        d.registers(out)
        assert np.array_equal(out.cpu().numpy().reshape(d.n, 64), a.registers())


def test_checkpoint_resume_identical():
    rp, ci = graphgen.rmat(12, 50_000, seed=12)
    with hanf.HyperANF(0) as h:
        h.load(rp, ci).init(5, 77)
        full = h.run()
        final = h.registers()
    with hanf.HyperANF(0) as h:
        h.load(rp, ci).init(5, 77)
        h.step(3)
        regs = h.registers()
        prefix = h.nt()
    with hanf.HyperANF(0) as h2:
        h2.load(rp, ci).init(5, 1)  # fixes m; counters are replaced
        hanf.hanf_write_registers(h2.ctx, regs, 3, prefix)
        nt = h2.run()
        assert np.array_equal(h2.registers(), final)
        np.testing.assert_allclose(nt, full, rtol=RTOL, atol=0)
        assert len(nt) == len(full)


def test_errors():
    rp, ci = graphgen.rmat(8, 1000, seed=1)
    with hanf.HyperANF(0) as h:
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_iterate(h.ctx)
        assert e.value.code == hanf.HANF_ESTATE
        bad = rp.copy()
        bad[0] = 1
        with pytest.raises(hanf.HanfError) as e:
            h.load(bad, ci)
        assert e.value.code == hanf.HANF_EINVAL
        bad = rp.copy()
        bad[5] = bad[6] + 5  # row_ptr decreases from 5 to 6
        with pytest.raises(hanf.HanfError) as e:
            h.load(bad, ci)
        assert e.value.code == hanf.HANF_EINVAL
        bad = rp.copy()
        bad[-1] += 1  # row_ptr[n] != arcs
        with pytest.raises(hanf.HanfError) as e:
            h.load(bad, ci)
        assert e.value.code == hanf.HANF_EINVAL
        badc = ci.copy()
        badc[10] = len(rp) - 1
        with pytest.raises(hanf.HanfError):
            h.load(rp, badc)
        badc[10] = -1
        with pytest.raises(hanf.HanfError):
            h.load(rp, badc)
        # sizes beyond HANF_MAX_NODES / HANF_MAX_ARCS are refused before the arrays are read
        lib = hanf.lib()
        prp, pci = rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p)
        for n_bad, arcs_bad in ((hanf.HANF_MAX_NODES + 1, len(ci)), (len(rp) - 1, hanf.HANF_MAX_ARCS + 1)):
            assert lib.hanf_load_csr(h.ctx, n_bad, arcs_bad, prp, pci, hanf.HANF_HOST_PTRS) == hanf.HANF_EINVAL
            assert "HANF_MAX" in hanf.hanf_last_error(h.ctx)
        h.load(rp, ci)
        for b in (3, 9):
            with pytest.raises(hanf.HanfError) as e:
                h.init(b, 1)
            assert e.value.code == hanf.HANF_EINVAL
        h.init(6, 1)
        # argument errors of a resume leave the run in progress untouched
        h.step(2)
        regs2, nt2 = h.registers().copy(), h.nt()
        pre = np.asarray(nt2, np.float64)
        pin, ppre = regs2.ctypes.data_as(ctypes.c_void_p), pre.ctypes.data_as(ctypes.c_void_p)
        for bytes_, t_, len_, flags_ in ((regs2.size - 1, 2, 3, 0), (regs2.size, -1, 0, 0),
                                         (regs2.size, 2, 2, 0), (regs2.size, 2, 3, 7)):
            assert lib.hanf_write_registers(h.ctx, pin, bytes_, t_, ppre, len_, flags_) == hanf.HANF_EINVAL
        assert lib.hanf_write_registers(h.ctx, pin, regs2.size, 2, ppre, 3,
                                        hanf.HANF_DEVICE_PTRS) == hanf.HANF_EINVAL  # host memory
        h.step(1)
        want = [x for _, _, x in oracle.run_steps(rp, ci, 6, 1)][:4]
        got = h.nt()
        assert len(want) == 4 and len(got) >= 4
        np.testing.assert_allclose(got[:4], want, rtol=RTOL, atol=0)
        bad_regs = np.full((len(rp) - 1, 64), 32, np.uint8)
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_write_registers(h.ctx, bad_regs, 0, [1.0])
        assert e.value.code == hanf.HANF_EINVAL
    # pass cap
    rp, ci = graphgen.directed_path(200)
    with hanf.HyperANF(0, max_passes=5) as h:
        h.load(rp, ci).init(6, 1)
        with pytest.raises(hanf.HanfError) as e:
            h.run()
        assert e.value.code == hanf.HANF_EMAXITER
        assert len(h.nt()) == 6


def test_forced_allocation_failure():
    rp, ci = graphgen.rmat(8, 1000, seed=1)
    for k in (2, 5, 9):
        os.environ["HANF_TEST_FAIL_ALLOC"] = str(k)
        try:
            h = hanf.HyperANF(0)
        finally:
            del os.environ["HANF_TEST_FAIL_ALLOC"]
        with pytest.raises(hanf.HanfError) as e:
            h.load(rp, ci).init(6, 1)
        assert e.value.code == hanf.HANF_ENOMEM
        h.close()


@pytest.mark.parametrize("case", ["rmat14", "web", "star", "cycle", "packed", "persistent"])
def test_forward_scan_systolic_every_iteration(case):
    """Systolic passes without a transposed graph (HANF_OPT_FORWARD = 1): the nodes to
    recompute are found by a forward scan of the successor lists. Registers, estimates,
    N_hat, T and the work counters equal the oracle's at every t; each systolic pass's
    signalled arcs equal the oracle's count of arcs into modified counters."""
    if case == "rmat14":
        rp, ci = graphgen.workload_graph(graphgen.WORKLOADS["rmat14"])
        step_parity(rp, ci, 4, 1, forward=1)
    elif case == "web":
        rp, ci = graphgen.web(1 << 14, host_mean=100.0, seed=61, keep_kind=True)
        step_parity(rp, ci, 7, 2, forward=1, systolic=2)
    elif case == "star":  # one heavy row split into chunks
        rp, ci = graphgen.star_out(20000)
        step_parity(rp, ci, 6, 3, forward=1, systolic=1)
    elif case == "cycle":
        rp, ci = graphgen.directed_cycle(700)
        step_parity(rp, ci, 5, 4, forward=1)
    elif case == "packed":
        rp, ci = graphgen.rmat(12, 50000, seed=62)
        step_parity(rp, ci, 6, 5, forward=1, packed5=1)
    else:  # every pass through the persistent kernel over listed units
        rp, ci = graphgen.rmat(12, 50000, seed=63)
        step_parity(rp, ci, 6, 6, forward=1, union_policy=2, chunk_arcs=256)
