"""Batched runs: every component (graph, seed) of a batch must equal its own run, register
for register, with N_hat within 1e-12 and the same fixpoint T."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_graphs():
    gs = [graphgen.erdos_renyi(200 + 37 * i, 5 * (200 + 37 * i), seed=60 + i) for i in range(6)]
    gs += [graphgen.rmat(9 + (i % 3), 3000 + 500 * i, seed=70 + i) for i in range(6)]
    gs += [graphgen.empty(1), graphgen.empty(70), graphgen.directed_path(150), graphgen.star_out(3000),
           graphgen.directed_cycle(65), graphgen.clique_path_clique(9, 5), graphgen.complete(40)]
    return gs


@pytest.mark.parametrize("b,S,per_row,fmt", [(4, 3, 0, 2), (6, 2, 0, 2), (8, 1, 0, 2), (6, 8, 0, 2), (8, 8, 0, 2),
                                             (6, 8, 0, 0), (8, 8, 0, 0), (4, 40, 0, 2), (6, 8, 1, 2), (6, 8, 2, 2),
                                             (5, 5, 4, 2)])
def test_batch_components_equal_their_runs(b, S, per_row, fmt):
    """Seeds side by side in node rows: 3 seeds (a row of 4, one empty), 8 seeds of m = 64
    (rows of 512 registers), m = 256 with 8 seeds (two copies of rows of 4), 40 seeds of
    m = 16 (two copies of rows of 32), and forced 1, 2 and 4 seeds per row. fmt: the register
    format option (2: chosen by row width, 5-bit for the rows of 512 registers and more; 0:
    one register per byte for those too)."""
    gs = _mixed_graphs()
    seeds = [1000 * g + 17 * s + 1 for g in range(len(gs)) for s in range(S)]
    _say(f"[batch] {len(gs)} graphs x {S} seeds, b={b}, seeds per row {per_row or 'auto'}, format {fmt}")
    with hanf.Batch(0, seeds_per_row=per_row, packed5=fmt) as bt:
        bt.load_graphs(gs, S).init(b, seeds)
        bt.run()
        T = bt.fixpoints()
        assert (T >= 0).all()
        for g, (rp, ci) in enumerate(gs):
            for s in range(S):
                c = g * S + s
                nt_ref, T_ref, regs_ref = oracle.run(rp, ci, b, seeds[c], want_regs=True)
                assert T[c] == T_ref, (g, s)
                np.testing.assert_allclose(bt.nt(c), nt_ref, rtol=1e-12, atol=0)
                assert np.array_equal(bt.registers(c), regs_ref), (g, s)
                assert np.array_equal(bt.estimates(c), oracle.sizes(regs_ref, b)), (g, s)
                st = bt.stats(c)
                with hanf.HyperANF(0) as h:
                    h.load(rp, ci).init(b, seeds[c])
                    nt_plain = h.run()
                    sp = h.stats()
                np.testing.assert_allclose(nt_plain, bt.nt(c), rtol=1e-12, atol=0)
                for k in ("ed", "ied", "avg_dist", "spid"):
                    if np.isnan(sp[k]):
                        assert np.isnan(st[k])
                    else:
                        assert st[k] == pytest.approx(sp[k], rel=1e-9, abs=1e-12), k


@pytest.mark.parametrize("sys_div,S,b,counting", [(1, 2, 6, 0), (4, 2, 6, 0), (1, 8, 8, 0), (2, 3, 4, 0),
                                                  (1, 8, 8, 1)])
def test_batch_systolic_components_equal_their_runs(sys_div, S, b, counting):
    """Systolic passes over a batch (transposed base built on the device by the bucket sort,
    or by per-node counters, laid out with the graph, also in two copies for 8 seeds of
    m = 256)."""
    gs = _mixed_graphs()
    seeds = [500 + 3 * c for c in range(len(gs) * S)]
    with hanf.Batch(0, systolic=sys_div, transpose_counting=counting) as bt:
        bt.load_graphs(gs, S).build_transpose().init(b, seeds)
        bt.run()
        assert any(r["systolic"] for r in bt.pass_log())
        T = bt.fixpoints()
        for g, (rp, ci) in enumerate(gs):
            for s in range(S):
                c = g * S + s
                nt_ref, T_ref, regs_ref = oracle.run(rp, ci, b, seeds[c], want_regs=True)
                assert T[c] == T_ref, (g, s)
                np.testing.assert_allclose(bt.nt(c), nt_ref, rtol=1e-12, atol=0)
                assert np.array_equal(bt.registers(c), regs_ref), (g, s)


@pytest.mark.parametrize("S,b", [(8, 6), (8, 8), (3, 4)])
def test_batch_symmetric_self_transpose(S, b):
    """Symmetric graphs declared their own transpose (no copy): systolic passes over rows of
    seeds, also laid out in two copies (8 seeds of m = 256)."""
    gs = [graphgen.rmat(9 + (i % 3), 2500 + 400 * i, symmetric=True, seed=90 + i) for i in range(6)]
    gs += [graphgen.complete(30), graphgen.empty(5)]
    seeds = [77 + 5 * c for c in range(len(gs) * S)]
    with hanf.Batch(0, systolic=1) as bt:
        bt.load_graphs(gs, S).transpose_self().init(b, seeds)
        bt.run()
        assert any(r["systolic"] for r in bt.pass_log())
        T = bt.fixpoints()
        for g, (rp, ci) in enumerate(gs):
            for s in range(S):
                c = g * S + s
                nt_ref, T_ref, regs_ref = oracle.run(rp, ci, b, seeds[c], want_regs=True)
                assert T[c] == T_ref, (g, s)
                np.testing.assert_allclose(bt.nt(c), nt_ref, rtol=1e-12, atol=0)
                assert np.array_equal(bt.registers(c), regs_ref), (g, s)


def test_batch_step_by_step_registers():
    """Registers of every component at every t, while other components still change."""
    gs = [graphgen.directed_path(40), graphgen.rmat(10, 6000, seed=3), graphgen.erdos_renyi(500, 1500, seed=4)]
    seeds = [11, 12, 13]
    refs = [[c.copy() for _, c, _ in oracle.run_steps(rp, ci, 6, sd)] for (rp, ci), sd in zip(gs, seeds)]
    with hanf.Batch(0) as bt:
        bt.load_graphs(gs, 1).init(6, seeds)
        for t in range(max(len(r) for r in refs) + 1):
            for g in range(3):
                want = refs[g][min(t, len(refs[g]) - 1)]
                assert np.array_equal(bt.registers(g), want), (t, g)
            st, _, _ = bt.step(1)
            if st == hanf.HANF_DONE:
                break
        assert list(bt.fixpoints()) == [len(r) - 1 for r in refs]


def test_batch_device_pointers():
    import torch
    gs = [graphgen.rmat(9, 2000, seed=5 + i) for i in range(5)]
    go, ao, rp, ci = hanf.Batch.union(gs)
    seeds = list(range(1, 11))
    with hanf.Batch(0) as a, hanf.Batch(0) as d:
        a.load_union(go, ao, rp, ci, 2).init(6, seeds)
        d.load_union(go, ao, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), 2).init(6, seeds)
        a.run()
        d.run()
        assert np.array_equal(a.fixpoints(), d.fixpoints())
        for c in range(10):
            assert np.array_equal(a.registers(c), d.registers(c))
            assert np.array_equal(a.nt(c), d.nt(c))


def test_batch_errors():
    rp, ci = graphgen.erdos_renyi(100, 300, seed=1)
    with hanf.HyperANF(0) as h:
        offs = np.array([0, 50, 100], np.int32)  # arcs cross the cut at 50
        aoff = np.array([0, rp[50], rp[100]], np.int32)
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_load_batch(h.ctx, offs, aoff, rp, ci, 2)
        assert e.value.code == hanf.HANF_EINVAL
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_load_batch(h.ctx, np.array([0, 0, 100], np.int32), np.array([0, 0, rp[100]], np.int32),
                                 rp, ci, 1)
        assert e.value.code == hanf.HANF_EINVAL
        with pytest.raises(hanf.HanfError) as e:  # arc offsets disagree with row_ptr
            hanf.hanf_load_batch(h.ctx, np.array([0, 100], np.int32), np.array([0, rp[100] - 1], np.int32),
                                 rp, ci, 1)
        assert e.value.code == hanf.HANF_EINVAL
        hanf.hanf_load_batch(h.ctx, np.array([0, 100], np.int32), np.array([0, rp[100]], np.int32), rp, ci, 2)
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_init_counters(h.ctx, 6, 1)
        assert e.value.code == hanf.HANF_EINVAL
        hanf.hanf_init_batch(h.ctx, 6, [1, 2])
        with pytest.raises(hanf.HanfError):
            hanf.hanf_batch_read_nt(h.ctx, 2)
        bad = ci.copy()
        bad[7] = 100  # out of its graph's ids
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_load_batch_list(h.ctx, [(rp, ci), (rp, bad)], 1)
        assert e.value.code == hanf.HANF_EINVAL
        badr = rp.copy()
        badr[3] = badr[4] + 1
        with pytest.raises(hanf.HanfError) as e:
            hanf.hanf_load_batch_list(h.ctx, [(badr, ci)], 1)
        assert e.value.code == hanf.HANF_EINVAL


@pytest.mark.timeout(900)
def test_batch_512_graphs_8_seeds():
    """The many-graph workload at full size: 512 graphs (lognormal 2^8..2^16 nodes, half
    Erdos-Renyi with 8n arcs, half R-MAT with 16n arcs) x 8 seeds, 64 registers. Every
    component's T and N_hat against its plain run; registers and N_hat of 48 sampled
    components against the oracle."""
    gs = graphgen.batch_graphs()
    S, b = 8, 6
    seeds = [(g << 8) + s + 1 for g in range(len(gs)) for s in range(S)]
    _say(f"[batch512] nodes={sum(len(r) - 1 for r, _ in gs)} arcs={sum(len(c) for _, c in gs)}")
    with hanf.Batch(0) as bt:
        bt.load_graphs(gs, S).init(b, seeds)
        bt.run()
        T = bt.fixpoints()
        assert (T >= 0).all()
        rng = np.random.default_rng(5)
        sample = set(rng.choice(len(gs) * S, 48, replace=False).tolist())
        with hanf.HyperANF(0) as h:
            for g, (rp, ci) in enumerate(gs):
                h.load(rp, ci)
                for s in range(S):
                    c = g * S + s
                    h.init(b, seeds[c])
                    nt_plain = h.run()
                    assert len(nt_plain) == T[c] + 1, c
                    np.testing.assert_allclose(bt.nt(c), nt_plain, rtol=1e-12, atol=0)
                    if c in sample:
                        nt_ref, T_ref, regs_ref = oracle.run(rp, ci, b, seeds[c], want_regs=True)
                        assert T_ref == T[c]
                        np.testing.assert_allclose(bt.nt(c), nt_ref, rtol=1e-12, atol=0)
                        assert np.array_equal(bt.registers(c), regs_ref)
                if g % 64 == 0:
                    _say(f"[batch512] graph {g} ok")


@pytest.mark.parametrize("distinct", [False, True])
def test_batch_seed_statistics(distinct):
    """The statistics of many runs per graph (Section 6's protocol): every component's
    hanf_stats values from the one-launch hanf_batch_stats_all equal the oracle's on its own
    N_hat (Sections 4-5 and Algorithm 3 with eps), and seed_summary's mean and standard
    deviation over the seeds equal those of the oracle's per-seed values."""
    from oracle import stats as ostats
    gs = [graphgen.rmat(10, 8000, seed=3), graphgen.erdos_renyi(900, 4000, seed=5),
          graphgen.clique_path_clique(12, 6), graphgen.directed_cycle(80), graphgen.empty(5)]
    S, b, eps = 6, 6, 0.05
    seeds = [31 * c + 7 for c in range(len(gs) * S)]
    keys = ("ed", "ied", "avg_dist", "spid")
    with hanf.Batch(0) as bt:
        bt.load_graphs(gs, S).init(b, seeds)
        bt.run()
        st = bt.stats_all(0.9, eps, distinct)
        summ = bt.seed_summary(0.9, distinct)  # computed by the library (hanf_batch_seed_summary)
    ref = {k: np.zeros((len(gs), S)) for k in keys}
    for g, (rp, ci) in enumerate(gs):
        for s in range(S):
            c = g * S + s
            nt_ref, T_ref, _ = oracle.run(rp, ci, b, seeds[c])
            r = ostats.stats(list(nt_ref), 0.9, distinct)
            assert st["T"][c] == T_ref == r["T"]
            for k in keys + ("var", "n_max"):
                if np.isnan(r[k]):
                    assert np.isnan(st[k][c]), (g, s, k)
                else:
                    assert st[k][c] == pytest.approx(r[k], rel=1e-9, abs=1e-12), (g, s, k)
            lo, hi = ostats.diameter_interval(list(nt_ref), eps, 0.9)
            assert st["d_lo"][c] == (-1 if lo is None else lo), (g, s)
            assert st["d_hi"][c] == (-1 if hi is None else hi), (g, s)
            for k in keys:
                ref[k][g, s] = r[k]
    assert (summ["runs"] == S).all()
    for k in keys:
        np.testing.assert_allclose(summ[k + "_mean"], ref[k].mean(axis=1), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(summ[k + "_std"], ref[k].std(axis=1, ddof=1), rtol=1e-7, atol=1e-12)


def test_seed_summary_of_single_runs():
    """With one run per graph the means are that run's statistics and the sample standard
    deviations are undefined (NaN)."""
    gs = [graphgen.rmat(9, 3000, seed=8), graphgen.directed_cycle(40)]
    with hanf.Batch(0) as bt:
        bt.load_graphs(gs, 1).init(6, [5, 6])
        bt.run()
        st = bt.stats_all(0.9)
        summ = bt.seed_summary(0.9)
    for k in ("ed", "ied", "avg_dist", "spid"):
        assert np.array_equal(summ[k + "_mean"], st[k])
        assert np.isnan(summ[k + "_std"]).all()
