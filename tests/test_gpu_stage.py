"""Light tiles staged in LDS (HANF_OPT_STAGE): in passes over every successor, a tile's
counters are copied to LDS and successors inside the tile's id range are maximised in from
there. The results must not change: registers byte-equal to the oracle's at every t, every
node's estimate bit for bit, N_hat(t) within 1e-12, T and the work counters exactly the
oracle's (the step parity of test_gpu_parity.py), for every register count the staged
kernels serve, on graphs with and without locality, ragged last tiles and heavy rows."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

hanf = pytest.importorskip("paper_1011_5599_amd")
from test_gpu_parity import step_parity  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


GRAPHS = {
    "web_2^14": lambda: graphgen.web(1 << 14, host_mean=200.0, seed=31, keep_kind=True),
    "web_ragged": lambda: graphgen.web(3001, host_mean=50.0, deg_mean=8.0, seed=32, keep_kind=True),
    "rmat_12": lambda: graphgen.rmat(12, 40_000, seed=33),
    "cycle_1000": lambda: graphgen.directed_cycle(1000),
    "path_130": lambda: graphgen.directed_path(130),
    "star_out_3000": lambda: graphgen.star_out(3000),
    "clique_path_clique": lambda: graphgen.clique_path_clique(20, 37),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("b", [4, 6, 7, 8])
@pytest.mark.parametrize("mode", ["stage", "count_near"])
def test_staged_every_iteration(name, b, mode):
    """mode stage: staged tiles (near successors counted too); count_near: the instrumented
    kernels without staging. step_parity also checks every pass's near count against numpy."""
    rp, ci = GRAPHS[name]()
    step_parity(rp, ci, b, seed=5 + b, **{mode: 1})
    with hanf.HyperANF(0, **{mode: 1}) as h:
        h.load(rp, ci).init(b, 5 + b)
        h.run()
        log = h.pass_log()
    dense = [r for r in log if r["gather_all"]]
    assert dense and all(0 <= r["arcs_local"] <= r["arcs_near"] <= r["arcs_gathered"] for r in log)
    assert all(r["arcs_local"] == 0 for r in log if not r["gather_all"])  # staging only there
    if mode == "count_near":
        assert all(r["arcs_local"] == 0 for r in log)
    elif name.startswith("web") or name in ("cycle_1000", "path_130"):
        assert dense[0]["arcs_local"] > 0, dense[0]


@pytest.mark.parametrize("b", [6, 7])
def test_staged_with_systolic_passes(b):
    """Staged dense passes followed by systolic ones (transposed graph built on the device)."""
    rp, ci = graphgen.web(1 << 13, host_mean=100.0, seed=34, keep_kind=True)
    step_parity(rp, ci, b, seed=3, transpose="build", stage=1)


def test_staging_is_off_by_default_and_changes_nothing():
    """Staging is off by default; forced on, a web-like graph (its intra-host arcs mostly
    inside a tile) reads a third or more of its first pass's successors from LDS, R-MAT ids
    none beyond their own tile; N_hat (same sums, same order), registers and the gathered
    counts are identical either way, and equal the oracle's."""
    cases = {"web": graphgen.web(1 << 16, seed=35, keep_kind=True),
             "rmat": graphgen.rmat(16, 1 << 20, seed=36)}
    for name, (rp, ci) in cases.items():
        b, seed = 7, 9
        out = {}
        for stage in (None, 0, 1):
            opts = {} if stage is None else {"stage": stage}
            with hanf.HyperANF(0, **opts) as h:
                h.load(rp, ci).init(b, seed)
                nt = h.run()
                out[stage] = (nt, h.registers().copy(), h.pass_log())
        first = out[1][2][0]
        _say(f"[stage] {name}: first pass local {first['arcs_local']} near {first['arcs_near']} of "
             f"{first['arcs_gathered']}")
        for stage in (None, 1):
            assert np.array_equal(out[stage][0], out[0][0])  # same sums in the same order
            assert np.array_equal(out[stage][1], out[0][1])
            assert [r["arcs_gathered"] for r in out[stage][2]] == [r["arcs_gathered"] for r in out[0][2]]
        assert all(r["arcs_local"] == 0 and r["arcs_near"] == -1 for r in out[None][2] + out[0][2])
        if name == "web":  # (the intra-host arcs of a node of ~20 reach beyond +-16 ids)
            assert first["arcs_local"] > 0.3 * first["arcs_gathered"], first
        assert first["arcs_local"] <= first["arcs_near"] <= first["arcs_gathered"]
        nt_o, T_o, _ = oracle.run(rp, ci, b, seed, nthreads=8)
        assert len(out[1][0]) == T_o + 1
        np.testing.assert_allclose(out[1][0], nt_o, rtol=1e-12, atol=0)


def test_staged_batch_components():
    """Batched runs of one seed per row (64-byte rows) staged: every component equals the
    oracle's run."""
    gs = [graphgen.web(600 + 50 * i, host_mean=40.0, deg_mean=6.0, seed=40 + i, keep_kind=True) for i in range(6)]
    gs += [graphgen.rmat(9, 3000, seed=50), graphgen.directed_cycle(70), graphgen.empty(5)]
    b, S = 6, 1
    seeds = [100 + g for g in range(len(gs))]
    with hanf.Batch(0, stage=1, seeds_per_row=1) as bt:
        bt.load_graphs(gs, S).init(b, seeds)
        bt.run()
        T = bt.fixpoints()
        for g, (rp, ci) in enumerate(gs):
            nt_ref, T_ref, regs_ref = oracle.run(rp, ci, b, seeds[g], want_regs=True)
            assert T[g] == T_ref, g
            np.testing.assert_allclose(bt.nt(g), nt_ref, rtol=1e-12, atol=0)
            assert np.array_equal(bt.registers(g), regs_ref), g
        assert bt.pass_log()[0]["arcs_local"] > 0
