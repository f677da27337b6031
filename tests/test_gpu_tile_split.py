"""Light tiles shared by several wavefronts (HANF_OPT_TILE_SPLIT): in passes over every
successor, 2, 4 or 8 wavefronts take a tile's rounds of nodes in turn. The results must not
change: registers byte-equal to the oracle's at every t, every node's estimate bit for bit,
N_hat(t) within 1e-12, T and the work counters exactly the oracle's (the step parity of
test_gpu_parity.py), on ragged last tiles, tiles with fewer rounds than wavefronts, heavy
rows split into chunks, and with the instrumented (near-counting) kernels."""
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
    "web_2^14": lambda: graphgen.web(1 << 14, host_mean=200.0, seed=61, keep_kind=True),
    "web_ragged": lambda: graphgen.web(3001, host_mean=50.0, deg_mean=8.0, seed=62, keep_kind=True),
    "rmat_12": lambda: graphgen.rmat(12, 40_000, seed=63),
    "cycle_1000": lambda: graphgen.directed_cycle(1000),
    "star_out_3000": lambda: graphgen.star_out(3000),
    "clique_path_clique": lambda: graphgen.clique_path_clique(20, 37),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("b", [4, 6, 7, 8])
@pytest.mark.parametrize("split", [1, 2, 4, 8])
@pytest.mark.parametrize("sweep", [0, 1])
def test_split_tiles_every_iteration(name, b, split, sweep):
    """sweep 1: the union step from a grid that claims work units per XCD (option 105)."""
    if split == 1 and not sweep:
        pytest.skip("the default schedule (test_gpu_parity.py)")
    rp, ci = GRAPHS[name]()
    step_parity(rp, ci, b, seed=11 + b, tile_split=split, sweep=sweep)


@pytest.mark.parametrize("split", [1, 2, 8])
@pytest.mark.parametrize("sweep", [0, 1])
def test_split_tiles_with_systolic_and_near_counts(split, sweep):
    """Split dense passes, then systolic passes (transposed graph built on the device); and
    the instrumented kernels, whose near counts step_parity checks against numpy."""
    rp, ci = graphgen.web(1 << 13, host_mean=100.0, seed=64, keep_kind=True)
    step_parity(rp, ci, 7, seed=3, transpose="build", tile_split=split, sweep=sweep)
    step_parity(rp, ci, 7, seed=4, tile_split=split, count_near=1, sweep=sweep)


def test_split_changes_nothing():
    """Every split, with and without the sweep kernel, gives the same N_hat (same sums in the
    same order), registers, pass kinds and gathered counts as one wavefront per tile, with the
    tile sizes of large graphs, and equals the oracle."""
    cases = {"web": graphgen.web(1 << 16, seed=65, keep_kind=True),
             "rmat": graphgen.rmat(16, 1 << 20, seed=66)}
    for name, (rp, ci) in cases.items():
        b, seed = 7, 9
        out = {}
        for split, sweep in ((0, 0), (1, 0), (2, 0), (4, 0), (8, 0), (1, 1), (2, 1), (8, 1)):
            with hanf.HyperANF(0, tile_split=split, sweep=sweep) as h:
                h.load(rp, ci).init(b, seed)
                nt = h.run()
                log = h.pass_log()
                out[split, sweep] = (nt, h.registers().copy(),
                              [(r["gather_all"], r["arcs_gathered"], r["changed"]) for r in log])
        one = out[1, 0]
        _say(f"[tile_split] {name}: {len(one[0]) - 1} passes, kinds {[k for k, _, _ in one[2]]}")
        for key, res in out.items():
            assert np.array_equal(res[0], one[0]), key
            assert np.array_equal(res[1], one[1]), key
            assert res[2] == one[2], key
        nt_o, T_o, _ = oracle.run(rp, ci, b, seed, nthreads=8)
        assert len(one[0]) == T_o + 1
        np.testing.assert_allclose(one[0], nt_o, rtol=1e-12, atol=0)


def test_split_option_checked():
    with hanf.HyperANF(0) as h:
        for bad in (3, 5, 16, -1):
            with pytest.raises(hanf.HanfError):
                hanf.hanf_set_option(h.ctx, hanf.HANF_OPT_TILE_SPLIT, bad)
