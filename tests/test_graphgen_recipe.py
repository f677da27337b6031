"""The seeded input generators against their recipe, on the CPU at small sizes: valid CSR
with sorted successor lists and no duplicates or self-loops, exact arc counts, symmetric
R-MAT equal to its own transpose, R-MAT skew, the web-like graph's out-degree law after
duplicate removal, its local arcs and its power-law in-degree of the inter-host arcs, and
determinism under the graph seed; the per-arc intra/inter choice gives 80% intra-host
arcs."""
import numpy as np
import pytest

import graphgen


def check_csr(rp, ci):
    n = len(rp) - 1
    assert rp[0] == 0 and rp[-1] == len(ci) and np.all(np.diff(rp) >= 0)
    assert len(ci) == 0 or (ci.min() >= 0 and ci.max() < n)
    src = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(src == ci), "self-loop"
    same_row = src[1:] == src[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row]), "successors not strictly increasing"
    return n, src


def test_rmat_directed():
    rp, ci = graphgen.rmat(14, 1 << 18, seed=14)
    n, _ = check_csr(rp, ci)
    assert n == 1 << 14 and len(ci) == 1 << 18
    deg = np.diff(rp)
    assert deg.max() > 50 * deg.mean()          # (a,b,c,d) = (.57,.19,.19,.05): heavy hubs
    rp2, ci2 = graphgen.rmat(14, 1 << 18, seed=14)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    rp3, ci3 = graphgen.rmat(14, 1 << 18, seed=15)
    assert not np.array_equal(ci, ci3)


def test_rmat_symmetric_is_its_own_transpose():
    rp, ci = graphgen.rmat(12, 1 << 15, symmetric=True, seed=3)
    n, src = check_csr(rp, ci)
    assert len(ci) == 2 << 15
    fwd = np.sort(src.astype(np.int64) * n + ci)
    bwd = np.sort(ci.astype(np.int64) * n + src)
    assert np.array_equal(fwd, bwd)


def test_rmat_node_cap_rejects_far_endpoints():
    rp, ci = graphgen.rmat(10, 8000, seed=9, n=700)
    n, _ = check_csr(rp, ci)
    assert n == 700 and len(ci) == 8000


def test_erdos_renyi_exact_arc_count():
    rp, ci = graphgen.erdos_renyi(3000, 24000, seed=5)
    n, _ = check_csr(rp, ci)
    assert n == 3000 and len(ci) == 24000
    deg = np.diff(rp)
    assert abs(deg.var() / deg.mean() - 1.0) < 0.15    # binomial out-degrees: variance ~ mean


@pytest.fixture(scope="module")
def web16():
    return graphgen.web(1 << 16, seed=5)


def test_web_out_degree_law_after_dedupe(web16):
    rp, ci = web16
    n, _ = check_csr(rp, ci)
    deg = np.diff(rp)
    assert abs(deg.mean() - 20.0) < 0.5                 # LogNormal with mean 20
    logs = np.log(deg[deg > 0])
    assert abs(logs.std() - 1.0) < 0.05                 # sigma 1
    assert abs(logs.mean() - (np.log(20.0) - 0.5)) < 0.05


def intra_host_share_and_inter_indeg(rp, ci, hosts):
    n = len(rp) - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    intra = hosts[ci] == hosts[src]
    return intra.mean(), np.sort(np.bincount(ci[~intra], minlength=n))[::-1], int((~intra).sum())


def check_inter_power_law(inter_in, inter, n):
    # Inter-host targets: weight rank^(-1/(gamma-1)) with gamma = 2.1 (Chung-Lu), so the
    # r-th largest inter-host in-degree is about inter * r^(-1/1.1) / sum_k k^(-1/1.1).
    # Ranks 30..1000: past the top few, whose in-degree saturates at one arc per source.
    ex = -1 / 1.1
    norm = np.sum(np.arange(1, n + 1, dtype=np.float64) ** ex)
    r = np.arange(30, 1001)
    slope = np.polyfit(np.log(r), np.log(inter_in[r - 1]), 1)[0]
    assert abs(slope - ex) < 0.05
    for k in (30, 100, 300, 1000):
        assert inter_in[k - 1] == pytest.approx(inter * k ** ex / norm, rel=0.15), k


def test_web_hosts(web16):
    hosts = graphgen.web_hosts(1 << 16, seed=5)
    assert hosts[0] == 0 and np.all(np.diff(hosts) >= 0) and np.all(hosts <= np.arange(1 << 16))
    first = np.unique(hosts)
    sizes = np.diff(np.append(first, 1 << 16))
    assert np.all(hosts[first] == first)
    assert 500 < sizes[:-1].mean() < 2000               # LogNormal sizes of mean 1000


def test_web_default_draws(web16):
    rp, ci = web16
    n = len(rp) - 1
    share, inter_in, inter = intra_host_share_and_inter_indeg(rp, ci, graphgen.web_hosts(n, seed=5))
    # Intra-host with probability 0.8 per draw; a duplicate target is drawn again with a
    # new intra/inter choice, and nearby ids repeat far more often than power-law targets,
    # so only a little over half of the kept arcs are intra-host.
    assert 0.5 < share < 0.6
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    assert (np.abs(ci.astype(np.int64) - src) <= 64).mean() > 0.95 * share   # and nearby
    check_inter_power_law(inter_in, inter, n)


def test_web_kind_kept_per_arc(web16):
    n = 1 << 16
    rp, ci = graphgen.web(n, seed=5, keep_kind=True)
    check_csr(rp, ci)
    assert np.array_equal(rp, web16[0])                 # the same out-degrees
    share, inter_in, inter = intra_host_share_and_inter_indeg(rp, ci, graphgen.web_hosts(n, seed=5))
    assert abs(share - 0.8) < 0.01
    check_inter_power_law(inter_in, inter, n)


def test_web_is_deterministic(web16):
    rp, ci = graphgen.web(1 << 16, seed=5)
    assert np.array_equal(rp, web16[0]) and np.array_equal(ci, web16[1])
    assert not np.array_equal(graphgen.web(1 << 16, seed=6)[1][:1000], ci[:1000])


def test_batch_workload_recipe():
    sizes = graphgen.batch_sizes(512, seed=4)
    assert len(sizes) == 512 and min(sizes) >= 1 << 8 and max(sizes) <= 1 << 16
    assert 0.75 < np.median(sizes) / 4096 < 1.3        # lognormal, median 2^12
    graphs = graphgen.batch_graphs(16, seed=4)
    for i, ((rp, ci), n) in enumerate(zip(graphs, graphgen.batch_sizes(16, seed=4))):
        m, _ = check_csr(rp, ci)
        assert m == n
        # first half Erdos-Renyi with 8n arcs, second half R-MAT with 16n arcs
        assert len(ci) == (8 * n if i < 8 else 16 * n)


def test_disjoint_union_layout():
    gs = [graphgen.directed_cycle(5), graphgen.empty(3), graphgen.erdos_renyi(40, 200, seed=2)]
    off, rp, ci = graphgen.disjoint_union(gs)
    assert list(off) == [0, 5, 8, 48]
    check_csr(rp, ci)
    for g, (a, b) in zip(gs, zip(off[:-1], off[1:])):
        grp = rp[a:b + 1] - rp[a]
        assert np.array_equal(grp, g[0])
        assert np.array_equal(ci[rp[a]:rp[b]] - a, g[1])


def test_serve_request_recipe():
    reqs = graphgen.serve_requests(40, trace_seed=5, hi=1 << 13, median=1 << 11, sigma=1.0)
    assert [r["rid"] for r in reqs] == list(range(40))
    assert {r["log2m"] for r in reqs} <= {4, 6, 8} and len({r["log2m"] for r in reqs}) == 3
    assert {r["kind"] for r in reqs} == {"rmat", "web"}
    for r in reqs:
        rp, ci = r["graph"]
        n, _ = check_csr(rp, ci)
        assert n == r["n"] and (1 << 10) <= n <= (1 << 13)
        assert r["seed"] == r["rid"] + 1
        if r["kind"] == "rmat":
            assert len(ci) == 16 * n


def test_benchmark_graph_at_full_size():
    """The symmetric R-MAT graph of scale 22 the benchmark runs on: 2^22 nodes, 2^26 arcs
    (2^25 distinct edges, both directions), its largest degree and its nodes without arcs
    as generated from graph seed 22."""
    rp, ci = graphgen.workload_graph(graphgen.WORKLOADS["rmat22sym"])
    deg = np.diff(rp)
    assert len(rp) - 1 == 1 << 22 and len(ci) == 1 << 26
    assert int(deg.max()) == 99_802 and int((deg == 0).sum()) == 2_168_332
    assert not np.any(np.repeat(np.arange(1 << 22, dtype=np.int32), deg) == ci)


def test_limit_graph_recipe():
    """The arc-limit graph's recipe on a small instance (the full one, 2^21 * 1023 + 2^20 =
    2^31 - 2^20 arcs, is generated by the GPU test): heavy rows first with their arithmetic
    targets, one-successor rows after them; parameters whose targets would overflow int32
    are refused. (Node 0's first arc is a self-loop, which the library accepts.)"""
    H, D, L = 1 << 6, 15, 1 << 5
    rp, ci = graphgen.limit_graph(heavy_log2=6, degree=D, light_log2=5)
    n, arcs = len(rp) - 1, len(ci)
    assert rp.dtype == ci.dtype == np.int32 and rp[0] == 0 and rp[-1] == arcs
    assert ci.min() >= 0 and ci.max() < n
    assert n == H + L and arcs == H * D + L
    assert np.array_equal(np.diff(rp), [D] * H + [1] * L)
    for v in (0, 1, H // 2, H - 1):
        assert ci[rp[v]:rp[v + 1]].tolist() == [(v * D + j) % n for j in range(D)]
    for u in (H, H + 1, n - 1):
        assert ci[rp[u]:rp[u + 1]].tolist() == [(7 * u + 3) % n]
    assert (1 << 21) * 1023 + (1 << 20) == (1 << 31) - (1 << 20)
    with pytest.raises(ValueError):
        graphgen.limit_graph(heavy_log2=22, degree=1023, light_log2=1)
