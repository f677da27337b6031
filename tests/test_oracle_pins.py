"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the passage of Boldi, Rosa, Vigna, "HyperANF" (arXiv:1011.5599) it
checks. None of these compares the oracle with itself: the expected values are
printed in the paper, published (the splitmix64 vector), closed forms, brute force
(BFS), or library routines (numerical integration).
"""
import json
import math
import os
import random

import numpy as np
import pytest

import graphgen
import oracle
from oracle import exact, stats


def _load_vector(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64_seed1234567.txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    seed = int(lines[0].split()[1])
    return seed, [int(x) for x in lines[1:]]


@pytest.fixture(scope="module")
def paper(golden_dir):
    with open(os.path.join(golden_dir, "paper_values.json")) as f:
        return json.load(f)


# ------------------------------------------------------------------ hash and Algorithm 1

def test_hash_matches_published_splitmix64(golden_dir):
    """h_s(x) = output x+1 of splitmix64 from state s (reading of Section 3.1's ideal hash)."""
    seed, outs = _load_vector(golden_dir)
    assert [oracle.hash64(seed, x) for x in range(len(outs))] == outs


def test_rho_plus_paper_example(paper):
    """Section 3.1: rho+(00101) = 3."""
    ex = paper["rho_plus_example"]
    bits = ex["bits"]
    for b in (0, 4, 6, 8):
        # the 64-b bits after the leftmost b start with 00101, the rest arbitrary ones
        tail_len = 64 - b
        h = (int(bits, 2) << (tail_len - len(bits))) | ((1 << (tail_len - len(bits))) - 1)
        h |= ((1 << b) - 1) << tail_len  # leftmost b bits all ones: must not matter
        assert oracle.rho_plus(h, b) == ex["value"]


def test_rho_plus_edges_brute_force():
    """rho+ = leading zeroes of h^b(x) plus one, checked against the binary string."""
    rng = random.Random(5)
    for b in range(4, 9):
        for _ in range(300):
            h = rng.getrandbits(64) >> rng.randrange(64)
            h |= rng.getrandbits(b) << (64 - b)
            tail = format(h, "064b")[b:]
            want = (len(tail) - len(tail.lstrip("0"))) + 1
            assert oracle.rho_plus(h, b) == want
            assert oracle.register_index(h, b) == int(format(h, "064b")[:b], 2)
        assert oracle.rho_plus(0, b) == 64 - b + 1
        assert oracle.rho_plus(1 << (63 - b), b) == 1


def test_add_saturates_and_is_max():
    """Algorithm 1 add: M[i] <- max(M[i], rho+); registers saturate at 31 (5-bit)."""
    b, seed = 4, 77
    for x in range(2000):
        M = np.zeros(1 << b, np.uint8)
        M[:] = 3
        oracle.add(M, b, seed, x)
        h = oracle.hash64(seed, x)
        i = oracle.register_index(h, b)
        r = min(oracle.rho_plus(h, b), 31)
        want = np.full(1 << b, 3, np.uint8)
        want[i] = max(3, r)
        assert np.array_equal(M, want)


def test_add_crafted_hashes():
    """Algorithm 1 add on hashes built bit by bit: the register is the leftmost b bits, the
    value rho+ of the rest, saturated at 31 (registers of ceil(log log n) = 5 bits)."""
    for b in range(4, 9):
        tail = 64 - b
        for idx in (0, 1, (1 << b) - 1):
            for zeros in (0, 1, 7, 15, 16, 29, 30, 31, 40, tail - 1, tail):
                h = idx << tail
                if zeros < tail:
                    h |= 1 << (tail - 1 - zeros)
                M = np.zeros(1 << b, np.uint8)
                oracle.add_hashed(M, b, h)
                want = np.zeros(1 << b, np.uint8)
                want[idx] = min(zeros + 1, 31)
                assert np.array_equal(M, want), (b, idx, zeros)
                M2 = np.full(1 << b, 30, np.uint8)
                oracle.add_hashed(M2, b, h)
                assert M2[idx] == max(30, min(zeros + 1, 31))


def test_alpha_matches_integral_definition():
    """alpha_m of the HyperLogLog paper, (m * int_0^inf log2((2+u)/(1+u))^m du)^-1, against
    the published constants the oracle uses (the paper defers alpha_m to that paper)."""
    from scipy.integrate import quad
    for b in range(4, 9):
        m = 1 << b
        val, _ = quad(lambda u: math.log2((2 + u) / (1 + u)) ** m, 0, math.inf, limit=500)
        exact_alpha = 1.0 / (m * val)
        assert abs(oracle.alpha(m) / exact_alpha - 1) < 5e-4, (m, oracle.alpha(m), exact_alpha)


def test_size_empty_and_single():
    """Empty counter estimates 0 (linear counting, V = m); one non-zero register estimates
    m ln(m/(m-1)) for any value, since the raw value is below 5m/2."""
    for b in range(4, 9):
        m = 1 << b
        assert oracle.size(np.zeros(m, np.uint8), b) == 0.0
        for r in (1, 5, 31):
            M = np.zeros(m, np.uint8)
            M[m // 3] = r
            assert oracle.size(M, b) == m * math.log(m / (m - 1))


def test_size_large_range_uses_raw():
    """All registers high: V = 0, so the raw alpha_m m^2 / sum 2^-M applies."""
    for b in range(4, 9):
        m = 1 << b
        M = np.full(m, 20, np.uint8)
        assert oracle.size(M, b) == pytest.approx(oracle.alpha(m) * m * m / (m * 2.0 ** -20),
                                                  rel=1e-15)


def test_sketch_of_union_random_sets():
    """Section 3.2: the counter of the stream AB is the register max of those of A and B."""
    rng = random.Random(11)
    for b in (4, 6, 8):
        for _ in range(20):
            A = rng.sample(range(10 ** 6), rng.randrange(0, 400))
            B = rng.sample(range(10 ** 6), rng.randrange(0, 400))
            MA = np.zeros(1 << b, np.uint8)
            MB = np.zeros(1 << b, np.uint8)
            MAB = np.zeros(1 << b, np.uint8)
            for x in A:
                oracle.add(MA, b, 3, x)
                oracle.add(MAB, b, 3, x)
            for x in B:
                oracle.add(MB, b, 3, x)
                oracle.add(MAB, b, 3, x)
            oracle.union(MA, MB)
            assert np.array_equal(MA, MAB)


# ------------------------------------------------------------------ broadword (Section 3.3)

@pytest.mark.parametrize("k", [5, 8])
def test_broadword_max_exhaustive(k):
    """Section 3.3's x <_k^u y and mask formulas give the block-wise max, for every pair of
    block values, in every block position (L_8 read as 0x0101010101010101)."""
    rng = random.Random(k)
    nb = 64 // k
    assert oracle.broadword_L(8) == 0x0101010101010101
    for pos in range(nb):
        for x in range(1 << k):
            for y in range(1 << k):
                X = Y = want = 0
                for i in range(nb):
                    a = x if i == pos else rng.randrange(1 << k)
                    c = y if i == pos else rng.randrange(1 << k)
                    X |= a << (i * k)
                    Y |= c << (i * k)
                    want |= max(a, c) << (i * k)
                assert oracle.broadword_max(X, Y, k) == want
                less = oracle.broadword_less(X, Y, k)
                assert bool((less >> (pos * k + k - 1)) & 1) == (x < y)


# ------------------------------------------------------------------ Algorithm 2

def _tiny_graphs():
    gs = []
    for s in range(6):
        gs.append(("er%d" % s, graphgen.erdos_renyi(60 + 30 * s, 150 + 90 * s, seed=100 + s)))
    for s in range(4):
        gs.append(("rmat%d" % s, graphgen.rmat(7 + (s % 2), 300 + 100 * s, seed=200 + s)))
    gs.append(("rmatsym", graphgen.rmat(7, 300, symmetric=True, seed=301)))
    gs.append(("cycle", graphgen.directed_cycle(37)))
    gs.append(("path", graphgen.directed_path(23)))
    gs.append(("cpc", graphgen.clique_path_clique(6, 4)))
    gs.append(("star_out", graphgen.star_out(50)))
    gs.append(("star_in", graphgen.star_in(50)))
    return gs


TINY = _tiny_graphs()


@pytest.mark.parametrize("name,g", TINY, ids=[t[0] for t in TINY])
def test_counter_equals_counter_of_ball(name, g):
    """Section 3.2: after t iterations c[v] is in the state of a counter fed with B(v,t).
    Checked for every node and every t up to stabilisation, register for register, against
    a counter built by BFS; the ball sizes against a Python BFS."""
    rp, ci = g
    n = len(rp) - 1
    for b, seed in ((4, 1), (6, 9)):
        for t, c, _ in oracle.run_steps(rp, ci, b, seed):
            for v in range(n):
                M, sz = oracle.ball_counter(rp, ci, b, seed, v, t)
                assert np.array_equal(c[v], M), (name, b, t, v)
                if v % 17 == 0:
                    assert sz == len(exact.ball(rp, ci, v, t))


@pytest.mark.parametrize("name,g", TINY, ids=[t[0] for t in TINY])
def test_stabilisation_bound_and_monotone_registers(name, g):
    """Alg. 2's loop stops when no counter changes; the footnote of Section 4 says it may
    stop before the largest distance (collisions) but never after it. Registers never
    decrease."""
    rp, ci = g
    D = len(exact.neighbourhood_function(rp, ci)) - 1
    for b, seed in ((4, 3), (6, 4)):
        prev = None
        T = None
        for t, c, _ in oracle.run_steps(rp, ci, b, seed):
            if prev is not None:
                assert (c >= prev).all()
            prev = c.copy()
            T = t
        assert T <= D


@pytest.mark.parametrize("name,g", TINY, ids=[t[0] for t in TINY])
def test_skip_unmodified_and_threads_identical(name, g):
    """Section 3.3: skipping counters unmodified in the last iteration, and the task
    decomposition over threads, leave every counter identical at every t."""
    rp, ci = g
    b, seed = 5, 21
    dense = [(t, c.copy(), s) for t, c, s in oracle.run_steps(rp, ci, b, seed, skip_unmodified=False)]
    skip = [(t, c.copy(), s) for t, c, s in oracle.run_steps(rp, ci, b, seed, nthreads=3)]
    assert len(dense) == len(skip)
    for (t1, c1, s1), (t2, c2, s2) in zip(dense, skip):
        assert t1 == t2 and np.array_equal(c1, c2) and s1 == s2
    nt, T, regs = oracle.run(rp, ci, b, seed, want_regs=True, nthreads=2)
    assert T == dense[-1][0]
    assert np.array_equal(regs, dense[-1][1])
    assert np.array_equal(nt, np.array([s for _, _, s in dense]))


def test_permuted_successors_duplicates_self_loops_change_nothing():
    """Max is associative, commutative and idempotent: successor order, duplicate arcs and
    self-loops do not change any counter (Algorithm 2)."""
    rp, ci = graphgen.erdos_renyi(120, 500, seed=9)
    n = len(rp) - 1
    rng = np.random.default_rng(3)
    arcs = [(u, int(w)) for u in range(n) for w in ci[rp[u]:rp[u + 1]]]
    extra = arcs + [arcs[i] for i in rng.integers(0, len(arcs), 200)] + [(u, u) for u in range(0, n, 3)]
    rng.shuffle(extra)
    # keep the shuffled order inside each row
    rows = [[] for _ in range(n)]
    for u, w in extra:
        rows[u].append(w)
    rp2 = np.zeros(n + 1, np.int32)
    rp2[1:] = np.cumsum([len(r) for r in rows])
    ci2 = np.array([w for r in rows for w in r], np.int32)
    a = oracle.run(rp, ci, 6, 5, want_regs=True)
    b = oracle.run(rp2, ci2, 6, 5, want_regs=True)
    assert a[1] == b[1] and np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_no_arcs():
    """No arcs: the first pass changes nothing, T = 0, output [N_hat(0)]."""
    rp, ci = graphgen.empty(100)
    nt, T, _ = oracle.run(rp, ci, 4, 1)
    assert T == 0 and len(nt) == 1
    assert nt[0] == pytest.approx(100 * 16 * math.log(16 / 15), rel=1e-15)


def test_complete_digraph_stabilises_fast():
    rp, ci = graphgen.complete(40)
    nt, T, _ = oracle.run(rp, ci, 6, 2)
    assert T <= 1


@pytest.mark.parametrize("b,n", [(4, 16384), (6, 4194304), (7, 1 << 24)])
def test_initial_estimate_closed_form(b, n):
    """Every counter starts with exactly one non-zero register, so each estimates
    m ln(m/(m-1)) (small-range rule) and N_hat(0) = n m ln(m/(m-1)), whatever the seed.
    Checked on a prefix of the nodes (the value per node is what matters) and, for the
    smallest size, on all of them."""
    m = 1 << b
    n_check = min(n, 1 << 15)
    for seed in (1, 7, 123456789):
        c = oracle.init(n_check, b, seed)
        assert (np.count_nonzero(c, axis=1) == 1).all()
        got = oracle.sum_sizes(c, b)
        assert got == pytest.approx(n_check * m * math.log(m / (m - 1)), rel=1e-13)
    closed = n * m * math.log(m / (m - 1))
    assert closed == pytest.approx({4: 16918.386085, 6: 4227417.383993, 7: 16843095.345915}[b],
                                   rel=1e-10)


# ------------------------------------------------------------------ exact N(t) and statistics

@pytest.mark.parametrize("k,l", [(2, 1), (3, 2), (5, 3), (8, 6), (4, 10)])
def test_clique_path_clique_closed_form(k, l):
    """Section 4: the exact neighbourhood function of two k-cliques joined by a one-way path
    of l nodes, against BFS."""
    rp, ci = graphgen.clique_path_clique(k, l)
    N = exact.neighbourhood_function(rp, ci)

    def closed(t):
        if t == 0:
            return 2 * k + l
        if t <= l:
            return (t + 1) * (2 * k + l - t / 2) - 2 * k + 2 * k * k
        return (l + 1) * (2 * k + l / 2) - 2 * k + 3 * k * k

    assert len(N) - 1 == l + 1
    for t in range(len(N) + 3):
        assert N[min(t, len(N) - 1)] == closed(t)


@pytest.mark.parametrize("l", [2, 5, 10])
def test_effective_diameter_stop_rule(l, paper):
    """Section 4: with k = 2l^2+5l+2 the effective diameter (alpha = 0.9) is l+1 when run to
    stabilisation and 1 if the iteration stops at t = l."""
    k = 2 * l * l + 5 * l + 2
    alpha = paper["alpha_default"]["value"]

    def closed(t):
        if t == 0:
            return 2 * k + l
        if t <= l:
            return (t + 1) * (2 * k + l - t / 2) - 2 * k + 2 * k * k
        return (l + 1) * (2 * k + l / 2) - 2 * k + 3 * k * k

    full = [closed(t) for t in range(l + 2)]
    assert stats.stats(full, alpha)["ed"] == l + 1
    assert stats.stats(full[: l + 1], alpha)["ed"] == 1
    if l == 2:  # also through an actual run (exact N by BFS) of the small instance
        rp, ci = graphgen.clique_path_clique(k, l)
        assert list(exact.neighbourhood_function(rp, ci)) == full


@pytest.mark.parametrize("n", [2, 5, 12, 40])
def test_cycle_moments_closed_form(n):
    """Directed cycle: N(t) = n(t+1) for t < n (BFS), so h(t) = 1/n for t = 0..n-1:
    average distance (n-1)/2, variance (n^2-1)/12, spid (n+1)/6 (Sections 4-5)."""
    rp, ci = graphgen.directed_cycle(n)
    N = exact.neighbourhood_function(rp, ci)
    assert list(N) == [n * (t + 1) for t in range(n)]
    s = stats.stats(list(N))
    assert s["avg_dist"] == pytest.approx((n - 1) / 2, rel=1e-12)
    assert s["var"] == pytest.approx((n * n - 1) / 12, rel=1e-12, abs=1e-12)
    assert s["spid"] == pytest.approx((n + 1) / 6, rel=1e-12)
    # interpolated effective diameter: H(t) = (t+1)/n crosses 0.9 at t = 0.9n - 1
    assert s["ied"] == pytest.approx(max(0.0, 0.9 * n - 1), rel=1e-12, abs=1e-12)
    assert s["ed"] == math.ceil(0.9 * n - 1 - 1e-12)


@pytest.mark.parametrize("n", [2, 5, 12, 40])
def test_cycle_moments_distinct_pairs_closed_form(n):
    """Directed cycle, pairs at distance >= 1 only (self-pairs dropped from the distance
    distribution): H(t) = t/(n-1), so h(t) = 1/(n-1) for t = 1..n-1, average distance n/2,
    variance n(n-2)/12, spid (n-2)/6, and H crosses 0.9 at t = 0.9(n-1)."""
    rp, ci = graphgen.directed_cycle(n)
    s = stats.stats(list(exact.neighbourhood_function(rp, ci)), distinct=True)
    assert s["avg_dist"] == pytest.approx(n / 2, rel=1e-12)
    assert s["var"] == pytest.approx(n * (n - 2) / 12, rel=1e-12, abs=1e-12)
    assert s["spid"] == pytest.approx((n - 2) / 6, rel=1e-12, abs=1e-12)
    assert s["ied"] == pytest.approx(0.9 * (n - 1), rel=1e-12)
    assert s["ed"] == math.ceil(0.9 * (n - 1) - 1e-12)


def test_diameter_interval_algorithm3():
    """Algorithm 3 on a hand-checked sequence: H = [.1 .3 .6 .85 .95 1]; with alpha = .9 and
    eps = .02: D- = largest t with H <= .864 -> 3; D+ = smallest t with H >= .936 -> 4."""
    nt = [10, 30, 60, 85, 95, 100]
    assert stats.diameter_interval(nt, 0.02, 0.9) == (3, 4)


def test_rsd_and_memory_numbers(paper):
    """Section 3: eta_m <= 1.06/sqrt(m) gives the printed 9.37% (m=128), 13.25% (m=64),
    6.62% (m=256); m ~ 1.12/eta^2 registers of ceil(log2 log2 n) bits for 10^9 nodes give
    the printed 74.5 GB."""
    c = paper["rsd_bound_coefficient"]["value"]
    for m, pct in paper["rsd_percent"].items():
        if m.startswith("_"):
            continue
        assert abs(100 * c / math.sqrt(int(m)) - pct) <= 0.005 + 1e-12  # printed to 2 decimals
    mem = paper["memory_example"]
    eta = mem["rsd_percent"] / 100
    m = 1 << round(math.log2(1.12 / eta ** 2))
    bits = math.ceil(math.log2(math.log2(mem["nodes"])))
    assert m == 128 and bits == 5
    assert round(m * bits * mem["nodes"] / 8 / 2 ** 30, 1) == mem["gigabytes"]


def test_vp_confidences(paper):
    """Section 3.4: k eta with confidence 1 - 4/(9k^2): 2 eta ~ 90%, 3 eta ~ 95%."""
    for k, conf in paper["vp_confidence"].items():
        if k.startswith("_"):
            continue
        assert abs((1 - 4 / (9 * int(k) ** 2)) - conf) < 0.012


# ------------------------------------------------------------------ statistical (Theorem 1)

def _error_samples(graphs, b, seeds):
    errs = []
    means = []
    for rp, ci in graphs:
        N = exact.neighbourhood_function(rp, ci)
        runs = []
        for seed in seeds:
            nt, T, _ = oracle.run(rp, ci, b, seed)
            ext = [nt[min(t, T)] for t in range(len(N))]
            runs.append(ext)
            errs.extend(abs(x / y - 1) for x, y in zip(ext, N))
        means.extend(np.mean(runs, axis=0) / N - 1)
    return np.array(errs), np.array(means)


@pytest.mark.parametrize("b,beta", [(4, 1.106), (6, 1.06), (7, 1.06)])
def test_error_against_exact_neighbourhood_function(b, beta):
    """Theorem 1 and the Vysochanskii-Petunin bound (Section 3.4): each N_hat(t) is within
    k eta_m of N(t) with probability >= 1 - 4/(9k^2). Over 60 seeds and 8 small graphs, the
    fraction within 2 eta is >= 0.889 and within 3 eta >= 0.951; the seed-mean is within
    eta/2 of N(t) (almost unbiased). eta_m = 1.06/sqrt(m), and 1.106/sqrt(16) at m = 16
    (the paper assumes m >= 64)."""
    gs = [graphgen.erdos_renyi(150, 450, seed=400 + s) for s in range(4)]
    gs += [graphgen.rmat(8, 900, seed=500 + s) for s in range(2)]
    gs += [graphgen.directed_cycle(60), graphgen.clique_path_clique(7, 5)]
    eta = beta / math.sqrt(1 << b)
    errs, means = _error_samples(gs, b, range(1, 61))
    assert (errs <= 2 * eta).mean() >= 1 - 4 / 36
    assert (errs <= 3 * eta).mean() >= 1 - 4 / 81
    assert np.abs(means).max() <= eta / 2


# ------------------------------------------------------------------ the parity workload itself

@pytest.fixture(scope="module")
def rmat14_balls():
    """The directed R-MAT scale 14 parity workload (16,384 nodes, 262,144 arcs, m = 16,
    hash seed 1): the oracle's counters at every t and the exact N(t) by BFS."""
    spec = graphgen.WORKLOADS["rmat14"]
    rp, ci = graphgen.workload_graph(spec)
    b, seed = spec["log2m"], spec["seed"]
    counters = [c for _, c, _ in oracle.run_steps(rp, ci, b, seed)]
    bad, first, N = oracle.balls_check(rp, ci, b, seed, counters, nthreads=os.cpu_count() or 1)
    return rp, ci, b, seed, counters, bad, first, N


def test_rmat14_every_counter_is_its_ball(rmat14_balls):
    """Section 3.2: c_t[v] is the counter of B(v, t). Checked for all 16,384 nodes of the
    parity workload at every t (and for every later distance against the stable c_T), by a
    breadth-first search from each node."""
    rp, ci, b, seed, counters, bad, first, N = rmat14_balls
    assert len(counters) >= 4
    assert bad == 0, f"{bad} (node, t) pairs differ; first {first}"


def test_rmat14_ball_check_catches_a_changed_register(rmat14_balls):
    rp, ci, b, seed, counters, _, _, _ = rmat14_balls
    planted = [c.copy() for c in counters]
    planted[2][1234, 5] += 1
    bad, first, _ = oracle.balls_check(rp, ci, b, seed, planted, nthreads=os.cpu_count() or 1)
    assert bad >= 1 and first == (1234, 2)


def test_rmat14_within_theorem1_over_seeds(rmat14_balls):
    """Theorem 1 with the Vysochanskii-Petunin bound (Section 3.4) on the parity workload:
    over 32 hash seeds, N_hat(t) is within 2 eta of the exact N(t) (BFS) for at least
    1 - 4/36 of the (seed, t) points and within 3 eta for at least 1 - 4/81, with
    eta = 1.106/sqrt(16) at m = 16; the seed mean is within eta/2 (almost unbiased).
    N(0) = n exactly (Section 4: self-pairs count) and N(t) ends at the reachable pairs."""
    rp, ci, b, _, _, _, _, N = rmat14_balls
    n = len(rp) - 1
    assert N[0] == n and np.all(np.diff(N) > 0)
    eta = 1.106 / math.sqrt(1 << b)
    errs, runs = [], []
    for seed in range(1, 33):
        nt, T, _ = oracle.run(rp, ci, b, seed, nthreads=os.cpu_count() or 1)
        ext = np.array([nt[min(t, T)] for t in range(len(N))])
        runs.append(ext)
        errs.extend(np.abs(ext / N - 1))
    errs = np.array(errs)
    assert (errs <= 2 * eta).mean() >= 1 - 4 / 36
    assert (errs <= 3 * eta).mean() >= 1 - 4 / 81
    assert np.abs(np.mean(runs, axis=0) / N - 1).max() <= eta / 2


@pytest.mark.parametrize("b", [4, 6])
def test_estimate_falls_only_at_the_small_range_switch(b):
    """Section 4 calls the estimated distance function monotone. Registers only grow, so the
    raw estimate alpha m^2 / sum_j 2^-M[j] never falls; with the small-range rule a node's
    estimate can still fall, but only in the pass where its counter leaves the
    linear-counting range (raw <= 5m/2 with an empty register) for the raw estimate.
    Checked node by node over whole runs on small random graphs."""
    m = 1 << b
    a = oracle.alpha(m)
    dips = 0
    for gseed in range(40):
        rp, ci = graphgen.erdos_renyi(60, 150, seed=gseed)
        prev = None
        for t, c, s in oracle.run_steps(rp, ci, b, 1000 + gseed):
            E = oracle.sizes(c, b)
            raw = a * m * m / np.power(2.0, -c.astype(np.float64)).sum(axis=1)
            lc = (raw <= 2.5 * m) & ((c == 0).sum(axis=1) > 0)
            if prev is not None:
                pE, praw, plc = prev
                assert (raw >= praw).all(), t
                fell = E < pE
                assert not (fell & ~(plc & ~lc)).any(), t
                dips += int(fell.sum())
            prev = (E, raw, lc)
    if b == 4:
        assert dips > 0  # the case the monotonicity remark passes over does occur at m = 16
