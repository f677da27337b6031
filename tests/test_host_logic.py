"""Host-side logic without a GPU: the schedule autotuner's search and the grouping of
profiler dispatches into passes."""
from paper_1011_5599_amd import prof, tune


def test_coordinate_descent_finds_the_separable_minimum():
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30], "c": [0, 1]}
    best_at = {"a": 3, "b": 20, "c": 1}
    calls = []

    def measure(cfg):
        calls.append(dict(cfg))
        return sum((cfg[k] - best_at[k]) ** 2 for k in space) + 1.0

    cfg, t, trials = tune.coordinate_descent(measure, space, {"a": 1, "b": 10, "c": 0}, sweeps=1, repeats=2)
    assert cfg == best_at
    assert t == 1.0
    # each distinct setting measured `repeats` times, none twice over
    assert trials == len({tuple(sorted(c.items())) for c in calls})
    assert len(calls) == 2 * trials


def test_coordinate_descent_keeps_start_when_nothing_is_faster():
    cfg, t, _ = tune.coordinate_descent(lambda c: 1.0, {"x": [1, 2, 3]}, {"x": 2})
    assert cfg == {"x": 2} and t == 1.0


def _d(i, name, v):
    return (i, name, v)


def test_union_per_pass_groups_runs_and_drops_passes_after_the_fixpoint():
    U = "void hanf::(anonymous namespace)::k_union<4, 4>(hanf::PassArgs, int)"
    L = "void hanf::(anonymous namespace)::k_union_list<4, 4>(hanf::PassArgs, int)"
    top = "hanf::(anonymous namespace)::k_reduce_top(hanf::PassArgs, int)"
    init = "void hanf::(anonymous namespace)::k_init<4>(hanf::PassArgs, unsigned long)"
    other = "hanf::(anonymous namespace)::k_reduce_blocks(hanf::PassArgs, int)"
    seq = []
    for run in range(2):
        seq += [init, top]                       # initial estimate
        for p in range(4):                       # 4 enqueued passes, the last one after the fixpoint
            seq += [U, L, other, top]
    disp = [(i, name, float(10 * (i % 7) + 1)) for i, name in enumerate(seq)]
    passes = prof.union_per_pass(disp, passes_per_run=3)
    assert len(passes) == 6
    # every pass sums its k_union and k_union_list values
    expect = []
    for run in range(2):
        base = run * 18
        for p in range(3):
            i = base + 2 + 4 * p
            expect.append(disp[i][2] + disp[i + 1][2])
    assert passes == expect


def test_kernel_name_shortening():
    assert prof._short("void hanf::(anonymous namespace)::k_union<8, 4>(hanf::PassArgs, int)") == "k_union<8, 4>"
    assert prof._short("hanf::(anonymous namespace)::k_reduce_top(hanf::PassArgs, int)") == "k_reduce_top"
    assert prof._is_union("void hanf::(anonymous namespace)::k_union_list<2, 4>(hanf::PassArgs, int)")
    assert not prof._is_union("hanf::(anonymous namespace)::k_reduce_top(hanf::PassArgs, int)")
