"""CPU pins of the reference the node-order tests compare the device against: in-degree
class levels and the hubs-first order, checked on hand-worked cases (no GPU)."""
import numpy as np

from test_gpu_order import degree_levels, expected_order


def test_levels_by_hand():
    # below 8 the level is the in-degree; from 8 on, 8 levels per octave from the three
    # bits below the leading one: 8..15 -> 8..15, 16/17 -> 16, 18/19 -> 17, ..., 31 -> 23,
    # 32..35 -> 24, 60..63 -> 31, 64..71 -> 32
    d = [0, 1, 2, 7, 8, 15, 16, 17, 18, 19, 30, 31, 32, 35, 36, 63, 64, 71, 72, 1000]
    want = [0, 1, 2, 7, 8, 15, 16, 16, 17, 17, 23, 23, 24, 24, 25, 31, 32, 32, 33, 8 * 7 + 7]
    assert degree_levels(d).tolist() == want
    # the largest in-degree an int32 graph can have still gets a level below 240
    assert degree_levels([2**31 - 1]).tolist() == [8 * 28 + 7]


def test_order_by_hand():
    # in-degrees of nodes 0..7; levels equal the in-degrees here (all below 8)
    indeg = np.array([1, 5, 0, 5, 7, 2, 5, 1])
    # K = 1: level 7 holds one node (4) -> hubs [4]
    order, hubs = expected_order(indeg, 1)
    assert hubs == 1 and order.tolist() == [4, 0, 1, 2, 3, 5, 6, 7]
    # K = 3: level 7 (1 node) fits, level 5 (3 more: 4 in all) does not -> still [4]
    order, hubs = expected_order(indeg, 3)
    assert hubs == 1 and order.tolist() == [4, 0, 1, 2, 3, 5, 6, 7]
    # K = 4: levels 7 and 5 -> hubs 4, then 1, 3, 6 by id; the rest by id
    order, hubs = expected_order(indeg, 4)
    assert hubs == 4 and order.tolist() == [4, 1, 3, 6, 0, 2, 5, 7]
    # K = 7: every node with an arc in (levels 7, 5, 2, 1); node 2 (none) last
    order, hubs = expected_order(indeg, 7)
    assert hubs == 7 and order.tolist() == [4, 1, 3, 6, 5, 0, 7, 2]
    # K = 0, or a top level larger than K: the caller's order
    assert expected_order(indeg, 0)[0].tolist() == list(range(8))
    assert expected_order(np.full(10, 3), 5)[0].tolist() == list(range(10))
    # a permutation in every case
    for K in range(10):
        assert sorted(expected_order(indeg, K)[0].tolist()) == list(range(8))
