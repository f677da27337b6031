"""Exact neighbourhood function by breadth-first search — TEST INFRASTRUCTURE ONLY.

N(t) = number of pairs (x, y) with d(x, y) <= t, self-pairs included (N(0) = n), the
definition that Algorithm 2 and the two-clique closed form of Section 4 use. Only for
tiny graphs: all-pairs distances come from scipy's unweighted shortest paths, or from
a pure-Python BFS for the smallest cases.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def bfs_distances(row_ptr, col_idx, source: int):
    """Distances from `source` following arcs forward; -1 = unreachable."""
    n = len(row_ptr) - 1
    dist = [-1] * n
    dist[source] = 0
    q = deque([source])
    while q:
        u = q.popleft()
        for a in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            w = int(col_idx[a])
            if dist[w] < 0:
                dist[w] = dist[u] + 1
                q.append(w)
    return dist


def ball(row_ptr, col_idx, v: int, t: int):
    """B(v, t): the nodes reachable from v in at most t arcs."""
    d = bfs_distances(row_ptr, col_idx, v)
    return [u for u, x in enumerate(d) if 0 <= x <= t]


def distance_matrix(row_ptr, col_idx):
    n = len(row_ptr) - 1
    if n <= 64:
        return np.array([bfs_distances(row_ptr, col_idx, s) for s in range(n)], dtype=np.int64)
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    data = np.ones(len(col_idx), dtype=np.float64)
    A = sp.csr_matrix((data, np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))
    D = shortest_path(A, method="D", directed=True, unweighted=True)
    out = np.where(np.isinf(D), -1, D).astype(np.int64)
    return out


def neighbourhood_function(row_ptr, col_idx):
    """Exact N(0..D), D = the largest finite distance."""
    D = distance_matrix(row_ptr, col_idx)
    finite = D[D >= 0]
    dmax = int(finite.max()) if finite.size else 0
    counts = np.bincount(finite, minlength=dmax + 1)
    return np.cumsum(counts).astype(np.float64)
