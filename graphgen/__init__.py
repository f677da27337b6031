"""Seeded synthetic input graphs (CSR int32) shared by the tests and the benchmark.

This module builds inputs only: it holds none of HyperANF's arithmetic. Large
generators (R-MAT, Erdos-Renyi, web-like) live in ``graphgen.cpp`` (built with
g++ into ``libgraphgen.so``); small structured graphs are built here in numpy.

A graph is returned as ``(row_ptr, col_idx)``: ``row_ptr`` int32[n+1],
``col_idx`` int32[arcs]; the successors of v are ``col_idx[row_ptr[v]:row_ptr[v+1]]``,
sorted ascending.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile graphgen.cpp into libgraphgen.so (g++, OpenMP)."""
    src = os.path.join(_HERE, "graphgen.cpp")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        out = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
               ctypes.POINTER(i32p), ctypes.POINTER(i32p)]
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64] + out
        lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64] + out
        lib.gg_web.argtypes = ([ctypes.c_int32] + [ctypes.c_double] * 7 + [ctypes.c_uint64, ctypes.c_int32]
                               + out)
        lib.gg_web_hosts.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, i32p]
        for f in (lib.gg_rmat, lib.gg_er, lib.gg_web, lib.gg_web_hosts):
            f.restype = ctypes.c_int
        lib.gg_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _call(fn, *args):
    lib = _load()
    n = ctypes.c_int32()
    arcs = ctypes.c_int64()
    rp = ctypes.POINTER(ctypes.c_int32)()
    ci = ctypes.POINTER(ctypes.c_int32)()
    rc = fn(*args, ctypes.byref(n), ctypes.byref(arcs), ctypes.byref(rp), ctypes.byref(ci))
    if rc != 0:
        raise ValueError(f"graph generator failed with code {rc}")
    try:
        row_ptr = np.ctypeslib.as_array(rp, shape=(n.value + 1,)).copy()
        col_idx = (np.ctypeslib.as_array(ci, shape=(arcs.value,)).copy()
                   if arcs.value > 0 else np.zeros(0, np.int32))
    finally:
        lib.gg_free(ctypes.cast(rp, ctypes.c_void_p))
        lib.gg_free(ctypes.cast(ci, ctypes.c_void_p))
    return row_ptr, col_idx


def rmat(scale: int, target: int, a=0.57, b=0.19, c=0.19, symmetric=False, seed=1, n=0):
    """R-MAT on 2^scale ids: `target` distinct arcs (directed) or edges (symmetric, 2x arcs).
    With n > 0 the graph has n nodes: samples with an endpoint >= n are rejected."""
    lib = _load()
    return _call(lib.gg_rmat, scale, target, a, b, c, int(symmetric), seed, n)


def erdos_renyi(n: int, target: int, seed=1):
    """Directed G(n, M): exactly `target` distinct non-loop arcs."""
    lib = _load()
    return _call(lib.gg_er, n, target, seed)


def web(n: int, host_mean=1000.0, host_sigma=1.0, deg_mean=20.0, deg_sigma=1.0, p_intra=0.8,
        geo_p=0.25, gamma=2.1, seed=24, keep_kind=False):
    """Web-like directed graph: lognormal hosts, local intra-host arcs, power-law in-degree.
    A duplicate target is drawn again: with keep_kind=False with a new intra/inter choice
    (fewer than p_intra of the kept arcs are then intra-host), with keep_kind=True within
    the arc's own kind (p_intra holds for the kept arcs, up to nodes whose nearby ids run
    out)."""
    lib = _load()
    return _call(lib.gg_web, n, host_mean, host_sigma, deg_mean, deg_sigma, p_intra, geo_p,
                 gamma, seed, int(keep_kind))


def web_hosts(n: int, host_mean=1000.0, host_sigma=1.0, seed=24) -> np.ndarray:
    """First id of each node's host in `web` with the same arguments (int32[n])."""
    lib = _load()
    out = np.zeros(n, np.int32)
    if lib.gg_web_hosts(n, host_mean, host_sigma, seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) != 0:
        raise ValueError("web_hosts: bad arguments")
    return out


# ---------------------------------------------------------------- small structured graphs

def from_arcs(n: int, arcs) -> tuple[np.ndarray, np.ndarray]:
    """CSR from an iterable of (u, v) arcs; keeps duplicates and self-loops as given,
    successor lists sorted."""
    a = np.asarray(list(arcs), dtype=np.int64).reshape(-1, 2)
    order = np.lexsort((a[:, 1], a[:, 0])) if len(a) else np.zeros(0, np.int64)
    a = a[order]
    row_ptr = np.zeros(n + 1, np.int64)
    if len(a):
        np.add.at(row_ptr, a[:, 0] + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, a[:, 1].astype(np.int32).copy()


def empty(n: int):
    return np.zeros(n + 1, np.int32), np.zeros(0, np.int32)


def directed_cycle(n: int):
    return from_arcs(n, [(i, (i + 1) % n) for i in range(n)])


def directed_path(n: int):
    return from_arcs(n, [(i, i + 1) for i in range(n - 1)])


def complete(n: int):
    return from_arcs(n, [(i, j) for i in range(n) for j in range(n) if i != j])


def star_out(n: int):
    """Node 0 points to every other node (one heavy row)."""
    return from_arcs(n, [(0, j) for j in range(1, n)])


def star_in(n: int):
    """Every node points to node 0."""
    return from_arcs(n, [(j, 0) for j in range(1, n)])


def clique_path_clique(k: int, l: int):
    """Two k-cliques joined by a one-way path of l nodes: left clique nodes 0..k-1, path
    nodes k..k+l-1, right clique k+l..2k+l-1. Every left node points to the first path node,
    the path runs forward, the last path node points to every right node."""
    n = 2 * k + l
    arcs = []
    for base in (0, k + l):
        arcs += [(base + i, base + j) for i in range(k) for j in range(k) if i != j]
    p0, pl = k, k + l - 1
    arcs += [(i, p0) for i in range(k)]
    arcs += [(k + i, k + i + 1) for i in range(l - 1)]
    arcs += [(pl, k + l + j) for j in range(k)]
    return from_arcs(n, arcs)


def limit_graph(heavy_log2: int = 21, degree: int = 1023, light_log2: int = 20):
    """A graph with exactly the library's largest arc count, 2^31 - 2^20, at the default sizes
    (2^21 * 1023 + 2^20 = 2,146,435,072 arcs, 8.6 GB of col_idx), with arc positions near
    2^31 in both kinds of rows: the first 2^heavy_log2 nodes have
    `degree` successors each, (v * degree + j) mod N for j < degree (an expander: every node
    is reached within a few steps); the last 2^light_log2 nodes have one successor each,
    (7 u + 3) mod N, and their rows sit at the end of col_idx. N is the node count.
    Deterministic, no random draws."""
    H, L = 1 << heavy_log2, 1 << light_log2
    N = H + L
    if (H - 1) * degree + degree - 1 >= 1 << 31:
        raise ValueError("v * degree + j must fit in int32")
    row_ptr = np.empty(N + 1, np.int64)
    row_ptr[: H + 1] = np.arange(H + 1, dtype=np.int64) * degree
    row_ptr[H + 1:] = H * degree + np.arange(1, L + 1, dtype=np.int64)
    col_idx = np.empty(H * degree + L, np.int32)
    j = np.arange(degree, dtype=np.int32)
    step = 1 << 16
    for s in range(0, H, step):
        v = np.arange(s, min(H, s + step), dtype=np.int32)
        col_idx[s * degree:(s + v.size) * degree] = ((v[:, None] * np.int32(degree) + j) % np.int32(N)).ravel()
    u = np.arange(H, N, dtype=np.int64)
    col_idx[H * degree:] = ((7 * u + 3) % N).astype(np.int32)
    return row_ptr.astype(np.int32), col_idx


# ---------------------------------------------------------------- the named workloads

WORKLOADS = {
    # directed R-MAT scale 14, 262,144 distinct arcs; log2m 4, hash seed 1
    "rmat14": dict(kind="rmat", scale=14, target=262_144, symmetric=False, graph_seed=14,
                   log2m=4, seed=1),
    # symmetric R-MAT scale 22, 2^25 edges -> 2^26 arcs; log2m 6, hash seed 7
    "rmat22sym": dict(kind="rmat", scale=22, target=1 << 25, symmetric=True, graph_seed=22,
                      log2m=6, seed=7),
    # web-like, 2^24 nodes, 80% of the kept arcs intra-host (the intra/inter choice is kept
    # when a duplicate target is redrawn); log2m 7, hash seed 1
    "web24": dict(kind="web", n=1 << 24, graph_seed=24, keep_kind=True, log2m=7, seed=1),
}


def batch_sizes(count: int = 512, seed: int = 4, lo: int = 1 << 8, hi: int = 1 << 16,
                median: float = 4096.0, sigma: float = 1.0):
    """Node counts round(exp(X)), X ~ Normal(ln median, sigma), redrawn outside [lo, hi]."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        x = int(round(math.exp(rng.normal(math.log(median), sigma))))
        if lo <= x <= hi:
            out.append(x)
    return out


def batch_graphs(count: int = 512, seed: int = 4):
    """The many-graph workload: `count` graphs with lognormal node counts in [2^8, 2^16]
    (median 2^12); the first half directed Erdos-Renyi with 8 n distinct arcs, the second
    half directed R-MAT (a=.57, b=.19, c=.19) on the next power of two, endpoints >= n
    rejected, 16 n distinct arcs. Graph i uses graph seed 1000 + i."""
    sizes = batch_sizes(count, seed)
    graphs = []
    for i, n in enumerate(sizes):
        if i < count // 2:
            graphs.append(erdos_renyi(n, 8 * n, seed=1000 + i))
        else:
            scale = max(1, (n - 1).bit_length())
            graphs.append(rmat(scale, 16 * n, seed=1000 + i, n=n))
    return graphs


def serve_requests(count: int = 96, trace_seed: int = 5, lo: int = 1 << 10, hi: int = 1 << 22,
                   median: float = 1 << 16, sigma: float = 1.5):
    """The request stream of the serving workload: node counts round(exp(X)),
    X ~ Normal(ln median, sigma), clipped to [lo, hi]; generator R-MAT (16 n distinct arcs on
    the next power of two, endpoints >= n rejected) or web-like (out-degree mean 20), with
    probability 1/2 each; log2m uniform over {4, 6, 8}; hash seed = request id. Returns a list
    of dicts (rid, kind, n, log2m, seed, graph)."""
    rng = np.random.default_rng(trace_seed)
    out = []
    for rid in range(count):
        n = int(min(hi, max(lo, round(math.exp(rng.normal(math.log(median), sigma))))))
        kind = "rmat" if rng.random() < 0.5 else "web"
        log2m = int(rng.choice([4, 6, 8]))
        gseed = 50_000 + rid
        if kind == "rmat":
            g = rmat(max(1, (n - 1).bit_length()), 16 * n, seed=gseed, n=n)
        else:
            g = web(n, seed=gseed)
        out.append(dict(rid=rid, kind=kind, n=n, log2m=log2m, seed=rid + 1, graph=g))
    return out


def disjoint_union(graphs):
    """(graph_off[G+1], row_ptr[N+1], col_idx[E]) of graphs laid side by side (global ids)."""
    offs = [0]
    for rp, _ in graphs:
        offs.append(offs[-1] + len(rp) - 1)
    rps = []
    cis = []
    arc_base = 0
    for (rp, ci), o in zip(graphs, offs[:-1]):
        rps.append(rp[:-1].astype(np.int64) + arc_base)
        cis.append(ci.astype(np.int64) + o)
        arc_base += len(ci)
    row_ptr = np.concatenate(rps + [np.array([arc_base], np.int64)]).astype(np.int32)
    col_idx = np.concatenate(cis).astype(np.int32) if cis else np.zeros(0, np.int32)
    return np.array(offs, np.int32), row_ptr, col_idx


def workload_graph(spec: dict):
    """Generate the graph for a workload spec (see WORKLOADS)."""
    if spec["kind"] == "rmat":
        return rmat(spec["scale"], spec["target"], symmetric=spec["symmetric"],
                    seed=spec["graph_seed"])
    if spec["kind"] == "web":
        return web(spec["n"], seed=spec["graph_seed"], keep_kind=spec.get("keep_kind", False))
    if spec["kind"] == "er":
        return erdos_renyi(spec["n"], spec["target"], seed=spec["graph_seed"])
    raise ValueError(spec["kind"])
