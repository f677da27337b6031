"""Autotuner for the work schedule of the HyperANF kernels.

The union kernel's schedule has knobs: the largest node handled by one lane group
(`light_max`), the arcs per wavefront chunk (`chunk_arcs`), nodes per light tile
(`tile_nodes`), loads in flight per lane (`unroll`), the gather-all switch
(`dense_switch`), and, for batched runs, how many seeds share a node row (`seeds_per_row`)
and how many graphs share one batch (`group`). The
best values depend on the degree distribution, m and the batch mix. The tuner runs the
caller's workload under candidate settings and keeps the fastest, by coordinate descent
from the defaults. Every setting gives identical results (max is order-free), so tuning
only changes time.
"""
from __future__ import annotations

import json
import os
import time

SPACE = {
    "light_max": [16, 32, 64, 128],
    "chunk_arcs": [256, 512, 1024, 2048],
    "tile_nodes": [0, 64, 128, 256],
    "unroll": [0, 2, 4, 8],
    "dense_switch": [0, 2, 4, 8],
}

DEFAULTS = {"light_max": 0, "chunk_arcs": 0, "tile_nodes": 0, "unroll": 0, "dense_switch": 4}
# 0: the library default for the run's row width (light_max and chunk_arcs grow with it) and
# register format (unroll)
# batched runs also tune `seeds_per_row` (0 = as many seeds per node row as fit) and `group`


def coordinate_descent(measure, space=None, start=None, sweeps=1, repeats=2, log=None):
    """Minimises measure(config) -> seconds over `space` (dict of candidate lists) by
    trying each knob's values with the others fixed, `sweeps` times. Each measurement is
    the minimum of `repeats` calls. Returns (best config, best time, trials)."""
    space = dict(SPACE if space is None else space)
    cur = dict(DEFAULTS if start is None else start)
    for k in space:
        cur.setdefault(k, space[k][0])
    cache = {}

    def timed(cfg):
        key = tuple(sorted(cfg.items()))
        if key not in cache:
            cache[key] = min(measure(dict(cfg)) for _ in range(repeats))
            if log:
                log(f"[tune] {cfg} -> {1e3 * cache[key]:.3f} ms")
        return cache[key]

    best = timed(cur)
    for _ in range(sweeps):
        for k, vals in space.items():
            for v in vals:
                if v == cur[k]:
                    continue
                cand = dict(cur)
                cand[k] = v
                t = timed(cand)
                if t < best:
                    best, cur = t, cand
    return cur, best, len(cache)


def load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(path, key, cfg, seconds):
    data = load_cache(path)
    data[key] = {"config": cfg, "seconds": seconds, "when": time.time()}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
