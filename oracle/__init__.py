"""HyperANF CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow CPU reference for the GPU library: only ``tests/``, the smoke entry
point and the benchmark's CPU-baseline leg may import it. The product package
never imports it and shares no code with it.

* ``hanf_oracle.c`` (built with gcc into ``liboracle.so``): Algorithm 1 (HyperLogLog
  add/size), Algorithm 2 (the HyperANF iteration), the paper's task decomposition for
  multi-threaded passes and modified-counter skipping (Section 3.3), and the
  ball counter that Section 3.2 equates with c_t[v].
* ``stats.py``: distance cdf, density, effective diameter, moments and spid
  (Sections 4 and 5), Algorithm 3's effective-diameter interval.
* ``exact.py``: exact neighbourhood function by breadth-first search, for tiny graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, no FP contraction)."""
    src = os.path.join(_HERE, "hanf_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_hash.restype = ctypes.c_uint64
        L.orc_register_index.argtypes = [ctypes.c_uint64, ctypes.c_int]
        L.orc_register_index.restype = ctypes.c_int
        L.orc_rho_plus.argtypes = [ctypes.c_uint64, ctypes.c_int]
        L.orc_rho_plus.restype = ctypes.c_int
        L.orc_add.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_add.restype = None
        L.orc_add_hashed.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64]
        L.orc_add_hashed.restype = None
        L.orc_alpha.argtypes = [ctypes.c_int]
        L.orc_alpha.restype = ctypes.c_double
        L.orc_size.argtypes = [u8p, ctypes.c_int]
        L.orc_size.restype = ctypes.c_double
        L.orc_union.argtypes = [u8p, u8p, ctypes.c_int]
        L.orc_union.restype = None
        L.orc_init.argtypes = [ctypes.c_int32, ctypes.c_int, ctypes.c_uint64, u8p]
        L.orc_init.restype = None
        L.orc_sizes.argtypes = [ctypes.c_int32, ctypes.c_int, u8p, ctypes.POINTER(ctypes.c_double)]
        L.orc_sizes.restype = None
        L.orc_sum_sizes.argtypes = [ctypes.c_int32, ctypes.c_int, u8p]
        L.orc_sum_sizes.restype = ctypes.c_double
        L.orc_sum_sizes_mt.argtypes = [ctypes.c_int32, ctypes.c_int, u8p, ctypes.c_int]
        L.orc_sum_sizes_mt.restype = ctypes.c_double
        L.orc_pass.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int, u8p, u8p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_int64)]
        L.orc_pass.restype = ctypes.c_int64
        L.orc_run.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int, ctypes.c_uint64,
                              ctypes.c_int32, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
        L.orc_run.restype = ctypes.c_int
        L.orc_ball_counter.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_int32, ctypes.c_int32, u8p,
                                       ctypes.POINTER(ctypes.c_int64)]
        L.orc_ball_counter.restype = ctypes.c_int
        L.orc_balls_check.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int, ctypes.c_uint64,
                                      u8p, ctypes.c_int32, ctypes.c_int,
                                      np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"),
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.orc_balls_check.restype = ctypes.c_int64
        for f in (L.orc_broadword_L,):
            f.argtypes = [ctypes.c_int]
            f.restype = ctypes.c_uint64
        for f in (L.orc_broadword_less, L.orc_broadword_max):
            f.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
            f.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)  # a valid pointer; never read when there are no arcs
    return rp, ci


def hash64(seed: int, x: int) -> int:
    return _load().orc_hash(seed, x)


def register_index(h: int, b: int) -> int:
    return _load().orc_register_index(h, b)


def rho_plus(h: int, b: int) -> int:
    return _load().orc_rho_plus(h, b)


def alpha(m: int) -> float:
    return _load().orc_alpha(m)


def add(M: np.ndarray, b: int, seed: int, x: int) -> None:
    _load().orc_add(M, b, seed, x)


def add_hashed(M: np.ndarray, b: int, h: int) -> None:
    _load().orc_add_hashed(M, b, h)


def size(M: np.ndarray, b: int) -> float:
    return _load().orc_size(np.ascontiguousarray(M, dtype=np.uint8), b)


def union(M: np.ndarray, N: np.ndarray) -> None:
    _load().orc_union(M, np.ascontiguousarray(N, dtype=np.uint8), M.size)


def broadword_L(k: int) -> int:
    return _load().orc_broadword_L(k)


def broadword_less(x: int, y: int, k: int) -> int:
    return _load().orc_broadword_less(x, y, k)


def broadword_max(x: int, y: int, k: int) -> int:
    return _load().orc_broadword_max(x, y, k)


def init(n: int, b: int, seed: int) -> np.ndarray:
    """Counters after Algorithm 2's initialisation, shape (n, 2^b) uint8."""
    c = np.zeros((max(n, 1), 1 << b), np.uint8)
    _load().orc_init(n, b, seed, c)
    return c[:n]


def sizes(c: np.ndarray, b: int) -> np.ndarray:
    """size() of every counter (Algorithm 1), one per row of c."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    out = np.zeros(max(c.shape[0], 1), np.float64)
    _load().orc_sizes(c.shape[0], b, c if c.size else np.zeros(1, np.uint8),
                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out[: c.shape[0]]


def sum_sizes(c: np.ndarray, b: int, nthreads: int = 1) -> float:
    """N_hat = sum of size() over the counters, in node order (Neumaier summation); the
    sizes may be computed by several threads (the same value)."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    if nthreads > 1 and c.shape[0] > 0:
        return _load().orc_sum_sizes_mt(c.shape[0], b, c, nthreads)
    return _load().orc_sum_sizes(c.shape[0], b, c if c.size else np.zeros(1, np.uint8))


def step(row_ptr, col_idx, b: int, cur: np.ndarray, modified=None, nthreads: int = 1):
    """One synchronous pass. Returns (next, changed_flags, n_changed, n_unions)."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    cur = np.ascontiguousarray(cur, dtype=np.uint8)
    nxt = np.empty_like(cur)
    mod_out = np.zeros(max(n, 1), np.uint8)
    mod_ptr = None
    if modified is not None:
        modified = np.ascontiguousarray(modified, dtype=np.uint8)
        mod_ptr = modified.ctypes.data
    maxed = ctypes.c_int64()
    changed = _load().orc_pass(n, rp, ci, b, cur, nxt, mod_ptr, mod_out.ctypes.data, nthreads,
                               ctypes.byref(maxed))
    return nxt, mod_out[:n], int(changed), int(maxed.value)


def run(row_ptr, col_idx, b: int, seed: int, max_passes: int | None = None,
        skip_unmodified: bool = True, nthreads: int = 1, want_regs: bool = False,
        want_nt: bool = True):
    """Algorithm 2 to stabilisation. Returns (nt[0..T] or None, T, final counters or None)."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    if max_passes is None:
        max_passes = n + 1
    cap = max_passes + 2
    nt = np.zeros(cap, np.float64)
    T = ctypes.c_int32()
    regs = np.zeros((n, 1 << b), np.uint8) if want_regs else None
    rc = _load().orc_run(n, rp, ci, b, seed, max_passes, int(skip_unmodified), nthreads,
                         nt.ctypes.data if want_nt else None, cap,
                         ctypes.byref(T), regs.ctypes.data if want_regs else None)
    if rc != 0:
        raise RuntimeError(f"oracle run failed with code {rc}")
    return (nt[: T.value + 1].copy() if want_nt else None), T.value, regs


def run_steps(row_ptr, col_idx, b: int, seed: int, max_passes: int | None = None,
              skip_unmodified: bool = True, nthreads: int = 1):
    """Algorithm 2 step by step, yielding (t, counters c_t, N_hat(t)) for t = 0..T; the
    generator ends after the pass that changes nothing."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    if max_passes is None:
        max_passes = n + 1
    cur = init(n, b, seed)
    mod = np.ones(n, np.uint8) if skip_unmodified else None
    t = 0
    while True:
        yield t, cur, sum_sizes(cur, b, nthreads)
        if t >= max_passes:
            raise RuntimeError("oracle did not stabilise")
        nxt, mod_out, changed, _ = step(rp, ci, b, cur, mod if skip_unmodified else None, nthreads)
        if changed == 0:
            return
        cur = nxt
        if skip_unmodified:
            mod = mod_out
        t += 1


def ball_counter(row_ptr, col_idx, b: int, seed: int, v: int, t: int):
    """Counter fed with every node of B(v, t); returns (registers, |B(v,t)|)."""
    rp, ci = _csr(row_ptr, col_idx)
    M = np.zeros(1 << b, np.uint8)
    sz = ctypes.c_int64()
    rc = _load().orc_ball_counter(rp.size - 1, rp, ci, b, seed, v, t, M, ctypes.byref(sz))
    if rc != 0:
        raise MemoryError("oracle ball counter")
    return M, int(sz.value)


def balls_check(row_ptr, col_idx, b: int, seed: int, counters, nthreads: int = 1):
    """Checks c_t[v] == counter of B(v, t) (Section 3.2) for every node v and every t, by a
    breadth-first search from every node; `counters` holds c_0 .. c_T (each n x m uint8).
    Returns (mismatches, (first bad v, t) or None, exact N(0..D)) where N(t) counts the
    pairs at distance <= t, self-pairs included, and D is the largest finite distance."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    T = len(counters) - 1
    regs = np.ascontiguousarray(np.stack([np.asarray(c, np.uint8).reshape(n, -1) for c in counters]))
    hist = np.zeros(n + 1, np.int64)
    bv, bt = ctypes.c_int32(), ctypes.c_int32()
    bad = _load().orc_balls_check(n, rp, ci, b, seed, regs.reshape(-1), T, nthreads, hist, hist.size,
                                  ctypes.byref(bv), ctypes.byref(bt))
    if bad < 0:
        raise MemoryError("oracle balls check")
    D = int(np.nonzero(hist)[0].max())
    return int(bad), ((bv.value, bt.value) if bad else None), np.cumsum(hist[: D + 1]).astype(np.float64)
