"""MI355X HyperANF: Python binding of libhanf.so (the C ABI declared in include/hanf.h).

HyperANF (Boldi, Rosa, Vigna, arXiv:1011.5599) approximates the neighbourhood function
N(t) of a graph with one HyperLogLog counter per node; every pass replaces each counter
by the register-wise max of itself and its successors' counters, until no counter
changes. The functions below marshal arguments to the library of the same names; every
step of the computation runs in its HIP kernels. Host arrays are numpy arrays; device
arrays are torch tensors on the context's device (torch serves as allocator and stream
provider only). There is no fallback: if libhanf.so is missing, importing the functions'
library raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhanf.so")

HANF_OK = 0
HANF_DONE = 1
HANF_BUSY = 2
HANF_EINVAL = -1
HANF_ENOMEM = -2
HANF_EDEVICE = -3
HANF_ESTATE = -4
HANF_ERANGE = -5
HANF_EMAXITER = -6

HANF_HOST_PTRS = 0
HANF_DEVICE_PTRS = 1
HANF_MAX_NODES = 2146435072  # 2^31 - 2^20: the most nodes, and arcs, of a graph or batch
HANF_MAX_ARCS = 2146435072

HANF_OPT_FRONTIER = 1
HANF_OPT_MAX_PASSES = 2
HANF_OPT_LIGHT_MAX = 3
HANF_OPT_CHUNK_ARCS = 4
HANF_OPT_TIMING = 5
HANF_OPT_BATCH = 6
HANF_OPT_TILE_NODES = 7
HANF_OPT_DENSE_SWITCH = 8
HANF_OPT_SYSTOLIC = 9
HANF_OPT_SEEDS_PER_ROW = 10
HANF_OPT_PACKED5 = 11
HANF_OPT_HUBS = 12
HANF_OPT_STAGE = 13
HANF_OPT_FORWARD = 14
HANF_FP_COPY_GRAPH = 1
HANF_FP_TRANSPOSE = 2
HANF_FP_PACKED5 = 4
HANF_FP_ORDER = 8
HANF_OPT_UNROLL = 100
HANF_OPT_UNION_POLICY = 101  # 0 auto, 1 one wavefront per work unit, 2 persistent sparse kernel
HANF_OPT_TRANSPOSE_COUNTING = 102  # 1: build transposes with per-node counters (test option)
HANF_OPT_STAGE_BYTES = 103  # LDS bytes per wavefront of a staged light tile (tuning option)
HANF_OPT_COUNT_NEAR = 104  # 1: instrumented union kernels count arcs_near (measurement option)

ERROR_NAMES = {HANF_EINVAL: "EINVAL", HANF_ENOMEM: "ENOMEM", HANF_EDEVICE: "EDEVICE",
               HANF_ESTATE: "ESTATE", HANF_ERANGE: "ERANGE", HANF_EMAXITER: "EMAXITER"}


class hanf_stats_t(ctypes.Structure):
    _fields_ = [("ed", ctypes.c_double), ("ied", ctypes.c_double), ("avg_dist", ctypes.c_double),
                ("var", ctypes.c_double), ("spid", ctypes.c_double), ("n_max", ctypes.c_double),
                ("d_lo", ctypes.c_double), ("d_hi", ctypes.c_double), ("T", ctypes.c_int32),
                ("distinct", ctypes.c_int32)]


class hanf_pass_t(ctypes.Structure):
    _fields_ = [("changed", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64),
                ("arcs_gathered", ctypes.c_int64), ("rows_written", ctypes.c_int64),
                ("rows_read", ctypes.c_int64),
                ("union_ms", ctypes.c_float), ("finalize_ms", ctypes.c_float),
                ("reduce_ms", ctypes.c_float), ("gather_all", ctypes.c_int32),
                ("systolic", ctypes.c_int32), ("arcs_signalled", ctypes.c_int64),
                ("signal_ms", ctypes.c_float), ("arcs_local", ctypes.c_int64), ("arcs_near", ctypes.c_int64),
                ("flag_summary", ctypes.c_int32)]


class HanfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def lib():
    """The loaded libhanf.so. Raises if it has not been built.

    PyTorch ships its own copy of the HIP runtime, which its libraries load under the name
    libamdhip64.so. libhanf.so needs libamdhip64.so.7, the soname of both copies. Importing
    torch first makes libhanf.so bind to the runtime torch already loaded, so the process
    has one HIP runtime and torch's tensors and streams can be handed to the library. Two
    runtimes in one process are refused."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(or python -m paper_1011_5599_amd.build)")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes loaded in one process: {rts}")
        vp = ctypes.c_void_p
        i32, i64, u32, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        sig = {
            "hanf_create": ([ctypes.c_int, vp, ctypes.POINTER(vp)], ctypes.c_int),
            "hanf_destroy": ([vp], None),
            "hanf_set_option": ([vp, ctypes.c_int, i64], ctypes.c_int),
            "hanf_load_csr": ([vp, i32, i64, vp, vp, u32], ctypes.c_int),
            "hanf_load_transpose": ([vp, i32, i64, vp, vp, u32], ctypes.c_int),
            "hanf_build_transpose": ([vp], ctypes.c_int),
            "hanf_transpose_self": ([vp], ctypes.c_int),
            "hanf_init_counters": ([vp, i32, u64], ctypes.c_int),
            "hanf_iterate": ([vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)], ctypes.c_int),
            "hanf_read_nt": ([vp, vp, i32, ctypes.POINTER(i32)], ctypes.c_int),
            "hanf_read_registers": ([vp, vp, i64, u32], ctypes.c_int),
            "hanf_read_estimates": ([vp, vp, i64, u32], ctypes.c_int),
            "hanf_read_order": ([vp, vp, i32, u32], ctypes.c_int),
            "hanf_batch_read_estimates": ([vp, i32, vp, i64, u32], ctypes.c_int),
            "hanf_write_registers": ([vp, vp, i64, i32, vp, i32, u32], ctypes.c_int),
            "hanf_stats": ([vp, dbl, dbl, i32, ctypes.POINTER(hanf_stats_t)], ctypes.c_int),
            "hanf_read_pass_log": ([vp, vp, i32, ctypes.POINTER(i32)], ctypes.c_int),
            "hanf_footprint": ([i32, i64, i32, i32, ctypes.POINTER(i64)], ctypes.c_int),
            "hanf_last_error": ([vp], ctypes.c_char_p),
            "hanf_bytemax_words": ([ctypes.c_int, vp, vp, vp, i64], ctypes.c_int),
            "hanf_gathermax_lanes": ([ctypes.c_int, vp, ctypes.c_int32, ctypes.c_int32, vp, i64], ctypes.c_int),
            "hanf_max5_groups": ([ctypes.c_int, vp, vp, vp, i64], ctypes.c_int),
            "hanf_stats_nt": ([vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp],
                              ctypes.c_int),
            "hanf_load_batch": ([vp, i32, vp, vp, vp, vp, i32, u32], ctypes.c_int),
            "hanf_load_batch_list": ([vp, i32, vp, vp, vp, vp, i32, u32], ctypes.c_int),
            "hanf_enqueue": ([vp, i32], ctypes.c_int),
            "hanf_poll": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
            "hanf_init_batch": ([vp, i32, vp], ctypes.c_int),
            "hanf_batch_info": ([vp, ctypes.POINTER(i32), vp], ctypes.c_int),
            "hanf_batch_read_nt": ([vp, i32, vp, i32, ctypes.POINTER(i32)], ctypes.c_int),
            "hanf_batch_read_registers": ([vp, i32, vp, i64, u32], ctypes.c_int),
            "hanf_batch_stats": ([vp, i32, dbl, dbl, i32, ctypes.POINTER(hanf_stats_t)], ctypes.c_int),
            "hanf_batch_stats_all": ([vp, dbl, dbl, i32, vp], ctypes.c_int),
            "hanf_batch_stats_all_noalloc": ([vp, dbl, dbl, i32, vp], ctypes.c_int),
            "hanf_batch_seed_summary": ([vp, dbl, i32, vp], ctypes.c_int),
            "hanf_device_bytes": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
            "hanf_trim": ([vp], ctypes.c_int),
        }
        missing = []
        for name, (args, res) in sig.items():
            try:
                f = getattr(L, name)
            except AttributeError:  # a library built from older sources: that call raises
                missing.append(name)
                continue
            f.argtypes = args
            f.restype = res
        for name in missing:
            setattr(L, name, _missing_symbol(name))
        _lib = L
    return _lib


def _missing_symbol(name):
    def call(*_args):
        raise ImportError(f"{LIB_PATH} does not export {name}: rebuild it from the current sources")
    return call


def hanf_last_error(ctx=None) -> str:
    msg = lib().hanf_last_error(ctx)
    return msg.decode() if msg else ""


def _check(rc: int, ctx=None, ok=(HANF_OK,)) -> int:
    if rc not in ok:
        raise HanfError(rc, hanf_last_error(ctx))
    return rc


def _is_tensor(x) -> bool:
    return hasattr(x, "data_ptr") and hasattr(x, "is_cuda")


def _ptr(x, dtype):
    """(pointer, flags, keepalive) for a numpy array (host) or a torch tensor (device)."""
    if _is_tensor(x):
        if not x.is_cuda:
            x = x.numpy()
        else:
            if not x.is_contiguous():
                raise ValueError("device tensor must be contiguous")
            return x.data_ptr(), HANF_DEVICE_PTRS, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, HANF_HOST_PTRS, a


# ------------------------------------------------------------------ the C ABI, by name

def hanf_create(device: int = 0, stream=None):
    """Context on HIP device `device`; `stream` is a hipStream_t handle (int), e.g.
    torch.cuda.current_stream().cuda_stream, or None for a library-owned stream."""
    out = ctypes.c_void_p()
    _check(lib().hanf_create(device, stream, ctypes.byref(out)))
    return out


def hanf_destroy(ctx) -> None:
    lib().hanf_destroy(ctx)


def hanf_set_option(ctx, option: int, value: int) -> None:
    _check(lib().hanf_set_option(ctx, option, int(value)), ctx)


def hanf_load_csr(ctx, row_ptr, col_idx):
    """CSR int32 graph: numpy arrays (copied) or torch tensors on the device (borrowed:
    keep them alive). Returns the objects to keep alive."""
    p_rp, f1, k1 = _ptr(row_ptr, np.int32)
    p_ci, f2, k2 = _ptr(col_idx, np.int32)
    if f1 != f2:
        raise ValueError("row_ptr and col_idx must both be host or both be device arrays")
    n = (k1.numel() if _is_tensor(k1) else k1.size) - 1
    arcs = k2.numel() if _is_tensor(k2) else k2.size
    _check(lib().hanf_load_csr(ctx, n, arcs, p_rp, p_ci if arcs > 0 else None, f1), ctx)
    return (k1, k2)


def hanf_load_transpose(ctx, row_ptr_t, col_idx_t):
    """Predecessor lists of the loaded graph (CSR int32, numpy or device tensors; device
    tensors are borrowed). Returns the objects to keep alive."""
    p_rp, f1, k1 = _ptr(row_ptr_t, np.int32)
    p_ci, f2, k2 = _ptr(col_idx_t, np.int32)
    if f1 != f2:
        raise ValueError("row_ptr_t and col_idx_t must both be host or both be device arrays")
    n = (k1.numel() if _is_tensor(k1) else k1.size) - 1
    arcs = k2.numel() if _is_tensor(k2) else k2.size
    _check(lib().hanf_load_transpose(ctx, n, arcs, p_rp, p_ci if arcs > 0 else None, f1), ctx)
    return (k1, k2)


def hanf_build_transpose(ctx) -> None:
    _check(lib().hanf_build_transpose(ctx), ctx)


def hanf_transpose_self(ctx) -> None:
    _check(lib().hanf_transpose_self(ctx), ctx)


def hanf_init_counters(ctx, log2m: int, seed: int) -> None:
    _check(lib().hanf_init_counters(ctx, log2m, seed & 0xFFFFFFFFFFFFFFFF), ctx)


def hanf_iterate(ctx, max_steps: int = 0):
    """Returns (status, steps_done, changed_last); status HANF_OK or HANF_DONE."""
    steps = ctypes.c_int32()
    changed = ctypes.c_int64()
    rc = lib().hanf_iterate(ctx, max_steps, ctypes.byref(steps), ctypes.byref(changed))
    _check(rc, ctx, ok=(HANF_OK, HANF_DONE))
    return rc, steps.value, changed.value


def hanf_enqueue(ctx, passes: int) -> None:
    _check(lib().hanf_enqueue(ctx, passes), ctx)


def hanf_poll(ctx):
    """(status, t): status HANF_BUSY, HANF_OK (more passes needed) or HANF_DONE."""
    t = ctypes.c_int32()
    rc = lib().hanf_poll(ctx, ctypes.byref(t))
    _check(rc, ctx, ok=(HANF_OK, HANF_DONE, HANF_BUSY))
    return rc, t.value


def hanf_read_nt(ctx) -> np.ndarray:
    n = ctypes.c_int32()
    rc = lib().hanf_read_nt(ctx, None, 0, ctypes.byref(n))
    _check(rc, ctx, ok=(HANF_OK, HANF_ERANGE))
    out = np.zeros(max(n.value, 1), np.float64)
    _check(lib().hanf_read_nt(ctx, out.ctypes.data, out.size, ctypes.byref(n)), ctx)
    return out[: n.value]


def hanf_read_registers(ctx, n: int, log2m: int, out=None):
    """Current counters as an (n, m) uint8 array (numpy), or into `out` (numpy or device
    tensor of n*m bytes)."""
    nbytes = n << log2m
    if out is None:
        out = np.empty((n, 1 << log2m), np.uint8)
    if _is_tensor(out) and out.is_cuda:
        _check(lib().hanf_read_registers(ctx, out.data_ptr(), nbytes, HANF_DEVICE_PTRS), ctx)
    else:
        if not out.flags["C_CONTIGUOUS"] or out.dtype != np.uint8 or out.size != nbytes:
            raise ValueError("out must be a contiguous uint8 array of n*m bytes")
        _check(lib().hanf_read_registers(ctx, out.ctypes.data, nbytes, HANF_HOST_PTRS), ctx)
    return out


def hanf_write_registers(ctx, regs, t: int, nt_prefix) -> None:
    p, flags, keep = _ptr(regs, np.uint8)
    nbytes = keep.numel() if _is_tensor(keep) else keep.size
    pre = np.ascontiguousarray(nt_prefix, dtype=np.float64)
    _check(lib().hanf_write_registers(ctx, p, nbytes, t, pre.ctypes.data, pre.size, flags), ctx)


def hanf_device_bytes(ctx) -> tuple[int, int]:
    """(held, pooled): device bytes the context holds, and the part kept for reuse."""
    held, pooled = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().hanf_device_bytes(ctx, ctypes.byref(held), ctypes.byref(pooled)), ctx)
    return held.value, pooled.value


def hanf_trim(ctx) -> None:
    """Returns the context's pooled device buffers to HIP."""
    _check(lib().hanf_trim(ctx), ctx)


def hanf_stats_nt(nt, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False) -> dict:
    """Statistics of a caller's N_hat(0..T) (host function, no device)."""
    a = np.ascontiguousarray(nt, dtype=np.float64)
    s = hanf_stats_t()
    _check(lib().hanf_stats_nt(a.ctypes.data, a.size, alpha, eps, int(distinct), ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in hanf_stats_t._fields_}


def hanf_stats(ctx, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False) -> dict:
    s = hanf_stats_t()
    _check(lib().hanf_stats(ctx, alpha, eps, int(distinct), ctypes.byref(s)), ctx)
    return {f: getattr(s, f) for f, _ in hanf_stats_t._fields_}


def hanf_read_pass_log(ctx) -> list[dict]:
    n = ctypes.c_int32()
    rc = lib().hanf_read_pass_log(ctx, None, 0, ctypes.byref(n))
    _check(rc, ctx, ok=(HANF_OK, HANF_ERANGE))
    arr = (hanf_pass_t * max(n.value, 1))()
    _check(lib().hanf_read_pass_log(ctx, ctypes.cast(arr, ctypes.c_void_p), n.value, ctypes.byref(n)), ctx)
    return [{f: getattr(arr[i], f) for f, _ in hanf_pass_t._fields_}
            for i in range(n.value)]


def hanf_footprint(n: int, arcs: int, log2m: int, copy_graph: bool = True, transpose: bool = False,
                   packed5: bool = False, order: bool = False) -> int:
    out = ctypes.c_int64()
    flags = ((HANF_FP_COPY_GRAPH if copy_graph else 0) | (HANF_FP_TRANSPOSE if transpose else 0)
             | (HANF_FP_PACKED5 if packed5 else 0) | (HANF_FP_ORDER if order else 0))
    _check(lib().hanf_footprint(n, arcs, log2m, flags, ctypes.byref(out)))
    return out.value


def hanf_max5_groups(device: int, x, y, out) -> None:
    """Device uint8 tensors of 40-byte groups (64 packed 5-bit registers each);
    out = register-wise max of x and y."""
    if x.numel() % 40 or y.numel() != x.numel() or out.numel() != x.numel():
        raise ValueError("x, y and out must hold the same whole number of 40-byte groups")
    _check(lib().hanf_max5_groups(device, x.data_ptr(), y.data_ptr(), out.data_ptr(), x.numel() // 40))


def hanf_gathermax_lanes(device: int, x, k: int, from_first: bool, out) -> None:
    """Device tensors: x of count * k * 4 int32 words (16-byte lanes), out of count * 4;
    out lane i = register-wise max of lanes i*k .. i*k+k of x, by the union step's gather
    accumulator."""
    if out.numel() % 4 or x.numel() != out.numel() * int(k):
        raise ValueError("hanf_gathermax_lanes: x must hold k lanes of 4 words per lane of out")
    _check(lib().hanf_gathermax_lanes(device, x.data_ptr(), int(k), 1 if from_first else 0, out.data_ptr(),
                                      out.numel() // 4))


def hanf_bytemax_words(device: int, x, y, out) -> None:
    """Device tensors of int32/uint32 words; out[i] = register-wise max of x[i], y[i]."""
    _check(lib().hanf_bytemax_words(device, x.data_ptr(), y.data_ptr(), out.data_ptr(), x.numel()))


def hanf_load_batch(ctx, graph_off, arc_off, row_ptr, col_idx, n_seeds: int) -> None:
    """graph_off[G+1], arc_off[G+1] (host); one CSR over all graphs with global ids: numpy
    arrays (copied) or device tensors (read during the call)."""
    go = np.ascontiguousarray(graph_off, dtype=np.int32)
    ao = np.ascontiguousarray(arc_off, dtype=np.int32)
    p_rp, f1, k1 = _ptr(row_ptr, np.int32)
    p_ci, f2, k2 = _ptr(col_idx, np.int32)
    if f1 != f2:
        raise ValueError("row_ptr and col_idx must both be host or both be device arrays")
    _check(lib().hanf_load_batch(ctx, go.size - 1, go.ctypes.data, ao.ctypes.data, p_rp,
                                 p_ci if int(ao[-1]) > 0 else None, n_seeds, f1), ctx)


def hanf_load_batch_list(ctx, graphs, n_seeds: int):
    """graphs: list of (row_ptr, col_idx) with their own node ids, all numpy (copied) or all
    device tensors (read during the call). Returns the objects to keep alive until then."""
    ptrs = [(_ptr(rp, np.int32), _ptr(ci, np.int32)) for rp, ci in graphs]
    flags = {p[0][1] for p in ptrs} | {p[1][1] for p in ptrs}
    if len(flags) != 1:
        raise ValueError("all arrays must be host arrays or all device tensors")
    G = len(graphs)
    rps = (ctypes.c_void_p * G)(*[p[0][0] for p in ptrs])
    cis = (ctypes.c_void_p * G)(*[p[1][0] for p in ptrs])
    sizes = lambda k: (k.numel() if _is_tensor(k) else k.size)  # noqa: E731
    nn = np.array([sizes(p[0][2]) - 1 for p in ptrs], np.int32)
    na = np.array([sizes(p[1][2]) for p in ptrs], np.int64)
    _check(lib().hanf_load_batch_list(ctx, G, ctypes.cast(rps, ctypes.c_void_p), ctypes.cast(cis, ctypes.c_void_p),
                                      nn.ctypes.data, na.ctypes.data, n_seeds, flags.pop()), ctx)
    return ptrs


def hanf_init_batch(ctx, log2m: int, seeds) -> None:
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    _check(lib().hanf_init_batch(ctx, log2m, sd.ctypes.data), ctx)


def hanf_batch_info(ctx, with_T: bool = True):
    """(number of components, fixpoint T per component or None); T = -1 while changing."""
    n = ctypes.c_int32()
    _check(lib().hanf_batch_info(ctx, ctypes.byref(n), None), ctx)
    if not with_T:
        return n.value, None
    T = np.zeros(n.value, np.int32)
    _check(lib().hanf_batch_info(ctx, ctypes.byref(n), T.ctypes.data), ctx)
    return n.value, T


def hanf_batch_read_nt(ctx, comp: int) -> np.ndarray:
    n = ctypes.c_int32()
    rc = lib().hanf_batch_read_nt(ctx, comp, None, 0, ctypes.byref(n))
    _check(rc, ctx, ok=(HANF_OK, HANF_ERANGE))
    out = np.zeros(max(n.value, 1), np.float64)
    _check(lib().hanf_batch_read_nt(ctx, comp, out.ctypes.data, out.size, ctypes.byref(n)), ctx)
    return out[: n.value]


def hanf_batch_read_registers(ctx, comp: int, n: int, log2m: int, out=None):
    """Counters of component `comp` as an (n, m) uint8 array, or into `out` (a device
    tensor of n*m bytes)."""
    if out is not None and _is_tensor(out) and out.is_cuda:
        if out.numel() != n << log2m or out.element_size() != 1:
            raise ValueError("out must be a byte device tensor of n*m bytes")
        _check(lib().hanf_batch_read_registers(ctx, comp, out.data_ptr(), n << log2m, HANF_DEVICE_PTRS), ctx)
        return out
    out = np.empty((n, 1 << log2m), np.uint8)
    _check(lib().hanf_batch_read_registers(ctx, comp, out.ctypes.data, out.size, HANF_HOST_PTRS), ctx)
    return out


def hanf_read_estimates(ctx, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _check(lib().hanf_read_estimates(ctx, out.ctypes.data, n, HANF_HOST_PTRS), ctx)
    return out


def hanf_read_order(ctx, n: int, out=None):
    """The library's node order: out[i] = the caller's id of row i (int32; `out` may be a
    device tensor of n int32)."""
    if out is not None:
        _check(lib().hanf_read_order(ctx, out.data_ptr(), n, HANF_DEVICE_PTRS), ctx)
        return out
    arr = np.empty(n, np.int32)
    _check(lib().hanf_read_order(ctx, arr.ctypes.data, n, HANF_HOST_PTRS), ctx)
    return arr


def hanf_batch_read_estimates(ctx, comp: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _check(lib().hanf_batch_read_estimates(ctx, comp, out.ctypes.data, n, HANF_HOST_PTRS), ctx)
    return out


def hanf_batch_stats(ctx, comp: int, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False) -> dict:
    s = hanf_stats_t()
    _check(lib().hanf_batch_stats(ctx, comp, alpha, eps, int(distinct), ctypes.byref(s)), ctx)
    return {f: getattr(s, f) for f, _ in hanf_stats_t._fields_}


STATS_DTYPE = np.dtype({"names": [f for f, _ in hanf_stats_t._fields_],
                        "formats": [np.float64 if t is ctypes.c_double else np.int32 for _, t in hanf_stats_t._fields_],
                        "offsets": [getattr(hanf_stats_t, f).offset for f, _ in hanf_stats_t._fields_],
                        "itemsize": ctypes.sizeof(hanf_stats_t)})  # numpy view of hanf_stats_t


def hanf_batch_stats_all(ctx, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False) -> dict:
    """Statistics of every component: dict of numpy arrays (ed, ied, avg_dist, var, spid,
    n_max, d_lo, d_hi, T)."""
    n, _ = hanf_batch_info(ctx, with_T=False)
    # a structured array with the C struct's layout receives the records directly
    arr = np.zeros(max(n, 1), STATS_DTYPE)
    _check(lib().hanf_batch_stats_all(ctx, alpha, eps, int(distinct), arr.ctypes.data), ctx)
    return {f: arr[f][:n].copy() for f, _ in hanf_stats_t._fields_}


class hanf_seed_summary_t(ctypes.Structure):
    _fields_ = [("ed", ctypes.c_double), ("ied", ctypes.c_double), ("avg_dist", ctypes.c_double),
                ("spid", ctypes.c_double), ("ed_sd", ctypes.c_double), ("ied_sd", ctypes.c_double),
                ("avg_dist_sd", ctypes.c_double), ("spid_sd", ctypes.c_double), ("runs", ctypes.c_int32),
                ("distinct", ctypes.c_int32)]


def hanf_batch_seed_summary(ctx, n_graphs: int, alpha: float = 0.9, distinct: bool = False) -> dict:
    """Per graph: {k_mean, k_std} for k in ed, ied, avg_dist, spid, and runs."""
    arr = (hanf_seed_summary_t * max(n_graphs, 1))()
    _check(lib().hanf_batch_seed_summary(ctx, alpha, int(distinct), ctypes.cast(arr, ctypes.c_void_p)), ctx)
    out = {}
    for k in ("ed", "ied", "avg_dist", "spid"):
        out[k + "_mean"] = np.array([getattr(arr[g], k) for g in range(n_graphs)])
        out[k + "_std"] = np.array([getattr(arr[g], k + "_sd") for g in range(n_graphs)])
    out["runs"] = np.array([arr[g].runs for g in range(n_graphs)], np.int32)
    return out


def hanf_batch_stats_all_noalloc(ctx, out: np.ndarray, alpha: float = 0.9, eps: float = 0.0,
                                 distinct: bool = False) -> np.ndarray:
    """The same records written into the caller's `out` (STATS_DTYPE, at least one entry per
    component) by the library's entry point that allocates no device memory."""
    if out.dtype != STATS_DTYPE or not out.flags.c_contiguous:
        raise TypeError("out must be a C-contiguous array of STATS_DTYPE")
    n, _ = hanf_batch_info(ctx, with_T=False)
    if out.size < n:
        raise ValueError(f"out holds {out.size} records, the batch has {n} components")
    _check(lib().hanf_batch_stats_all_noalloc(ctx, alpha, eps, int(distinct), out.ctypes.data), ctx)
    return out


# ------------------------------------------------------------------ convenience wrapper

class HyperANF:
    """One graph and one run on one device: load, init, iterate to the fixpoint, read."""

    def __init__(self, device: int = 0, stream=None, **options):
        self.ctx = hanf_create(device, stream)
        self.n = 0
        self.log2m = 0
        self._keep = None
        names = {"frontier": HANF_OPT_FRONTIER, "max_passes": HANF_OPT_MAX_PASSES,
                 "light_max": HANF_OPT_LIGHT_MAX, "chunk_arcs": HANF_OPT_CHUNK_ARCS,
                 "timing": HANF_OPT_TIMING, "batch": HANF_OPT_BATCH,
                 "tile_nodes": HANF_OPT_TILE_NODES, "unroll": HANF_OPT_UNROLL,
                 "dense_switch": HANF_OPT_DENSE_SWITCH, "systolic": HANF_OPT_SYSTOLIC,
                 "seeds_per_row": HANF_OPT_SEEDS_PER_ROW, "packed5": HANF_OPT_PACKED5,
                 "hubs": HANF_OPT_HUBS, "stage": HANF_OPT_STAGE,
                 "forward": HANF_OPT_FORWARD,
                 "union_policy": HANF_OPT_UNION_POLICY,
                 "transpose_counting": HANF_OPT_TRANSPOSE_COUNTING, "stage_bytes": HANF_OPT_STAGE_BYTES,
                 "count_near": HANF_OPT_COUNT_NEAR}
        for k, v in options.items():
            hanf_set_option(self.ctx, names[k], int(v))

    def close(self):
        if self.ctx is not None:
            hanf_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, row_ptr, col_idx):
        self._keep = hanf_load_csr(self.ctx, row_ptr, col_idx)
        k = self._keep[0]
        self.n = (k.numel() if _is_tensor(k) else k.size) - 1
        return self

    def load_transpose(self, row_ptr_t, col_idx_t):
        """The graph's predecessor lists, for systolic passes; for a symmetric graph loaded
        from device tensors, pass the same tensors."""
        self._keep_t = hanf_load_transpose(self.ctx, row_ptr_t, col_idx_t)
        return self

    def build_transpose(self):
        """Builds the predecessor lists on the device, for systolic passes."""
        hanf_build_transpose(self.ctx)
        return self

    def transpose_self(self):
        """The graph (every graph of a batch) is symmetric: its successor lists serve as its
        predecessor lists in systolic passes."""
        hanf_transpose_self(self.ctx)
        return self

    def init(self, log2m: int, seed: int):
        hanf_init_counters(self.ctx, log2m, seed)
        self.log2m = log2m
        return self

    def step(self, k: int = 1):
        return hanf_iterate(self.ctx, k)

    def run(self):
        """Iterates to the fixpoint; returns N_hat(0..T)."""
        hanf_iterate(self.ctx, 0)
        return hanf_read_nt(self.ctx)

    def nt(self):
        return hanf_read_nt(self.ctx)

    def registers(self, out=None):
        return hanf_read_registers(self.ctx, self.n, self.log2m, out)

    def estimates(self):
        """Per-node estimates of the current counters."""
        return hanf_read_estimates(self.ctx, self.n)

    def order(self, out=None):
        """The library's node order (row i holds the caller's node order()[i])."""
        return hanf_read_order(self.ctx, self.n, out)

    def stats(self, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False):
        return hanf_stats(self.ctx, alpha, eps, distinct)

    def pass_log(self):
        return hanf_read_pass_log(self.ctx)


class Batch(HyperANF):
    """Many independent runs in the same passes: every graph of `graphs` (a list of
    (row_ptr, col_idx)) with each of its seeds; component g * n_seeds + s."""

    @staticmethod
    def union(graphs):
        """(graph_off, arc_off, row_ptr, col_idx) of graphs laid side by side (global ids)."""
        sizes = [len(rp) - 1 for rp, _ in graphs]
        arcs = [len(ci) for _, ci in graphs]
        goff = np.zeros(len(graphs) + 1, np.int64)
        goff[1:] = np.cumsum(sizes)
        aoff = np.zeros(len(graphs) + 1, np.int64)
        aoff[1:] = np.cumsum(arcs)
        row_ptr = np.concatenate([np.asarray(rp[:-1], np.int64) + a for (rp, _), a in zip(graphs, aoff[:-1])]
                                 + [aoff[-1:]])
        col_idx = (np.concatenate([np.asarray(ci, np.int64) + o for (_, ci), o in zip(graphs, goff[:-1])])
                   if aoff[-1] else np.zeros(0, np.int64))
        return goff, aoff, row_ptr.astype(np.int32), col_idx.astype(np.int32)

    def load_union(self, graph_off, arc_off, row_ptr, col_idx, n_seeds: int):
        """Loads graphs already laid side by side (see union); row_ptr / col_idx may be device
        tensors."""
        hanf_load_batch(self.ctx, graph_off, arc_off, row_ptr, col_idx, n_seeds)
        go = np.asarray(graph_off)
        self.sizes = list(np.diff(go))
        self.n_seeds = n_seeds
        return self

    def load_graphs(self, graphs, n_seeds: int):
        """Loads a list of (row_ptr, col_idx), each with its own node ids (numpy or device
        tensors), with no concatenation on the host."""
        hanf_load_batch_list(self.ctx, graphs, n_seeds)
        self.sizes = [len(rp) - 1 for rp, _ in graphs]
        self.n_seeds = n_seeds
        return self

    def init(self, log2m: int, seeds):
        hanf_init_batch(self.ctx, log2m, seeds)
        self.log2m = log2m
        return self

    def fixpoints(self):
        return hanf_batch_info(self.ctx)[1]

    def nt(self, comp: int):
        return hanf_batch_read_nt(self.ctx, comp)

    def registers(self, comp: int):
        return hanf_batch_read_registers(self.ctx, comp, self.sizes[comp // self.n_seeds], self.log2m)

    def estimates(self, comp: int):
        return hanf_batch_read_estimates(self.ctx, comp, self.sizes[comp // self.n_seeds])

    def stats(self, comp: int, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False):
        return hanf_batch_stats(self.ctx, comp, alpha, eps, distinct)

    def stats_all(self, alpha: float = 0.9, eps: float = 0.0, distinct: bool = False):
        return hanf_batch_stats_all(self.ctx, alpha, eps, distinct)

    def seed_summary(self, alpha: float = 0.9, distinct: bool = False):
        """A-posteriori statistics over the seeds of each graph (the paper's many low-precision
        runs, Section 6), computed by the library: mean and sample standard deviation of ed,
        ied, average distance and spid, per graph (keys k_mean, k_std)."""
        return hanf_batch_seed_summary(self.ctx, len(self.sizes), alpha, distinct)


def rsd(log2m: int, beta: float = 1.06) -> float:
    """Relative standard deviation bound beta/sqrt(m) of Section 3.1."""
    return beta / math.sqrt(1 << log2m)
