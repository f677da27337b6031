#!/usr/bin/env python3
"""HyperANF benchmark on one MI355X.

One step is a whole HyperANF run on a graph already resident in HBM: graph ingest
(device-side validation and work schedule), counter initialisation, passes until no
counter changes, and the statistics (distance distribution, effective diameter, spid).
The default workload is the web-like graph of 2^24 nodes (lognormal hosts of mean 1000,
out-degree mean 20, 80% of the arcs intra-host to nearby ids, the rest to a power-law
in-degree target) with 128 registers per counter and hash seed 1. The same run also times
the symmetric R-MAT graph of scale 22 (2^26 arcs, 64 registers, hash seed 7), the batched
workload (512 graphs x 8 hash seeds) against plain runs one after another, and the
serving workload (a Poisson stream of requests) against sequential first-come runs, each
under its own key, and each checked for equal results.

Prints one JSON line. `value` = edge-register updates per second over the whole step of the
default workload: m * (successor counters actually maximised in, summed over the passes) /
step time. `method_updates_per_s` counts only the unions the paper's modified-counter
tracking performs (Section 3.3), taken from a run with the gather-all switch off.
`roofline` is for the union step (the dominant kernel), timed with HIP events on the
library's stream: `achieved` counts the bytes it must move through device memory (the
algorithmic bytes less the successor counters read from a light tile's counters staged in
LDS), `algorithmic_cache_inclusive` the same rate with every successor counter counted.
`cpu_baseline` times the CPU oracle on a bounded sample of the default workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes(rec, n, m):
    """Bytes a union pass must move: col_idx of every arc scanned (4 B), m bytes (the bytes
    of one counter: m registers, or 5m/8 when packed) per successor counter maximised in, per
    own counter read and per new counter written; plus,
    in a pass over every node, row_ptr (4 B/node) and one flag bit per node read and
    written, or, in a systolic pass (only signalled nodes visited), two row_ptr entries per
    node whose counter was read."""
    rows = m * (rec["arcs_gathered"] + rec["rows_read"] + rec["rows_written"])
    if rec.get("systolic"):
        return 8 * rec["rows_read"] + 4 * rec["arcs_scanned"] + rows
    return 4 * (n + 1) + 4 * rec["arcs_scanned"] + rows + n // 4


def model_bytes(rec, n, m, near=None):
    """Bytes a union pass must move through HBM (the roofline's bytes): the algorithmic
    bytes less the successor counters that need not come from HBM: those within the near
    window of their node (`near`, counted by the instrumented kernels: rows that the XCD
    sweeping that id range read moments before as their own counters, held in its L2), or,
    when no near count is given, those read from a light tile's counters staged in LDS."""
    cached = rec.get("arcs_local", 0) if near is None or near < 0 else near
    return algorithmic_bytes(rec, n, m) - m * cached


def cpu_threads():
    """(nproc, threads to use): the CPUs this process may run on, capped by the thread
    count the machine's share sets (OMP_NUM_THREADS) when there is one."""
    nproc = len(os.sched_getaffinity(0))
    try:
        share = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        share = 0
    return nproc, (min(nproc, share) if share > 0 else nproc)


def measured_traffic(workload):
    """HBM bytes per union launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded
    under profiles/ (`workload` with a `_packed5` suffix for 5-bit registers and `_hubs` for
    the hubs-first node order from the first run, --opt hubs=K), or None when the kernel
    source changed since they were taken or no such run was recorded."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", f"k_union_{workload}_traffic.json")
    src = os.path.join(ROOT, "paper_1011_5599_amd", "csrc", "hanf_kernels.hip")
    try:
        rec = json.load(open(rec_path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    return rec["traffic_bytes_per_launch"] if rec.get("kernel_source_sha256") == sha else None


def run_cpu_baseline(rp, ci, b, seed, passes, threads):
    """The oracle on the same job: initialisation, N_hat(t) every iteration, passes (with
    modified-counter skipping, multi-threaded over node segments) until no counter changes,
    or `passes` passes when passes > 0."""
    import numpy as np

    import oracle
    n = len(rp) - 1
    t0 = time.perf_counter()
    c = oracle.init(n, b, seed)
    mod = np.ones(n, np.uint8)
    maxed_total = 0
    done = 0
    while True:
        oracle.sum_sizes(c, b, threads)
        if passes > 0 and done >= passes:
            break
        nxt, mod, changed, maxed = oracle.step(rp, ci, b, c, mod, nthreads=threads)
        maxed_total += maxed
        done += 1
        if changed == 0:
            break
        c = nxt
    el = time.perf_counter() - t0
    what = "the whole run to the fixpoint" if passes <= 0 else f"initialisation and the first {done} pass(es)"
    return dict(value=(1 << b) * maxed_total / el, unit="edge-register updates/s", cores=threads,
                kind="oracle", seconds=round(el, 3), unions=maxed_total,
                sample=f"{what} of the same graph ({done} passes, {maxed_total} successor unions, "
                       f"N_hat every iteration) in {el:.2f} s, {threads} threads over contiguous "
                       f"node segments")


def run_cpu_single_prefix(rp, ci, b, seed, frac_div):
    """One thread: the first pass (every successor) over the first n / frac_div nodes,
    from the initial counters (initialisation not timed)."""
    import numpy as np

    import oracle
    n = len(rp) - 1
    k = max(1, n // frac_div)
    c = oracle.init(n, b, seed)
    rp_k = np.ascontiguousarray(rp[:k + 1])
    t0 = time.perf_counter()
    # the oracle's pass over nodes 0..k-1; their successors may be any node of c
    _, _, _, maxed = oracle.step(rp_k, ci, b, c, None, nthreads=1)
    el = time.perf_counter() - t0
    return dict(value=(1 << b) * maxed / el, unit="edge-register updates/s", cores=1, seconds=round(el, 3),
                unions=maxed,
                sample=f"the first pass over the first {k} of {n} nodes ({maxed} successor unions), "
                       f"initialisation not timed, in {el:.2f} s on one thread")


def copy_ceiling_gbs(mib: int = 1024, reps: int = 5):
    """Bytes read + written per second by a plain 1 GiB device copy (torch), best of `reps`:
    a measured streaming ceiling beside the 8 TB/s HBM3E specification."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    nbytes = 2 * src.numel() * 4
    del src, dst
    torch.cuda.empty_cache()
    return nbytes / (best / 1000.0) / 1e9


def fifo_finish(arrivals, service):
    """Completion times of one-at-a-time, first-come-first-served runs: request i starts
    when it has arrived and request i-1 is done, and takes service[i]."""
    import numpy as np
    fin, t = np.zeros(len(arrivals)), 0.0
    for i, (a, s) in enumerate(zip(arrivals, service)):
        t = max(t, a) + s
        fin[i] = t
    return fin


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def run_batch_mode(args, steps=None, warmup=None):
    """Many-graph workload: 512 graphs (lognormal 2^8..2^16 nodes; half Erdos-Renyi with
    8n arcs, half R-MAT with 16n arcs) x 8 hash seeds, m = 64. All 4096 runs are submitted
    at once. Batched: the runs go through batched passes, with grouping and schedule chosen
    by the autotuner first. Plain: the same runs one after another through the plain path
    (graph loaded once per graph). Reports graphs/s (each graph with its 8 seeds) and the
    latency percentiles of the runs (completion time since submission). In batched passes
    the 8 seeds of a graph share one node row (8 x 64 registers), so one successor scan and
    one 512-byte gather serve all of them."""
    import numpy as np
    import torch

    import graphgen
    import paper_1011_5599_amd as hanf
    from paper_1011_5599_amd import tune

    S, b = 8, 6
    graphs = graphgen.batch_graphs()
    G = len(graphs)
    seeds = [(g << 8) + s + 1 for g in range(G) for s in range(S)]
    order = sorted(range(G), key=lambda g: -(len(graphs[g][0]) - 1))  # groups of similar sizes
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    ctxs = {}
    resident = {}  # (group size, group index) -> graphs of the group laid side by side, in HBM

    def run_batched(cfg):
        group = cfg.get("group", G)
        opts = {k: v for k, v in cfg.items() if k != "group"}
        for gi, lo in enumerate(range(0, G, group)):
            key = (group, gi)
            if key not in resident:
                ids = order[lo:lo + group]
                go, ao, rp, ci = hanf.Batch.union([graphs[g] for g in ids])
                resident[key] = (go, ao, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                                 [seeds[g * S + s] for g in ids for s in range(S)])
                ctxs[key] = hanf.Batch(0, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done_at = []
        for gi, lo in enumerate(range(0, G, group)):
            key = (group, gi)
            bt = ctxs[key]
            go, ao, drp, dci, sd = resident[key]
            for k, v in opts.items():
                hanf.hanf_set_option(bt.ctx, getattr(hanf, "HANF_OPT_" + k.upper()), v)
            bt.load_union(go, ao, drp, dci, S)
            bt.init(b, sd)
            bt.run()
            bt.stats_all()
            done_at += [time.perf_counter() - t0] * (len(sd))
        return time.perf_counter() - t0, done_at

    space = dict(tune.SPACE)
    space["group"] = [G, 256, 128, 64]
    space["seeds_per_row"] = [0, 4, 2, 1]  # 0: all 8 seeds of a graph in one row
    space["packed5"] = [2, 0, 1]  # chosen by row width (the default), bytes, 5-bit (320-byte rows)
    start = dict(tune.DEFAULTS)
    start["group"] = G
    t_tune = time.perf_counter()
    best, best_t, trials = tune.coordinate_descent(lambda cfg: run_batched(cfg)[0], space, start,
                                                   sweeps=1, repeats=2,
                                                   log=lambda m: print(m, file=sys.stderr, flush=True))
    t_tune = time.perf_counter() - t_tune
    print(f"[bench] tuned {best} in {trials} trials, {t_tune:.1f}s", file=sys.stderr, flush=True)
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    for _ in range(warmup):
        run_batched(best)
    torch.cuda.synchronize()
    times, lat = [], []
    for _ in range(steps):
        el, done = run_batched(best)
        times.append(el)
        lat += done
    batched_s = float(np.median(times))
    # every run's N_hat and T from the last batched step, to compare with its plain run
    group = best.get("group", G)
    batched_nt = {}
    for gi, lo in enumerate(range(0, G, group)):
        ids = order[lo:lo + group]
        bt = ctxs[(group, gi)]
        T = bt.fixpoints()
        for k, g in enumerate(ids):
            for s_ in range(S):
                c = k * S + s_
                batched_nt[(g, s_)] = (bt.nt(c), int(T[c]))
    # plain runs, one after another, each graph already in HBM
    dev_graphs = [(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()) for rp, ci in graphs]
    torch.cuda.synchronize()
    h = hanf.HyperANF(0, stream=stream)
    t0 = time.perf_counter()
    plain_lat = []
    plain_nt = {}
    for g, (rp, ci) in enumerate(dev_graphs):
        h.load(rp, ci)
        for s in range(S):
            h.init(b, seeds[g * S + s])
            plain_nt[(g, s)] = h.run()
            h.stats()
            plain_lat.append(time.perf_counter() - t0)
    plain_s = time.perf_counter() - t0
    for key, nt in plain_nt.items():  # equal results: N_hat within 1e-12, the same T
        bnt, bT = batched_nt[key]
        if bT != len(nt) - 1:
            raise AssertionError(f"batched run {key}: T={bT}, plain T={len(nt) - 1}")
        np.testing.assert_allclose(bnt, nt, rtol=1e-12, atol=0)
    h.close()
    for bt in ctxs.values():
        bt.close()
    nodes = sum(len(rp) - 1 for rp, _ in graphs)
    arcs = sum(len(ci) for _, ci in graphs)
    return {
        "metric": "graphs/s (512 graphs x 8 seeds, batched)",
        "value": G / batched_s,
        "unit": "graphs/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(1000 * batched_s, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "512 graphs, lognormal 2^8..2^16 nodes (median 2^12), half Erdos-Renyi 8n arcs, "
                               "half R-MAT 16n arcs, 8 hash seeds each, 64 registers",
                   "graphs": G, "seeds": S, "runs": G * S, "nodes": nodes, "arcs": arcs, "tuned": best,
                   "tuner_trials": trials, "tuner_s": round(t_tune, 2)},
        "runs_per_s": G * S / batched_s,
        "latency_ms": {"p50": 1000 * percentile(lat, 50), "p99": 1000 * percentile(lat, 99)},
        "plain": {"graphs_per_s": G / plain_s, "runs_per_s": G * S / plain_s, "seconds": plain_s,
                  "latency_ms": {"p50": 1000 * percentile(plain_lat, 50),
                                 "p99": 1000 * percentile(plain_lat, 99)}},
        "speedup_vs_plain": plain_s / batched_s,
        "equal_results": "every run's N_hat within 1e-12 of its plain run, the same T",
    }


def batched_leg(args):
    """The batched workload under its own key: graphs/s and latency batched (tuned) against
    plain runs one after another, equal results checked."""
    r = run_batch_mode(args, steps=3, warmup=1)
    keep = ("value", "unit", "ms_per_step", "config", "runs_per_s", "latency_ms", "plain", "speedup_vs_plain",
            "equal_results")
    out = {k: r[k] for k in keep}
    out["graphs_per_s"] = out.pop("value")
    return out


def run_seeds_mode(args):
    """Many runs on one graph (the paper's protocol of many low-precision runs, Section 6):
    the workload graph with `--seeds` hash seeds, once as one batch whose node rows hold the
    seeds' counters side by side, once as plain runs one after another. Both start from the
    graph in HBM and end with every run's statistics; every run's N_hat is checked equal.
    Reports edge-register updates/s over all runs (m x successor counters maximised in,
    summed over the runs' own passes)."""
    import numpy as np
    import torch

    import graphgen
    import paper_1011_5599_amd as hanf

    spec = graphgen.WORKLOADS[args.workload]
    rp, ci = graphgen.workload_graph(spec)
    b, S = spec["log2m"], args.seeds
    m = 1 << b
    sym = bool(spec.get("symmetric"))
    drp, dci = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    seeds = [spec["seed"] + s for s in range(S)]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    opts = {k: int(v) for k, v in (kv.split("=") for kv in args.opt)}  # for the batched runs
    fmt = opts.get("packed5", 2)  # the library chooses 5-bit rows from 512 registers on
    row_seeds = 1
    while (row_seeds < S and row_seeds < 32 and 2 * row_seeds * m <= 1024
           and (not opts.get("seeds_per_row") or row_seeds < opts["seeds_per_row"])):
        row_seeds *= 2
    packed = fmt == 1 or (fmt == 2 and m >= 64 and row_seeds * m >= 512)
    bt = hanf.Batch(0, stream=stream, **opts)
    h = hanf.HyperANF(0, stream=stream, timing=1)

    def rows():
        bt.load_graphs([(drp, dci)], S)
        if sym:
            bt.transpose_self()
        bt.init(b, seeds)
        bt.run()
        return bt.stats_all()

    def plain():
        out = []
        for sd in seeds:
            h.load(drp, dci)
            if sym:
                h.transpose_self()
            h.init(b, sd)
            nt = h.run()
            h.stats()
            out.append((nt, sum(r["arcs_gathered"] for r in h.pass_log())))
        return out

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), res

    t_rows, _ = timed(rows)
    t_plain, res = timed(plain)
    for s_, (nt, _) in enumerate(res):
        np.testing.assert_allclose(bt.nt(s_), nt, rtol=1e-12, atol=0)
    updates = m * sum(g for _, g in res)
    bt.close()
    h.close()
    return {
        "metric": f"edge-register updates/s ({S} runs of one graph, seeds side by side)",
        "value": updates / t_rows, "unit": "edge-register updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000 * t_rows, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": spec_name(args.workload), "seeds": S, "log2m": b,
                   "row_bytes": row_seeds * (5 * m // 8 if packed else m),
                   "transpose": "self" if sym else "none",
                   "registers": "5-bit packed" if packed else "one per byte", "options": opts},
        "plain": {"ms_per_step": round(1000 * t_plain, 3), "updates_per_s": updates / t_plain},
        "speedup_vs_plain": t_plain / t_rows,
    }


def run_serve_mode(args, count=None, rates=(0.25, 0.5, 1.0, 2.0)):
    """Serving workload: a Poisson stream of requests, graphs of 2^10..2^22 nodes (lognormal,
    median 2^16), R-MAT or web-like, log2m in {4, 6, 8}, hash seed = request id. Each request
    is first run alone through the plain path to get its service time; sequential serving
    (first come, first served, one run at a time) is evaluated with those times. The
    continuous-batching server is then run in real time at arrival rates from 0.25x to 2x the
    sequential capacity. Latency = completion - arrival."""
    import numpy as np
    import torch

    import graphgen
    import paper_1011_5599_amd as hanf
    from paper_1011_5599_amd import serve

    count = args.requests if count is None else count
    specs = graphgen.serve_requests(count)
    torch.cuda.init()
    h = hanf.HyperANF(0)
    service = []
    for sp in specs:  # warm-up of every size class, then timed runs alone
        rp, ci = sp["graph"]
        h.load(rp, ci).init(sp["log2m"], sp["seed"])
        h.run()
    alone = []
    for sp in specs:
        rp, ci = sp["graph"]
        t0 = time.perf_counter()
        h.load(rp, ci).init(sp["log2m"], sp["seed"])
        nt = h.run()
        h.stats()
        service.append(time.perf_counter() - t0)
        alone.append(nt)
    h.close()
    service = np.array(service)
    capacity = count / service.sum()
    rng = np.random.default_rng(7)
    gaps = rng.exponential(1.0, count)
    rows = []
    for factor in rates:
        lam = factor * capacity
        arrivals = np.cumsum(gaps) / lam
        arrivals -= arrivals[0]
        fin = fifo_finish(arrivals, service)
        seq_lat = fin - arrivals
        reqs = [serve.Request(sp["rid"], sp["graph"][0], sp["graph"][1], sp["log2m"], sp["seed"], float(a))
                for sp, a in zip(specs, arrivals)]
        kw = {"passes_per_poll": args.passes_per_poll} if getattr(args, "passes_per_poll", 0) else {}
        srv = serve.Server(0, max_batches=args.max_batches, size_classes=bool(args.size_classes), **kw)
        srv.warm_up(reqs)
        srv.batch_sizes, srv.max_flights = [], 0
        srv.serve_trace(reqs)
        srv.close()
        for r, nt in zip(reqs, alone):  # each result equal to the same request run alone
            if r.error is not None or r.T != len(nt) - 1:
                raise AssertionError(f"request {r.rid}: served T={r.T} error={r.error}, alone T={len(nt) - 1}")
            np.testing.assert_allclose(r.nt, nt, rtol=1e-12, atol=0)
        lat = np.array([r.latency for r in reqs])
        wait = np.array([r.admitted - r.arrival for r in reqs])    # queued before admission
        run = np.array([r.finish - r.admitted for r in reqs])      # admitted to completed
        span = max(r.finish for r in reqs) - min(r.arrival for r in reqs)
        rows.append({
            "rate_x_capacity": factor, "rate_req_per_s": lam,
            "served": {"p50_ms": 1000 * float(np.percentile(lat, 50)), "p99_ms": 1000 * float(np.percentile(lat, 99)),
                       "wait_p50_ms": 1000 * float(np.percentile(wait, 50)),
                       "run_p50_ms": 1000 * float(np.percentile(run, 50)),
                       "graphs_per_s": count / span, "batches": len(srv.batch_sizes),
                       "mean_batch": float(np.mean(srv.batch_sizes)), "max_in_flight": srv.max_flights,
                       "host_s": {k: round(v, 3) for k, v in srv.host_s.items()}},
            "sequential": {"p50_ms": 1000 * float(np.percentile(seq_lat, 50)),
                           "wait_p50_ms": 1000 * float(np.percentile(seq_lat - service, 50)),
                           "p99_ms": 1000 * float(np.percentile(seq_lat, 99)),
                           "graphs_per_s": count / (fin[-1] - arrivals[0])},
        })
        sv, sq = rows[-1]["served"], rows[-1]["sequential"]
        print(f"[bench] rate {factor}x: served p50 {sv['p50_ms']:.1f} ms (wait {sv['wait_p50_ms']:.1f}, "
              f"run {sv['run_p50_ms']:.1f}) p99 {sv['p99_ms']:.1f} ms; sequential p50 {sq['p50_ms']:.1f} ms "
              f"(wait {sq['wait_p50_ms']:.1f}) p99 {sq['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    top = rows[-1]
    return {
        "metric": "graphs/s served at 2x sequential capacity (Poisson arrivals)",
        "value": top["served"]["graphs_per_s"], "unit": "graphs/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"{count} requests, 2^10..2^22 nodes lognormal (median 2^16, sigma 1.5), "
                               "R-MAT or web-like, log2m in {4,6,8}",
                   "nodes": int(sum(sp["n"] for sp in specs)),
                   "arcs": int(sum(len(sp["graph"][1]) for sp in specs)),
                   "sequential_capacity_req_per_s": capacity,
                   "policy": {"size_classes": bool(args.size_classes), "max_batches": args.max_batches,
                              "passes_per_poll": srv.passes_per_poll},
                   "service_ms": {"p50": 1000 * float(np.percentile(service, 50)),
                                  "p99": 1000 * float(np.percentile(service, 99))}},
        "rates": rows,
        "equal_results": "every served request's N_hat within 1e-12 of the same request run alone, the same T",
    }


def served_leg(args):
    """The serving workload under its own key: 48 requests at 1x and 2x the sequential
    capacity, served against sequential first-come runs, equal results checked."""
    r = run_serve_mode(args, count=48, rates=(1.0, 2.0))
    out = {k: r[k] for k in ("config", "rates", "equal_results")}
    out["graphs_per_s_at_2x"] = r["value"]
    top = r["rates"][-1]
    out["p50_ms_at_2x"] = top["served"]["p50_ms"]
    out["p99_ms_at_2x"] = top["served"]["p99_ms"]
    out["sequential_at_2x"] = top["sequential"]
    return out


def run_plain(name, args, h_opts, tmode_arg="auto", runs_per_load=1, log_prefix="[bench]"):
    """Times whole runs of workload `name` (the graph resident in HBM, ingest included in
    each step). Returns (result dict, graph) where the dict carries the workload's rate,
    roofline and per-pass figures."""
    import numpy as np
    import torch

    import graphgen
    import paper_1011_5599_amd as hanf

    spec = graphgen.WORKLOADS[name]
    t0 = time.perf_counter()
    rp, ci = graphgen.workload_graph(spec)
    gen_s = time.perf_counter() - t0
    n, arcs = len(rp) - 1, len(ci)
    b, seed = spec["log2m"], spec["seed"]
    m = 1 << b
    print(f"{log_prefix} workload={name} n={n} arcs={arcs} m={m} gen={gen_s:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    trp = torch.from_numpy(rp).to(dev)
    tci = torch.from_numpy(ci).to(dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    opts = dict(h_opts)
    h = hanf.HyperANF(0, stream=stream.cuda_stream, **opts)
    packed = opts.get("packed5") == 1  # single runs keep byte registers unless told otherwise
    rowb = (5 * m) // 8 if packed else m  # bytes of one counter
    tmode = tmode_arg
    if tmode == "auto":
        tmode = "self" if spec.get("symmetric") else "none"
    if tmode == "self" and not spec.get("symmetric"):
        print("bench.py: --transpose self needs a symmetric workload", file=sys.stderr)
        sys.exit(2)
    R = max(1, runs_per_load)

    def step(ctx):
        ctx.load(trp, tci)
        if tmode == "self":
            ctx.transpose_self()
        elif tmode == "build":
            ctx.build_transpose()
        run_logs = []
        for r in range(R):
            ctx.init(b, seed + r)
            nt = ctx.run()
            run_logs.append(ctx.pass_log())
        return nt, ctx.stats(), run_logs

    for i in range(args.warmup):
        step(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logs = []
    for i in range(args.steps):
        nt, st, run_logs = step(h)
        logs.extend(run_logs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    print(f"{log_prefix} {name}: {args.steps} steps in {elapsed:.3f}s, T={st['T']}", file=sys.stderr, flush=True)

    log = logs[-1]
    gathered = sum(r["arcs_gathered"] for lg in logs[-R:] for r in lg)  # the last step's R runs
    updates = m * gathered
    out = {
        "value": updates / (ms_per_step / 1000.0),
        "ms_per_step": round(ms_per_step, 4),
        "config": {"workload": spec_name(name), "n": n, "arcs": arcs, "log2m": b,
                   "hash_seed": seed, "T": st["T"], "passes": len(log), "transpose": tmode,
                   "runs_per_load": R,
                   "registers": "5-bit packed" if packed else "one per byte",
                   "staged_tiles": any(r.get("arcs_local", 0) > 0 for r in log),
                   "pass_kinds": "".join({1: "S", 2: "M"}.get(r["systolic"]) or ("D" if r["gather_all"] else "F")
                                         for r in log)},
        "gathered_unions": gathered,
        "dense_equivalent_updates_per_s": m * arcs * sum(len(lg) for lg in logs[-R:]) / (ms_per_step / 1000.0),
        "graphs_per_s": R * 1000.0 / ms_per_step,
        "stats": {k: st[k] for k in ("ed", "ied", "avg_dist", "var", "spid")},
    }
    # per-pass near successors, from the same run through the instrumented kernels (untimed;
    # the same passes, checked): the roofline's bytes leave out those cached rows
    near = [None] * len(log)
    extra = not getattr(args, "no_extra_runs", False)
    if extra and not packed:
        iopts = {k: v for k, v in opts.items() if k != "timing"}
        with hanf.HyperANF(0, stream=stream.cuda_stream, count_near=1, **iopts) as hn:
            nt_n, _, nlogs = step(hn)
        np.testing.assert_allclose(nt_n, nt, rtol=1e-12, atol=0)
        nlog = nlogs[-1]
        if ([r["arcs_gathered"] for r in nlog] == [r["arcs_gathered"] for r in log]
                and all(r["arcs_near"] >= 0 for r in nlog)):
            near = [r["arcs_near"] for r in nlog]
    if extra:
        # the unions of the paper's modified-counter tracking alone: the same run with the
        # gather-all switch off (untimed); its results must be the timed run's
        with hanf.HyperANF(0, stream=stream.cuda_stream, dense_switch=0, **{k: v for k, v in opts.items()
                                                                             if k not in ("dense_switch", "timing")}) as hm:
            nt_m, _, mlogs = step(hm)
        np.testing.assert_allclose(nt_m, nt, rtol=1e-12, atol=0)
        method = sum(r["arcs_gathered"] for lg in mlogs for r in lg)
        out["method_unions"] = method
        out["method_updates_per_s"] = m * method / (ms_per_step / 1000.0)
    out["pass_model_bytes"] = [model_bytes(r, n, rowb, near[i]) for i, r in enumerate(log)]
    out["pass_algorithmic_bytes"] = [algorithmic_bytes(r, n, rowb) for r in log]
    out["pass_near"] = near
    if not args.no_timing:
        all_recs = [r for lg in logs for r in lg]
        union_ms = sum(r["union_ms"] for r in all_recs)
        # every timed run makes the same passes as the last one (R = 1), so the near counts of
        # the instrumented run apply pass by pass
        near_of = (lambda i: near[i % len(log)]) if R == 1 else (lambda i: None)
        byts = sum(model_bytes(r, n, rowb, near_of(i)) for i, r in enumerate(all_recs))
        algo = sum(algorithmic_bytes(r, n, rowb) for r in all_recs)
        launches = len(all_recs)
        achieved = byts / (union_ms / 1000.0) / 1e9
        algo_gbs = algo / (union_ms / 1000.0) / 1e9
        out["roofline"] = dict(
            bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
            frac=round(achieved / HBM_PEAK_GBS, 4),
            traffic=measured_traffic(name + ("_packed5" if packed else "")
                                     + ("_hubs" if opts.get("hubs", -1) > 0 else "")),
            traffic_kind="bytes beyond L2 per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a "
                         "device copy): HBM and Infinity Cache, an upper bound on HBM bytes",
            kernel="union step (k_union; k_union_list in systolic passes)", launches=launches,
            avg_launch_us=round(1000.0 * union_ms / launches, 2),
            avg_model_bytes=int(byts / launches),
            model="per pass: col_idx of the arcs scanned, row_ptr and modified flags, own counters "
                  "read, new counters written, and the successor counters gathered except those "
                  "within the near window of their node (held in the L2 of the XCD sweeping that "
                  "id range; counted per pass by the instrumented kernels)",
            near_window=(2 << 20) // rowb, near_counted=near[0] is not None,
            algorithmic_cache_inclusive=dict(avg_bytes=int(algo / launches), gbs=round(algo_gbs, 1),
                                             frac=round(algo_gbs / HBM_PEAK_GBS, 4)))
        p0 = [lg[0] for lg in logs]
        ms0 = sum(r["union_ms"] for r in p0) / len(p0)
        b0 = model_bytes(p0[0], n, rowb, near[0])
        a0 = algorithmic_bytes(p0[0], n, rowb)
        out["full_pass"] = dict(union_ms=round(ms0, 4), model_gb=round(b0 / 1e9, 4),
                                gbs=round(b0 / (ms0 / 1000.0) / 1e9, 1),
                                frac=round(b0 / (ms0 / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
                                algorithmic_gb=round(a0 / 1e9, 4),
                                algorithmic_gbs=round(a0 / (ms0 / 1000.0) / 1e9, 1),
                                near_share=(None if near[0] is None
                                            else round(near[0] / max(1, p0[0]["arcs_gathered"]), 4)),
                                updates_per_s=m * p0[0]["arcs_gathered"] / (ms0 / 1000.0))
        last = [r for lg in logs[-R:] for r in lg]  # the last step's passes
        out["per_step_kernel_ms"] = dict(signal_ms=round(sum(r["signal_ms"] for r in last), 4),
                                         finalize_ms=round(sum(r["finalize_ms"] for r in last), 4),
                                         reduce_ms=round(sum(r["reduce_ms"] for r in last), 4),
                                         union_ms=round(sum(r["union_ms"] for r in last), 4))
        out["pass_union_ms"] = [round(r["union_ms"], 4) for r in log]
        out["pass_signal_ms"] = [round(r["signal_ms"], 4) for r in log]
    h.close()
    del trp, tci
    torch.cuda.empty_cache()
    return out, (rp, ci, b, seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="web24")
    ap.add_argument("--cpu-passes", type=int, default=1,
                    help="CPU baseline: oracle passes timed on all threads (0 = the whole run)")
    ap.add_argument("--cpu-single-div", type=int, default=32,
                    help="CPU baseline: the single-thread leg runs the first pass over n / this many nodes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--no-extra-runs", action="store_true",
                    help="no untimed diagnostic runs (method unions, near counts): for kernel traces")
    ap.add_argument("--opt", action="append", default=[], help="library option name=value")
    ap.add_argument("--legs", default="rmat22sym,batched,served",
                    help="plain mode: comma-separated extra legs after the main workload "
                         "(rmat22sym, batched, served; empty for none)")
    ap.add_argument("--mode", choices=["plain", "batch", "serve", "seeds"], default="plain",
                    help="plain: one graph (the default workload) and the extra legs; batch: 512 graphs "
                         "x 8 seeds; serve: Poisson request stream; seeds: many runs of the workload graph")
    ap.add_argument("--seeds", type=int, default=8, help="seeds mode: runs of the graph")
    ap.add_argument("--requests", type=int, default=96, help="serve mode: number of requests")
    ap.add_argument("--max-batches", type=int, default=4, help="serve mode: batches in flight")
    ap.add_argument("--size-classes", type=int, default=1, choices=(0, 1),
                    help="serve mode: batch only requests whose footprints are within 4x")
    ap.add_argument("--passes-per-poll", type=int, default=0,
                    help="serve mode: passes enqueued per batch between polls (0: the server's default)")
    ap.add_argument("--rates", default="0.25,0.5,1,2",
                    help="serve mode: arrival rates, as multiples of the sequential capacity")
    ap.add_argument("--runs-per-load", type=int, default=1, metavar="R",
                    help="plain mode: runs (hash seeds seed .. seed + R - 1) after each ingest of the "
                         "graph; a step is the ingest and its R runs")
    ap.add_argument("--transpose", choices=["auto", "self", "build", "none"], default="auto",
                    help="transposed graph for systolic passes: auto = self for symmetric workloads, "
                         "none otherwise")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times): the reference for "
                         "scaling HBM byte counters of a profiler")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(json.dumps({"copy_calibration_bytes": (args.copy_calibration << 20),
                          "copy_gbs_read_plus_write": round(copy_ceiling_gbs(args.copy_calibration), 1)}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py: the benchmark runs on one GPU only; runs on several GPUs are not implemented "
              f"(asked for {max(args.gpus, world)}).", file=sys.stderr)
        sys.exit(2)

    if args.mode == "batch":
        print(json.dumps(run_batch_mode(args)))
        return
    if args.mode == "serve":
        print(json.dumps(run_serve_mode(args, rates=tuple(float(x) for x in args.rates.split(",")))))
        return
    if args.mode == "seeds":
        print(json.dumps(run_seeds_mode(args)))
        return

    opts = dict(timing=0 if args.no_timing else 1)
    for kv in args.opt:
        k, v = kv.split("=")
        opts[k] = int(v)
    main_res, (rp, ci, b, seed) = run_plain(args.workload, args, opts, args.transpose, args.runs_per_load)
    out = {
        "metric": "edge-register updates/s",
        "value": main_res["value"],
        "unit": "edge-register updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": main_res["config"],
        "roofline": main_res.get("roofline"),
        "cpu_baseline": None,
    }
    for k, v in main_res.items():
        if k not in out:
            out[k] = v
    if out["roofline"] is not None:
        # context for the peak: a plain device copy measured on the same GPU, after the timed region
        cgbs = copy_ceiling_gbs()
        out["roofline"]["copy_ceiling"] = {"gbs": round(cgbs, 1), "frac_of_peak": round(cgbs / HBM_PEAK_GBS, 4),
                                           "achieved_over_copy": round(out["roofline"]["achieved"] / cgbs, 4)}
    if not args.no_cpu_baseline:
        nproc, threads = cpu_threads()
        cpu = run_cpu_baseline(rp, ci, b, seed, args.cpu_passes, threads)
        cpu["nproc"] = nproc
        cpu["single_thread"] = run_cpu_single_prefix(rp, ci, b, seed, args.cpu_single_div)
        out["cpu_baseline"] = cpu
        print(f"[bench] cpu baseline: {cpu['sample']}; single thread: {cpu['single_thread']['sample']}",
              file=sys.stderr, flush=True)
    del rp, ci
    legs = [x for x in args.legs.split(",") if x]
    if "rmat22sym" in legs and args.workload != "rmat22sym":
        res, g = run_plain("rmat22sym", args, dict(timing=opts["timing"]), "auto", 1)
        if not args.no_cpu_baseline:
            nproc, threads = cpu_threads()
            res["cpu_baseline"] = run_cpu_baseline(*g, 0, threads)
            res["cpu_baseline"]["nproc"] = nproc
        out["rmat22sym"] = res
        del g
    if "batched" in legs:
        out["batched"] = batched_leg(args)
    if "served" in legs:
        out["served"] = served_leg(args)
    print(json.dumps(out))


def spec_name(name):
    return {
        "rmat22sym": "symmetric R-MAT scale 22 (a=.57,b=.19,c=.19), 2^26 arcs, 64 registers, hash seed 7",
        "rmat14": "directed R-MAT scale 14, 262144 arcs, 16 registers, hash seed 1",
        "web24": "web-like 2^24 nodes, lognormal hosts (mean 1000), out-degree mean 20, 80% of the arcs "
                 "intra-host to nearby ids, the rest to power-law in-degree targets (2.1), 128 registers, "
                 "hash seed 1",
    }.get(name, name)


if __name__ == "__main__":
    main()
