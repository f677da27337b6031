"""Summaries of rocprofv3 runs of bench.py, written under profiles/.

* the kernel-time table of a `rocprofv3 --kernel-trace --stats` run, with the union step's
  average time per pass beside bench.py's own HIP-event figure from the same run;
* the bytes the union step moves beyond L2 per pass, from two `rocprofv3 --pmc` runs
  (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
  for a plain device copy of known size (`bench.py --copy-calibration MIB`). These count the
  L2's requests to the memory fabric, so reads served by the Infinity Cache are included:
  an upper bound on the bytes that reach HBM. Beside them, per pass, the algorithmic bytes
  and the bytes of the roofline model bench.py reports.

The union step of a pass is every k_union / k_union_list dispatch between two k_reduce_top
dispatches (in a systolic pass both may be launched, one of them leaving at once); passes
enqueued after the fixpoint (they return at once) are left out.

    python -m paper_1011_5599_amd.prof --workload rmat22sym --trace DIR --trace-json FILE \\
        --fetch DIR --write DIR --pmc-json FILE --copy-fetch DIR --copy-write DIR \\
        --copy-mib 1024 --commands FILE --out-md profiles/k_union_rmat22sym.md \\
        --out-json profiles/k_union_rmat22sym_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_1011_5599_amd", "csrc", "hanf_kernels.hip")


def _short(name: str) -> str:
    """Kernel name without namespaces and argument lists."""
    base = name.replace("hanf::(anonymous namespace)::", "").replace("void ", "")
    return base.split("(")[0]


def _is_union(name: str) -> bool:
    s = _short(name)
    return s.startswith("k_union<") or s.startswith("k_union_list<")


def kernel_table(trace_dir: str):
    with open(os.path.join(trace_dir, "run_kernel_stats.csv")) as f:
        rows = list(csv.DictReader(f))
    return [dict(name=_short(r["Name"]), calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                 total_ms=float(r["TotalDurationNs"]) / 1e6, pct=float(r["Percentage"])) for r in rows]


def _dispatches(path: str):
    """(dispatch id, kernel name, value) in dispatch order; value = duration ns (trace) or the
    counter value (counter collection)."""
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if "Counter_Value" in r:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
            else:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"],
                            float(r["End_Timestamp"]) - float(r["Start_Timestamp"])))
    out.sort()
    return out


def union_per_pass(dispatches, passes_per_run, max_runs=None):
    """Sums of the union-step values of every executed pass: a run starts at k_init, its
    first k_reduce_top is the initial estimate, and each later k_reduce_top closes a pass.
    Only the first `passes_per_run` passes of a run count: passes enqueued after the fixpoint
    return at once. With max_runs, runs after the first max_runs (bench.py's untimed
    diagnostic runs) are left out."""
    out, run, cur = [], None, None
    runs = 0
    for _, name, val in dispatches:
        s = _short(name)
        if s.startswith("k_init"):
            if run:
                out += run[:passes_per_run]
            if max_runs is not None and runs >= max_runs:
                return out
            runs += 1
            run, cur = [], None
        elif run is None:
            continue
        elif s.startswith("k_reduce_top"):
            if cur is not None:
                run.append(cur)
            cur = 0.0
        elif _is_union(name) and cur is not None:
            cur += val
    if run:
        out += run[:passes_per_run]
    return out


def counter_runs(path: str):
    """{counter name: [(dispatch id, kernel name, value)]} of a counter-collection CSV that may
    hold several counters per dispatch."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            out.setdefault(r["Counter_Name"], []).append(
                (int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    for v in out.values():
        v.sort()
    return out


def copy_scale(copy_dir: str, copy_bytes: int) -> float:
    rows = [(n, v) for _, n, v in _dispatches(os.path.join(copy_dir, "run_counter_collection.csv"))
            if "copyBuffer" in n or "copy" in _short(n).lower()]
    if not rows:
        raise SystemExit(f"no copy kernel in {copy_dir}")
    kib = sum(v for _, v in rows) / len(rows)
    return copy_bytes / (kib * 1024.0)


def derived_utilisation(c, label="first pass", cus=256, simds=1024, xcds=8):
    """Utilisation of the vector memory path and the vector ALUs in one pass (`label`), from
    counters of separate runs (so only roughly comparable): GRBM_GUI_ACTIVE counts busy
    cycles per XCD (summed over the 8); TA and TD busy cycles are per compute unit; a
    wavefront's VALU instruction occupies its SIMD for one quad-cycle."""
    if "GRBM_GUI_ACTIVE" not in c:
        return []
    cyc = c["GRBM_GUI_ACTIVE"] / xcds
    rows = []
    if "TA_TA_BUSY_sum" in c:
        rows.append(("texture addresser (TA) busy", c["TA_TA_BUSY_sum"] / cus / cyc))
    if "TD_TD_BUSY_sum" in c:
        rows.append(("texture data (TD) busy", c["TD_TD_BUSY_sum"] / cus / cyc))
    if "TD_TC_STALL_sum" in c:
        rows.append(("TD stalled waiting for the L1 cache", c["TD_TC_STALL_sum"] / cus / cyc))
    if "TCP_PENDING_STALL_CYCLES_sum" in c:
        rows.append(("L1 cache stalled on pending L2 requests", c["TCP_PENDING_STALL_CYCLES_sum"] / cus / cyc))
    if "SQ_INSTS_VALU" in c:
        rows.append(("VALU issue (instructions x 4 cycles / SIMD cycles)", 4 * c["SQ_INSTS_VALU"] / simds / cyc))
    L = [f"Derived, {label} (cycles per XCD from GRBM_GUI_ACTIVE / 8; counters from separate runs):", "",
         "| quantity | value |", "|---|---:|"]
    L += [f"| {k} | {v:.0%} |" for k, v in rows]
    if "TCP_TCC_READ_REQ_LATENCY_sum" in c and c.get("TCP_TCC_READ_REQ_sum"):
        L.append(f"| L1 to L2 read latency, average (cycles) | {c['TCP_TCC_READ_REQ_LATENCY_sum'] / c['TCP_TCC_READ_REQ_sum']:.0f} |")
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        L.append(f"| L2 hit rate | {c['TCC_HIT_sum'] / (c['TCC_HIT_sum'] + c['TCC_MISS_sum']):.0%} |")
    return L + [""]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--trace", required=True, help="rocprofv3 --kernel-trace --stats output dir")
    ap.add_argument("--trace-json", required=True, help="bench.py JSON line of the trace run")
    ap.add_argument("--fetch", help="rocprofv3 --pmc FETCH_SIZE output dir")
    ap.add_argument("--write", help="rocprofv3 --pmc WRITE_SIZE output dir")
    ap.add_argument("--pmc-json", help="bench.py JSON line of the counter runs")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--counters", action="append", default=[],
                    help="rocprofv3 --pmc output dir of a run with other counters (repeatable); its "
                         "bench.py JSON line is DIR.json")
    ap.add_argument("--commands", required=True, help="text file with the commands that were run")
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json")
    args = ap.parse_args()

    bench = json.loads(open(args.trace_json).read().strip().splitlines()[-1])
    table = kernel_table(args.trace)
    trace = _dispatches(os.path.join(args.trace, "run_kernel_trace.csv"))
    per_pass_ns = union_per_pass(trace, bench["config"]["passes"], bench["steps"] + bench["warmup"])
    step_avg_us = sum(per_pass_ns) / len(per_pass_ns) / 1e3 if per_pass_ns else float("nan")
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()

    L = [f"# Union step on {args.workload}" + (f" ({args.title})" if args.title else ""), ""]
    L += ["Run from the repository root on one MI355X (gfx950), ROCm 7.2, after "
          "`python -c 'import __graft_entry__ as g; g.build()'`. Commands:", "", "```"]
    L += [ln.rstrip() for ln in open(args.commands) if ln.strip()]
    L += ["```", "", "## Kernel trace", ""]
    runs = bench["steps"] + bench["warmup"]
    L += [f"{runs} HyperANF runs ({bench['warmup']} warm-up + {bench['steps']} timed), "
          f"{bench['config']['passes']} passes each (T = {bench['config']['T']}, pass kinds "
          f"{bench['config'].get('pass_kinds', '?')}: D all successors, F modified-flag frontier, "
          f"S systolic through the transposed graph, M systolic marked by a forward scan).", ""]
    L += ["| kernel | calls | avg µs | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in table:
        L.append(f"| {r['name']} | {r['calls']} | {r['avg_us']:.1f} | {r['total_ms']:.3f} | {r['pct']:.2f} |")
    rl = bench.get("roofline") or {}
    L += ["", f"Union step (k_union and k_union_list dispatches of a pass): rocprofv3 average over "
              f"{len(per_pass_ns)} passes {step_avg_us:.2f} µs; bench.py's HIP events in the same run "
              f"(timed runs, {rl.get('launches')} passes) {rl.get('avg_launch_us')} µs.", ""]

    rec = None
    if args.fetch and args.write and args.pmc_json and args.copy_fetch and args.copy_write:
        pmc = json.loads(open(args.pmc_json).read().strip().splitlines()[-1])
        alg = pmc["pass_algorithmic_bytes"]
        model = pmc.get("pass_model_bytes", alg)
        pr = pmc["config"]["passes"]
        runs_pmc = pmc["steps"] + pmc["warmup"]
        fetch = union_per_pass(_dispatches(os.path.join(args.fetch, "run_counter_collection.csv")), pr, runs_pmc)
        write = union_per_pass(_dispatches(os.path.join(args.write, "run_counter_collection.csv")), pr, runs_pmc)
        copy_bytes = args.copy_mib << 20
        fs = copy_scale(args.copy_fetch, copy_bytes)
        ws = copy_scale(args.copy_write, copy_bytes)
        n = min(len(fetch), len(write), len(alg))
        L += ["## Bytes beyond L2 (FETCH_SIZE, WRITE_SIZE)", ""]
        L += [f"Calibration: a plain {args.copy_mib} MiB device copy reads FETCH_SIZE and WRITE_SIZE such "
              f"that FETCH_SIZE is scaled by {fs:.3f} and WRITE_SIZE by {ws:.3f} to bytes. The counters "
              "count the L2's requests to the memory fabric: reads the Infinity Cache serves are "
              "included, so these bytes bound the HBM bytes from above. Model: the roofline's bytes "
              "(algorithmic, less the successor counters within the near window of their node).", ""]
        L += ["| pass t | FETCH_SIZE KiB | WRITE_SIZE KiB | beyond L2 GB | algorithmic GB | model GB | "
              "beyond L2 / model |", "|---:|---:|---:|---:|---:|---:|---:|"]
        tot_hbm = tot_alg = tot_mod = 0.0
        for t in range(n):
            hbm = fetch[t] * 1024 * fs + write[t] * 1024 * ws
            tot_hbm += hbm
            tot_alg += alg[t]
            tot_mod += model[t]
            L.append(f"| {t} | {fetch[t]:.0f} | {write[t]:.0f} | {hbm / 1e9:.3f} | {alg[t] / 1e9:.3f} | "
                     f"{model[t] / 1e9:.3f} | {hbm / model[t]:.2f} |")
        L += ["", f"Per pass (average of {n}): {tot_hbm / n / 1e9:.3f} GB moved beyond L2, "
                  f"{tot_alg / n / 1e9:.3f} GB algorithmic, {tot_mod / n / 1e9:.3f} GB in the model "
                  f"(beyond L2 / model {tot_hbm / tot_mod:.2f}).", ""]
        rec = dict(kernel="union step (k_union, k_union_list)", workload=args.workload,
                   kernel_source_sha256=sha, traffic_bytes_per_launch=int(tot_hbm / n),
                   traffic_kind="bytes beyond L2 (FETCH_SIZE + WRITE_SIZE, scaled by a device copy; "
                                "Infinity Cache hits included)",
                   algorithmic_bytes_per_launch=int(tot_alg / n), model_bytes_per_launch=int(tot_mod / n),
                   fetch_scale=fs, write_scale=ws, launches=n)
    if args.counters:
        L += ["## Other counters of the union step", "",
              "Summed over the union dispatches of a pass (k_union, k_union_list); the first pass "
              "(every successor gathered), the last pass (the fixpoint's, which changes no counter) "
              "and the average over the passes of one run.", "",
              "| counter | first pass | last pass | average per pass |", "|---|---:|---:|---:|"]
        first, last = {}, {}
        for d in args.counters:
            cj = json.loads(open(d.rstrip("/") + ".json").read().strip().splitlines()[-1])
            pr, runs_c = cj["config"]["passes"], cj["steps"] + cj["warmup"]
            for name, rows in sorted(counter_runs(os.path.join(d, "run_counter_collection.csv")).items()):
                per = union_per_pass(rows, pr, runs_c)
                if per:
                    L.append(f"| {name} | {per[0]:.4g} | {per[-1]:.4g} | {sum(per) / len(per):.4g} |")
                    first[name] = per[0]
                    last[name] = per[-1]
        L += [""]
        L += derived_utilisation(first, "first pass")
        L += derived_utilisation(last, "last pass")
    L += [f"Kernel source at measurement: `paper_1011_5599_amd/csrc/hanf_kernels.hip` sha256 `{sha[:16]}…` "
          "(bench.py reports `traffic` only while the source is unchanged)."]
    with open(args.out_md, "w") as f:
        f.write("\n".join(L) + "\n")
    if rec and args.out_json:
        with open(args.out_json, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
