#!/usr/bin/env python
"""Benchmark of the aggregate-batch hot path on one MI355X.

Workload (default): the retail-shaped snowflake -- Inv(locn, date, ksn, units)
84M rows (locn uniform over 1.3k, date uniform over 124, ksn Zipf(1.0) over
5.6k), Items 5.6k, Stores 1.3k, Demog 1.3k, Weather 1.1M (full locn x date
grid) -- with the ridge covariance batch over 43 continuous features plus 6
one-hot categoricals: 1,269 aggregate queries (one SUM each), FP32 scans,
FP64 merges and results.  Synthetic data, seed 0.

One step = one ``lmfao_run``: every view and every query of the plan, on the
GPU, inputs already resident in HBM (prepare -- sorting and trie pieces -- is
done once before the timed region and reported separately).  The timed steps
replay the run as a HIP graph captured during the warm-up (``--no-graph``
launches directly); the per-kernel durations behind ``roofline`` come from as
many further runs launched directly with HIP events around each launch.

metric: join-tuple-aggregates/s = |D| * A / t_step, with |D| = 84M join tuples
(every fact row joins exactly once) and A = 1,269 SUM expressions.

Other workloads: ``--config grocery`` (BF16x3 contraction), ``cart`` (CART
node batch), ``chain`` (Rk-means step 1 with learned hash-table sizing),
``tiny``.  ``--plain-steps K`` also times the plain per-view form.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 exits: the
benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def _cpu_baseline(problem, n_rows, budget_s):
    """The oracle, as it stands, on a bounded prefix of the fact table."""
    import oracle
    import workloads as W
    fact = max(problem["schema"], key=lambda r: r["n_rows"])["name"]
    sample = W.fact_prefix(problem, fact, n_rows)
    t0 = time.perf_counter()
    res = oracle.evaluate(sample)
    dt = time.perf_counter() - t0
    n_aggs = sum(len(q["aggs"]) for q in problem["batch"])
    return {"value": n_rows * n_aggs / dt, "unit": "join-tuple-aggregates/s", "cores": 1,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"first {n_rows} of {problem['schema'][0]['n_rows']} {fact} rows, full dimension "
                      f"tables, all {len(problem['batch'])} queries (numpy FP64 with 80-bit accumulation, "
                      f"single thread)"}, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="retail", choices=["retail", "tiny", "grocery", "cart", "chain"])
    ap.add_argument("--precision", default=None, choices=["f64", "f32", "bf16x3", "bf16x2"],
                    help="arithmetic (default: the configuration's own)")
    ap.add_argument("--sizing", default=None, choices=["bound", "learned"],
                    help="hash-table sizing (default: learned for chain, bound otherwise)")
    ap.add_argument("--no-graph", action="store_true", help="launch every run directly (no HIP graph replay)")
    ap.add_argument("--scan-blocks", type=int, default=0, help="most workgroups of a scan launch (0 = 2048 generated, 512 built-in)")
    ap.add_argument("--contract-splits", type=int, default=0,
                    help="piece ranges per output tile column of a contraction (0 = 1024)")
    ap.add_argument("--one-hot-max", type=int, default=0, help="outputs keyed by outer codes only: largest key space expanded one-hot (0 = per group)")
    ap.add_argument("--plain-steps", type=int, default=0,
                    help="also time this many steps of the plain per-view form on the same input")
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the fact table (testing only)")
    ap.add_argument("--cpu-rows", type=int, default=150_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (scale for HBM byte counters)")
    ap.add_argument("--form", default="fused", choices=["fused", "per_view"],
                    help="fused: one pass per group of outputs (the method); per_view: one pass per output")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_2008_08657_amd as E

    if args.calibrate_copy:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE counters read the
        # bytes moved, giving the scale of those counters on this device
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)
        return

    E.load_library()
    t_gen = time.perf_counter()
    bw = W.bench_workload(args.config, args.scale)
    problem, workload = bw["problem"], bw["workload"]
    precision = args.precision or bw["precision"]
    sizing = args.sizing or bw["sizing"]
    fact = max(problem["schema"], key=lambda r: r["n_rows"])
    n_join = fact["n_rows"]   # every fact row joins exactly once (complete foreign keys)
    n_aggs = sum(len(q["aggs"]) for q in problem["batch"])
    t_gen = time.perf_counter() - t_gen

    plan = E.Plan(problem, precision=precision, policy=problem["policy"], form=args.form, sizing=sizing,
                  graph=not args.no_graph, one_hot_max=args.one_hot_max, scan_blocks=args.scan_blocks,
                  contract_splits=args.contract_splits)
    cols = E.device_columns(problem)
    torch.cuda.synchronize()
    t_prep = time.perf_counter()
    prep = E.Prepared(plan, cols)
    t_prep = time.perf_counter() - t_prep
    del cols
    torch.cuda.empty_cache()

    for _ in range(args.warmup):
        prep.run(sync=False)
    prep.run(sync=True)   # checks the kernels' error flags once
    torch.cuda.synchronize()

    # timed region: K runs replayed from the captured HIP graph (the warm-up
    # captured it), bracketed by device synchronisation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prep.run(sync=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_per_step = 1e3 * t / args.steps
    graph = prep.describe()["graph"]

    # per-launch durations: K more runs launched directly with HIP events
    # around every timed launch, on the run's stream
    prep.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prep.run(sync=False)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    prep.set_timing(False)
    timing = prep.timing()          # mean ms per timed launch over those runs
    desc = prep.describe()

    # dominant kernel: the timed launch with the largest mean duration
    steps = {s["name"]: s for s in desc["steps"]}
    kern = max((x for x in timing if x[0] != "run"), key=lambda x: x[1])
    kd = steps[kern[0]]
    kern_ms = kern[1]
    alg_bytes = kd["alg_read_bytes"] + kd["alg_write_bytes"]
    t_s = kern_ms * 1e-3
    mfma_peak = 2500.0 if precision.startswith("bf16") else 78.6   # the contraction's MFMA type
    if kd["kind"] in ("gemm", "contract") and kd["alg_flop"] / t_s / 1e12 / mfma_peak > alg_bytes / t_s / 8e12:
        # matrix-core contraction: priced against the MFMA peak of its type
        # (FP64, or bf16 for the split forms, counting useful flops only)
        peak = mfma_peak
        achieved = kd["alg_flop"] / (kern_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": None,
                    "kernel": kern[0], "kernel_ms": round(kern_ms, 4), "alg_flop": kd["alg_flop"]}
    else:
        achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                    "frac": round(achieved / 8000.0, 4), "traffic": None,
                    "kernel": kern[0], "kernel_ms": round(kern_ms, 4),
                    "alg_bytes": int(alg_bytes)}

    # HBM traffic of the dominant kernel from committed counter runs, valid
    # only while its generated source is the one that was profiled
    group = kern[0].rsplit(":", 1)[0]
    src = next((x.split("\n", 1)[1] for x in prep.kernel_sources() if x.split("\n", 1)[0] == group), None)
    digest = None
    if src is not None:
        # the kernel's source and its launch grid: counters taken at another
        # grid do not describe this launch
        from paper_2008_08657_amd.profiling import source_digest
        digest = source_digest(src + f"\n// grid {kd['grid']}")
    roofline["kernel_source_digest"] = digest
    prof_dir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
    if digest and os.path.isdir(prof_dir):
        for fn in sorted(os.listdir(prof_dir)):
            if not (fn.startswith("traffic_") and fn.endswith(".json")):
                continue
            with open(os.path.join(prof_dir, fn)) as f:
                rec = json.load(f)
            if rec.get("workload") == args.config and rec.get("step") == kern[0] and \
                    rec.get("source_digest") == digest:
                roofline["traffic"] = int(rec["bytes"])
                roofline["traffic_source"] = fn

    # sanity on the GPU results: COUNT equals |D| (closed form)
    check = {}
    if not args.no_check and not problem["batch"][0]["where"] and not problem["batch"][0]["groupby"]:
        r0 = prep.result(0)
        check["count_equals_join_size"] = bool(int(r0["count"][0]) == n_join
                                                and float(r0["sum"][0, 0]) == float(n_join))

    hashes = desc.get("hash_tables", [])
    sizing_info = {"tables": len(hashes), "slots": sum(h["slots"] for h in hashes),
                   "regrowths": desc.get("hash_regrowths", 0)} if hashes else None

    plain = None
    if args.plain_steps > 0 and args.form == "fused":
        # the plain form on the same input: one pass per output, no sharing
        del prep
        torch.cuda.empty_cache()
        cols = E.device_columns(problem)
        pplan = E.Plan(problem, precision=precision, policy=problem["policy"], form="per_view", sizing=sizing,
                       codegen=False)
        pprep = E.Prepared(pplan, cols)
        del cols
        torch.cuda.empty_cache()
        pprep.run(sync=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            pprep.run(sync=False)
        torch.cuda.synchronize()
        pms = 1e3 * (time.perf_counter() - t0) / args.plain_steps
        plain = {"form": "per_view", "steps": args.plain_steps, "ms_per_step": round(pms, 4),
                 "value": n_join * n_aggs / (pms * 1e-3), "fused_speedup": round(pms / ms_per_step, 2)}
        del pprep, pplan

    cpu = None
    if not args.no_cpu_baseline:
        cpu, _ = _cpu_baseline(problem, min(args.cpu_rows, n_join), 30.0)

    out = {
        "metric": "join-tuple-aggregates/s",
        "value": n_join * n_aggs / (ms_per_step * 1e-3),
        "unit": "join-tuple*aggregates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision,
        "data": "synthetic",
        "config": {"workload": workload, "join_tuples": n_join, "aggregates": n_aggs,
                   "queries": len(problem["batch"]), "precision": precision,
                   "form": args.form, "root_policy": problem["policy"], "seed": 0, "sizing": sizing,
                   "prepare_s": round(t_prep, 2), "generate_s": round(t_gen, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "graph": {"captured": bool(graph["captured"]), "ms_per_step_direct": round(1e3 * t_eager / args.steps, 4)},
        "kernels_ms": {k: round(v, 4) for k, v in timing},
        "kernels_launch": {k: [steps[k]["grid"], steps[k]["grid_y"], steps[k]["lds"]]
                           for k, _ in timing if k in steps},
        "plain": plain,
        "hash_sizing": sizing_info,
        "check": check,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
