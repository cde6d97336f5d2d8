#!/usr/bin/env python
"""Benchmark of the aggregate-batch hot path on one MI355X.

Headline workload (default ``--config chain``): step 1 of Rk-means on a
3-relation chain join -- R1(a, b, x1..x40) 50M rows, R2(b, c, y1..y30) 5M
rows, R3(c, z1..z30) 200k rows, foreign keys b and c, attribute domains
log-uniform in [10, 1e6] -- with SUM(1) grouped by each of the 100 attributes
and by 10 attribute pairs (110 aggregates), hash tables sized by the learned
estimator.  This is the largest single-GPU configuration and the one whose
batch uses every part of the metric (fused form, learned sizing).  The
retail-shaped snowflake (Inv 84M rows, 1,269 covariance aggregates, FP32) is
measured in the same run as a labelled sub-record (``--sub``).

One step = one ``lmfao_run``: every view and every query of the plan, on the
GPU, inputs already resident in HBM (``lmfao_prepare`` -- sorting, trie
pieces, hash tables -- runs once before the timed region and is reported
separately).  The timed steps replay the run as a HIP graph captured during
the warm-up; per-launch durations come from as many further runs launched
directly with HIP events around each launch on the run's stream.

Reported beside the throughput (join-tuple-aggregates/s = |D| * A / t_step):

* ``roofline``: the launch with the largest mean duration, its algorithmic
  bytes counted as every column of the relation that its outputs reference
  (rows x column bytes, read once, whether the kernel reads it or prepare
  folded it into piece keys) plus its writes, against 8 TB/s; the bytes the
  kernel itself must read are printed beside it (``needed_bytes``);
* ``largest_pass``: the same accounting over all launches of the relation
  pass with the most bytes;
* ``plain``: the plain per-view form (one pass per output) on the same input;
* ``hash_sizing``: learned, bound and exact-count sizing of the hash tables:
  slots, zero-filled bytes, regrowths and step time, and whether the results
  are identical;
* ``accuracy``: every output against the full-size expected results of
  ``tests/golden/`` (written by the tier-B oracle): worst scaled and plain
  relative error, integers exact;
* ``cpu_baseline``: the tier-B oracle (C, OpenMP, all host cores) on a
  bounded sample of the same workload.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the benchmark measures
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(ROOT, "tests", "golden")
HBM_PEAK_GBS = 8000.0
T0 = time.perf_counter()


def _log(msg):
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(problem, target_s=15.0):
    """The tier-B oracle (the plain definition, enumerating the join on all
    host cores) on the first rows of the fact relation, sized from a 1%
    calibration run to take about ``target_s`` seconds."""
    from oracle import tierb
    fact = max(problem["schema"], key=lambda r: r["n_rows"])
    n_fact = fact["n_rows"]
    n_aggs = sum(len(q["aggs"]) for q in problem["batch"])
    st = {}
    cal = max(1000, n_fact // 100)
    _log(f"cpu baseline: calibration on {cal} {fact['name']} rows")
    tierb.evaluate(problem, root=fact["name"], root_rows=cal, stats=st)
    rows = int(min(n_fact, max(cal, cal * target_s / max(st["seconds"], 1e-3))))
    st = {}
    _log(f"cpu baseline: {rows} {fact['name']} rows")
    tierb.evaluate(problem, root=fact["name"], root_rows=rows, stats=st)
    return {"value": rows * n_aggs / st["seconds"], "unit": "join-tuple*aggregates/s", "cores": st["threads"],
            "kind": "oracle", "seconds": round(st["seconds"], 3),
            "sample": f"tuples of D extending the first {rows} of {n_fact} {fact['name']} rows (full other "
                      f"relations), all {len(problem['batch'])} queries; tier-B oracle (C, OpenMP, FP64 "
                      f"Neumaier sums, no factorisation)",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def _digest(keys, count):
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(keys, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(count, dtype="<i8").tobytes())
    return h.hexdigest()


def _accuracy(prep, config, problem):
    """Every output against the golden results of the full-size workload."""
    import numpy as np
    path = os.path.join(GOLDEN, f"full_{config}.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(z["meta"]).decode())
    import workloads as W
    if meta["problem_digest"] != W.problem_digest(problem):
        return {"golden": os.path.relpath(path, ROOT), "error": "generator changed since the golden was written"}
    worst = worst_plain = 0.0
    cells = floored = digests = 0
    exact = True
    for qi, m in enumerate(meta["queries"]):
        r = prep.result(qi)
        if r["keys"].shape[0] != m["groups"] or int(r["count"].sum()) != m["total_count"]:
            exact = False
            continue
        if not m["stored"]:
            exact &= _digest(r["keys"], r["count"]) == m["sha256"]
            digests += 1
            continue
        exact &= bool(np.array_equal(r["keys"], z[f"q{qi}_keys"]) and np.array_equal(r["count"], z[f"q{qi}_count"]))
        o, a, ab = z[f"q{qi}_sum"], r["sum"], z[f"q{qi}_abs"]
        if o.size == 0:
            continue
        scale = np.maximum(np.abs(o), 1e-3 * ab)
        scale = np.where(scale == 0, 1.0, scale)
        worst = max(worst, float((np.abs(a - o) / scale).max()))
        nz = np.abs(o) > 0
        if nz.any():
            worst_plain = max(worst_plain, float((np.abs(a - o)[nz] / np.abs(o)[nz]).max()))
        floored += int((1e-3 * ab > np.abs(o)).sum())
        cells += int(o.size)
    return {"golden": os.path.relpath(path, ROOT), "oracle": meta.get("oracle"), "queries": len(meta["queries"]),
            "float_cells": cells, "max_scaled_err": worst, "max_rel_err": worst_plain,
            "cells_on_floor": floored, "compared_by_digest": digests, "integers_exact": bool(exact),
            "tol": 1e-5}


def _results_digest(prep, n_queries):
    h = hashlib.sha256()
    for q in range(n_queries):
        r = prep.result(q)
        for k in ("keys", "count", "sum"):
            h.update(r[k].tobytes())
    return h.hexdigest()


def _time_steps(prep, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prep.run(sync=False)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def _roofline(desc, timing):
    steps = {s["name"]: s for s in desc["steps"]}
    kern = max((x for x in timing if x[0] != "run"), key=lambda x: x[1])
    kd = steps[kern[0]]
    t_s = kern[1] * 1e-3
    needed = kd["alg_read_bytes"] + kd["alg_write_bytes"]
    alg = kd.get("pass_read_bytes", kd["alg_read_bytes"]) + kd["alg_write_bytes"]
    achieved = alg / t_s / 1e9
    return kern, kd, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kern[0],
                      "kernel_ms": round(kern[1], 4), "alg_bytes": int(alg), "needed_bytes": int(needed),
                      "needed_frac": round(needed / t_s / 1e9 / HBM_PEAK_GBS, 4)}


def _largest_pass(desc, timing):
    """All launches of one relation's pass: every column of the relation that
    the launches reference, read once, over their summed mean durations."""
    ms = dict(timing)
    passes = {}
    for s in desc["steps"]:
        if "relation" not in s or s["name"] not in ms:
            continue
        p = passes.setdefault(s["relation"], {"rows": s["relation_rows"], "cols": {}, "ms": 0.0, "launches": 0})
        p["cols"].update(zip(s["pass_cols"], s["pass_col_bytes"]))
        p["ms"] += ms[s["name"]]
        p["launches"] += 1
    if not passes:
        return None
    rel, p = max(passes.items(), key=lambda kv: kv[1]["rows"] * sum(kv[1]["cols"].values()))
    byts = p["rows"] * sum(p["cols"].values())
    gbs = byts / (p["ms"] * 1e-3) / 1e9
    return {"relation": rel, "rows": p["rows"], "columns": len(p["cols"]), "bytes": int(byts),
            "launches": p["launches"], "ms": round(p["ms"], 4), "achieved": round(gbs, 1), "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def _traffic(prep, kern, kd, config):
    """HBM bytes of the dominant launch from committed counter runs, valid only
    while its source (the generated kernel, or the library's kernel file for
    built-in kernels) and grid are the ones that were profiled."""
    from paper_2008_08657_amd.profiling import source_digest, builtin_source
    group = kern[0].rsplit(":", 1)[0]
    src = next((x.split("\n", 1)[1] for x in prep.kernel_sources() if x.split("\n", 1)[0] == group), None)
    if src is None or kd.get("lean", 0) != 2:
        src = builtin_source() + f"\n// step {kern[0]}"
    digest = source_digest(src + f"\n// grid {kd['grid']}")
    prof_dir = os.path.join(ROOT, "profiles")
    for fn in sorted(os.listdir(prof_dir)) if os.path.isdir(prof_dir) else []:
        if not (fn.startswith("traffic_") and fn.endswith(".json")):
            continue
        with open(os.path.join(prof_dir, fn)) as f:
            rec = json.load(f)
        if rec.get("workload") == config and rec.get("step") == kern[0] and rec.get("source_digest") == digest:
            return int(rec["bytes"]), digest
    return None, digest


def measure(E, W, config, args, full=True):
    """One workload: fused-form throughput, per-launch roofline, accuracy,
    plain form and (with hash tables) the sizing comparison."""
    import torch
    t_gen = time.perf_counter()
    _log(f"{config}: generating")
    bw = W.bench_workload(config, args.scale)
    problem = bw["problem"]
    if args.precision and full:
        bw["precision"] = args.precision
    if args.sizing and full:
        bw["sizing"] = args.sizing
    fact = max(problem["schema"], key=lambda r: r["n_rows"])
    n_join = fact["n_rows"]   # every fact row joins exactly once (complete foreign keys)
    n_aggs = sum(len(q["aggs"]) for q in problem["batch"])
    t_gen = time.perf_counter() - t_gen
    opts = W.bench_plan_options(bw, graph=not args.no_graph)
    cols = E.device_columns(problem)
    tuning = None
    if args.scan_blocks or args.contract_splits or args.one_hot_max or args.no_tune:
        opts.update(scan_blocks=args.scan_blocks, contract_splits=args.contract_splits,
                    one_hot_max=args.one_hot_max)
    else:
        # launch shapes from the autotuner (its JSON cache; a miss is tuned now)
        _log(f"{config}: launch shapes (autotuner, cache {os.path.relpath(args.tune_cache, ROOT)})")
        t0 = time.perf_counter()
        tuned = E.tune(problem, cols, cache_path=args.tune_cache, runs=5, **opts)
        opts = tuned["options"]
        tuning = {"scan_blocks": opts["scan_blocks"], "contract_splits": opts["contract_splits"],
                  "one_hot_max": opts["one_hot_max"], "tuned_ms": round(tuned["tuned_ms"], 4),
                  "base_ms": round(tuned["base_ms"], 4), "seconds": round(time.perf_counter() - t0, 1)}
    plan = E.Plan(problem, **opts)
    torch.cuda.synchronize()
    _log(f"{config}: prepare")
    t_prep = time.perf_counter()
    prep = E.Prepared(plan, cols)
    t_prep = time.perf_counter() - t_prep
    del cols
    torch.cuda.empty_cache()

    _log(f"{config}: warm-up and timed steps")
    for _ in range(args.warmup):
        prep.run(sync=False)
    prep.run(sync=True)   # checks the kernels' error flags (and regrows a hash table that overflowed)
    for _ in range(2):
        prep.run(sync=False)   # recapture after a regrowth
    # timed region: K graph replays bracketed by device synchronisation
    ms_per_step = _time_steps(prep, args.steps)
    graph = prep.describe()["graph"]
    # per-launch durations: K direct runs with HIP events around every launch
    prep.set_timing(True)
    ms_direct = _time_steps(prep, args.steps)
    prep.set_timing(False)
    timing = prep.timing()
    desc = prep.describe()
    kern, kd, roof = _roofline(desc, timing)
    traffic, digest = _traffic(prep, kern, kd, config)
    roof["traffic"] = traffic
    roof["kernel_source_digest"] = digest
    rec = {
        "value": n_join * n_aggs / (ms_per_step * 1e-3),
        "ms_per_step": round(ms_per_step, 4),
        "dtype": {"f64": "f64", "f32": "f32", "bf16x3": "bf16x3", "bf16x2": "bf16x2"}[bw["precision"]]
        if config != "chain" else "int32",
        "config": {"workload": bw["workload"], "join_tuples": n_join, "aggregates": n_aggs,
                   "queries": len(problem["batch"]), "precision": bw["precision"], "form": "fused",
                   "root_policy": problem["policy"], "seed": 0, "sizing": bw["sizing"],
                   "prepare_s": round(t_prep, 2), "generate_s": round(t_gen, 2)},
        "roofline": roof,
        "largest_pass": _largest_pass(desc, timing),
        "graph": {"captured": bool(graph["captured"]), "ms_per_step_direct": round(ms_direct, 4)},
        "kernels_ms": {k: round(v, 4) for k, v in timing},
        "hash_tables": {"tables": len(desc.get("hash_tables", [])),
                        "slots": sum(h["slots"] for h in desc.get("hash_tables", [])),
                        "regrowths": desc.get("hash_regrowths", 0),
                        "picked_by_estimator": desc.get("picked_hash", 0)},
        "tuning": tuning,
    }
    if not args.no_check and args.scale == 1.0:
        t0 = time.perf_counter()
        _log(f"{config}: comparing with the golden results")
        rec["accuracy"] = _accuracy(prep, config, problem)
        if rec["accuracy"] is not None:
            rec["accuracy"]["seconds"] = round(time.perf_counter() - t0, 1)
    has_hash = bool(desc.get("hash_tables"))
    del prep, plan
    torch.cuda.empty_cache()

    if has_hash and args.sizing_steps > 0:
        rec["hash_sizing"] = _sizing(E, W, bw, args)
    if args.plain_steps > 0:
        _log(f"{config}: plain per-view form")
        cols = E.device_columns(problem)
        pplan = E.Plan(problem, **dict(W.bench_plan_options(bw, form="per_view", graph=False), codegen=False))
        pprep = E.Prepared(pplan, cols)
        del cols
        torch.cuda.empty_cache()
        pprep.run(sync=True)
        pms = _time_steps(pprep, args.plain_steps)
        rec["plain"] = {"form": "per_view", "steps": args.plain_steps, "ms_per_step": round(pms, 4),
                        "value": n_join * n_aggs / (pms * 1e-3), "fused_speedup": round(pms / ms_per_step, 2)}
        del pprep, pplan
        torch.cuda.empty_cache()
    if full and not args.no_cpu_baseline:
        rec["cpu_baseline"] = _cpu_baseline(problem)
    return rec


def _sizing(E, W, bw, args):
    """The same batch with hash tables sized by the learned estimator, by the
    group-count bound and by an exact-count pass: table slots, zero-filled
    bytes, regrowths and step time; results must be identical."""
    import torch
    problem = bw["problem"]
    out, digests = {}, {}
    for sizing in ("learned", "bound", "exact"):
        _log(f"sizing comparison: {sizing}")
        cols = E.device_columns(problem)
        plan = E.Plan(problem, **dict(W.bench_plan_options(dict(bw, sizing=sizing), graph=not args.no_graph)))
        t0 = time.perf_counter()
        prep = E.Prepared(plan, cols)
        t_prep = time.perf_counter() - t0
        del cols
        torch.cuda.empty_cache()
        prep.run(sync=True)
        for _ in range(2):
            prep.run(sync=False)
        ms = _time_steps(prep, args.sizing_steps)
        d = prep.describe()
        hs = d.get("hash_tables", [])
        out[sizing] = {"ms_per_step": round(ms, 4), "slots": sum(h["slots"] for h in hs),
                       "table_bytes": sum(h["slots"] for h in hs) * 24, "fill_bytes": d.get("fill_bytes"),
                       "regrowths": d.get("hash_regrowths", 0), "prepare_s": round(t_prep, 2)}
        prep.run(sync=True)
        digests[sizing] = _results_digest(prep, len(problem["batch"]))
        del prep, plan
        torch.cuda.empty_cache()
    out["identical_results"] = len(set(digests.values())) == 1
    out["learned_vs_bound_speedup"] = round(out["bound"]["ms_per_step"] / out["learned"]["ms_per_step"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="chain", choices=["retail", "tiny", "grocery", "cart", "chain"])
    ap.add_argument("--sub", default="retail",
                    help="comma-separated workloads measured as labelled sub-records ('' for none)")
    ap.add_argument("--precision", default=None, choices=["f64", "f32", "bf16x3", "bf16x2"],
                    help="arithmetic of the headline workload (default: its own)")
    ap.add_argument("--sizing", default=None, choices=["bound", "learned", "exact"],
                    help="hash-table sizing of the headline workload (default: its own)")
    ap.add_argument("--no-graph", action="store_true", help="launch every run directly (no HIP graph replay)")
    ap.add_argument("--scan-blocks", type=int, default=0)
    ap.add_argument("--contract-splits", type=int, default=0)
    ap.add_argument("--one-hot-max", type=int, default=0)
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the plain per-view form timed on the same input (0 = skip)")
    ap.add_argument("--sizing-steps", type=int, default=5,
                    help="steps timed per hash-table sizing in the sizing comparison (0 = skip)")
    ap.add_argument("--no-tune", action="store_true", help="the library's default launch shapes (no autotuner)")
    ap.add_argument("--tune-cache", default=None, help="JSON cache of the autotuner (default: the package's)")
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the fact table (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the comparison with the golden results")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (scale for HBM byte counters)")
    ap.add_argument("--form", default="fused", choices=["fused"], help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

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
    if args.tune_cache is None:
        args.tune_cache = E.TUNED_SHAPES
    head = measure(E, W, args.config, args, full=True)
    subs = {}
    for c in [x for x in args.sub.split(",") if x and x != args.config]:
        sub_args = argparse.Namespace(**vars(args))
        sub_args.sizing_steps = 0
        subs[c] = measure(E, W, c, sub_args, full=False)
    out = {
        "metric": "join-tuple-aggregates/s",
        "value": head["value"],
        "unit": "join-tuple*aggregates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
    }
    out.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step", "dtype")})
    out["sub"] = subs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
