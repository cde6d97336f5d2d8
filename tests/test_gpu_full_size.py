"""Parity at the benchmark's full size, in the launch configuration it times.

The retail-shaped snowflake (Inv 84M rows, 1,269 queries, FP32) runs exactly
as the benchmark runs it: the same generator call, the same plan options, the
warm-up run that captures the HIP graph, then graph replays.  The oracle cannot
evaluate the whole batch at this size in reasonable time, so a seeded sample
of outputs is compared instead: query 0 (COUNT and SUM(1) of the whole join),
two further aggregates without group-by and one grouped query, each reduced
to one aggregate, whole (every group), from one materialisation of the join
over the columns they need.  Keys and counts must be identical, sums within
the FP32 bound of the other parity tests.
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W

from parity import compare

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5


def sampled_batch(batch, seed):
    rng = np.random.default_rng(seed)
    plain = [i for i, q in enumerate(batch) if i and not q["groupby"]]
    grouped = [i for i, q in enumerate(batch) if q["groupby"]]
    picks = [0] + sorted(rng.choice(plain, 2, replace=False).tolist()) + [int(rng.choice(grouped))]
    out = []
    for qi in picks:
        ai = 0 if qi == 0 else int(rng.integers(len(batch[qi]["aggs"])))
        out.append((qi, ai))
    return out


def test_retail_full_size_sampled():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2008_08657_amd as E
    E.load_library()
    t0 = time.perf_counter()
    bw = W.bench_workload("retail")
    problem = bw["problem"]
    print(f"[full] retail generated in {time.perf_counter() - t0:.1f} s", flush=True)

    plan = E.Plan(problem, precision=bw["precision"], policy=problem["policy"], form="fused",
                  sizing=bw["sizing"], graph=True)
    cols = E.device_columns(problem)
    prep = E.Prepared(plan, cols)
    del cols
    prep.run(sync=False)          # warm-up: captures the graph
    prep.run(sync=True)           # replay, error flags checked
    assert prep.describe()["graph"]["captured"]
    picks = sampled_batch(problem["batch"], seed=2008)
    gpu = {}
    for qi, ai in picks:
        r = prep.result(qi)
        gpu[qi] = {"keys": r["keys"], "count": r["count"], "sum": r["sum"][:, ai:ai + 1]}
    del prep, plan
    torch.cuda.empty_cache()
    print(f"[full] GPU run done; sampled (query, aggregate): {picks}", flush=True)

    sub = []
    needed = set()
    for qi, ai in picks:
        q = dict(problem["batch"][qi])
        q["aggs"] = [q["aggs"][ai]]
        sub.append(q)
        needed |= set(q["groupby"]) | {w[0] for w in q["where"]} | {a for a, _ in q["aggs"][0]}
    t0 = time.perf_counter()
    D = oracle.materialize_join(problem, needed)
    print(f"[full] oracle join materialised in {time.perf_counter() - t0:.1f} s", flush=True)

    n_join = problem["schema"][0]["n_rows"]
    for (qi, ai), q in zip(picks, sub):
        t0 = time.perf_counter()
        r = oracle.evaluate_query(D, q)
        if qi == 0:
            assert int(r["count"][0]) == n_join      # complete foreign keys: |D| = |Inv|
        worst = compare(gpu[qi], r, F32_TOL, f"retail full size, query {qi} aggregate {ai}")
        print(f"[full] query {qi} aggregate {ai}: {r['keys'].shape[0]} groups, worst scaled error {worst:.2e} "
              f"(oracle {time.perf_counter() - t0:.1f} s)", flush=True)
