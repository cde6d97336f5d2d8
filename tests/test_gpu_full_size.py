"""Parity at the benchmark's full sizes, in the launch configuration it times.

Each measured workload (``workloads.bench_workload``: the retail-shaped
snowflake, the grocery-shaped star in BF16x3, the CART node batch and the
Rk-means step-1 chain) runs exactly as ``bench.py`` runs it: the same
generator call, the same plan options (``workloads.bench_plan_options``) with
the autotuner's launch shapes, a warm-up run that captures the HIP graph,
then a graph replay.  EVERY output is
compared with the expected results that ``tests/golden/make_full_size.py``
wrote from the streaming tier-B oracle (the plain definition, enumerating the
natural join on all host cores):

* keys and counts identical, float sums within 1e-5 of
  max(|oracle|, 1e-3 * sum |terms|);
* outputs with too many groups to store (the chain's large integer
  group-bys) by their group count, total count and a SHA-256 over the keys
  and counts, which the GPU result must reproduce bit for bit.

The golden files record the digest of the generated columns: a mismatch
means the generator changed and the files must be written again.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import workloads as W

from parity import compare

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-5


def load_golden(config):
    z = np.load(os.path.join(GOLDEN, f"full_{config}.npz"), allow_pickle=False)
    meta = json.loads(bytes(z["meta"]).decode())
    return z, meta


def result_digest(keys, count):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(keys, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(count, dtype="<i8").tobytes())
    return h.hexdigest()


def check_against_golden(prep, problem, config):
    z, meta = load_golden(config)
    worst, digests = 0.0, 0
    for qi, m in enumerate(meta["queries"]):
        r = prep.result(qi)
        where = f"{config} full size, query {qi}"
        assert r["keys"].shape[0] == m["groups"], f"{where}: {r['keys'].shape[0]} groups, expected {m['groups']}"
        assert int(r["count"].sum()) == m["total_count"], where
        if m["stored"]:
            ref = {"keys": z[f"q{qi}_keys"], "count": z[f"q{qi}_count"], "sum": z[f"q{qi}_sum"],
                   "abs": z[f"q{qi}_abs"]}
            worst = max(worst, compare(r, ref, TOL, where))
        else:
            assert result_digest(r["keys"], r["count"]) == m["sha256"], f"{where}: keys or counts differ"
            aggs = problem["batch"][qi]["aggs"]
            for k, f in enumerate(aggs):
                if not f:   # SUM(1) equals the count exactly
                    np.testing.assert_array_equal(r["sum"][:, k], r["count"].astype(np.float64), err_msg=where)
            digests += 1
    return worst, digests, len(meta["queries"])


@pytest.mark.parametrize("config", ["retail", "grocery", "cart", "chain"])
def test_full_size_every_output(config):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2008_08657_amd as E
    E.load_library()
    t0 = time.perf_counter()
    bw = W.bench_workload(config)
    problem = bw["problem"]
    _, meta = load_golden(config)
    assert W.problem_digest(problem) == meta["problem_digest"], \
        f"the {config} generator changed: run tests/golden/make_full_size.py {config}"
    print(f"[full] {config} generated in {time.perf_counter() - t0:.1f} s", flush=True)
    cols = E.device_columns(problem)
    # the launch shapes bench.py times: the autotuner's (from its cache)
    opts = E.tune(problem, cols, cache_path=E.TUNED_SHAPES, runs=5, **W.bench_plan_options(bw))["options"]
    plan = E.Plan(problem, **opts)
    prep = E.Prepared(plan, cols)
    del cols
    torch.cuda.empty_cache()
    prep.run(sync=False)          # warm-up: captures the graph
    prep.run(sync=True)           # a replay (or a run after a regrowth), error flags checked
    # the timed path: the largest relation's scans run the kernels generated
    # for their groups (hipRTC), not the built-in fallback
    d = prep.describe()
    assert not d["codegen_failures"], d["codegen_failures"]
    scans = [s for s in d["steps"] if s["kind"] == "scan"]
    top = max(s["rows"] for s in scans)
    assert all(s["lean"] == 2 for s in scans if s["rows"] == top), [s["name"] for s in scans]
    t0 = time.perf_counter()
    worst, digests, n = check_against_golden(prep, problem, config)
    print(f"[full] {config}: {n} queries, {n - digests} compared cell by cell (worst scaled error {worst:.2e}), "
          f"{digests} by digest; read back in {time.perf_counter() - t0:.1f} s", flush=True)
    del prep, plan
    torch.cuda.empty_cache()
