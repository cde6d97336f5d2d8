"""The launch-shape autotuner (``lmfao_tune``): a first call times variants
of scan_blocks, contract_splits and one_hot_max and writes the JSON cache
keyed by plan hash; a second call returns the cached shapes without timing;
the tuned plan's results equal the oracle's."""
import json
import time

import pytest

import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu


def test_tune_writes_and_reuses_its_cache(tmp_path):
    import oracle
    import paper_2008_08657_amd as E
    p = W.retail_snowflake(seed=4, n_inv=100_000)
    cols = E.device_columns(p)
    cache = str(tmp_path / "shapes.json")
    base = dict(precision="f32", policy="fact", graph=True)
    t0 = time.perf_counter()
    first = E.tune(p, cols, cache_path=cache, runs=3, **base)
    t_first = time.perf_counter() - t0
    entries = json.load(open(cache))["entries"]
    assert len(entries) == 1
    (key, ent), = entries.items()
    assert ent["ms"] <= ent["base_ms"] + 1e-9
    assert first["tuned_ms"] == pytest.approx(ent["ms"], rel=1e-5)
    t0 = time.perf_counter()
    second = E.tune(p, cols, cache_path=cache, runs=3, **base)
    t_second = time.perf_counter() - t0
    assert second["options"] == first["options"]
    assert t_second < t_first
    plan = E.Plan(p, **first["options"])
    prep = E.Prepared(plan, cols)
    prep.run(sync=True)
    qs = list(range(0, len(p["batch"]), 97))
    ref = oracle.evaluate(p, qs)
    for i, q in enumerate(qs):
        compare(prep.result(q), ref[i], 1e-5, f"tuned query {q}")
