"""The seeded input generators behind the benchmark and the parity tests."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("name, precision", [("retail", "f32"), ("grocery", "bf16x3"), ("cart", "f32"),
                                             ("chain", "f32"), ("tiny", "f64")])
def test_bench_workload_configurations(name, precision):
    bw = W.bench_workload(name, scale=2e-5)
    assert bw["precision"] == precision
    assert bw["sizing"] == ("learned" if name == "chain" else "bound")
    p = bw["problem"]
    for rel in p["schema"]:
        for a in rel["attrs"]:
            assert len(p["data"][rel["name"]][a["name"]]) == rel["n_rows"]
    # same seed, same data
    q = W.bench_workload(name, scale=2e-5)["problem"]
    assert W.problem_digest(p) == W.problem_digest(q)


def test_bench_workload_rejects_unknown_names():
    with pytest.raises(ValueError):
        W.bench_workload("nope")


def test_tagged_star_join_size_counts_tags():
    # every fact row joins once per tag of its item (Stores and Items are keyed)
    p = W.tagged_star(seed=1, n_fact=20_000, n_items=500, dup_frac=0.1)
    tags = np.bincount(p["data"]["Tags"]["item"], minlength=500)
    assert set(np.unique(tags)) == {1, 2}
    ref = oracle.evaluate(p)
    assert int(ref[0]["count"][0]) == int(tags[p["data"]["S"]["item"]].sum())
    # grouped by cat, the counts add up to the join size
    assert int(ref[1]["count"].sum()) == int(ref[0]["count"][0])
