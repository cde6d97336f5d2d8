"""Integer range of join multiplicities on the GPU path.

A many-to-many join multiplies tuple counts: two relations of n and m rows
that share one key value join into n*m tuples (paper, section 2: D is the
natural join with bag semantics).  The scans sum multiplicities in 32-bit
counters per piece and per workgroup and widen to 64 bits in the contraction
and merges, so a COUNT far above 2^31 is exact as long as each 32-bit partial
stays in range; a run whose multiplicities could overflow a partial must
report LMFAO_EOVERFLOW instead of a wrapped result.  Expected values here are
closed forms (n*m, sums of products of independent sums).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2008_08657_amd as E
    E.load_library()
    return E


def one_key_pair(n, m, seed=0, n_cat=4):
    rng = np.random.default_rng(seed)
    x = np.round(rng.standard_normal(n), 3)
    y = np.round(rng.standard_normal(m), 3)
    cat = rng.integers(0, n_cat, n).astype(np.int32)
    schema = [
        {"name": "A", "n_rows": n, "attrs": [{"name": "k", "dtype": "i32", "domain": 2, "key": False},
                                              {"name": "x", "dtype": "f64", "domain": 0, "key": False},
                                              {"name": "cat", "dtype": "i32", "domain": n_cat, "key": False}]},
        {"name": "B", "n_rows": m, "attrs": [{"name": "k", "dtype": "i32", "domain": 2, "key": False},
                                              {"name": "y", "dtype": "f64", "domain": 0, "key": False}]},
    ]
    data = {"A": {"k": np.zeros(n, np.int32), "x": x, "cat": cat},
            "B": {"k": np.zeros(m, np.int32), "y": y}}
    aggs = [[], [("x", 1)], [("y", 1)], [("x", 1), ("y", 1)]]
    batch = [{"groupby": [], "where": [], "aggs": aggs, "root": "A"},
             {"groupby": ["cat"], "where": [], "aggs": [[]], "root": "A"}]
    return {"schema": schema, "tree": [(0, 1)], "batch": batch, "data": data, "policy": "groupby"}


def test_count_above_2_31_is_exact(eng):
    # 100k x 100k rows sharing one key: COUNT = 1e10
    n = m = 100_000
    p = one_key_pair(n, m)
    print(f"[case] one-key join {n} x {m}", flush=True)
    plan = eng.Plan(p, precision="f64", row_piece_max=-1)
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    r0, r1 = prep.result(0), prep.result(1)
    assert r0["count"].tolist() == [n * m]
    sx, sy = math.fsum(p["data"]["A"]["x"]), math.fsum(p["data"]["B"]["y"])
    want = [float(n * m), sx * m, sy * n, sx * sy]
    ax = float(np.abs(p["data"]["A"]["x"]).sum())
    ay = float(np.abs(p["data"]["B"]["y"]).sum())
    floor = [float(n * m), ax * m, ay * n, ax * ay]
    for got, w, f in zip(r0["sum"][0], want, floor):
        assert abs(got - w) <= 1e-12 * max(abs(w), 1e-3 * f), (got, w)
    cat = p["data"]["A"]["cat"]
    assert r1["keys"][:, 0].tolist() == sorted(set(cat.tolist()))
    assert r1["count"].tolist() == [int((cat == c).sum()) * m for c in sorted(set(cat.tolist()))]


def test_multiplicity_beyond_32_bit_partials_is_reported(eng):
    # 1M fact rows times a multiplicity of 2.5M on one key: a workgroup of the
    # scan sums thousands of rows, each worth 2.5M tuples, into 32-bit
    # counters -- the run must refuse instead of wrapping
    n, m = 1_000_000, 2_500_000
    p = one_key_pair(n, m, seed=1)
    print(f"[case] one-key join {n} x {m} (expects LMFAO_EOVERFLOW)", flush=True)
    plan = eng.Plan(p, precision="f64", row_piece_max=-1)
    prep = eng.Prepared(plan, eng.device_columns(p))
    with pytest.raises(eng.LmfaoError) as ei:
        prep.run(sync=True)
    assert ei.value.status == 5, str(ei.value)
    assert "32-bit" in str(ei.value)
    # the result readers see the same flag
    with pytest.raises(eng.LmfaoError):
        prep.result(0)


def one_key_grouped(n, m, dom, all_one_cell=False, seed=0):
    """A (n rows: key k = 0, g over a domain of `dom` values) joined with B (m
    rows, all k = 0): SUM(1) GROUP BY g rooted at A counts every A row m
    times -- the partition count with each row weighted by the count of B
    tuples per key."""
    rng = np.random.default_rng(seed)
    g = np.zeros(n, np.int32) if all_one_cell else rng.integers(0, dom, n).astype(np.int32)
    schema = [
        {"name": "A", "n_rows": n, "attrs": [{"name": "k", "dtype": "i32", "domain": 2, "key": False},
                                              {"name": "g", "dtype": "i32", "domain": dom, "key": False}]},
        {"name": "B", "n_rows": m, "attrs": [{"name": "k", "dtype": "i32", "domain": 2, "key": False}]},
    ]
    data = {"A": {"k": np.zeros(n, np.int32), "g": g}, "B": {"k": np.zeros(m, np.int32)}}
    batch = [{"groupby": ["g"], "where": [], "aggs": [[]], "root": "A"}]
    return {"schema": schema, "tree": [(0, 1)], "batch": batch, "data": data, "policy": "groupby"}


def test_weighted_partition_count_beyond_2_32_in_total(eng):
    # 300k A rows over 20,000 cells, each worth 40k B tuples: 1.2e10 tuples
    # in all, about 6e5 per cell -- exact, with cells and chunks summed in
    # 64 bits (closed form: rows of the cell times m)
    n, m, dom = 300_000, 40_000, 20_000
    p = one_key_grouped(n, m, dom)
    print(f"[case] weighted partition {n} x {m} over {dom} cells", flush=True)
    plan = eng.Plan(p, precision="f64")
    assert any(g.get("partitioned") for g in plan.describe()["groups"])
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    r = prep.result(0)
    g = p["data"]["A"]["g"]
    vals, cnt = np.unique(g, return_counts=True)
    assert r["keys"][:, 0].tolist() == vals.tolist()
    assert r["count"].tolist() == (cnt.astype(np.int64) * m).tolist()


def test_weighted_partition_one_cell_beyond_2_32(eng):
    # every one of 200k A rows in one cell, each worth 40k B tuples: 8e9 in
    # the cell, each of the direct pass's three row chunks below 2^32 in LDS
    n, m, dom = 200_000, 40_000, 20_000
    p = one_key_grouped(n, m, dom, all_one_cell=True)
    print(f"[case] weighted partition, one cell of {n} x {m}", flush=True)
    plan = eng.Plan(p, precision="f64")
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    r = prep.result(0)
    assert r["keys"][:, 0].tolist() == [0] and r["count"].tolist() == [n * m]


def test_weighted_partition_cell_beyond_32_bits_is_reported(eng):
    # the same with 100k B tuples per row: a chunk of about 66.7k rows adds
    # 6.7e9 to the cell's 32-bit LDS count -- the run must refuse
    n, m, dom = 200_000, 100_000, 20_000
    p = one_key_grouped(n, m, dom, all_one_cell=True)
    print(f"[case] weighted partition, one cell of {n} x {m} (expects LMFAO_EOVERFLOW)", flush=True)
    plan = eng.Plan(p, precision="f64")
    prep = eng.Prepared(plan, eng.device_columns(p))
    with pytest.raises(eng.LmfaoError) as ei:
        prep.run(sync=True)
    assert ei.value.status == 5, str(ei.value)
    with pytest.raises(eng.LmfaoError):
        prep.result(0)
