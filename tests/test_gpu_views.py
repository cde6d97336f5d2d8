"""Parity of every intermediate view the GPU computes with the oracle's
``evaluate_view`` (paper, section 2, view generation layer: the view along an
edge is the join of the subtree below it, grouped by the edge's join
attributes, holding the partial aggregates the queries above need).

The plan description names, per view, the relation it leaves and enters, its
key attributes, the value columns stored per key (attribute values for a view
with at most one subtree tuple per key, aggregate monomials otherwise), the
group-by attributes it carries as codes, and the conditions pushed into it.
``lmfao_view_copy`` returns the dense arrays over the key domain (last key
attribute fastest).  Keys with a nonzero count must be exactly the oracle's
groups, with identical counts and codes; value columns match to the plan's
tolerance; every other key must hold count 0.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from parity import compare

pytestmark = pytest.mark.gpu

OPS = {0: "<=", 1: "<", 2: ">", 3: ">=", 4: "==", 5: "!="}


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2008_08657_amd as E
    E.load_library()
    return E


def with_derived(problem, plan_desc):
    """Adds the plan's derived bucket codes (the number of thresholds below
    the value, or at most the value) as columns, so the oracle can group and
    carry them like any attribute."""
    if not plan_desc.get("derived"):
        return problem
    p = dict(problem, data={k: dict(v) for k, v in problem["data"].items()},
             schema=[dict(r, attrs=list(r["attrs"])) for r in problem["schema"]])
    for d in plan_desc["derived"]:
        rel = next(r for r in p["schema"] if r["name"] == d["relation"])
        x = np.asarray(p["data"][d["relation"]][d["source"]], dtype=np.float64)
        thr = np.asarray(d["threshold_values"], dtype=np.float64)
        side = "left" if d["kind"] == 0 else "right"
        p["data"][d["relation"]][d["name"]] = np.searchsorted(thr, x, side=side).astype(np.int32)
        rel["attrs"].append({"name": d["name"], "dtype": "i32", "domain": len(thr) + 1, "key": False})
    return p


def domains(problem):
    out = {}
    for r in problem["schema"]:
        for a in r["attrs"]:
            if a["dtype"] == "i32" and a["domain"]:
                out[a["name"]] = int(a["domain"])
    return out


def check_views(E, problem, tol, name, **kw):
    print(f"[case] views {name} {kw}", flush=True)
    plan = E.Plan(problem, **kw)
    prep = E.Prepared(plan, E.device_columns(problem))
    prep.run(sync=True)
    desc = plan.describe()
    p = with_derived(problem, desc)
    dom = domains(p)
    worst = 0.0
    assert desc["views"], f"{name}: plan has no views"
    for v in desc["views"]:
        got = prep.view(v["id"])
        key = v["key"]
        n_keys = int(np.prod([dom[k] for k in key]))
        assert got["count"].shape == (n_keys,) == (v["n_keys"],)
        present = np.nonzero(got["count"])[0]
        # dense index -> key tuple, last key attribute fastest
        keys = np.zeros((len(present), len(key)), dtype=np.int64)
        rem = present.copy()
        for j in range(len(key) - 1, -1, -1):
            keys[:, j] = rem % dom[key[j]]
            rem //= dom[key[j]]
        aggs = [[(a, 1) for a in m.split("*")] for m in v["stored_values"]]
        where = [(c[0], OPS[c[1]], c[2]) for c in v["conditions"]]
        ref = oracle.evaluate_view(p, v["from"], v["to"], key, aggs, carried=v["stored_codes"],
                                   where=where)
        gpu = {"keys": keys, "count": got["count"][present], "sum": got["values"][present]}
        where_s = f"{name} view {v['id']} {v['from']}->{v['to']}"
        worst = max(worst, compare(gpu, ref, tol, where_s))
        if v["stored_codes"]:
            np.testing.assert_array_equal(got["codes"][present].astype(np.int64), ref["codes"],
                                          err_msg=f"{where_s}: carried codes")
    print(f"[case] views {name}: {len(desc['views'])} views, worst scaled error {worst:.2e}", flush=True)
    return desc


def test_views_tiny_star(eng):
    check_views(eng, W.tiny_star(seed=0, n_fact=30_000), 1e-12, "tiny_star", precision="f64", policy="fact")


@pytest.mark.parametrize("policy", ["groupby", "fact"])
def test_views_worked_example(eng, policy):
    d = check_views(eng, W.favorita_example(0, n_sales=400), 1e-12, "favorita", precision="f64", policy=policy,
                    row_piece_max=-1, min_segment=1)
    if policy == "groupby":
        assert len(d["views"]) == 6


def test_views_retail_small(eng):
    p = W.retail_snowflake(seed=2, n_inv=300_000)
    check_views(eng, p, 1e-5, "retail", precision="f32", policy="fact")


def test_views_tagged_star_many_to_many(eng):
    check_views(eng, W.tagged_star(seed=1, n_fact=100_000), 1e-12, "tagged_star", precision="f64", policy="fact",
                row_piece_max=-1)


@pytest.mark.parametrize("seed", [41, 69, 79, 82])
def test_views_random_many_to_many(eng, seed):
    # seeds whose batch the groupby root policy plans (others carry a group-by
    # attribute through a many-to-many view, which the planner rejects)
    p = W.random_acyclic(seed, n_rel=4, max_rows=400, max_dom=20)
    check_views(eng, p, 1e-12, f"random_{seed}", precision="f64", policy="groupby", row_piece_max=-1,
                min_segment=1)


def test_views_cart_node_with_conditions(eng):
    p = W.cart_node(seed=1, n_inv=200_000)
    d = check_views(eng, p, 1e-5, "cart_node", precision="f32", policy="fact")
    assert any(v["conditions"] for v in d["views"]) or d["derived"]


def test_views_rkmeans_chain(eng):
    p = W.rkmeans_chain(seed=3, n1=200_000, n2=20_000, n3=2_000, max_dom=5_000)
    check_views(eng, p, 1e-5, "chain", precision="f32", policy="fact")
