"""Host-only tests of the planner through the C ABI (no GPU needed).

Structural pins from the paper's worked example (section 2, Figure 2 and
Figure 3): with Sales and Items as roots the batch decomposes into exactly the
six directional views V_{T->S}, V_{R->T}, V_{O->T}, V_{H->S}, V_{I->S},
V_{S->I}; the views and queries fall into seven groups whose dependency graph
has the edges G1->G5, G2->G5, G5->G6, G3->G6, G4->G6, G6->G7; with the
attribute order item < date < store at Sales, V_{I->S} is looked up at the
item level, V_{H->S} at the date level and V_{T->S} at the store level.
"""
import json

import numpy as np
import pytest

import workloads as W

E = pytest.importorskip("paper_2008_08657_amd")


def plan(problem, **kw):
    return E.Plan(problem, **kw).describe()


def views_by_edge(d):
    return {(v["from"], v["to"]): v for v in d["views"]}


def test_worked_example_views_and_groups():
    p = W.favorita_example()
    d = plan(p, policy="groupby")
    # roots of the example: Q1, Q2 at Sales, Q3 at Items
    assert [q["root"] for q in d["queries"]] == ["Sales", "Sales", "Items"]
    edges = set(views_by_edge(d))
    assert edges == {("Transactions", "Sales"), ("StoRes", "Transactions"), ("Oil", "Transactions"),
                     ("Holidays", "Sales"), ("Items", "Sales"), ("Sales", "Items")}
    assert len(d["views"]) == 6
    groups = d["groups"]
    assert len(groups) == 7

    def gid(node, kind, target=None):
        for g in groups:
            if g["node"] != node:
                continue
            for o in g["outputs"]:
                if o["kind"] == "view" and kind == "view":
                    v = d["views"][o["id"]]
                    if v["to"] == target:
                        return g["id"]
                if o["kind"] == "query" and kind == "query":
                    return g["id"]
        raise KeyError((node, kind, target))

    g1 = gid("StoRes", "view", "Transactions")
    g2 = gid("Oil", "view", "Transactions")
    g3 = gid("Holidays", "view", "Sales")
    g4 = gid("Items", "view", "Sales")
    g5 = gid("Transactions", "view", "Sales")
    g6 = gid("Sales", "query")
    g7 = gid("Items", "query")
    assert g4 != g7
    # group 6 holds Q1, Q2 and V_{S->I}
    out6 = groups[g6]["outputs"]
    assert sorted(o["kind"] for o in out6) == ["query", "query", "view"]
    dag = {(dep, g["id"]) for g in groups for dep in g["deps"]}
    assert dag == {(g1, g5), (g2, g5), (g5, g6), (g3, g6), (g4, g6), (g6, g7)}


def test_worked_example_merged_components():
    d = plan(W.favorita_example(), policy="groupby")
    v = views_by_edge(d)
    # V_{T->S} serves Q2 (h from Oil) and Q3 (price from Oil): one view, two components
    assert sorted(v[("Transactions", "Sales")]["components"]) == ["h", "price"]
    assert v[("Sales", "Items")]["components"] == ["units*price"]
    assert v[("Items", "Sales")]["components"] == ["g"]


def test_worked_example_attribute_order_levels():
    p = W.favorita_example()
    d = plan(p, policy="groupby", order={"Sales": ["item", "date", "store"]},
             row_piece_max=-1, min_segment=1)
    sales = [g for g in d["groups"] if g["node"] == "Sales"][0]
    assert d["relations"][0]["order"] == ["item", "date", "store"]
    lv = {}
    for pv in sales["program"]["views"]:
        v = d["views"][pv["view"]]
        lv[v["from"]] = pv["level"]
    # looked up once per item, per date, per (date, store) respectively
    assert lv == {"Items": 1, "Holidays": 2, "Transactions": 3}


def test_fact_policy_roots_group_by_at_fact():
    d = plan(W.favorita_example(), policy="fact")
    # class is reached from Sales through the Items key, so Q3 stays at Sales
    assert [q["root"] for q in d["queries"]] == ["Sales", "Sales", "Sales"]


def test_root_override():
    p = W.favorita_example()
    p["batch"][0] = dict(p["batch"][0], root="Transactions")
    d = plan(p, policy="groupby")
    assert d["queries"][0]["root"] == "Transactions"


def test_retail_plan_shape():
    p = W.retail_snowflake(n_inv=1000)
    for r in p["schema"]:
        if r["name"] == "Inv":
            r["n_rows"] = 84_000_000
    d = plan(p, precision="f32", policy="fact")
    assert len(d["queries"]) == 1269
    v = views_by_edge(d)
    assert v[("Items", "Inv")]["unique"] and v[("Weather", "Inv")]["unique"]
    assert v[("Stores", "Inv")]["unique"] and v[("Demog", "Stores")]["unique"]
    assert not v[("Inv", "Items")]["unique"]
    inv = [g for g in d["groups"] if g["node"] == "Inv" and "program" in g]
    assert len(inv) == 1, "the fact relation is scanned once"
    prog = inv[0]["program"]
    assert prog["cut"] == 2 and not prog["row_pieces"]
    assert d["relations"][0]["order"] == ["locn", "date", "ksn"]
    outer = {d["views"][x["view"]]["from"]: x["outer"] for x in prog["views"]}
    assert outer == {"Weather": True, "Stores": True, "Items": False}


def test_rk_means_step1_batch_is_n_queries():
    # step 1 of Rk-means: one SUM(1) GROUP BY X_j query per attribute
    p = W.tiny_star(n_fact=100)
    attrs = ["store", "item", "cat"]
    p["batch"] = [{"groupby": [a], "where": [], "aggs": [[]], "root": None} for a in attrs]
    d = plan(p, policy="groupby")
    assert len(d["queries"]) == len(attrs)


def test_partition_count_takes_tables_weighted_by_count_views():
    # SUM(1) grouped by attributes of R2 (or R3) is rooted there; the view
    # from R1 into R2 holds several R1 tuples per key b, and its count weights
    # each R2 row: such tables are counted by partition at R2 and R3 (section
    # 3, Rk-means step 1), not by per-row atomics in a scan
    p = W.rkmeans_chain(seed=12, n1=400_000, n2=6_000, n3=500, n_x=4, n_y=6, n_z=6, max_dom=1_000_000)
    d = plan(p, precision="f32", policy="fact")
    assert {g["node"] for g in d["groups"] if g.get("partitioned")} >= {"R1", "R2", "R3"}
    assert {q["root"] for q in d["queries"]} == {"R1", "R2", "R3"}


@pytest.mark.parametrize("mutate, status", [
    (lambda p: p.update(tree=[(0, 1)]), "EINVAL"),                                   # not connected
    (lambda p: p.update(tree=[(0, 1), (0, 2), (1, 2)]), "EINVAL"),                   # cycle
    (lambda p: p["batch"].append({"groupby": [], "where": [], "aggs": [[("nope", 1)]], "root": None}), "EINVAL"),
    (lambda p: p["batch"].append({"groupby": [], "where": [], "aggs": [[("units", 2), ("f1", 1)]], "root": None}),
     "EUNSUPPORTED"),                                                                # degree 3
    (lambda p: p["batch"].append({"groupby": ["store", "item", "cat"], "where": [], "aggs": [[]], "root": None}),
     "EUNSUPPORTED"),                                                                # 3 group-bys
    (lambda p: p["batch"].append({"groupby": ["units"], "where": [], "aggs": [[]], "root": None}),
     "EUNSUPPORTED"),                                                                # float group-by
])
def test_validation_errors(mutate, status):
    p = W.tiny_star(n_fact=100)
    mutate(p)
    with pytest.raises(E.LmfaoError) as ei:
        E.Plan(p, policy="fact")
    assert str(ei.value).startswith(status)


def test_running_intersection_violation():
    p = W.tiny_star(n_fact=100)
    # give Stores an attribute 'cat' too: Items and Stores are not adjacent
    p["schema"][1]["attrs"].append({"name": "cat", "dtype": "i32", "domain": 20, "key": False})
    with pytest.raises(E.LmfaoError) as ei:
        E.Plan(p, policy="fact")
    assert "running-intersection" in str(ei.value)


def test_plan_json_roundtrip():
    d = plan(W.tiny_star(n_fact=100), policy="fact")
    assert json.loads(json.dumps(d)) == d
    assert d["supported"] is True


def _cart_small(**kw):
    return W.cart_node(seed=0, n_inv=2_000, n_locn=12, n_dates=6, n_ksn=50, n_weather_dates=8, **kw)


def test_cart_candidates_become_bucket_group_bys():
    p = _cart_small()
    d = plan(p, precision="f32", policy="fact")
    # the node condition is the batch-wide filter
    assert sorted(c[0] for c in d["filter"]) == sorted(c[0] for c in p["node"])
    # one derived bucket attribute per thresholded feature, in its owner relation
    assert len(d["derived"]) == 42
    owner = {a["name"]: r["name"] for r in p["schema"] for a in r["attrs"]}
    for x in d["derived"]:
        assert x["kind"] == 0 and x["thresholds"] <= 20 and x["relation"] == owner[x["source"]]
    uq = d["user_queries"]
    assert len(uq) == len(p["batch"]) == 2544
    # X <= t_k selects buckets [0, k]: ranges of one feature's thresholds are nested
    first = [u for u, q in zip(uq, p["batch"]) if len(q["where"]) > len(p["node"])
             and q["where"][-1][0] == "i1" and q["aggs"] == [[]]]
    his = [u["hi"] for u in first]
    assert all(u["lo"] == 0 for u in first) and his == sorted(his)
    # one planned query per (feature, statistic), shared by all its thresholds
    assert len({u["planned"] for u in first}) == 1


def test_condition_rewrite_ops():
    p = W.tiny_star(n_fact=100)
    base = {"groupby": [], "aggs": [[("units", 1)]], "root": None}
    p["batch"] = [dict(base, where=[("f1", op, 0.25)]) for op in ("<=", "<", ">", ">=")]
    p["batch"] += [dict(base, where=[("cat", op, 3)]) for op in ("==", "!=")]
    d = plan(p, policy="fact")
    uq = d["user_queries"]
    assert [u["lo"] for u in uq[:4]] == [0, 0, 1, 1] and [u["hi"] for u in uq[:4]] == [1, 1, 2, 2]
    assert (uq[4]["lo"], uq[4]["hi"], uq[4]["except"]) == (3, 4, -1)
    assert (uq[5]["lo"], uq[5]["hi"], uq[5]["except"]) == (0, 20, 3)
    assert sorted(x["kind"] for x in d["derived"]) == [0, 1]
    assert d["filter"] == []


def test_two_private_conditions_are_unsupported():
    p = W.tiny_star(n_fact=100)
    p["batch"] = [{"groupby": [], "aggs": [[]], "root": None, "where": [("f1", "<=", 0.0), ("g1", ">", 0.0)]},
                  {"groupby": [], "aggs": [[]], "root": None, "where": []}]
    with pytest.raises(E.LmfaoError) as ei:
        E.Plan(p, policy="fact")
    assert str(ei.value).startswith("EUNSUPPORTED")


def test_per_view_form_has_one_output_per_group():
    p = W.favorita_example()
    fused = plan(p, policy="groupby")
    solo = plan(p, policy="groupby", form="per_view")
    assert len(fused["groups"]) == 7
    assert all(len(g["outputs"]) == 1 for g in solo["groups"])
    n_out = len(solo["views"]) + len(solo["queries"])
    assert len(solo["groups"]) == n_out == 9


def test_wide_chain_groups_are_split_to_fit_the_kernels():
    # Rk-means step 1 at full size: 40 + 30 + 30 attributes grouped one by one
    # and in pairs; the planner halves groups whose scan would exceed one
    # kernel's columns or histograms, moves hashed outputs and outputs with no
    # scan form (an inner and a large outer key) to groups evaluated row by row
    p = W.rkmeans_chain(seed=0, n1=2000, n2=200, n3=20)
    for r, n in zip(p["schema"], (50_000_000, 5_000_000, 200_000)):
        r["n_rows"] = n
    d = E.Plan(p, precision="f32", policy="fact").describe()
    outs = [o for g in d["groups"] for o in g["outputs"]]
    queries = sorted(o["id"] for o in outs if o["kind"] == "query")
    assert queries == list(range(len(p["batch"])))
    by_rel = {}
    for g in d["groups"]:
        by_rel.setdefault(g["node"], []).append(g)
    assert len(by_rel["R1"]) > 2
    # SUM(1) group-bys whose table a scan cannot keep in LDS (dense past 12k
    # cells, hashed, or past what the scan's other tables leave of its LDS
    # budget) are counted by radix partition, in groups of their own
    part = [o["id"] for g in by_rel["R1"] if g.get("partitioned") for o in g["outputs"]]
    doms = p["domains"]
    cells_of = {}
    for qi, q in enumerate(p["batch"]):
        cells_of[qi] = int(np.prod([doms[a] for a in q["groupby"]])) if q["groupby"] else 0
    eligible_large = {qi for qi, q in enumerate(p["batch"])
                      if cells_of[qi] > 12288 and all(not f for f in q["aggs"]) and
                      all(a.startswith("x") or a == "b" for a in q["groupby"])}
    assert eligible_large <= set(part)
    for qi in part:
        assert all(not f for f in p["batch"][qi]["aggs"])
        assert cells_of[qi] > 12288 or len(p["batch"][qi]["groupby"]) == 1
    assert any(len(p["batch"][qi]["groupby"]) == 2 and
               doms[p["batch"][qi]["groupby"][0]] * doms[p["batch"][qi]["groupby"][1]] > 1 << 24 for qi in part)
    for g in d["groups"]:
        prog = g.get("program") or {}
        assert len(prog.get("scan_cols", [])) <= 16
    # without partitioning, hashed outputs are evaluated row by row
    d = E.Plan(p, precision="f32", policy="fact", partition=False).describe()
    r1 = [g for g in d["groups"] if g["node"] == "R1"]
    assert not any(g.get("partitioned") for g in d["groups"])
    assert any((g.get("program") or {}).get("row_pieces") for g in r1)


@pytest.mark.parametrize("kw", [{"scan_blocks": -1}, {"contract_splits": -4}])
def test_negative_launch_options_are_rejected(kw):
    with pytest.raises(E.LmfaoError) as ei:
        E.Plan(W.tiny_star(n_fact=100), policy="fact", **kw)
    assert str(ei.value).startswith("EINVAL")


@pytest.mark.parametrize("which", ["tiny", "grocery", "chain", "random8", "random9"])
def test_root_cost_policy_never_costs_more_than_its_start(which):
    # the search starts at the FACT roots and accepts only moves that lower
    # the modelled bytes; a plan outside the supported class falls back to
    # FACT (equal cost)
    p = {"tiny": lambda: W.tiny_star(seed=0, n_fact=100_000),
         "grocery": lambda: W.grocery_star(seed=0, n_sales=500_000),
         "chain": lambda: W.rkmeans_chain(seed=0, n1=200_000, n2=20_000, n3=1_000),
         "random8": lambda: W.random_acyclic(8), "random9": lambda: W.random_acyclic(9)}[which]()
    fact = E.Plan(p, precision="f32", policy="fact").describe()
    cost = E.Plan(p, precision="f32", policy="cost").describe()
    assert cost["root_cost_bytes"] <= fact["root_cost_bytes"] * (1 + 1e-12)
    assert len(cost["queries"]) == len(fact["queries"])


def test_root_cost_policy_shares_the_fact_scan_on_the_tiny_star():
    # every query of the tiny star can read the fact relation S once; the
    # dimension roots of FACT cost a pass over each dimension and more views
    p = W.tiny_star(seed=0, n_fact=100_000)
    d = E.Plan(p, precision="f64", policy="cost").describe()
    assert {q["root"] for q in d["queries"]} == {"S"}
    assert len(d["views"]) == 2
