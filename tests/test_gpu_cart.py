"""Regression-tree growth by CART on the GPU (section 3 of the paper,
decision trees) against the oracle's tree (``oracle/cart.py``).

Every node of a depth-3 tree over a small retail-shaped snowflake: the node
batch is planned and prepared once; each node's path condition is written
into the row weights of the relations holding its attributes and the batch
is replayed from the captured HIP graph; the split is chosen on the GPU
(``lmfao_cart_grow``).  Splits, node sizes and (FP64) node sums and costs
must match the oracle, which materialises the join and grows the tree from
the plain definition with the same tie rule.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _oracle_tree(p, depth, min_leaf, tie_eps):
    import oracle.cart as cart
    cands = [(c["attr"], 0 if c["op"] == "<=" else 1, c["value"]) for c in p["cart"]["candidates"]]
    return cart.grow_tree(p, p["label"], cands, max_depth=depth, min_leaf=min_leaf, tie_eps=tie_eps)


def _grow(p, depth, min_leaf, tie_eps, precision="f64", graph=True):
    import paper_2008_08657_amd as E
    plan = E.Plan(p, precision=precision, policy="fact", row_weights=p["row_weights"], graph=graph)
    cols = E.device_columns(p)
    prep = E.Prepared(plan, cols)
    spec = dict(p["cart"], max_depth=depth, min_leaf=min_leaf, tie_eps=tie_eps)
    nodes = prep.cart_grow(spec, cols)
    return nodes, prep, plan, cols


@pytest.mark.parametrize("graph", [True, False])
def test_tree_matches_oracle(graph):
    import torch
    assert torch.cuda.is_available()
    p = W.cart_tree(seed=0, n_inv=200_000)
    depth, min_leaf, eps = 3, 50, 1e-9
    print(f"[cart] {len(p['cart']['candidates'])} candidates, {len(p['batch'])} queries, graph={graph}", flush=True)
    got, prep, plan, cols = _grow(p, depth, min_leaf, eps, graph=graph)
    want = _oracle_tree(p, depth, min_leaf, eps)
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        where = f"node {i} (depth {w['depth']})"
        assert (g["parent"], g["depth"], g["split"], g["left"], g["right"]) == \
            (w["parent"], w["depth"], w["split"], w["left"], w["right"]), where
        assert g["n"] == w["n"], where
        scale = max(1.0, abs(w["sum_y2"]))
        assert abs(g["sum_y"] - w["sum_y"]) <= 1e-9 * scale, where
        assert abs(g["sum_y2"] - w["sum_y2"]) <= 1e-9 * scale, where
        assert abs(g["cost"] - w["cost"]) <= 1e-9 * scale, where
    assert sum(1 for g in got if g["split"] >= 0) >= 3
    assert sum(g["n"] for g in got if g["split"] < 0) == 200_000


def test_best_split_and_costs_of_the_root_batch():
    import torch
    import oracle.cart as cart
    import oracle
    import paper_2008_08657_amd as E
    p = W.cart_tree(seed=1, n_inv=120_000, n_thr=6)
    plan = E.Plan(p, precision="f64", policy="fact", row_weights=p["row_weights"])
    cols = E.device_columns(p)
    prep = E.Prepared(plan, cols)
    prep.run(sync=True)
    n_c = len(p["cart"]["candidates"])
    costs = torch.empty(n_c, dtype=torch.float64, device="cuda")
    spec = dict(p["cart"], min_leaf=10, tie_eps=1e-9)
    got = prep.cart_best_split(spec, costs)
    cands = [(c["attr"], 0 if c["op"] == "<=" else 1, c["value"]) for c in p["cart"]["candidates"]]
    D = oracle.materialize_join(p, sorted({c[0] for c in cands} | {p["label"]}))
    mask = np.ones(len(D[p["label"]]), dtype=bool)
    ref = cart.split_costs(D, p["label"], mask, cands, 10)
    n, sy, sy2 = cart.node_stats(D, p["label"], mask)
    assert got["n"] == n == 120_000
    c = costs.cpu().numpy()
    for i, (cost, nl, nr, ok) in enumerate(ref):
        if ok:
            assert abs(c[i] - cost) <= 1e-9 * max(1.0, sy2), i
        else:
            assert np.isinf(c[i]), i
    assert got["best"] == cart.best_split(ref, cart.var_term(n, sy, sy2), 1e-9)
