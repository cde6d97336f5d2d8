"""Pins of the CART oracle (``oracle/cart.py``) against what the definition
and the mathematics fix, on materialised joins of tiny inputs (section 3 of
the paper, decision trees):

* VAR from the aggregates equals numpy's two-pass population variance times
  the fragment size;
* the chosen split equals a brute-force search that partitions the tuples
  with Python's own comparisons and scores each side with ``numpy.var``;
* a response that is exactly an indicator of one threshold is split there at
  cost 0 (closed form);
* children partition their parent, and the leaves partition D;
* a planted mistake (the complement of ``x <= t`` taken as ``x >= t``) fails
  the brute-force pin.
"""
import numpy as np
import pytest

import oracle
import oracle.cart as cart
import workloads as W


def _problem(n=400, seed=3):
    p = W.tiny_star(seed=seed, n_fact=n, n_stores=6, n_items=30)
    return p


def _candidates(p, n_thr=4):
    owner = {a["name"]: r["name"] for r in p["schema"] for a in r["attrs"]}
    cands = []
    for x in ("f1", "g1", "g2"):
        for t in W.quantile_thresholds(p["data"][owner[x]][x], n_thr):
            cands.append((x, 0, t))
    for v in range(20):
        cands.append(("cat", 1, v))
    return cands


def _brute_force(p, y, cands, path, min_leaf, tie_eps):
    """Partitions the node's tuples with scalar comparisons and scores each
    candidate with numpy's variance; same selection rule as the oracle."""
    D = oracle.materialize_join(p)
    n = len(D[y])
    rows = []
    for i in range(n):
        ok = True
        for k, holds in path:
            attr, kind, value = cands[k]
            v = D[attr][i]
            c = (v <= value) if kind == 0 else (v == value)
            ok = ok and (c if holds else not c)
        if ok:
            rows.append(i)
    yy = np.asarray(D[y], dtype=np.float64)
    node_y = yy[rows]
    node_var = float(np.var(node_y) * len(node_y)) if len(node_y) else 0.0
    costs = []
    for attr, kind, value in cands:
        left, right = [], []
        for i in rows:
            v = D[attr][i]
            c = (v <= value) if kind == 0 else (v == value)
            (left if c else right).append(yy[i])
        cl = float(np.var(left) * len(left)) if left else 0.0
        cr = float(np.var(right) * len(right)) if right else 0.0
        costs.append((cl + cr, len(left), len(right), len(left) >= min_leaf and len(right) >= min_leaf))
    return costs, node_var


def test_var_from_aggregates_equals_numpy_variance():
    p = _problem()
    D = oracle.materialize_join(p)
    y = np.asarray(D["units"], dtype=np.float64)
    rng = np.random.default_rng(0)
    for _ in range(5):
        mask = rng.random(len(y)) < rng.uniform(0.1, 0.9)
        n, sy, sy2 = cart.node_stats(D, "units", mask)
        assert n == int(mask.sum())
        ref = float(np.var(y[mask]) * mask.sum())
        assert abs(cart.var_term(n, sy, sy2) - ref) <= 1e-9 * max(1.0, abs(ref))
    assert cart.var_term(0, 0.0, 0.0) == 0.0


@pytest.mark.parametrize("min_leaf", [1, 40])
def test_root_and_child_splits_match_brute_force(min_leaf):
    p = _problem()
    cands = _candidates(p)
    nodes = cart.grow_tree(p, "units", cands, max_depth=2, min_leaf=min_leaf)
    assert nodes[0]["split"] >= 0
    checked = 0
    for nd in nodes:
        if nd["split"] < 0:
            continue
        costs, node_var = _brute_force(p, "units", cands, nd["path"], min_leaf, 1e-9)
        want = cart.best_split(costs, node_var, 1e-9)
        assert _matches(nodes, nd, costs, want, node_var)
        checked += 1
    assert checked >= 2


def _matches(nodes, nd, costs, want, node_var):
    """The oracle's split of node nd is the brute-force choice, with its cost
    and both children's sizes."""
    return (nd["split"] == want and abs(nd["cost"] - costs[want][0]) <= 1e-9 * max(1.0, node_var)
            and nodes[nd["left"]]["n"] == costs[want][1] and nodes[nd["right"]]["n"] == costs[want][2])


def test_indicator_response_is_split_at_its_threshold_with_zero_cost():
    p = _problem(n=300, seed=5)
    owner = {a["name"]: r["name"] for r in p["schema"] for a in r["attrs"]}
    g1 = p["data"][owner["g1"]]["g1"]
    t0 = float(np.median(g1))
    # y = 1 where the tuple's item has g1 <= t0, else 0, stored on the fact
    items = p["data"]["S"]["item"]
    p["data"]["S"]["units"] = (g1[items] <= t0).astype(np.float64)
    cands = [("g1", 0, t) for t in sorted({t0, float(np.min(g1)), float(np.max(g1))})] + [("f1", 0, 0.0)]
    nodes = cart.grow_tree(p, "units", cands, max_depth=1, min_leaf=1)
    k = nodes[0]["split"]
    assert cands[k] == ("g1", 0, t0)
    assert abs(nodes[0]["cost"]) <= 1e-12


def test_children_partition_the_parent_and_leaves_partition_D():
    p = _problem(n=500, seed=7)
    nodes = cart.grow_tree(p, "units", _candidates(p), max_depth=3, min_leaf=5)
    for nd in nodes:
        if nd["split"] >= 0:
            L, R = nodes[nd["left"]], nodes[nd["right"]]
            assert L["n"] + R["n"] == nd["n"]
            assert abs(L["sum_y"] + R["sum_y"] - nd["sum_y"]) <= 1e-9 * max(1.0, abs(nd["sum_y"]))
    assert sum(nd["n"] for nd in nodes if nd["split"] < 0) == 500


def test_planted_complement_mistake_fails_the_brute_force_pin(monkeypatch):
    p = _problem()
    cands = _candidates(p)
    # ties on the threshold values exist in the data (thresholds are data values)
    real = cart._holds

    def wrong(col, kind, value, negate):
        if negate and kind == 0:
            return col >= value   # the complement of <= taken as >=
        return real(col, kind, value, negate)

    monkeypatch.setattr(cart, "_holds", wrong)
    nodes = cart.grow_tree(p, "units", cands, max_depth=2, min_leaf=1)
    caught = False
    for nd in nodes:
        if nd["split"] < 0:
            continue
        costs, node_var = _brute_force(p, "units", cands, nd["path"], 1, 1e-9)
        caught |= not _matches(nodes, nd, costs, cart.best_split(costs, node_var, 1e-9), node_var)
    assert caught
