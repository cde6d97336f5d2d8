"""Pins of the CPU oracle against things other than itself.

Each pin is chosen so that a plausible mistake in the oracle (a dropped join
multiplicity, a wrong power, a group-key mix-up, a lost dangling tuple, an
operand swap) fails at least one of them:

* brute force: every combination of one tuple per relation is enumerated in
  plain Python, kept iff all equally named attributes agree (the definition of
  the natural join), and summed with ``math.fsum``;
* closed forms: COUNT of a complete foreign-key star equals the fact size;
* library special cases: a single relation's covariance batch equals ``X^T X``
  (numpy matmul), a group-by on a key equals ``numpy.bincount``, a foreign-key
  two-relation join equals fancy indexing;
* invariants: group marginals add up to the ungrouped aggregate, SUM(a*b)
  equals SUM(b*a); a view's counts times the opposite view's counts, summed
  over the edge key, give |D| (a join tree factorises COUNT at every edge).

Conditions in the brute force are evaluated with Python's own scalar
comparison operators (``operator.le`` and so on), never with the oracle's
``OPS`` table, and a float32 column compares against the constant rounded to
float32 (the oracle's stated reading).

The planted-mistake tests at the end patch the oracle on the CPU and check that
the pins notice.
"""
import itertools
import math
import operator

import numpy as np
import pytest

import oracle
import workloads as W


PY_OPS = {"<=": operator.le, "<": operator.lt, ">": operator.gt, ">=": operator.ge,
          "==": operator.eq, "!=": operator.ne}


def _py_const(problem, attr, c):
    """The constant as the brute force compares it: rounded to float32 for a
    float32 column, else a Python float / int."""
    for r in problem["schema"]:
        for a in r["attrs"]:
            if a["name"] == attr and a["dtype"] == "f32":
                return float(np.float32(c))
    return c


def brute_force(problem, qi=None, rels=None, query=None):
    """Reference by enumeration: sum over all tuple combinations (of the
    relations named in ``rels``, default all) that agree on every shared
    attribute name."""
    rels = [r for r in problem["schema"] if rels is None or r["name"] in rels]
    data = problem["data"]
    q = problem["batch"][qi] if query is None else query
    where = [(a, PY_OPS[op], _py_const(problem, a, c)) for a, op, c in q.get("where", [])]
    groups = {}
    ranges = [range(r["n_rows"]) for r in rels]
    for combo in itertools.product(*ranges):
        tup = {}
        ok = True
        for r, i in zip(rels, combo):
            for a in r["attrs"]:
                v = data[r["name"]][a["name"]][i]
                v = int(v) if a["dtype"] == "i32" else float(v)
                if a["name"] in tup and tup[a["name"]] != v:
                    ok = False
                    break
                tup[a["name"]] = v
            if not ok:
                break
        if not ok:
            continue
        if not all(cmp(tup[a], c) for a, cmp, c in where):
            continue
        g = tuple(tup[a] for a in q.get("groupby", []))
        slot = groups.setdefault(g, [0, [[] for _ in q["aggs"]]])
        slot[0] += 1
        funcs = problem.get("functions", {})
        for k, factors in enumerate(q["aggs"]):
            t = 1.0
            for a, p in factors:
                # a user-defined factor: its table at the tuple's argument value
                v = float(funcs[a]["values"][tup[funcs[a]["attr"]]]) if a in funcs else tup[a]
                t *= v ** p
            slot[1][k].append(t)
    keys = sorted(groups)
    return keys, [groups[k][0] for k in keys], [[math.fsum(v) for v in groups[k][1]] for k in keys]


def assert_matches_brute(problem):
    res = oracle.evaluate(problem)
    for qi, r in enumerate(res):
        keys, counts, sums = brute_force(problem, qi)
        assert [tuple(int(x) for x in k) for k in r["keys"]] == keys
        assert list(r["count"]) == counts
        if keys:
            np.testing.assert_allclose(r["sum"], np.array(sums), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random_many_to_many(seed):
    p = W.random_acyclic(seed, n_rel=3 + seed % 2, max_rows=5, max_dom=3)
    assert_matches_brute(p)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_random_foreign_keys(seed):
    p = W.random_acyclic(100 + seed, n_rel=4, max_rows=6, max_dom=4, unique_dims=True)
    assert_matches_brute(p)


def test_brute_force_with_predicates():
    p = W.random_acyclic(7, n_rel=3, max_rows=6, max_dom=3)
    p["batch"] = [dict(q, where=[("x0", "<=", 0.1), ("c1", "!=", 1)]) for q in p["batch"]]
    assert_matches_brute(p)


def _operator_problem(seed):
    """A random join whose batch exercises all six comparison operators, on a
    float and an integer attribute, with constants equal to values the data
    holds (so that < and <=, > and >= select different tuples)."""
    p = W.random_acyclic(seed, n_rel=3, max_rows=6, max_dom=3)
    x0 = p["data"]["R0"]["x0"]
    c1 = p["data"]["R1"]["c1"]
    tx = float(np.sort(x0)[len(x0) // 2])
    tc = int(c1[0])
    batch = []
    for op in ("<=", "<", ">", ">=", "==", "!="):
        for q in p["batch"][:2]:
            batch.append(dict(q, where=[("x0", op, tx)]))
            batch.append(dict(q, where=[("c1", op, tc)]))
    p["batch"] = batch
    return p


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_all_comparison_operators(seed):
    assert_matches_brute(_operator_problem(seed))


def test_float32_condition_compares_in_float32():
    # a constant between two float32 neighbours: in float32 it rounds onto the
    # data value, in float64 it lies above it
    v = np.float32(0.1)
    c = float(v) + 1e-12
    schema = [{"name": "R", "n_rows": 3, "attrs": [
        {"name": "x", "dtype": "f32", "domain": 0, "key": False}]}]
    data = {"R": {"x": np.array([v, np.float32(0.5), np.float32(-1)], dtype=np.float32)}}
    batch = [{"groupby": [], "where": [("x", "<", c)], "aggs": [[]], "root": None},
             {"groupby": [], "where": [("x", "==", c)], "aggs": [[]], "root": None}]
    p = {"schema": schema, "tree": [], "batch": batch, "data": data}
    res = oracle.evaluate(p)
    assert res[0]["count"].tolist() == [1]      # only -1 < 0.1f
    assert res[1]["count"].tolist() == [1]      # 0.1f == round_f32(c)
    assert_matches_brute(p)


def test_brute_force_worked_example_schema():
    # the worked example's six-relation schema (Sales, Holidays, StoRes, Items,
    # Transactions, Oil) with its three queries, on a tiny instance
    p = W.favorita_example(0, n_sales=12)
    # shrink the dimension grid so brute force stays small
    assert_matches_brute(p)


def test_count_equals_fact_size_closed_form():
    p = W.tiny_star(seed=3, n_fact=5_000, n_stores=7, n_items=40)
    r = oracle.evaluate(p, queries=[0])[0]
    assert p["batch"][0]["aggs"] == [[]]  # SUM(1) is the first query
    assert r["count"].tolist() == [5_000]
    assert r["sum"][0, 0] == 5_000.0


def test_single_relation_is_xtx():
    rng = np.random.default_rng(5)
    n = 300
    X = rng.standard_normal((n, 4))
    schema = [{"name": "R", "n_rows": n, "attrs": [
        {"name": f"x{j}", "dtype": "f64", "domain": 0, "key": False} for j in range(4)]}]
    data = {"R": {f"x{j}": X[:, j] for j in range(4)}}
    batch = W.covariance_batch([f"x{j}" for j in range(4)], (), split=False)
    p = {"schema": schema, "tree": [], "batch": batch, "data": data}
    r = oracle.evaluate(p)[0]
    Xe = np.concatenate([np.ones((n, 1)), X], axis=1)
    sigma = Xe.T @ Xe
    want = [sigma[j, k] for j in range(5) for k in range(j, 5)]
    np.testing.assert_allclose(r["sum"][0], want, rtol=1e-12, atol=1e-10)


def test_groupby_key_is_bincount():
    p = W.tiny_star(seed=1, n_fact=3_000, n_stores=9, n_items=30)
    p["batch"] = [{"groupby": ["store"], "where": [], "aggs": [[], [("units", 1)]], "root": None}]
    r = oracle.evaluate(p)[0]
    s = p["data"]["S"]
    cnt = np.bincount(s["store"], minlength=9)
    present = np.nonzero(cnt)[0]
    assert r["keys"][:, 0].tolist() == present.tolist()
    assert r["count"].tolist() == cnt[present].tolist()
    np.testing.assert_allclose(r["sum"][:, 1], np.bincount(s["store"], s["units"], 9)[present],
                               rtol=1e-12)


def test_fk_join_is_fancy_indexing():
    p = W.tiny_star(seed=2, n_fact=2_000, n_stores=6, n_items=25)
    p["batch"] = [{"groupby": [], "where": [], "root": None,
                   "aggs": [[("units", 1), ("g2", 1)], [("f1", 1), ("g3", 1)], [("g1", 2)]]}]
    r = oracle.evaluate(p)[0]
    s, st, it = p["data"]["S"], p["data"]["Stores"], p["data"]["Items"]
    g1, g2, g3 = (it[k][s["item"]] for k in ("g1", "g2", "g3"))
    f1 = st["f1"][s["store"]]
    want = [np.sum(s["units"] * g2), np.sum(f1 * g3), np.sum(g1 * g1)]
    np.testing.assert_allclose(r["sum"][0], want, rtol=1e-11)


def test_group_marginals_add_up():
    p = W.tiny_star(seed=4, n_fact=4_000, n_stores=8, n_items=50)
    res = oracle.evaluate(p)
    half = len(p["batch"]) // 2
    for k in range(half):
        r0, r1 = res[k], res[half + k]
        assert p["batch"][half + k]["groupby"] == ["cat"]
        assert int(r1["count"].sum()) == int(r0["count"][0])
        np.testing.assert_allclose(r1["sum"].sum(axis=0), r0["sum"][0], rtol=1e-9, atol=1e-9)


def test_product_symmetry():
    p = W.tiny_star(seed=6, n_fact=1_000, n_stores=5, n_items=20)
    p["batch"] = [{"groupby": ["cat"], "where": [], "root": None,
                   "aggs": [[("f2", 1), ("g1", 1)], [("g1", 1), ("f2", 1)]]}]
    r = oracle.evaluate(p)[0]
    np.testing.assert_array_equal(r["sum"][:, 0], r["sum"][:, 1])


# ---------------------------------------------------------------------------
# planted mistakes: each one must be caught by a pin above
# ---------------------------------------------------------------------------

def _brute_mismatch(problem):
    try:
        assert_matches_brute(problem)
    except AssertionError:
        return True
    return False


def test_planted_dropped_multiplicity_is_caught(monkeypatch):
    real = oracle._equi_join

    def dedup_join(left, right, on):  # keeps only the first partner of each tuple
        out = real(left, right, on)
        if not on:
            return out
        key = np.stack([out[a] for a in sorted(left)], axis=1)
        _, first = np.unique(key, axis=0, return_index=True)
        return {a: v[np.sort(first)] for a, v in out.items()}

    monkeypatch.setattr(oracle, "_equi_join", dedup_join)
    p = W.random_acyclic(3, n_rel=3, max_rows=6, max_dom=2)
    assert _brute_mismatch(p)


def test_planted_power_ignored_is_caught(monkeypatch):
    def term_no_power(D, factors, sel):
        t = np.ones(int(sel.sum()), dtype=np.float64)
        for attr, _ in factors:
            t = t * D[attr][sel].astype(np.float64)
        return t

    monkeypatch.setattr(oracle, "_term", term_no_power)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((50, 2))
    p = {"schema": [{"name": "R", "n_rows": 50, "attrs": [
        {"name": "a", "dtype": "f64", "domain": 0, "key": False},
        {"name": "b", "dtype": "f64", "domain": 0, "key": False}]}],
        "tree": [], "data": {"R": {"a": X[:, 0], "b": X[:, 1]}},
        "batch": W.covariance_batch(["a", "b"], (), split=False)}
    r = oracle.evaluate(p)[0]
    Xe = np.concatenate([np.ones((50, 1)), X], axis=1)
    sigma = Xe.T @ Xe
    want = [sigma[j, k] for j in range(3) for k in range(j, 3)]
    assert not np.allclose(r["sum"][0], want)


def test_planted_wrong_group_key_is_caught(monkeypatch):
    real = oracle.evaluate_query

    def swapped(D, query):
        q = dict(query)
        if q.get("groupby"):
            q["groupby"] = ["store"]  # wrong attribute
        return real(D, q)

    monkeypatch.setattr(oracle, "evaluate_query", swapped)
    p = W.tiny_star(seed=1, n_fact=2_000, n_stores=9, n_items=30)
    res = oracle.evaluate(p)
    r1 = res[len(p["batch"]) // 2]   # first query grouped by cat
    # marginals still add up, but the bincount pin on cat does not
    it = p["data"]["Items"]
    cat = it["cat"][p["data"]["S"]["item"]]
    cnt = np.bincount(cat, minlength=20)
    assert r1["count"].tolist() != cnt[np.nonzero(cnt)[0]].tolist()


def test_planted_operator_swap_is_caught(monkeypatch):
    # < evaluated as <= : every pin that goes through the oracle's own OPS
    # table would still pass; the brute force's scalar operators do not
    monkeypatch.setitem(oracle.OPS, "<", np.less_equal)
    assert any(_brute_mismatch(_operator_problem(seed)) for seed in range(4))


def test_planted_ge_as_gt_is_caught(monkeypatch):
    monkeypatch.setitem(oracle.OPS, ">=", np.greater)
    assert any(_brute_mismatch(_operator_problem(seed)) for seed in range(4))


# ---------------------------------------------------------------------------
# views: the join of the subtree below an edge, grouped by the edge key
# ---------------------------------------------------------------------------

def _edge_views(problem, u, v, aggs, where=()):
    nu, nv = problem["schema"][u]["name"], problem["schema"][v]["name"]
    key = sorted({a["name"] for a in problem["schema"][u]["attrs"]}
                 & {a["name"] for a in problem["schema"][v]["attrs"]})
    return nu, nv, key


@pytest.mark.parametrize("seed", range(8))
def test_view_matches_brute_force_over_the_subtree(seed):
    p = W.random_acyclic(200 + seed, n_rel=4, max_rows=5, max_dom=3)
    for u, v in p["tree"]:
        for a, b in ((u, v), (v, u)):
            na, nb, key = _edge_views(p, a, b, [])
            sub = oracle.subtree(p, na, nb)
            feats = [f"x{int(r[1:])}" for r in sub]
            aggs = [[], [(feats[0], 1)], [(feats[-1], 2)], [(feats[0], 1), (feats[-1], 1)]]
            r = oracle.evaluate_view(p, na, nb, key, aggs)
            keys, counts, sums = brute_force(p, rels=sub, query={"groupby": key, "aggs": aggs})
            assert [tuple(int(x) for x in k) for k in r["keys"]] == keys
            assert r["count"].tolist() == counts
            if keys:
                np.testing.assert_allclose(r["sum"], np.array(sums), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_views_factorise_count_at_every_edge(seed):
    # for an edge (u, v) of a join tree with join attributes K,
    # |D| = sum over k of |D_u(k)| * |D_v(k)|: every tuple of D is one tuple of
    # the u side and one of the v side that agree on K
    p = W.random_acyclic(300 + seed, n_rel=4, max_rows=6, max_dom=3)
    total = oracle.evaluate(dict(p, batch=[{"groupby": [], "where": [], "aggs": [[]], "root": None}]))[0]
    n_d = int(total["count"].sum())
    for u, v in p["tree"]:
        nu, nv, key = _edge_views(p, u, v, [])
        a = oracle.evaluate_view(p, nu, nv, key, [[]])
        b = oracle.evaluate_view(p, nv, nu, key, [[]])
        ca = {tuple(k): c for k, c in zip(a["keys"].tolist(), a["count"].tolist())}
        cb = {tuple(k): c for k, c in zip(b["keys"].tolist(), b["count"].tolist())}
        assert sum(ca[k] * cb.get(k, 0) for k in ca) == n_d


def test_view_carried_attribute_and_condition():
    # a foreign-key dimension: the view of Items toward S carries cat, which
    # is a function of the key item
    p = W.tiny_star(seed=2, n_fact=500, n_stores=5, n_items=30)
    r = oracle.evaluate_view(p, "Items", "S", ["item"], [[("g1", 1)]], carried=["cat"],
                             where=[("g2", ">", 0.0)])
    it = p["data"]["Items"]
    keep = it["g2"] > 0
    assert r["keys"][:, 0].tolist() == np.nonzero(keep)[0].tolist()
    assert r["codes"][:, 0].tolist() == it["cat"][keep].tolist()
    np.testing.assert_array_equal(r["sum"][:, 0], it["g1"][keep])
    assert r["count"].tolist() == [1] * int(keep.sum())


def test_planted_wrong_subtree_side_is_caught(monkeypatch):
    real = oracle.subtree

    def flipped(problem, a, b):   # the other side of the edge
        return real(problem, b, a)

    monkeypatch.setattr(oracle, "subtree", flipped)
    p = W.random_acyclic(201, n_rel=4, max_rows=5, max_dom=3)
    caught = False
    for u, v in p["tree"]:
        na, nb, key = _edge_views(p, u, v, [])
        r = oracle.evaluate_view(p, na, nb, key, [[]])
        keys, counts, _ = brute_force(p, rels=real(p, na, nb), query={"groupby": key, "aggs": [[]]})
        if [tuple(int(x) for x in k) for k in r["keys"]] != keys or r["count"].tolist() != counts:
            caught = True
    assert caught


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_user_defined_factors(seed):
    # SUM(g(x) * h(y)) and SUM(g(x)^2) grouped and ungrouped, with g, h
    # tables over integer attributes (section 2, the example query Q2)
    p = W.random_acyclic(seed)
    ints = [(a["name"], a["domain"]) for r in p["schema"] for a in r["attrs"] if a["dtype"] == "i32" and a.get("domain")]
    rng = np.random.default_rng(seed)
    (xa, xd), (ya, yd) = ints[0], ints[-1]
    p["functions"] = {"g": {"attr": xa, "values": rng.normal(size=xd)},
                      "h": {"attr": ya, "values": rng.normal(size=yd)}}
    gb = [ya] if ya != xa else []
    p["batch"] = [{"groupby": [], "where": [], "aggs": [[("g", 1), ("h", 1)], [("g", 2)], []]},
                  {"groupby": gb, "where": [], "aggs": [[("g", 1)], [("h", 1), ("g", 1)]]}]
    assert_matches_brute(p)
