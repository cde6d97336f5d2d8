"""Plain CPU oracle for batches of group-by aggregates over a natural join.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it and shares no code with it; the two meet only at the seeded
input generators in ``workloads``.

What it computes is the plain definition of the result, not the factorized
method (section 2 of the paper, "LMFAO by Example"): D is the natural join of
all relations of the schema, taken with bag semantics (every combination of
matching tuples is one tuple of D); a query ``SELECT G, SUM(f_1), ..., SUM(f_m)
FROM D WHERE P GROUP BY G`` maps every group value g that at least one tuple of
D satisfying P carries to the sums over those tuples of each aggregate
function.  Aggregate functions are products of attribute powers, which covers
the aggregates section 3 lists for ridge regression (SUM(X_j*X_k), one-hot
categoricals as group-by attributes), CART (SUM(1), SUM(Y), SUM(Y^2) under a
conjunctive condition) and Rk-means (SUM(1) grouped by each attribute).

Steps, in order:
  1. materialise D by successive equi-joins along the join tree (bag
     semantics; dangling tuples drop out) -- ``materialize_join``;
  2. evaluate the predicate P per tuple of D;
  3. group the qualifying tuples by G (``numpy.unique`` over the key columns,
     so groups come out in lexicographic order);
  4. per group and aggregate, add the FP64 product terms into an 80-bit
     extended-precision accumulator (``numpy.longdouble``) and, separately,
     the sum of absolute terms (used to bound cancellation when comparing
     against a float kernel); counts are exact int64.

Everything is FP64 (or wider) as the paper fixes no precision.  A condition's
constant is compared in the column's own type (numpy's rule for a Python float
against a float32 array).  Pins that tie this code to something other than
itself live in ``tests/test_oracle_pins.py`` (brute force over tuple
combinations, closed forms, invariants, library special cases).
"""
from __future__ import annotations

import numpy as np

__all__ = ["materialize_join", "evaluate", "evaluate_query", "evaluate_single",
           "evaluate_view", "subtree", "with_functions", "OPS"]

OPS = {
    "<=": np.less_equal, "<": np.less, ">": np.greater, ">=": np.greater_equal,
    "==": np.equal, "!=": np.not_equal,
}


def _columns(problem, rel_index):
    rel = problem["schema"][rel_index]
    cols = problem["data"][rel["name"]]
    return {a["name"]: np.asarray(cols[a["name"]]) for a in rel["attrs"]}


def _equi_join(left: dict, right: dict, on: list) -> dict:
    """Bag-semantics equi-join of two column dicts on the attribute names ``on``.

    For every left tuple and every right tuple that agree on all ``on``
    attributes, one output tuple.  Implemented with a sort of the right side and
    range lookups; tuples without a partner drop out."""
    n_left = len(next(iter(left.values()))) if left else 0
    n_right = len(next(iter(right.values()))) if right else 0
    if not on:  # cross product (disconnected pieces never occur in a tree, kept for completeness)
        li = np.repeat(np.arange(n_left), n_right)
        ri = np.tile(np.arange(n_right), n_left)
    else:
        # encode each key tuple as one int64 with a mixed radix over both sides
        lk = np.zeros(n_left, dtype=np.int64)
        rk = np.zeros(n_right, dtype=np.int64)
        for a in on:
            lv = left[a].astype(np.int64)
            rv = right[a].astype(np.int64)
            lo = min(lv.min(initial=0), rv.min(initial=0))
            span = max(lv.max(initial=0), rv.max(initial=0)) - lo + 1
            lk = lk * span + (lv - lo)
            rk = rk * span + (rv - lo)
        order = np.argsort(rk, kind="stable")
        rk_sorted = rk[order]
        lo_idx = np.searchsorted(rk_sorted, lk, side="left")
        hi_idx = np.searchsorted(rk_sorted, lk, side="right")
        cnt = hi_idx - lo_idx
        li = np.repeat(np.arange(n_left), cnt)
        start = np.repeat(lo_idx, cnt)
        offs = np.arange(len(li)) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        ri = order[start + offs]
    out = {a: v[li] for a, v in left.items()}
    for a, v in right.items():
        if a not in out:
            out[a] = v[ri]
    return out


def materialize_join(problem: dict, attrs=None) -> dict:
    """Step 1: the natural join D of all relations, as a dict of columns.

    Relations are joined in breadth-first order of the join tree starting at
    relation 0; each join is on every attribute name the new relation shares
    with what has been joined so far (the natural-join definition).  If
    ``attrs`` is given, only those columns (plus join attributes) are carried."""
    n = len(problem["schema"])
    adj = {i: [] for i in range(n)}
    for a, b in problem["tree"]:
        adj[a].append(b)
        adj[b].append(a)
    seen = [0]
    queue = [0]
    while queue:
        u = queue.pop(0)
        for v in sorted(adj[u]):
            if v not in seen:
                seen.append(v)
                queue.append(v)
    if len(seen) != n:
        raise ValueError("join tree does not connect every relation")
    all_names = [{a["name"] for a in r["attrs"]} for r in problem["schema"]]
    shared = set()
    for i in range(n):
        for j in range(i + 1, n):
            shared |= all_names[i] & all_names[j]
    keep = None if attrs is None else set(attrs) | shared
    table = None
    for i in seen:
        cols = _columns(problem, i)
        if keep is not None:
            cols = {k: v for k, v in cols.items() if k in keep}
        if table is None:
            table = cols
        else:
            on = sorted(set(table) & set(cols))
            table = _equi_join(table, cols, on)
    return table


def _mask(D, where, n):
    m = np.ones(n, dtype=bool)
    for attr, op, const in where:
        m &= OPS[op](D[attr], const)
    return m


def _term(D, factors, sel):
    t = np.ones(int(sel.sum()) if sel.dtype == bool else len(sel), dtype=np.float64)
    for attr, power in factors:
        v = D[attr][sel].astype(np.float64)
        for _ in range(int(power)):
            t = t * v
    return t


def evaluate_query(D: dict, query: dict) -> dict:
    """Steps 2-4 for one query over the materialised join D.

    Returns ``keys`` (int64, groups x |G|, lexicographically sorted), ``count``
    (int64 join tuples per group), ``sum`` (FP64 rounding of the extended
    precision sums, groups x aggregates) and ``abs`` (sum of |term|)."""
    n = len(next(iter(D.values()))) if D else 0
    sel = _mask(D, query.get("where", []), n)
    G = list(query.get("groupby", []))
    if G:
        keycols = np.stack([D[g][sel].astype(np.int64) for g in G], axis=1)
        if len(keycols):
            keys, inv = np.unique(keycols, axis=0, return_inverse=True)
            inv = inv.reshape(-1)
        else:
            keys, inv = np.zeros((0, len(G)), np.int64), np.zeros(0, np.int64)
    else:
        n_sel = int(sel.sum())
        keys = np.zeros((1 if n_sel else 0, 0), dtype=np.int64)
        inv = np.zeros(n_sel, dtype=np.int64)
    n_groups = keys.shape[0]
    count = np.bincount(inv, minlength=n_groups).astype(np.int64)
    aggs = query["aggs"]
    sums = np.zeros((n_groups, len(aggs)), dtype=np.float64)
    abss = np.zeros((n_groups, len(aggs)), dtype=np.float64)
    for k, factors in enumerate(aggs):
        t = _term(D, factors, sel)
        acc = np.zeros(n_groups, dtype=np.longdouble)
        np.add.at(acc, inv, t.astype(np.longdouble))
        sums[:, k] = acc.astype(np.float64)
        abss[:, k] = np.bincount(inv, weights=np.abs(t), minlength=n_groups)
    return {"keys": keys, "count": count, "sum": sums, "abs": abss}


def with_functions(problem: dict, D: dict, names) -> dict:
    """User-defined factors (section 2: aggregates such as SUM(g(item) *
    h(date)) with functions g, h of one attribute): problem["functions"][name]
    = {"attr": a, "values": v} tabulates the function at every value of the
    integer attribute a; the column ``name`` of D is v[t[a]] per tuple t."""
    funcs = problem.get("functions", {})
    for name in names:
        if name in funcs and name not in D:
            f = funcs[name]
            D[name] = np.asarray(f["values"], dtype=np.float64)[np.asarray(D[f["attr"]], dtype=np.int64)]
    return D


def _needed(problem: dict, names) -> set:
    """Attribute columns the names stand for (a function needs its argument)."""
    funcs = problem.get("functions", {})
    return {funcs[a]["attr"] if a in funcs else a for a in names}


def evaluate(problem: dict, queries=None) -> list:
    """Every query of the batch (or the listed query indices) over the
    materialised join of ``problem``."""
    batch = problem["batch"]
    idx = range(len(batch)) if queries is None else queries
    needed = set()
    for i in idx:
        q = batch[i]
        needed |= set(q.get("groupby", []))
        needed |= {w[0] for w in q.get("where", [])}
        for f in q["aggs"]:
            needed |= {a for a, _ in f}
    D = materialize_join(problem, _needed(problem, needed))
    with_functions(problem, D, needed)
    return [evaluate_query(D, batch[i]) for i in idx]


def evaluate_single(problem: dict, qi: int, ai: int) -> dict:
    """One aggregate of one query, materialising only the columns it needs
    (used for sampled checks at full size)."""
    q = dict(problem["batch"][qi])
    q["aggs"] = [q["aggs"][ai]]
    sub = dict(problem, batch=[q])
    return evaluate(sub)[0]


def subtree(problem: dict, from_rel: str, to_rel: str) -> list:
    """Relations on the ``from_rel`` side of the join-tree edge (from_rel,
    to_rel): those reached from ``from_rel`` without crossing that edge."""
    names = [r["name"] for r in problem["schema"]]
    a, b = names.index(from_rel), names.index(to_rel)
    adj = {i: set() for i in range(len(names))}
    for u, v in problem["tree"]:
        adj[u].add(v)
        adj[v].add(u)
    if b not in adj[a]:
        raise ValueError(f"{from_rel} and {to_rel} are not adjacent in the join tree")
    seen, stack = [a], [a]
    while stack:
        u = stack.pop()
        for v in sorted(adj[u]):
            if v not in seen and not (u == a and v == b):
                seen.append(v)
                stack.append(v)
    return [names[i] for i in seen]


def evaluate_view(problem: dict, from_rel: str, to_rel: str, key, aggs, carried=(), where=()) -> dict:
    """A view along the join-tree edge from ``from_rel`` to ``to_rel``
    (section 2, view generation layer: the view computes, over the join of
    the relations below the edge, the partial aggregates the queries above it
    need, grouped by the edge's join attributes).

    Plain definition: D_S = the natural join of the relations in the subtree
    of ``from_rel`` (bag semantics, as ``materialize_join``); the result is
    ``evaluate_query`` of ``SELECT key, SUM(aggs) FROM D_S WHERE where GROUP
    BY key``.  ``carried`` attributes must be functions of the key within D_S
    (a view that carries a group-by attribute up the tree); their value per
    group is returned in ``codes`` (groups x |carried|, int64), and a key
    whose tuples disagree on one raises ``ValueError``."""
    names = subtree(problem, from_rel, to_rel)
    order = {n: i for i, n in enumerate(names)}
    idx = {r["name"]: i for i, r in enumerate(problem["schema"])}
    sub = {
        "schema": [problem["schema"][idx[n]] for n in names],
        "data": {n: problem["data"][n] for n in names},
        "tree": [(order[problem["schema"][u]["name"]], order[problem["schema"][v]["name"]])
                 for u, v in problem["tree"]
                 if problem["schema"][u]["name"] in order and problem["schema"][v]["name"] in order],
    }
    needed = set(key) | set(carried) | {w[0] for w in where}
    for f in aggs:
        needed |= {a for a, _ in f}
    D = materialize_join(sub, needed)
    res = evaluate_query(D, {"groupby": list(key), "where": list(where), "aggs": list(aggs)})
    n = len(next(iter(D.values()))) if D else 0
    sel = _mask(D, list(where), n)
    codes = np.zeros((res["keys"].shape[0], len(carried)), dtype=np.int64)
    if carried and len(res["keys"]):
        kc = np.stack([D[k][sel].astype(np.int64) for k in key], axis=1)
        _, inv = np.unique(kc, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        for j, c in enumerate(carried):
            v = D[c][sel].astype(np.int64)
            lo = np.full(len(res["keys"]), np.iinfo(np.int64).max)
            hi = np.full(len(res["keys"]), np.iinfo(np.int64).min)
            np.minimum.at(lo, inv, v)
            np.maximum.at(hi, inv, v)
            if np.any(lo != hi):
                raise ValueError(f"carried attribute {c} is not a function of the key {list(key)}")
            codes[:, j] = lo
    res["codes"] = codes
    return res
