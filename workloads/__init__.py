"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates* inputs: relations (columns as numpy arrays), their
schema, a join tree and a batch of group-by aggregate queries.  It holds none of
the method's arithmetic: nothing here joins relations or evaluates aggregates.

A problem is a plain dict:

* ``schema``: list of relations ``{"name", "n_rows", "attrs": [{"name", "dtype",
  "domain", "key"}]}``.  ``dtype`` is ``"i32"``, ``"f32"`` or ``"f64"``.
  Integer attributes hold codes in ``[0, domain)``.  ``key`` marks the
  relation's primary key (the underlined attributes of the paper's schema
  figure).  Attributes with the same name in different relations are joined
  (natural join).
* ``tree``: list of ``(i, j)`` relation index pairs (the join tree).
* ``batch``: list of queries ``{"groupby": [attr...], "where": [(attr, op,
  const)...], "aggs": [[(attr, power)...], ...], "root": None | relation
  name}``.  An empty factor list is ``SUM(1)``.
* ``data``: ``{relation name: {attr name: numpy array}}``.
* ``policy``: root-assignment policy the workload is meant to run with.

Every random draw comes from ``numpy.random.Generator(PCG64)`` streams spawned
from ``SeedSequence(seed)``, one stream per relation, so a given seed always
yields byte-identical arrays.
"""
from __future__ import annotations

import hashlib
import itertools

import numpy as np

__all__ = [
    "zipf_keys", "tiny_star", "retail_snowflake", "grocery_star", "cart_node", "quantile_thresholds",
    "rkmeans_chain", "favorita_example", "random_acyclic", "covariance_batch",
    "problem_digest", "fact_prefix", "estimator_workload", "bench_workload", "bench_plan_options",
]


# --------------------------------------------------------------------------
# samplers
# --------------------------------------------------------------------------

def zipf_keys(rng: np.random.Generator, n: int, support: int, s: float) -> np.ndarray:
    """Keys k in [0, support) with P(k) proportional to (k+1)^-s (finite support,
    no permutation of the ranks)."""
    w = np.arange(1, support + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    k = np.searchsorted(cdf, u, side="right")
    return np.minimum(k, support - 1).astype(np.int32)


def _attr(name, dtype, domain=0, key=False):
    return {"name": name, "dtype": dtype, "domain": int(domain), "key": bool(key)}


def _rel(name, n_rows, attrs):
    return {"name": name, "n_rows": int(n_rows), "attrs": attrs}


def _spawn(seed: int, n: int):
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(n)]


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------

def covariance_batch(continuous, categorical=(), pairs=True, groupby_cont=True, split=True):
    """Aggregates of the ridge-regression covariance matrix with one-hot
    categoricals (section 3, linear regression), each entry one query as in
    the paper:

    * SELECT SUM(x_j * x_k) for j <= k over ``[1] + continuous`` (the intercept
      x_1 = 1 turns the first row into COUNT and SUM(x_k)),
    * for every categorical c: SELECT c, SUM(x_k) GROUP BY c for x_k in
      ``[1] + continuous``,
    * for every pair of categoricals: SELECT c, c', SUM(1) GROUP BY c, c'.

    With ``split=False`` the aggregates sharing a group-by are packed into one
    multi-aggregate query instead (same cells).
    """
    feats = [None] + list(continuous)
    aggs = []
    for j in range(len(feats)):
        for k in range(j, len(feats)):
            fj, fk = feats[j], feats[k]
            if fj is None and fk is None:
                aggs.append([])
            elif fj is None:
                aggs.append([(fk, 1)])
            elif fj == fk:
                aggs.append([(fj, 2)])
            else:
                aggs.append([(fj, 1), (fk, 1)])
    groups = [([], aggs)]
    if groupby_cont:
        for c in categorical:
            groups.append(([c], [[]] + [[(x, 1)] for x in continuous]))
    if pairs:
        for a, b in itertools.combinations(categorical, 2):
            groups.append(([a, b], [[]]))
    batch = []
    for g, ag in groups:
        if split:
            batch += [{"groupby": list(g), "where": [], "aggs": [a], "root": None} for a in ag]
        else:
            batch.append({"groupby": list(g), "where": [], "aggs": ag, "root": None})
    return batch


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def tiny_star(seed: int = 0, n_fact: int = 100_000, n_stores: int = 50,
              n_items: int = 2_000, zipf_s: float = 1.1):
    """Tiny star join, FP64: S(store, item, units) with Zipf(1.1) keys,
    Stores(store, f1..f4 ~ N(0,1)), Items(item, g1..g3 ~ N(0,1), cat in [0,20)).
    Batch: COUNT, SUM(x_i), SUM(x_i*x_j) over the 8 continuous features, and the
    same 45 aggregates grouped by cat."""
    r_s, r_st, r_it = _spawn(seed, 3)
    data = {
        "S": {
            "store": zipf_keys(r_s, n_fact, n_stores, zipf_s),
            "item": zipf_keys(r_s, n_fact, n_items, zipf_s),
            "units": r_s.lognormal(0.0, 1.0, n_fact),
        },
        "Stores": {"store": np.arange(n_stores, dtype=np.int32)},
        "Items": {"item": np.arange(n_items, dtype=np.int32)},
    }
    for j in range(1, 5):
        data["Stores"][f"f{j}"] = r_st.standard_normal(n_stores)
    for j in range(1, 4):
        data["Items"][f"g{j}"] = r_it.standard_normal(n_items)
    data["Items"]["cat"] = r_it.integers(0, 20, n_items).astype(np.int32)
    schema = [
        _rel("S", n_fact, [_attr("store", "i32", n_stores), _attr("item", "i32", n_items),
                           _attr("units", "f64")]),
        _rel("Stores", n_stores, [_attr("store", "i32", n_stores, True)]
             + [_attr(f"f{j}", "f64") for j in range(1, 5)]),
        _rel("Items", n_items, [_attr("item", "i32", n_items, True)]
             + [_attr(f"g{j}", "f64") for j in range(1, 4)] + [_attr("cat", "i32", 20)]),
    ]
    cont = ["units", "f1", "f2", "f3", "f4", "g1", "g2", "g3"]
    ungrouped = covariance_batch(cont, (), pairs=False, groupby_cont=False)
    grouped = [dict(q, groupby=["cat"]) for q in ungrouped]
    return {"name": "tiny_star", "schema": schema, "tree": [(0, 1), (0, 2)],
            "batch": ungrouped + grouped, "data": data, "policy": "fact",
            "precision": "f64"}


def retail_snowflake(seed: int = 0, n_inv: int = 84_000_000, n_locn: int = 1_300,
                     n_dates: int = 124, n_ksn: int = 5_600, n_weather_dates: int = 846,
                     zipf_s: float = 1.0, dtype: str = "f32"):
    """Snowflake with 5 relations shaped like a retail inventory workload:
    Inv(locn, date, ksn, units) with locn and date uniform and ksn Zipf(1.0);
    Items(ksn, i1..i5, icat1, icat2); Stores(locn, zip, s1..s30, scat1, scat2);
    Demog(zip, d1..d15); Weather(locn, date, w1..w8, wcat1, wcat2) over the
    full (locn, date) grid.  Join tree Inv-Items, Inv-Weather, Inv-Stores,
    Stores-Demog.  Batch: ridge covariance over 43 continuous features plus 6
    one-hot categoricals (COUNT/SUM/products, categorical group-bys, pairs)."""
    npdt = np.float32 if dtype == "f32" else np.float64
    r_inv, r_it, r_st, r_dm, r_we = _spawn(seed, 5)
    inv = {
        "locn": r_inv.integers(0, n_locn, n_inv, dtype=np.int32),
        "date": r_inv.integers(0, n_dates, n_inv, dtype=np.int32),
        "ksn": zipf_keys(r_inv, n_inv, n_ksn, zipf_s),
        "units": r_inv.lognormal(0.0, 1.0, n_inv).astype(npdt),
    }
    items = {"ksn": np.arange(n_ksn, dtype=np.int32)}
    for j in range(1, 6):
        items[f"i{j}"] = r_it.standard_normal(n_ksn).astype(npdt)
    items["icat1"] = r_it.integers(0, 10, n_ksn, dtype=np.int32)
    items["icat2"] = r_it.integers(0, 8, n_ksn, dtype=np.int32)
    stores = {"locn": np.arange(n_locn, dtype=np.int32),
              "zip": r_st.integers(0, n_locn, n_locn, dtype=np.int32)}
    for j in range(1, 31):
        stores[f"s{j}"] = r_st.standard_normal(n_locn).astype(npdt)
    stores["scat1"] = r_st.integers(0, 5, n_locn, dtype=np.int32)
    stores["scat2"] = r_st.integers(0, 4, n_locn, dtype=np.int32)
    demog = {"zip": np.arange(n_locn, dtype=np.int32)}
    for j in range(1, 16):
        demog[f"d{j}"] = r_dm.standard_normal(n_locn).astype(npdt)
    n_w = n_locn * n_weather_dates
    weather = {"locn": np.repeat(np.arange(n_locn, dtype=np.int32), n_weather_dates),
               "date": np.tile(np.arange(n_weather_dates, dtype=np.int32), n_locn)}
    for j in range(1, 9):
        weather[f"w{j}"] = r_we.standard_normal(n_w).astype(npdt)
    weather["wcat1"] = r_we.integers(0, 3, n_w, dtype=np.int32)
    weather["wcat2"] = r_we.integers(0, 2, n_w, dtype=np.int32)
    data = {"Inv": inv, "Items": items, "Stores": stores, "Demog": demog, "Weather": weather}
    f = dtype
    schema = [
        _rel("Inv", n_inv, [_attr("locn", "i32", n_locn), _attr("date", "i32", n_weather_dates),
                            _attr("ksn", "i32", n_ksn), _attr("units", f)]),
        _rel("Items", n_ksn, [_attr("ksn", "i32", n_ksn, True)]
             + [_attr(f"i{j}", f) for j in range(1, 6)]
             + [_attr("icat1", "i32", 10), _attr("icat2", "i32", 8)]),
        _rel("Stores", n_locn, [_attr("locn", "i32", n_locn, True), _attr("zip", "i32", n_locn)]
             + [_attr(f"s{j}", f) for j in range(1, 31)]
             + [_attr("scat1", "i32", 5), _attr("scat2", "i32", 4)]),
        _rel("Demog", n_locn, [_attr("zip", "i32", n_locn, True)]
             + [_attr(f"d{j}", f) for j in range(1, 16)]),
        _rel("Weather", n_w, [_attr("locn", "i32", n_locn, True),
                              _attr("date", "i32", n_weather_dates, True)]
             + [_attr(f"w{j}", f) for j in range(1, 9)]
             + [_attr("wcat1", "i32", 3), _attr("wcat2", "i32", 2)]),
    ]
    cont = (["units"] + [f"i{j}" for j in range(1, 6)] + [f"s{j}" for j in range(1, 15)]
            + [f"d{j}" for j in range(1, 16)] + [f"w{j}" for j in range(1, 9)])
    cats = ["icat1", "icat2", "scat1", "scat2", "wcat1", "wcat2"]
    return {"name": "retail_snowflake", "schema": schema,
            "tree": [(0, 1), (0, 4), (0, 2), (2, 3)],
            "batch": covariance_batch(cont, cats), "data": data, "policy": "fact",
            "precision": dtype}


def grocery_star(seed: int = 0, n_sales: int = 120_000_000, n_stores: int = 54,
                 n_items: int = 4_000, n_dates: int = 1_537, n_oil: int = 1_200,
                 n_hol: int = 350, dtype: str = "f32"):
    """Star join with 6 relations shaped like grocery sales (the schema of the
    paper's worked example): Sales(date, store, item, unit_sales, onpromo),
    Items(item, family, class, perishable), Stores(store, city, state, stype,
    cluster), Trans(date, store, txns), Oil(date, price), Holidays(date, htype,
    locale).  Join tree Sales-Trans, Trans-Stores, Trans-Oil, Sales-Items,
    Sales-Holidays.  Sales dates are drawn from the holiday dates so that every
    fact row joins."""
    npdt = np.float32 if dtype == "f32" else np.float64
    r_sa, r_it, r_st, r_tr, r_oi, r_ho = _spawn(seed, 6)
    oil_dates = np.sort(r_oi.choice(n_dates, n_oil, replace=False)).astype(np.int32)
    hol_dates = np.sort(r_ho.choice(oil_dates, n_hol, replace=False)).astype(np.int32)
    sales = {
        "date": hol_dates[r_sa.integers(0, n_hol, n_sales)].astype(np.int32),
        "store": r_sa.integers(0, n_stores, n_sales, dtype=np.int32),
        "item": zipf_keys(r_sa, n_sales, n_items, 1.0),
        "unit_sales": r_sa.lognormal(0.0, 1.0, n_sales).astype(npdt),
        "onpromo": (r_sa.random(n_sales) < 0.1).astype(np.int32),
    }
    cls = r_it.integers(0, 337, n_items, dtype=np.int32)
    items = {"item": np.arange(n_items, dtype=np.int32), "class": cls,
             "family": (cls % 33).astype(np.int32),
             "perishable": (r_it.random(n_items) < 0.25).astype(np.int32)}
    city = r_st.integers(0, 22, n_stores, dtype=np.int32)
    stores = {"store": np.arange(n_stores, dtype=np.int32), "city": city,
              "state": (city % 16).astype(np.int32),
              "stype": r_st.integers(0, 5, n_stores, dtype=np.int32),
              "cluster": r_st.integers(0, 17, n_stores, dtype=np.int32)}
    trans = {"date": np.repeat(np.arange(n_dates, dtype=np.int32), n_stores),
             "store": np.tile(np.arange(n_stores, dtype=np.int32), n_dates)}
    trans["txns"] = r_tr.lognormal(7.0, 0.5, n_dates * n_stores).astype(npdt)
    oil = {"date": oil_dates, "price": r_oi.uniform(30.0, 110.0, n_oil).astype(npdt)}
    hol = {"date": hol_dates, "htype": r_ho.integers(0, 6, n_hol, dtype=np.int32),
           "locale": r_ho.integers(0, 3, n_hol, dtype=np.int32)}
    data = {"Sales": sales, "Trans": trans, "Stores": stores, "Oil": oil,
            "Items": items, "Holidays": hol}
    f = dtype
    schema = [
        _rel("Sales", n_sales, [_attr("date", "i32", n_dates), _attr("store", "i32", n_stores),
                                _attr("item", "i32", n_items), _attr("unit_sales", f),
                                _attr("onpromo", "i32", 2)]),
        _rel("Trans", n_dates * n_stores, [_attr("date", "i32", n_dates, True),
                                           _attr("store", "i32", n_stores, True),
                                           _attr("txns", f)]),
        _rel("Stores", n_stores, [_attr("store", "i32", n_stores, True), _attr("city", "i32", 22),
                                  _attr("state", "i32", 16), _attr("stype", "i32", 5),
                                  _attr("cluster", "i32", 17)]),
        _rel("Oil", n_oil, [_attr("date", "i32", n_dates, True), _attr("price", f)]),
        _rel("Items", n_items, [_attr("item", "i32", n_items, True), _attr("family", "i32", 33),
                                _attr("class", "i32", 337), _attr("perishable", "i32", 2)]),
        _rel("Holidays", n_hol, [_attr("date", "i32", n_dates, True), _attr("htype", "i32", 6),
                                 _attr("locale", "i32", 3)]),
    ]
    cont = ["unit_sales", "txns", "price"]
    cats = ["onpromo", "family", "class", "perishable", "city", "state", "stype",
            "cluster", "htype", "locale"]
    return {"name": "grocery_star", "schema": schema,
            "tree": [(0, 1), (1, 2), (1, 3), (0, 4), (0, 5)],
            "batch": covariance_batch(cont, cats), "data": data, "policy": "fact",
            "precision": dtype}


def favorita_example(seed: int = 0, n_sales: int = 40):
    """Tiny instance of the worked example's schema (Sales, Holidays, StoRes,
    Items, Transactions, Oil) with the three example queries (Q2 and Q3 use
    plain attributes in place of the user-defined functions g and h).  Used for
    the planner's structural tests and brute-force oracle pins."""
    r = _spawn(seed, 6)
    n_dates, n_stores, n_items = 4, 3, 5
    sales = {"date": r[0].integers(0, n_dates, n_sales, dtype=np.int32),
             "store": r[0].integers(0, n_stores, n_sales, dtype=np.int32),
             "item": r[0].integers(0, n_items, n_sales, dtype=np.int32),
             "units": r[0].lognormal(0, 1, n_sales),
             "promo": r[0].integers(0, 2, n_sales, dtype=np.int32)}
    hol = {"date": np.arange(n_dates, dtype=np.int32), "htype": r[1].integers(0, 3, n_dates, dtype=np.int32)}
    stores = {"store": np.arange(n_stores, dtype=np.int32), "city": r[2].integers(0, 2, n_stores, dtype=np.int32)}
    items = {"item": np.arange(n_items, dtype=np.int32),
             "class": r[3].integers(0, 3, n_items, dtype=np.int32),
             "g": r[3].standard_normal(n_items)}
    trans = {"date": np.repeat(np.arange(n_dates, dtype=np.int32), n_stores),
             "store": np.tile(np.arange(n_stores, dtype=np.int32), n_dates),
             "txns": r[4].lognormal(0, 1, n_dates * n_stores)}
    oil = {"date": np.arange(n_dates, dtype=np.int32), "price": r[5].uniform(1, 2, n_dates),
           "h": r[5].standard_normal(n_dates)}
    data = {"Sales": sales, "Holidays": hol, "StoRes": stores, "Items": items,
            "Transactions": trans, "Oil": oil}
    schema = [
        _rel("Sales", n_sales, [_attr("date", "i32", n_dates), _attr("store", "i32", n_stores),
                                _attr("item", "i32", n_items), _attr("units", "f64"),
                                _attr("promo", "i32", 2)]),
        _rel("Holidays", n_dates, [_attr("date", "i32", n_dates, True), _attr("htype", "i32", 3)]),
        _rel("StoRes", n_stores, [_attr("store", "i32", n_stores, True), _attr("city", "i32", 2)]),
        _rel("Items", n_items, [_attr("item", "i32", n_items, True), _attr("class", "i32", 3),
                                _attr("g", "f64")]),
        _rel("Transactions", n_dates * n_stores, [_attr("date", "i32", n_dates, True),
                                                  _attr("store", "i32", n_stores, True),
                                                  _attr("txns", "f64")]),
        _rel("Oil", n_dates, [_attr("date", "i32", n_dates, True), _attr("price", "f64"),
                              _attr("h", "f64")]),
    ]
    # join tree of the example: S-T, T-R, T-O, S-I, S-H
    tree = [(0, 4), (4, 2), (4, 5), (0, 3), (0, 1)]
    batch = [
        {"groupby": [], "where": [], "aggs": [[("units", 1)]], "root": None},
        {"groupby": ["store"], "where": [], "aggs": [[("g", 1), ("h", 1)]], "root": None},
        {"groupby": ["class"], "where": [], "aggs": [[("units", 1), ("price", 1)]], "root": None},
    ]
    return {"name": "favorita_example", "schema": schema, "tree": tree, "batch": batch,
            "data": data, "policy": "groupby", "precision": "f64"}


def random_acyclic(seed: int, n_rel: int = 4, max_rows: int = 6, max_dom: int = 3,
                   dangling: bool = True, unique_dims: bool = False, n_queries: int = 4):
    """Small random acyclic schema for property tests: a random tree over
    ``n_rel`` relations, each edge joined on one fresh shared integer attribute
    (domain ``max_dom``), plus one float feature and one categorical per
    relation.  Join keys may repeat (many-to-many) and may dangle.  With
    ``unique_dims`` every non-root relation is keyed by its parent edge
    attribute, so each child row appears at most once per key (FK joins)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    parent = [-1] + [int(rng.integers(0, i)) for i in range(1, n_rel)]
    tree = [(parent[i], i) for i in range(1, n_rel)]
    attrs = [[] for _ in range(n_rel)]
    for i in range(1, n_rel):
        ja = f"k{i}"
        attrs[parent[i]].append(_attr(ja, "i32", max_dom))
        attrs[i].append(_attr(ja, "i32", max_dom, key=unique_dims))
    schema, data = [], {}
    for i in range(n_rel):
        name = f"R{i}"
        if unique_dims and i > 0:
            n = max_dom if not dangling else int(rng.integers(1, max_dom + 1))
        else:
            n = int(rng.integers(1, max_rows + 1))
        cols = {}
        for a in attrs[i]:
            if unique_dims and i > 0 and a["key"]:
                cols[a["name"]] = rng.permutation(max_dom)[:n].astype(np.int32)
            else:
                cols[a["name"]] = rng.integers(0, max_dom, n).astype(np.int32)
        cols[f"x{i}"] = np.round(rng.standard_normal(n), 3)
        cols[f"c{i}"] = rng.integers(0, 3, n).astype(np.int32)
        full = attrs[i] + [_attr(f"x{i}", "f64"), _attr(f"c{i}", "i32", 3)]
        schema.append(_rel(name, n, full))
        data[name] = cols
    feats = [f"x{i}" for i in range(n_rel)]
    cats = [f"c{i}" for i in range(n_rel)]
    batch = []
    for _ in range(n_queries):
        g = list(rng.choice(cats, size=int(rng.integers(0, 3)), replace=False))
        aggs = [[]]
        for _ in range(3):
            deg = int(rng.integers(1, 3))
            fs = list(rng.choice(feats, size=deg, replace=True))
            if deg == 2 and fs[0] == fs[1]:
                aggs.append([(str(fs[0]), 2)])
            else:
                aggs.append([(str(f), 1) for f in fs])
        batch.append({"groupby": [str(x) for x in g], "where": [], "aggs": aggs, "root": None})
    return {"name": f"random_acyclic_{seed}", "schema": schema, "tree": tree,
            "batch": batch, "data": data, "policy": "groupby", "precision": "f64"}


def fact_prefix(problem: dict, rel: str, n: int) -> dict:
    """Copy of ``problem`` whose relation ``rel`` keeps only its first ``n`` rows
    (used for bounded CPU-baseline samples)."""
    out = dict(problem)
    out["data"] = dict(problem["data"])
    out["data"][rel] = {k: v[:n] for k, v in problem["data"][rel].items()}
    out["schema"] = [dict(r, n_rows=(n if r["name"] == rel else r["n_rows"]))
                     for r in problem["schema"]]
    return out


def problem_digest(problem: dict) -> str:
    """SHA-256 over every generated column (determinism check and cache key)."""
    h = hashlib.sha256()
    for rname in sorted(problem["data"]):
        for aname in sorted(problem["data"][rname]):
            h.update(f"{rname}.{aname}".encode())
            h.update(np.ascontiguousarray(problem["data"][rname][aname]).tobytes())
    return h.hexdigest()


def quantile_thresholds(values, n_thr: int = 20):
    """Split thresholds of a continuous feature: the data values at the
    nearest-rank quantiles k/(n_thr+1), k = 1..n_thr, of its base column."""
    v = np.sort(np.asarray(values))
    n = len(v)
    idx = np.ceil(np.arange(1, n_thr + 1) * n / (n_thr + 1)).astype(np.int64) - 1
    return [float(x) for x in v[np.clip(idx, 0, n - 1)]]


def cart_node(seed: int = 0, n_inv: int = 84_000_000, n_thr: int = 20, n_node_conds: int = 3,
              label: str = "units", **retail_kw):
    """One node of a regression tree grown by CART on the retail-shaped
    snowflake (section 3, decision trees): for every split candidate the
    statistics SUM(1), SUM(y), SUM(y^2) of y = units under the node's path
    condition.  Candidates: X <= t for each of the 42 non-label continuous
    features and its ``n_thr`` quantile thresholds, and a group-by on each
    categorical attribute (the 6 one-hot categoricals and ksn) for = / !=
    splits; plus the node totals.  The path condition is ``n_node_conds``
    random conditions (continuous: <= or > one of its thresholds; categorical:
    = or != a random code)."""
    p = retail_snowflake(seed=seed, n_inv=n_inv, **retail_kw)
    owner = {}
    for r in p["schema"]:
        for a in r["attrs"]:
            owner.setdefault(a["name"], r["name"])
    dom = {a["name"]: a["domain"] for r in p["schema"] for a in r["attrs"]}
    cont = [x for x in (["units"] + [f"i{j}" for j in range(1, 6)] + [f"s{j}" for j in range(1, 15)]
                        + [f"d{j}" for j in range(1, 16)] + [f"w{j}" for j in range(1, 9)]) if x != label]
    cats = ["icat1", "icat2", "scat1", "scat2", "wcat1", "wcat2"]
    thr = {x: quantile_thresholds(p["data"][owner[x]][x], n_thr) for x in cont}
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4])))
    node = []
    for _ in range(n_node_conds):
        k = int(rng.integers(0, len(cont) + len(cats)))
        if k < len(cont):
            x = cont[k]
            node.append((x, "<=" if rng.random() < 0.5 else ">", thr[x][int(rng.integers(0, n_thr))]))
        else:
            c = cats[k - len(cont)]
            node.append((c, "==" if rng.random() < 0.5 else "!=", int(rng.integers(0, dom[c]))))
    stats = [[], [(label, 1)], [(label, 2)]]
    batch = []
    for x in cont:
        for t in thr[x]:
            batch += [{"groupby": [], "where": node + [(x, "<=", t)], "aggs": [a], "root": None} for a in stats]
    for c in cats + ["ksn"]:
        batch += [{"groupby": [c], "where": list(node), "aggs": [a], "root": None} for a in stats]
    batch += [{"groupby": [], "where": list(node), "aggs": [a], "root": None} for a in stats]
    p.update(name="cart_node", batch=batch, thresholds=thr, node=node)
    return p



def udf_grocery(seed: int = 0, n_sales: int = 200_000, **kw):
    """The grocery-shaped star with user-defined factors (section 2, the
    example's second query: SUM(g(item) * h(date))): g tabulated over the
    item domain and h over the date domain (values ~ N(0, 1)).  Batch: that
    query, SUM(g(item)) grouped by store, SUM(h(date)^2) grouped by family,
    SUM(g(item) * unit_sales), SUM(g(item)^2) and COUNT."""
    p = grocery_star(seed=seed, n_sales=n_sales, **kw)
    dom = {a["name"]: a["domain"] for r in p["schema"] for a in r["attrs"]}
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    p["functions"] = {"g": {"attr": "item", "values": rng.standard_normal(int(dom["item"]))},
                      "h": {"attr": "date", "values": rng.standard_normal(int(dom["date"]))}}
    p["batch"] = [
        {"groupby": [], "where": [], "aggs": [[("g", 1), ("h", 1)]], "root": None},
        {"groupby": ["store"], "where": [], "aggs": [[("g", 1)]], "root": None},
        {"groupby": ["family"], "where": [], "aggs": [[("h", 2)]], "root": None},
        {"groupby": [], "where": [], "aggs": [[("g", 1), ("unit_sales", 1)], [("g", 2)], []], "root": None},
    ]
    p["name"] = "udf_grocery"
    return p


def cart_tree(seed: int = 0, n_inv: int = 200_000, n_thr: int = 8, cont=None, cats=None, label: str = "units",
              **retail_kw):
    """The node batch of regression-tree growth by CART on the retail-shaped
    snowflake (section 3, decision trees), the same for every node: per
    continuous candidate attribute and distinct threshold (``n_thr`` quantile
    thresholds of its base column) a query with the condition x <= t and the
    aggregates SUM(1), SUM(y), SUM(y^2) of y = ``label``; per categorical
    attribute one query grouped by it with the same aggregates (a candidate
    x == v per code v); and the node totals.  A node's path condition is
    applied through per-row weights of the relations holding the candidate
    attributes (``row_weights``).  ``cart`` lists the candidates in
    tie-break order (attributes as listed, then values) with the query and
    group row holding each one's statistics."""
    p = retail_snowflake(seed=seed, n_inv=n_inv, **retail_kw)
    owner = {}
    for r in p["schema"]:
        for a in r["attrs"]:
            owner.setdefault(a["name"], r["name"])
    dom = {a["name"]: a["domain"] for r in p["schema"] for a in r["attrs"]}
    cont = list(cont) if cont is not None else ["i1", "i2", "s1", "s2", "d1", "w1", "w2"]
    cats = list(cats) if cats is not None else ["icat1", "scat1", "wcat1"]
    stats = [[], [(label, 1)], [(label, 2)]]
    batch, cands = [], []
    for x in cont:
        for t in sorted(set(quantile_thresholds(p["data"][owner[x]][x], n_thr))):
            cands.append({"attr": x, "op": "<=", "value": t, "query": len(batch), "group": 0})
            batch.append({"groupby": [], "where": [(x, "<=", t)], "aggs": stats, "root": None})
    for c in cats:
        q = len(batch)
        batch.append({"groupby": [c], "where": [], "aggs": stats, "root": None})
        for v in range(int(dom[c])):
            cands.append({"attr": c, "op": "==", "value": v, "query": q, "group": v})
    total = len(batch)
    batch.append({"groupby": [], "where": [], "aggs": stats, "root": None})
    p.update(name="cart_tree", batch=batch, label=label, cart={"candidates": cands, "total_query": total},
             row_weights=sorted({owner[x] for x in cont + cats}))
    return p


def rkmeans_chain(seed: int = 0, n1: int = 50_000_000, n2: int = 5_000_000, n3: int = 200_000,
                  n_x: int = 40, n_y: int = 30, n_z: int = 30, max_dom: int = 1_000_000, zipf: float = 0.0):
    """Step 1 of Rk-means (section 3, Rk-means) on a chain join R1(a, b, x*) -
    R2(b, c, y*) - R3(c, z*) with foreign keys b and c (every R1 row joins
    exactly once).  Attribute j takes values k ~ U[0, d_j) with d_j =
    round(10^U(1, log10 max_dom)); the values are integers, stored as int32
    codes with domain d_j.  Batch: SUM(1) GROUP BY X_j for each of the
    n_x + n_y + n_z attributes, plus SUM(1) GROUP BY X_i, X_j for 10 pairs
    (4 within R1, 2 within R2, 1 within R3, 2 across R1 x R2, 1 across
    R1 x R3) picked by seed from domain-sorted attributes so that their group
    counts spread from small to large.  ``zipf`` > 0 draws every attribute
    from Zipf(zipf) over its domain instead of uniformly."""
    r1, r2, r3, rd = _spawn(seed, 4)
    top = np.log10(max_dom)
    names = ([f"x{j}" for j in range(1, n_x + 1)] + [f"y{j}" for j in range(1, n_y + 1)]
             + [f"z{j}" for j in range(1, n_z + 1)])
    dom = {a: int(max(2, round(10 ** rd.uniform(1, top)))) for a in names}
    R1 = {"a": np.arange(n1, dtype=np.int32), "b": r1.integers(0, n2, n1, dtype=np.int32)}
    R2 = {"b": np.arange(n2, dtype=np.int32), "c": r2.integers(0, n3, n2, dtype=np.int32)}
    R3 = {"c": np.arange(n3, dtype=np.int32)}
    for rel, rng, pre, cnt, n in ((R1, r1, "x", n_x, n1), (R2, r2, "y", n_y, n2), (R3, r3, "z", n_z, n3)):
        for j in range(1, cnt + 1):
            a = f"{pre}{j}"
            rel[a] = (zipf_keys(rng, n, dom[a], zipf) if zipf > 0
                      else rng.integers(0, dom[a], n, dtype=np.int32))
    schema = [
        _rel("R1", n1, [_attr("a", "i32"), _attr("b", "i32", n2)]
             + [_attr(f"x{j}", "i32", dom[f"x{j}"]) for j in range(1, n_x + 1)]),
        _rel("R2", n2, [_attr("b", "i32", n2, True), _attr("c", "i32", n3)]
             + [_attr(f"y{j}", "i32", dom[f"y{j}"]) for j in range(1, n_y + 1)]),
        _rel("R3", n3, [_attr("c", "i32", n3, True)]
             + [_attr(f"z{j}", "i32", dom[f"z{j}"]) for j in range(1, n_z + 1)]),
    ]
    batch = [{"groupby": [a], "where": [], "aggs": [[]], "root": None} for a in names]
    xs = sorted((a for a in names if a[0] == "x"), key=lambda a: dom[a])
    ys = sorted((a for a in names if a[0] == "y"), key=lambda a: dom[a])
    zs = sorted((a for a in names if a[0] == "z"), key=lambda a: dom[a])

    # pairs by domain rank: small x small up to the two largest domains
    m = len(xs) // 2
    pairs = [(xs[0], xs[1]), (xs[m], xs[m + 1]), (xs[-1], xs[0]), (xs[-1], xs[-2]),
             (ys[0], ys[1]), (ys[-1], ys[-2]), (zs[0], zs[-1]),
             (xs[0], ys[-1]), (xs[-1], ys[0]), (xs[m], zs[len(zs) // 2])]
    batch += [{"groupby": [a, b], "where": [], "aggs": [[]], "root": None} for a, b in pairs]
    data = {"R1": R1, "R2": R2, "R3": R3}
    return {"name": "rkmeans_chain", "schema": schema, "tree": [(0, 1), (1, 2)], "batch": batch,
            "data": data, "policy": "fact", "precision": "f32", "domains": dom, "pairs": pairs}


def estimator_workload(seed: int, max_rows: int = 1_000_000):
    """A random small acyclic join for the group-count estimator's corpus.

    Shape (star, chain or snowflake) over 2-5 relations; relation 0 has
    10^U(4, log10 max_rows) rows, every other relation up to as many as its
    parent.  An edge is a foreign key into the child (probability 0.7: the
    child's key attribute is 0..n-1, the parent's reference uniform or Zipf) or
    a many-to-many join on an attribute with domain 10^U(1, 4), the parent
    referring to values the child holds.  Every relation
    has 1-3 integer attributes with domains 10^U(1, 6), uniform or Zipf(s in
    [0.8, 1.5]).  Batch: SUM(1) grouped by each such attribute and by up to 6
    random pairs of them that one relation reaches through foreign keys."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5eed])))
    n_rel = int(g.integers(2, 6))
    shape = ["star", "chain", "snowflake"][int(g.integers(0, 3))]
    parent = [-1] + [0 if shape == "star" else i - 1 if shape == "chain" else int(g.integers(0, i))
                     for i in range(1, n_rel)]
    rows = [int(10 ** g.uniform(4, np.log10(max_rows)))]
    for i in range(1, n_rel):
        rows.append(max(10, int(10 ** g.uniform(1, np.log10(rows[parent[i]])))))

    def values(n, dom):
        if g.random() < 0.5:
            return g.integers(0, dom, n, dtype=np.int32)
        z = zipf_keys(g, n, dom, float(g.uniform(0.8, 1.5)))
        return g.permutation(dom).astype(np.int32)[z] if dom <= 1 << 20 else z

    attrs = [[] for _ in range(n_rel)]
    data = [{} for _ in range(n_rel)]
    fk = [False] * n_rel
    for c in range(1, n_rel):
        p, k = parent[c], f"k{c}"
        if g.random() < 0.7:
            fk[c] = True
            attrs[c].append(_attr(k, "i32", rows[c], True))
            data[c][k] = np.arange(rows[c], dtype=np.int32)
            attrs[p].append(_attr(k, "i32", rows[c]))
            data[p][k] = values(rows[p], rows[c])
        else:
            # many-to-many: the parent refers to values the child holds
            dk = int(10 ** g.uniform(1, 4))
            attrs[c].append(_attr(k, "i32", dk))
            data[c][k] = values(rows[c], dk)
            held = np.unique(data[c][k])
            attrs[p].append(_attr(k, "i32", dk))
            data[p][k] = held[values(rows[p], len(held))]
    feats, owned = [], [[] for _ in range(n_rel)]
    for r in range(n_rel):
        for j in range(int(g.integers(1, 4))):
            a, dom = f"v{r}_{j}", int(10 ** g.uniform(1, 6))
            attrs[r].append(_attr(a, "i32", dom))
            data[r][a] = values(rows[r], dom)
            feats.append(a)
            owned[r].append(a)
    batch = [{"groupby": [a], "where": [], "aggs": [[]], "root": None} for a in feats]
    # pairs of attributes that one relation reaches through foreign keys (so
    # that every tuple of the join below it carries one value of each)
    closed = fk[:]   # the edge into c and every edge below c are foreign keys
    for c in range(n_rel - 1, 0, -1):
        closed[c] = fk[c] and all(closed[d] for d in range(c + 1, n_rel) if parent[d] == c)
    pairs = set()
    for _ in range(6):
        r = int(g.integers(0, n_rel))
        reach, stack = [r], [r]
        while stack:
            u = stack.pop()
            for c in range(1, n_rel):
                if parent[c] == u and closed[c]:
                    reach.append(c)
                    stack.append(c)
        cand = [a for u in reach for a in owned[u]]
        if len(cand) > 1:
            i, j = sorted(g.choice(len(cand), 2, replace=False).tolist())
            pairs.add((cand[i], cand[j]))
    batch += [{"groupby": [a, b], "where": [], "aggs": [[]], "root": None} for a, b in sorted(pairs)]
    names = [f"T{r}" for r in range(n_rel)]
    schema = [_rel(names[r], rows[r], attrs[r]) for r in range(n_rel)]
    return {"name": f"estimator_{shape}_{seed}", "schema": schema,
            "tree": [(parent[c], c) for c in range(1, n_rel)], "batch": batch,
            "data": {names[r]: data[r] for r in range(n_rel)}, "policy": "fact", "precision": "f32"}


def bench_workload(config: str, scale: float = 1.0) -> dict:
    """The measured workloads at their full sizes (``scale`` shrinks the fact
    relation): the relations, the batch, the arithmetic precision they run in,
    the hash-table sizing and a one-line description.  The benchmark and the
    full-size parity tests both build their inputs here, so both see the same
    data and the same launch configuration."""
    if config == "retail":
        problem = retail_snowflake(seed=0, n_inv=int(84_000_000 * scale))
        precision, sizing = "f32", "bound"
        workload = "retail-shaped snowflake (Inv 84M x 5 relations), covariance + 6 one-hot categoricals"
    elif config == "grocery":
        problem = grocery_star(seed=0, n_sales=int(120_000_000 * scale))
        precision, sizing = "bf16x3", "bound"
        workload = "grocery-shaped star (Sales 120M x 6 relations), covariance + 10 categoricals"
    elif config == "cart":
        problem = cart_node(seed=0, n_inv=int(84_000_000 * scale))
        precision, sizing = "f32", "bound"
        workload = ("CART node on the retail snowflake (Inv 84M): 840 thresholds + 7 "
                    "categorical group-bys x {SUM(1), SUM(y), SUM(y^2)} under a 3-condition path")
    elif config == "chain":
        n1 = int(50_000_000 * scale)
        problem = rkmeans_chain(seed=0, n1=n1, n2=max(1000, n1 // 10), n3=max(100, n1 // 250))
        precision, sizing = "f32", "learned"
        workload = ("Rk-means step 1 on a 3-relation chain (R1 50M, R2 5M, R3 200k; 100 "
                    "attributes, domains 10..1e6): SUM(1) by each attribute and 10 pairs")
    elif config == "tiny":
        problem = tiny_star(seed=0)
        precision, sizing = "f64", "bound"
        workload = "tiny star (S 100k x 3 relations), covariance grouped by cat"
    else:
        raise ValueError(f"unknown workload {config!r}")
    return {"problem": problem, "precision": precision, "sizing": sizing, "workload": workload}


def bench_plan_options(bw: dict, form: str = "fused", graph: bool = True) -> dict:
    """Plan options of a measured workload (``bench_workload``) as the
    benchmark runs it; the full-size parity tests use the same, so that they
    check the launch configuration that is timed."""
    p = bw["problem"]
    return {"precision": bw["precision"], "policy": p["policy"], "form": form, "sizing": bw["sizing"],
            "graph": graph}


def tagged_star(seed: int = 0, n_fact: int = 200_000, n_stores: int = 40, n_items: int = 3_000,
                dup_frac: float = 0.03, n_cat: int = 12):
    """Star S(store, item, units) with Stores(store, f1, f2), Items(item, g1,
    cat in [0, n_cat)) and Tags(item, tagw): every item has one tag and a
    fraction ``dup_frac`` of the items a second one, so the join multiplies a
    few fact rows by two.  Batch: COUNT, SUM(units), SUM(units*g1), SUM(f1),
    each ungrouped and grouped by cat, plus SUM(1) grouped by (store, cat)."""
    r_s, r_st, r_it, r_tg = _spawn(seed, 4)
    extra = np.sort(r_tg.choice(n_items, max(1, int(dup_frac * n_items)), replace=False)).astype(np.int32)
    tag_items = np.concatenate([np.arange(n_items, dtype=np.int32), extra])
    data = {
        "S": {"store": zipf_keys(r_s, n_fact, n_stores, 1.0), "item": zipf_keys(r_s, n_fact, n_items, 1.1),
              "units": r_s.lognormal(0.0, 1.0, n_fact)},
        "Stores": {"store": np.arange(n_stores, dtype=np.int32),
                   "f1": r_st.standard_normal(n_stores), "f2": r_st.standard_normal(n_stores)},
        "Items": {"item": np.arange(n_items, dtype=np.int32), "g1": r_it.standard_normal(n_items),
                  "cat": r_it.integers(0, n_cat, n_items).astype(np.int32)},
        "Tags": {"item": tag_items, "tagw": r_tg.standard_normal(len(tag_items))},
    }
    schema = [
        _rel("S", n_fact, [_attr("store", "i32", n_stores), _attr("item", "i32", n_items), _attr("units", "f64")]),
        _rel("Stores", n_stores, [_attr("store", "i32", n_stores, True), _attr("f1", "f64"), _attr("f2", "f64")]),
        _rel("Items", n_items, [_attr("item", "i32", n_items, True), _attr("g1", "f64"),
                                _attr("cat", "i32", n_cat)]),
        _rel("Tags", len(tag_items), [_attr("item", "i32", n_items), _attr("tagw", "f64")]),
    ]
    aggs = [[], [("units", 1)], [("units", 1), ("g1", 1)], [("f1", 1)]]
    batch = [{"groupby": [], "where": [], "aggs": aggs, "root": None},
             {"groupby": ["cat"], "where": [], "aggs": aggs, "root": None},
             {"groupby": ["store", "cat"], "where": [], "aggs": [[]], "root": None}]
    return {"name": "tagged_star", "schema": schema, "tree": [(0, 1), (0, 2), (0, 3)],
            "batch": batch, "data": data, "policy": "fact", "precision": "f64"}
