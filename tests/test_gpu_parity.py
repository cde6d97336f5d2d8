"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case runs the whole batch on the GPU and compares every query result
with the oracle, element by element (keys and counts exact, floats within the
tolerance of ``tests/parity.py``).  Sizes span several pieces and work items
and a ragged tail; the factorized scan is forced on small relations through
``row_piece_max=-1`` and shallow cut levels through ``min_segment``.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from parity import compare_all

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2008_08657_amd as E
    E.load_library()
    return E


def run_engine(E, problem, **kw):
    plan = E.Plan(problem, **kw)
    cols = E.device_columns(problem)
    prep = E.Prepared(plan, cols)
    prep.run(sync=True)
    res = prep.results()
    return plan, prep, res


def check(E, problem, tol, name, allow_unsupported=False, **kw):
    print(f"[case] {name} {kw}", flush=True)
    try:
        plan, prep, res = run_engine(E, problem, **kw)
    except E.LmfaoError as e:
        if allow_unsupported and e.status == 4:
            print(f"[case] {name}: outside the supported class ({e})", flush=True)
            return None, None
        raise
    ref = oracle.evaluate(problem)
    return compare_all(res, ref, tol, name), plan


def test_worked_example(eng):
    p = W.favorita_example(0, n_sales=200)
    worst, plan = check(eng, p, F64_TOL, "favorita_example", policy="groupby")
    d = plan.describe()
    assert len(d["groups"]) == 7


def test_worked_example_forced_scan(eng):
    p = W.favorita_example(1, n_sales=5_000)
    check(eng, p, F64_TOL, "favorita_scan", policy="groupby", row_piece_max=-1, min_segment=1)


@pytest.mark.parametrize("policy", ["fact", "groupby"])
def test_tiny_star_rows(eng, policy):
    p = W.tiny_star(seed=0, n_fact=30_000)
    check(eng, p, F64_TOL, "tiny_star_rows", policy=policy)


@pytest.mark.parametrize("min_segment", [1, 10_000_000])
def test_tiny_star_scan(eng, min_segment):
    # min_segment=1 cuts at the item level (pieces = item segments);
    # a huge min_segment cuts at level 0 (pieces = fixed-size chunks)
    p = W.tiny_star(seed=1, n_fact=50_001)
    check(eng, p, F64_TOL, "tiny_star_scan", policy="fact", row_piece_max=-1, min_segment=min_segment)


@pytest.mark.parametrize("contraction", ["mfma", "valu"])
def test_tiny_star_full_size(eng, contraction):
    # the 100k-row tiny star configuration, seed 0, FP64, in the bench's launch configuration
    p = W.tiny_star(seed=0)
    check(eng, p, F64_TOL, "tiny_star_full", policy="fact", row_piece_max=-1, min_segment=1,
          contraction=contraction)


@pytest.mark.parametrize("seed", range(6))
def test_random_foreign_keys(eng, seed):
    p = W.random_acyclic(200 + seed, n_rel=4, max_rows=400, max_dom=30, unique_dims=True, n_queries=6)
    # the fact heuristic keeps every group-by single-valued, so it always plans
    check(eng, p, F64_TOL, f"random_fk_{seed}_fact", policy="fact")
    check(eng, p, F64_TOL, f"random_fk_{seed}_fact_scan", policy="fact", row_piece_max=-1, min_segment=1)
    # the group-by heuristic may carry a group-by through a multi-valued view
    check(eng, p, F64_TOL, f"random_fk_{seed}_groupby", allow_unsupported=True, policy="groupby")
    check(eng, p, F64_TOL, f"random_fk_{seed}_groupby_scan", allow_unsupported=True, policy="groupby",
          row_piece_max=-1, min_segment=1)


@pytest.mark.parametrize("seed", range(6))
def test_random_many_to_many(eng, seed):
    p = W.random_acyclic(300 + seed, n_rel=3, max_rows=300, max_dom=20, n_queries=6)
    # group-bys only on the root's own attributes keep every view keyed by join attributes
    p["batch"] = [dict(q, groupby=[g for g in q["groupby"] if g == "c0"], root="R0") for q in p["batch"]]
    check(eng, p, F64_TOL, f"random_m2m_{seed}", policy="groupby")
    check(eng, p, F64_TOL, f"random_m2m_{seed}_scan", policy="groupby", row_piece_max=-1, min_segment=1)
    check(eng, p, F64_TOL, f"random_m2m_{seed}_valu", policy="groupby", contraction="valu")


@pytest.mark.parametrize("contraction", ["mfma", "valu"])
def test_retail_snowflake_small(eng, contraction):
    p = W.retail_snowflake(seed=0, n_inv=300_007, n_locn=60, n_dates=20, n_ksn=400,
                           n_weather_dates=30)
    check(eng, p, F32_TOL, "retail_small_f32", precision="f32", policy="fact", row_piece_max=5_000,
          min_segment=16, contraction=contraction)


def test_retail_snowflake_small_f64(eng):
    p = W.retail_snowflake(seed=1, n_inv=120_000, n_locn=40, n_dates=12, n_ksn=300,
                           n_weather_dates=15, dtype="f64")
    check(eng, p, F64_TOL, "retail_small_f64", precision="f64", policy="fact", row_piece_max=5_000,
          min_segment=16)


def test_grocery_star_small(eng):
    p = W.grocery_star(seed=0, n_sales=200_003, n_stores=9, n_items=300, n_dates=80, n_oil=60,
                       n_hol=30)
    check(eng, p, F32_TOL, "grocery_small_f32", precision="f32", policy="fact", row_piece_max=5_000,
          min_segment=16)


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x2"])
@pytest.mark.parametrize("shape", ["grocery", "retail"])
def test_bf16_split_contraction(eng, shape, precision):
    # float tiles of the contraction on the bf16 matrix cores, integer cells
    # exact.  BF16x3 (three parts, six products) meets the FP32 tolerance.
    # BF16x2 (two parts, three products) leaves out terms of about 2^-17 of
    # each product: 1e-5 relative where the sum does not cancel, and 2^-16 of
    # the sum of the terms' magnitudes everywhere
    if shape == "grocery":
        p = W.grocery_star(seed=3, n_sales=200_003, n_stores=9, n_items=300, n_dates=80, n_oil=60, n_hol=30)
    else:
        p = W.retail_snowflake(seed=4, n_inv=120_001, n_locn=40, n_dates=12, n_ksn=300, n_weather_dates=14)
    print(f"[case] {shape} {precision}", flush=True)
    plan, prep, res = run_engine(eng, p, precision=precision, policy="fact", row_piece_max=5_000, min_segment=16)
    ref = oracle.evaluate(p)
    if precision == "bf16x3":
        worst = compare_all(res, ref, F32_TOL, f"{shape}_{precision}")
    else:
        worst = compare_all(res, ref, 2.0 ** -16, f"{shape}_{precision}", floor=1.0)
        rel = [float(np.max(np.abs(g["sum"] - r["sum"]) / np.maximum(np.abs(r["sum"]), 1e-300)))
               for g, r in zip(res, ref) if r["sum"].size and np.all(r["sum"] != 0)]
        print(f"[{precision}] {shape}: worst error / sum|terms| {worst:.3e}; worst plain relative "
              f"{max(rel):.3e}", flush=True)
    print(f"[{precision}] {shape}: worst scaled error {worst:.3e}", flush=True)


def test_bf16x3_needs_matrix_cores(eng):
    p = W.tiny_star(seed=0, n_fact=1_000)
    with pytest.raises(eng.LmfaoError):
        eng.Plan(p, precision="bf16x3", contraction="valu")
    with pytest.raises(eng.LmfaoError):
        eng.Plan(p, precision="bf16x2", contraction="valu")


@pytest.mark.parametrize("shape", ["retail", "chain"])
def test_graph_replay(eng, shape):
    # the run captured into a HIP graph and replayed several times, with eager
    # runs and other device work between the replays; every replay is checked
    import torch
    if shape == "retail":
        p = W.retail_snowflake(seed=5, n_inv=60_001, n_locn=30, n_dates=10, n_ksn=200, n_weather_dates=12)
        kw = dict(row_piece_max=5_000, min_segment=16)
    else:
        p = W.rkmeans_chain(seed=6, n1=40_000, n2=4_000, n3=400, n_x=6, n_y=5, n_z=5, max_dom=1_000_000)
        kw = {}
    print(f"[case] graph replay {shape}", flush=True)
    plan = eng.Plan(p, precision="f32", policy="fact", graph=True, **kw)
    prep = eng.Prepared(plan, eng.device_columns(p))
    ref = oracle.evaluate(p)
    prep.run(sync=True)
    compare_all(prep.results(), ref, F32_TOL, f"{shape} eager")
    for i in range(3):
        prep.run(sync=False)
        torch.cuda.synchronize()
        compare_all(prep.results(), ref, F32_TOL, f"{shape} replay {i}")
        x = torch.arange(4096, device="cuda", dtype=torch.float32)
        assert float((x * 2).sum().item()) == 4095 * 4096.0
        prep.run(sync=True)
        compare_all(prep.results(), ref, F32_TOL, f"{shape} eager {i}")
    d = prep.describe()
    assert d["graph"]["failed"] == 0 and d["graph"]["captured"] == 1


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_direct_tables_with_values(eng, precision):
    # per-key sums grouped by a key too large for a per-piece histogram
    # (item, 3,000 values) are direct tables with value components (SUM(1),
    # SUM(units), SUM(units^2), SUM(units*g1)) written by the generated scan,
    # values summed in FP64 over runs of equal keys
    p = W.tiny_star(seed=7, n_fact=120_001, n_stores=40, n_items=3_000)
    p["batch"] = [{"groupby": ["item"], "where": [], "root": None,
                   "aggs": [[], [("units", 1)], [("units", 2)], [("units", 1), ("g1", 1)]]},
                  {"groupby": ["store"], "where": [], "root": None, "aggs": [[], [("units", 1)]]},
                  {"groupby": ["cat"], "where": [], "root": None, "aggs": [[("units", 1)], [("f1", 1)]]}]
    if precision == "f32":
        for r in p["schema"]:
            for a in r["attrs"]:
                if a["dtype"] == "f64":
                    a["dtype"] = "f32"
                    p["data"][r["name"]][a["name"]] = p["data"][r["name"]][a["name"]].astype(np.float32)
    # store outer, item inner: the item group-by is a table written by the scan
    plan, prep, res = run_engine(eng, p, precision=precision, policy="fact", row_piece_max=-1, min_segment=16,
                                 order={"S": ["store", "item"]})
    d = prep.describe()
    scans = [(s["name"], s["lean"]) for s in d["steps"] if s["kind"] == "scan"]
    print(f"[case] tables with values {precision}: scans {scans}", flush=True)
    assert any(lean == 2 for _, lean in scans), "the scan with value tables was not generated"
    compare_all(res, oracle.evaluate(p), F64_TOL if precision == "f64" else F32_TOL, f"tables_{precision}")


def test_repeat_runs_identical_counts(eng):
    p = W.tiny_star(seed=2, n_fact=40_000)
    plan = eng.Plan(p, policy="fact", row_piece_max=-1, min_segment=1)
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run()
    a = prep.results()
    prep.run()
    b = prep.results()
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x["keys"], y["keys"])
        np.testing.assert_array_equal(x["count"], y["count"])


def _with_conditions(p, seed):
    """A batch-wide filter (one condition per relation feature) plus one private
    condition per query, of every operator."""
    rng = np.random.default_rng(seed)
    n_rel = len(p["schema"])
    shared = [(f"x{i}", "<=" if i % 2 else ">", float(rng.normal(0, 0.8))) for i in range(1, n_rel)]
    shared.append(("c0", "!=", int(rng.integers(0, 3))))
    ops = ["<=", "<", ">", ">=", "==", "!="]
    out = []
    for k, q in enumerate(p["batch"]):
        if len(q["groupby"]) > 1:
            q = dict(q, groupby=q["groupby"][:1])
        op = ops[k % len(ops)]
        i = int(rng.integers(0, n_rel))
        if op in ("==", "!="):
            attr, const = f"c{i}", int(rng.integers(0, 3))
        else:
            attr, const = f"x{i}", float(rng.normal(0, 1))
        if attr in q["groupby"]:
            attr, const, op = f"x{i}", float(rng.normal(0, 1)), "<="
        out.append(dict(q, where=shared + [(attr, op, const)]))
        out.append(dict(q, where=list(shared)))
    p["batch"] = out
    return p


@pytest.mark.parametrize("seed", range(4))
def test_random_conditions(eng, seed):
    p = _with_conditions(W.random_acyclic(500 + seed, n_rel=3, max_rows=400, max_dom=25, unique_dims=True,
                                          n_queries=6), seed)
    check(eng, p, F64_TOL, f"random_cond_{seed}", policy="fact")
    # two inner group-by codes next to outer factors are outside the planned class at some seeds
    check(eng, p, F64_TOL, f"random_cond_{seed}_scan", allow_unsupported=True, policy="fact", row_piece_max=-1,
          min_segment=1)


def test_cart_node_rows(eng):
    # node condition as a filter, 840 thresholds as bucket group-bys; Inv small enough for row pieces
    p = W.cart_node(seed=0, n_inv=20_000, n_locn=40, n_dates=12, n_ksn=300, n_weather_dates=15)
    check(eng, p, F32_TOL, "cart_rows_f32", precision="f32", policy="fact")


def test_cart_node_scan(eng):
    p = W.cart_node(seed=1, n_inv=150_001, n_locn=50, n_dates=16, n_ksn=400, n_weather_dates=20)
    check(eng, p, F32_TOL, "cart_scan_f32", precision="f32", policy="fact", row_piece_max=5_000, min_segment=16)


@pytest.mark.parametrize("form", ["fused", "per_view"])
def test_forms_agree(eng, form):
    # the plain per-view form (one pass per output) and the fused form give the same results
    p = W.retail_snowflake(seed=2, n_inv=80_000, n_locn=30, n_dates=10, n_ksn=250, n_weather_dates=12)
    p["batch"] = p["batch"][::7]
    check(eng, p, F32_TOL, f"retail_{form}", precision="f32", policy="fact", form=form, row_piece_max=5_000,
          min_segment=16)


def test_rkmeans_chain_wide(eng):
    # 64 attributes over three relations, all scanned (row pieces only below
    # 5,000 rows): groups split to fit the scan kernels, cross pairs with a
    # large outer key evaluated row by row, hashed pairs in groups of their own
    p = W.rkmeans_chain(seed=3, n1=150_000, n2=80_000, n3=70_000, n_x=24, n_y=20, n_z=20, max_dom=30_000)
    print("[case] rkmeans wide", flush=True)
    plan = eng.Plan(p, precision="f32", policy="fact", row_piece_max=5_000, min_segment=16)
    assert len(plan.describe()["groups"]) > 3
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    compare_all(prep.results(), oracle.evaluate(p), F32_TOL, "rkmeans_wide")


def test_rkmeans_chain_large_domains(eng):
    # count tables over domains up to 10^6 (counted by radix partition; the
    # R1 groups are scanned, not evaluated row by row)
    p = W.rkmeans_chain(seed=8, n1=150_000, n2=80_000, n3=70_000, n_x=6, n_y=5, n_z=5, max_dom=1_000_000)
    print("[case] rkmeans large domains", flush=True)
    plan = eng.Plan(p, precision="f32", policy="fact", row_piece_max=5_000, min_segment=16)
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    kinds = {s["kind"] for s in prep.describe()["steps"]}
    assert "scan" in kinds
    compare_all(prep.results(), oracle.evaluate(p), F32_TOL, "rkmeans_large_domains")


@pytest.mark.parametrize("seed, max_dom", [(11, 20_000), (12, 1_000_000)])
def test_weighted_partition_count(eng, seed, max_dom):
    # SUM(1) group-bys rooted at R2 and R3 count each row with the count of
    # R1 tuples per key b carried by the view into it (about 65 per key):
    # the partition count multiplies rows by those counts, in tables of one
    # slice (domains up to 20,000), of several (up to 10^6), and hashed
    # (pairs past 2^24 cells)
    p = W.rkmeans_chain(seed=seed, n1=400_000, n2=6_000, n3=500, n_x=4, n_y=6, n_z=6, max_dom=max_dom)
    print(f"[case] weighted partition seed {seed} max_dom {max_dom}", flush=True)
    plan = eng.Plan(p, precision="f32", policy="fact")
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    names = [s["name"] for s in prep.describe()["steps"]]
    assert any(":R2:part_" in n for n in names) and any(":R3:part_" in n for n in names), names
    if max_dom > 1 << 15:
        assert any(":R2:part_slices" in n for n in names), names
        # pairs of R2 (R3) attributes past 2^24 cells: weighted hashed tables
        hashed = [p["batch"][h["query"]]["groupby"] for h in prep.describe()["hash_tables"]]
        assert any(all(a[0] in "yz" for a in g) for g in hashed), hashed
    compare_all(prep.results(), oracle.evaluate(p), F32_TOL, f"weighted_partition_{seed}")


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("hash_slots", [0, 1024])
def test_rkmeans_chain(eng, seed, hash_slots):
    # step 1 of Rk-means: SUM(1) grouped by each attribute and by pairs; pairs whose key
    # space is too large for a dense table go to hash tables (sized small on purpose
    # in the second case, so that the run must grow them and repeat)
    p = W.rkmeans_chain(seed=seed, n1=30_000, n2=3_000, n3=300, n_x=8, n_y=6, n_z=6, max_dom=30_000)
    print(f"[case] rkmeans seed {seed} hash_slots {hash_slots}", flush=True)
    plan = eng.Plan(p, precision="f32", policy="fact", hash_slots=hash_slots)
    prep = eng.Prepared(plan, eng.device_columns(p))
    prep.run(sync=True)
    res = prep.results()
    compare_all(res, oracle.evaluate(p), F32_TOL, f"rkmeans_{seed}_{hash_slots}")
    d = prep.describe()
    assert len(d["hash_tables"]) >= 1
    if hash_slots:
        assert d["hash_regrowths"] >= 1
    # a second run reuses the grown tables and gives the same groups
    prep.run(sync=True)
    again = prep.results()
    for x, y in zip(res, again):
        np.testing.assert_array_equal(x["keys"], y["keys"])
        np.testing.assert_array_equal(x["count"], y["count"])


@pytest.mark.parametrize("n_weather_dates, precision", [(300, "f32"), (300, "f64"), (7, "f32")])
def test_view_build_large_and_small_relations(eng, n_weather_dates, precision):
    # Weather over 260 x n_weather_dates (locn, date) keys: 78,000 rows take
    # the thread-per-row view build (16-byte stores of 8 values and 2 codes),
    # 1,820 the thread-per-element one
    p = W.retail_snowflake(seed=9, n_inv=150_001, n_locn=260, n_dates=min(12, n_weather_dates),
                           n_ksn=300, n_weather_dates=n_weather_dates)
    check(eng, p, F32_TOL if precision == "f32" else F64_TOL,
          f"view build, Weather {260 * n_weather_dates} rows, {precision}", precision=precision, policy="fact")


def test_register_histograms_with_multiplicities(eng):
    # a few items carry two tags: inside the scan some rows weigh cat's
    # register histogram with a multiplicity of 2.  Register histograms need
    # pieces of 64 rows or more on average: FP32, and more than 16384 * 64
    # rows so that the work items grow past one chunk.
    p = W.tagged_star(seed=4, n_fact=2_500_000)
    ref = oracle.evaluate(p)
    for order in ({"S": ["store", "item"]}, None):
        print(f"[case] tagged star, order {order}", flush=True)
        _, prep, res = run_engine(eng, p, precision="f32", policy="fact", order=order)
        compare_all(res, ref, F32_TOL, f"tagged star {order}")
        if order is not None:
            assert any(" rh0_0 = 0;" in src for src in prep.kernel_sources())


def _tiny_star_variant(n_fact, seed=11):
    return W.tiny_star(seed=seed, n_fact=n_fact, n_stores=7, n_items=90)


@pytest.mark.parametrize("n_fact", [1, 63, 64, 65, 4097])
def test_ragged_sizes(eng, n_fact):
    # one row, one row short of a 64-row chunk, exactly one chunk, one row
    # past it, one row past a 4,096-row work item
    p = _tiny_star_variant(n_fact)
    check(eng, p, F64_TOL, f"ragged {n_fact}", policy="fact")
    check(eng, p, F64_TOL, f"ragged {n_fact} scan", policy="fact", row_piece_max=-1, min_segment=1)


def test_empty_join(eng):
    # Items holds one item that no fact row uses: the join is empty, and every
    # query has no group (the ungrouped ones no row either)
    p = _tiny_star_variant(3_000)
    p["data"]["Items"] = {"item": np.array([89], np.int32), "g1": np.array([0.5]), "g2": np.array([-1.0]),
                          "g3": np.array([2.0]), "cat": np.array([3], np.int32)}
    p["schema"][2]["n_rows"] = 1
    p["data"]["S"]["item"] = np.minimum(p["data"]["S"]["item"], 88).astype(np.int32)
    ref = oracle.evaluate(p)
    assert all(r["keys"].shape[0] == 0 for r in ref)
    check(eng, p, F64_TOL, "empty join", policy="fact")
    check(eng, p, F64_TOL, "empty join scan", policy="fact", row_piece_max=-1, min_segment=1)


def test_filter_selects_nothing(eng):
    p = _tiny_star_variant(5_000)
    p["batch"] = [dict(q, where=[("units", "<", -1.0)]) for q in p["batch"][:6]] + p["batch"][:2]
    ref = oracle.evaluate(p)
    assert all(r["keys"].shape[0] == 0 for r in ref[:6])
    check(eng, p, F64_TOL, "filter selects nothing", policy="fact")


def test_dangling_keys(eng):
    # half of the items are missing from Items: their fact rows drop out
    p = _tiny_star_variant(20_000)
    keep = p["data"]["Items"]["item"] % 2 == 0
    p["data"]["Items"] = {k: v[keep] for k, v in p["data"]["Items"].items()}
    p["schema"][2]["n_rows"] = int(keep.sum())
    ref = oracle.evaluate(p)
    assert 0 < int(ref[0]["count"][0]) < 20_000
    check(eng, p, F64_TOL, "dangling keys", policy="fact")
    check(eng, p, F64_TOL, "dangling keys scan", policy="fact", row_piece_max=-1, min_segment=1)


@pytest.mark.parametrize("which", ["tiny", "grocery", "random8", "random9"])
def test_root_cost_policy_matches_oracle(which):
    # roots chosen by the cost model give the oracle's results
    import paper_2008_08657_amd as E
    p = {"tiny": lambda: W.tiny_star(seed=2, n_fact=50_000),
         "grocery": lambda: W.grocery_star(seed=1, n_sales=150_000),
         "random8": lambda: W.random_acyclic(8), "random9": lambda: W.random_acyclic(9)}[which]()
    prec, tol = ("f64", 1e-12) if which != "grocery" else ("f32", 1e-5)
    plan = E.Plan(p, precision=prec, policy="cost")
    prep = E.Prepared(plan, E.device_columns(p))
    prep.run(sync=True)
    ref = oracle.evaluate(p)
    compare_all([prep.result(q) for q in range(len(p["batch"]))], ref, tol, which)
