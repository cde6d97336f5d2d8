"""Pins of the streaming tier-B oracle (``oracle/tierb.c``) against the
tier-A oracle, which materialises the join and sums in 80-bit precision, and
against brute force and closed forms.

Tier B enumerates the tuples of D by nested loops along the join tree and
never builds D, so agreement on many-to-many joins with dangling tuples,
multi-attribute keys, conditions on every operator and large key spaces
(the open-addressing path) ties both implementations of the same definition
together.  Counts and keys are compared exactly; sums within 1e-12 of the
larger of |value| and 1e-3 * sum |terms|.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import tierb

from parity import compare_all


def agree(problem, **kw):
    a = oracle.evaluate(problem)
    b = tierb.evaluate(problem, **kw)
    assert len(a) == len(b)
    compare_all(b, a, 1e-12, problem.get("name", ""))
    for x, y in zip(a, b):
        np.testing.assert_allclose(y["abs"], x["abs"], rtol=1e-12, atol=1e-300)
    return b


@pytest.mark.parametrize("seed", range(10))
def test_random_many_to_many_with_dangling(seed):
    agree(W.random_acyclic(seed, n_rel=3 + seed % 3, max_rows=30, max_dom=4))


@pytest.mark.parametrize("seed", range(4))
def test_random_foreign_keys(seed):
    agree(W.random_acyclic(50 + seed, n_rel=5, max_rows=40, max_dom=6, unique_dims=True))


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_thread_counts_agree(threads):
    agree(W.tiny_star(seed=1, n_fact=20_000), threads=threads)


def test_worked_example_and_tagged_star():
    agree(W.favorita_example(0, n_sales=300))
    agree(W.tagged_star(seed=2, n_fact=20_000))


def test_every_operator_and_float32_conditions():
    p = W.cart_node(seed=2, n_inv=20_000)
    agree(p)


def test_retail_small():
    agree(W.retail_snowflake(seed=1, n_inv=30_000))


def test_large_key_spaces_use_the_map():
    # pair group-bys whose key space passes 2^24 cells go to the
    # open-addressing map; single attributes above 16k cells are owned by one
    # thread with a dense array
    p = W.rkmeans_chain(seed=4, n1=20_000, n2=2_000, n3=200, max_dom=100_000)
    agree(p)


def test_root_choice_does_not_matter():
    p = W.random_acyclic(7, n_rel=4, max_rows=25, max_dom=3)
    ref = oracle.evaluate(p)
    for r in range(len(p["schema"])):
        compare_all(tierb.evaluate(p, root=r), ref, 1e-12, f"root {r}")


def test_root_rows_prefix_equals_fact_prefix():
    p = W.tiny_star(seed=3, n_fact=10_000)
    got = tierb.evaluate(p, root="S", root_rows=2_500)
    ref = oracle.evaluate(W.fact_prefix(p, "S", 2_500))
    compare_all(got, ref, 1e-12, "prefix")


def test_closed_form_count_many_to_many():
    # two relations sharing one key value: COUNT = n * m
    n, m = 300, 200
    p = {"schema": [{"name": "A", "n_rows": n, "attrs": [{"name": "k", "dtype": "i32", "domain": 1, "key": False}]},
                    {"name": "B", "n_rows": m, "attrs": [{"name": "k", "dtype": "i32", "domain": 1, "key": False}]}],
         "tree": [(0, 1)], "data": {"A": {"k": np.zeros(n, np.int32)}, "B": {"k": np.zeros(m, np.int32)}},
         "batch": [{"groupby": [], "where": [], "aggs": [[]], "root": None}]}
    r = tierb.evaluate(p)[0]
    assert r["count"].tolist() == [n * m]
    assert r["sum"][0, 0] == n * m
