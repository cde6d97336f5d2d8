"""The memory and result model of the C ABI (``include/lmfao.h``):

* ``lmfao_prepare_in`` carves every device buffer of a prepared plan from a
  workspace the caller allocates with torch, sized by
  ``lmfao_prepared_workspace_bytes``; its results equal those of the
  library-allocated handle;
* ``lmfao_result_device`` gives each query's result compacted on the GPU
  (present groups in lexicographic key order) as device arrays, read here
  through torch without a copy, and equal to the oracle: dense tables, range
  queries and hash tables (sorted on the GPU);
* a workspace that is too small is refused with LMFAO_ENOMEM.
"""
import numpy as np
import pytest

import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu


def _device_result(prep, q):
    r = prep.result_device(q)
    return {k: v.cpu().numpy() for k, v in r.items()}


def test_workspace_from_torch_and_device_results():
    import torch
    import oracle
    import paper_2008_08657_amd as E
    p = W.retail_snowflake(seed=2, n_inv=150_000)
    plan = E.Plan(p, precision="f64", policy="fact")
    cols = E.device_columns(p)
    ref_prep = E.Prepared(plan, cols)
    need = ref_prep.workspace_bytes(with_results=True)
    assert need >= ref_prep.workspace_bytes(with_results=False) > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    prep = E.Prepared(plan, cols, workspace=ws)
    prep.run(sync=True)
    ref_prep.run(sync=True)
    base = ws.data_ptr()
    ref = oracle.evaluate(p)
    for q in range(len(p["batch"])):
        got = prep.result_device(q)
        for k in ("keys", "count", "sum"):
            if got[k].numel():
                assert base <= got[k].data_ptr() < base + need, f"query {q} {k} outside the workspace"
        g = {k: v.cpu().numpy() for k, v in got.items()}
        h = ref_prep.result(q)
        np.testing.assert_array_equal(g["keys"], h["keys"])
        np.testing.assert_array_equal(g["count"], h["count"])
        compare(g, ref[q], 1e-12, f"query {q}")


def test_too_small_workspace_is_refused():
    import torch
    import paper_2008_08657_amd as E
    p = W.tiny_star(seed=0, n_fact=5_000)
    plan = E.Plan(p, precision="f64", policy="fact")
    cols = E.device_columns(p)
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(E.LmfaoError) as ei:
        E.Prepared(plan, cols, workspace=ws)
    assert ei.value.status == 2   # LMFAO_ENOMEM


def test_device_results_of_hash_tables_and_ranges():
    import oracle
    import paper_2008_08657_amd as E
    # hashed pair outputs (key spaces past 2^24 cells) and dense tables
    p = W.rkmeans_chain(seed=3, n1=120_000, n2=12_000, n3=500, n_x=6, n_y=4, n_z=3)
    plan = E.Plan(p, precision="f32", policy="fact")
    prep = E.Prepared(plan, E.device_columns(p))
    prep.run(sync=True)
    ref = oracle.evaluate(p)
    hashed = 0
    for q in range(len(p["batch"])):
        g = _device_result(prep, q)
        compare(g, ref[q], 1e-5, f"chain query {q}")
        hashed += int(np.prod([p["domains"][a] for a in p["batch"][q]["groupby"]]) > (1 << 24))
    assert hashed >= 1
    # range conditions (CART candidates) come out of finalised bucket sums
    c = W.cart_node(seed=0, n_inv=60_000, n_thr=4)
    plan = E.Plan(c, precision="f64", policy="fact")
    prep = E.Prepared(plan, E.device_columns(c))
    prep.run(sync=True)
    ref = oracle.evaluate(c, list(range(0, len(c["batch"]), 7)))
    for i, q in enumerate(range(0, len(c["batch"]), 7)):
        compare(_device_result(prep, q), ref[i], 1e-12, f"cart query {q}")
