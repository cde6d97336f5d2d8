"""User-defined factors on the GPU (section 2 of the paper, the example's
query SUM(g(item) * h(date))): functions of one attribute, tabulated by the
caller, gathered into a column at prepare time and then planned like any
continuous factor; every query equals the oracle's, in FP64 and FP32."""
import pytest

import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_udf_factors_match_oracle(precision, tol):
    import oracle
    import paper_2008_08657_amd as E
    p = W.udf_grocery(seed=1, n_sales=150_000)
    plan = E.Plan(p, precision=precision, policy="fact")
    prep = E.Prepared(plan, E.device_columns(p))
    prep.run(sync=True)
    ref = oracle.evaluate(p)
    for q in range(len(p["batch"])):
        compare(prep.result(q), ref[q], tol, f"{precision} query {q}")
