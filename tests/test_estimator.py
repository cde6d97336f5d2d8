"""Host side of the group-count estimator: the weights blob, its validation by
lmfao_plan, and the host evaluation of the network against the FP64 oracle
of the same network."""
import numpy as np
import pytest

from oracle import mlp
import paper_2008_08657_amd as lm
from paper_2008_08657_amd import estimator as est
import workloads as W


def _blob(h=8, seed=0, margin=0.5):
    g = np.random.default_rng(seed)
    mean = g.standard_normal(est.D).astype(np.float32)
    std = (0.5 + g.random(est.D)).astype(np.float32)
    params = mlp.flatten(mlp.init(est.D, h, seed=seed + 1)).astype(np.float32)
    return est.pack(mean, std, params, h, margin), mean, std, params


def test_feature_count_matches_header():
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "lmfao.h")).read()
    assert f"#define LMFAO_EST_FEATURES {est.D}" in hdr


def test_host_network_matches_oracle():
    blob, mean, std, params = _blob()
    X = np.random.default_rng(3).standard_normal((50, est.D)).astype(np.float32) * 3
    y = est._predict_host(blob, X)
    p = mlp.unflatten(params.astype(np.float64), est.D, 8)
    yo, _ = mlp.forward(p, (X.astype(np.float64) - mean) / std)
    np.testing.assert_allclose(y, X[:, est.BOUND] - yo, rtol=1e-4, atol=1e-4)


def test_weights_file_round_trip(tmp_path):
    blob, mean, std, params = _blob(h=4)
    path = str(tmp_path / "w.json")
    est.save(path, mean, std, params, 4, 0.5, {"note": "test"})
    np.testing.assert_array_equal(est.load(path), blob)


def test_weights_for_another_layout_are_rejected(tmp_path):
    import json
    blob, mean, std, params = _blob(h=4)
    path = str(tmp_path / "w.json")
    est.save(path, mean, std, params, 4, 0.5, {})
    doc = json.load(open(path))
    doc["features"] = doc["features"][::-1]
    json.dump(doc, open(path, "w"))
    with pytest.raises(ValueError):
        est.load(path)


def test_plan_validates_the_blob():
    p = W.estimator_workload(1, max_rows=20_000)
    blob, *_ = _blob(h=8)
    lm.Plan(p, precision="f32", sizing="learned", estimator=blob)
    with pytest.raises(lm.LmfaoError):
        lm.Plan(p, precision="f32", sizing="learned", estimator=blob[:-1])
    bad = blob.copy()
    bad[1] = est.D + 1
    with pytest.raises(lm.LmfaoError):
        lm.Plan(p, precision="f32", sizing="learned", estimator=bad)


def test_corpus_workloads_are_seeded_and_valid():
    a = W.estimator_workload(7, max_rows=30_000)
    b = W.estimator_workload(7, max_rows=30_000)
    assert a["name"] == b["name"]
    for r in a["schema"]:
        for at in r["attrs"]:
            x = a["data"][r["name"]][at["name"]]
            np.testing.assert_array_equal(x, b["data"][r["name"]][at["name"]])
            assert x.min() >= 0 and x.max() < at["domain"]
            if at["key"]:
                assert len(np.unique(x)) == len(x)
    lm.Plan(a, precision="f32")
