"""Pins of the Rk-means oracle (``oracle/rkmeans.py``; section 3 of the
paper, Rk-means steps 2 and 3):

* the 1-D weighted k-means equals scikit-learn's Lloyd k-means started from
  the same centroids, with the weights as sample weights;
* weights act as multiplicities: integer weights equal replicating the values;
* k at least the number of values puts every value in a cluster of its own
  (zero cost), and two far-apart groups give their weighted means;
* at the fixed point every centroid is the weighted mean of its values and
  every value is nearest to its own centroid (checked with plain loops);
* the grid coreset's weights sum to |D| and equal a brute-force count over
  the tuples of D.
"""
import numpy as np
import pytest

import oracle
import oracle.rkmeans as rk
import workloads as W


@pytest.mark.parametrize("seed", range(5))
def test_kmeans_1d_equals_sklearn_lloyd(seed):
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(seed)
    m = int(rng.integers(20, 200))
    v = np.sort(rng.choice(10_000, m, replace=False)).astype(np.float64)
    w = rng.integers(1, 50, m).astype(np.float64)
    k = int(rng.integers(2, 8))
    c, a, steps = rk.kmeans_1d(v, w, k, max_iter=300)
    init = rk.initial_centroids(v, w, k)
    ref = KMeans(n_clusters=k, init=init.reshape(-1, 1), n_init=1, algorithm="lloyd", max_iter=300, tol=0.0)
    ref.fit(v.reshape(-1, 1), sample_weight=w)
    np.testing.assert_allclose(np.sort(c), np.sort(ref.cluster_centers_.ravel()), rtol=1e-12, atol=1e-9)


def test_weights_are_multiplicities():
    rng = np.random.default_rng(3)
    v = np.sort(rng.choice(1000, 60, replace=False)).astype(np.float64)
    w = rng.integers(1, 6, 60)
    c1, _, _ = rk.kmeans_1d(v, w, 4)
    rep = np.repeat(v, w)
    # the replicated list has duplicates; merge them back into weights
    u, cnt = np.unique(rep, return_counts=True)
    c2, _, _ = rk.kmeans_1d(u, cnt, 4)
    np.testing.assert_array_equal(c1, c2)


def test_closed_forms():
    v = np.array([1.0, 2.0, 5.0, 9.0])
    c, a, _ = rk.kmeans_1d(v, np.ones(4), 4)
    assert sorted(c) == [1.0, 2.0, 5.0, 9.0] and len(set(a)) == 4
    # two groups far apart: the weighted means
    v = np.array([0.0, 1.0, 2.0, 100.0, 101.0])
    w = np.array([1.0, 2.0, 1.0, 3.0, 1.0])
    c, a, _ = rk.kmeans_1d(v, w, 2)
    assert c[0] == pytest.approx((0 + 2 + 2) / 4.0) and c[1] == pytest.approx((300 + 101) / 4.0)
    assert list(a) == [0, 0, 0, 1, 1]


def test_fixed_point_property():
    rng = np.random.default_rng(9)
    v = np.sort(rng.normal(size=300))
    w = rng.uniform(0.5, 3.0, 300)
    c, a, steps = rk.kmeans_1d(v, w, 6, max_iter=1000)
    assert steps < 1000
    for i in range(6):
        num = sum(w[j] * v[j] for j in range(300) if a[j] == i)
        den = sum(w[j] for j in range(300) if a[j] == i)
        if den:
            assert c[i] == pytest.approx(num / den, rel=1e-12, abs=1e-12)
    for j in range(300):
        best = min(range(6), key=lambda i: (abs(v[j] - c[i]), i))
        assert a[j] == best


def test_grid_coreset_counts_tuples():
    p = W.rkmeans_chain(seed=2, n1=3000, n2=300, n3=40, n_x=3, n_y=2, n_z=2, max_dom=50)
    rng = np.random.default_rng(0)
    clusters = {a: rng.integers(0, 3, p["domains"][a]) for a in ("x1", "x2", "y1", "z2")}
    keys, wts = rk.grid_coreset(p, clusters)
    assert wts.sum() == 3000
    D = oracle.materialize_join(p, list(clusters))
    brute = {}
    for t in range(len(D["x1"])):
        g = tuple(int(clusters[a][D[a][t]]) for a in clusters)
        brute[g] = brute.get(g, 0) + 1
    assert sorted(brute) == [tuple(k) for k in keys]
    assert [brute[tuple(k)] for k in keys] == list(wts)
