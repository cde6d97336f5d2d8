"""Rk-means steps 2 and 3 (section 3 of the paper, "Rk-means").

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` may import this module; the GPU
library never calls it and shares no code with it.

Step 1 (one SUM(1) GROUP BY X_j query per attribute) is the ordinary batch
of the main oracle.  Step 2 clusters each projection pi_{X_j}(D), a list of
distinct values with their weights (the step-1 counts), into k clusters by
weighted k-means; the paper leaves the algorithm open, and the one taken here
(also stated in the library's header) is Lloyd's algorithm in FP64:

* start: centroid i (i = 0 .. k-1) is the first value, in ascending order,
  whose cumulative weight reaches (2i + 1) / (2k) of the total weight;
* assignment: every value goes to its nearest centroid, the lowest index on
  a tie;
* update: every centroid becomes the weighted mean of its values (a centroid
  with none keeps its place);
* stop when an assignment step changes nothing, or after ``max_iter``
  update steps.

The assignment relation A_j maps each value to its centroid's index.  Step 3
is the plain definition of the grid-coreset query, SELECT C_1, ..., C_n,
SUM(1) FROM D JOIN A_1 ... JOIN A_n GROUP BY C_1, ..., C_n: the natural join
is materialised, every tuple's cluster ids looked up, and the tuples grouped
by the id vector.
"""
from __future__ import annotations

import numpy as np

from . import materialize_join

__all__ = ["initial_centroids", "kmeans_1d", "assign", "grid_coreset"]


def initial_centroids(values: np.ndarray, weights: np.ndarray, k: int) -> np.ndarray:
    """Centroid i: the first value whose cumulative weight reaches
    (2i + 1) / (2k) of the total."""
    cum = np.cumsum(np.asarray(weights, dtype=np.float64))
    total = cum[-1]
    out = np.empty(k)
    for i in range(k):
        j = int(np.searchsorted(cum, (2 * i + 1) / (2 * k) * total, side="left"))
        out[i] = values[min(j, len(values) - 1)]
    return out


def assign(values: np.ndarray, centroids: np.ndarray) -> np.ndarray:
    """Index of the nearest centroid per value (lowest index on a tie)."""
    d = np.abs(np.asarray(values, dtype=np.float64)[:, None] - centroids[None, :])
    return np.argmin(d, axis=1)   # argmin returns the first minimum


def kmeans_1d(values, weights, k: int, max_iter: int = 100):
    """Lloyd's algorithm on one weighted projection.  Returns (centroids,
    assignment, update steps done)."""
    v = np.asarray(values, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    c = initial_centroids(v, w, k)
    a = assign(v, c)
    steps = 0
    while steps < max_iter:
        for i in range(k):
            m = a == i
            if m.any():
                c[i] = np.sum(w[m] * v[m]) / np.sum(w[m])
        steps += 1
        b = assign(v, c)
        if np.array_equal(a, b):
            break
        a = b
    return c, a, steps


def grid_coreset(problem: dict, clusters: dict):
    """Step 3: ``clusters[attr]`` is the cluster id of every value of the
    integer attribute (indexed by value).  Returns (keys, weights): the
    distinct cluster-id vectors over the tuples of D, in lexicographic order
    (attributes as listed in ``clusters``), and the number of tuples of each."""
    attrs = list(clusters)
    D = materialize_join(problem, attrs)
    ids = np.stack([np.asarray(clusters[a])[np.asarray(D[a], dtype=np.int64)] for a in attrs], axis=1)
    keys, counts = np.unique(ids.astype(np.int64), axis=0, return_counts=True)
    return keys, counts.astype(np.int64)
