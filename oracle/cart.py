"""Regression-tree growth by CART over a join, from the plain definition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` may import this module (with the
rest of ``oracle/``); the GPU library never calls it and shares no code with
it.

What it computes (section 3 of the paper, "Decision Trees"): a node of the
tree is the bag of tuples of D (the natural join, materialised here) that
satisfy the node's path condition, a conjunction of the split conditions on
the way from the root.  A split candidate is a condition c on one attribute:
``x <= t`` for a threshold t of a continuous attribute, or ``x == v`` for a
code v of a categorical one; its branches are T = {tuples of the node with
c} and the rest of the node (``x > t``, ``x != v``).  The paper chooses the
condition that minimises the variance of the response y over the branches;
the reading taken here is the sum over both branches of

    VAR(B) = sum_{t in B} y_t^2 - (sum_{t in B} y_t)^2 / |B|     (0 if B is empty)

i.e. |B| times the population variance of y over B.

Selection rule (shared with the GPU path, stated in its header): a candidate
is valid when both branches hold at least ``min_leaf`` tuples; among valid
candidates the least cost wins, and candidates whose cost is within
``tie_eps * max(VAR(node), 1)`` of the least are tied, the one listed first
winning.  A node is split while its depth is below ``max_depth`` and a valid
candidate exists; nodes are numbered breadth first, the root 0, the branch
where the condition holds before the other.

Arithmetic: the sums per branch are correctly rounded to FP64
(``math.fsum`` over the materialised tuples); the cost formula and the
comparisons are then done in FP64, the precision the kernel decides in.
Counts are Python integers.
"""
from __future__ import annotations

import math

import numpy as np

from . import materialize_join

__all__ = ["var_term", "node_stats", "split_costs", "best_split", "grow_tree"]


def var_term(n: int, sy: float, sy2: float) -> float:
    """VAR(B) from the branch aggregates |B|, SUM(y), SUM(y^2), in FP64."""
    if n <= 0:
        return 0.0
    return float(np.float64(sy2) - np.float64(sy) * np.float64(sy) / np.float64(n))


def _holds(col, kind: int, value, negate: bool):
    """Rows where the candidate's condition (kind 0: x <= value, kind 1:
    x == value) holds, or its complement when ``negate``."""
    m = col <= value if kind == 0 else col == value
    return ~m if negate else m


def _branch_sums(y: np.ndarray, mask: np.ndarray):
    v = y[mask].astype(np.float64)
    return int(mask.sum()), math.fsum(v.tolist()), math.fsum((v * v).tolist())


def node_stats(D: dict, y: str, mask: np.ndarray):
    """|node|, SUM(y), SUM(y^2) over the node's tuples (correctly rounded)."""
    return _branch_sums(np.asarray(D[y]), mask)


def split_costs(D: dict, y: str, mask: np.ndarray, candidates: list, min_leaf: int):
    """Per candidate (attr, kind, value): (cost, n_left, n_right, valid) over
    the node's tuples; cost = VAR(left) + VAR(right)."""
    yy = np.asarray(D[y])
    out = []
    for attr, kind, value in candidates:
        col = np.asarray(D[attr])
        left = mask & _holds(col, kind, value, False)
        right = mask & _holds(col, kind, value, True)
        nl, syl, sy2l = _branch_sums(yy, left)
        nr, syr, sy2r = _branch_sums(yy, right)
        cost = var_term(nl, syl, sy2l) + var_term(nr, syr, sy2r)
        out.append((cost, nl, nr, nl >= min_leaf and nr >= min_leaf))
    return out


def best_split(costs: list, node_var: float, tie_eps: float):
    """Index of the chosen candidate (-1 if none is valid) under the rule in
    the module docstring."""
    valid = [c for c, _, _, ok in costs if ok]
    if not valid:
        return -1
    least = min(valid)
    tol = tie_eps * max(abs(node_var), 1.0)
    for i, (c, _, _, ok) in enumerate(costs):
        if ok and c <= least + tol:
            return i
    return -1


def grow_tree(problem: dict, y: str, candidates: list, max_depth: int, min_leaf: int = 1, tie_eps: float = 1e-9):
    """Grows the tree breadth first.  ``candidates`` lists (attr, kind, value)
    with kind 0 for ``attr <= value`` and 1 for ``attr == value``.  Returns
    the nodes as dicts {parent, depth, split, left, right, n, sum_y, sum_y2,
    cost, path}; ``path`` lists (candidate index, holds) from the root."""
    attrs = sorted({a for a, _, _ in candidates} | {y})
    D = materialize_join(problem, attrs)
    n_all = len(np.asarray(D[y]))
    nodes = [{"parent": -1, "depth": 0, "path": []}]
    mask_of = [np.ones(n_all, dtype=bool)]
    i = 0
    while i < len(nodes):
        nd, mask = nodes[i], mask_of[i]
        n, sy, sy2 = node_stats(D, y, mask)
        nd.update(n=n, sum_y=sy, sum_y2=sy2, split=-1, left=-1, right=-1, cost=var_term(n, sy, sy2))
        if nd["depth"] < max_depth and n > 0:
            costs = split_costs(D, y, mask, candidates, min_leaf)
            k = best_split(costs, var_term(n, sy, sy2), tie_eps)
            if k >= 0:
                attr, kind, value = candidates[k]
                col = np.asarray(D[attr])
                nd.update(split=k, cost=costs[k][0], left=len(nodes), right=len(nodes) + 1)
                for holds in (True, False):
                    nodes.append({"parent": i, "depth": nd["depth"] + 1, "path": nd["path"] + [(k, holds)]})
                    mask_of.append(mask & _holds(col, kind, value, not holds))
        i += 1
    return nodes
