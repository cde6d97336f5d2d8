"""Group-count estimator for hash-table sizing: corpus, training, weights.

Not part of the paper's method.  Outputs whose dense key space is too large
for a dense table are aggregated in hash tables; their initial capacity can
come from a small perceptron that predicts log2(1 + groups) from features the
engine computes at prepare time (``lmfao_prepared_features``; the layout is
declared with ``LMFAO_EST_FEATURES``).  A table that overflows is grown and the
run repeated, so results never depend on the prediction.

* corpus: the engine's own runs on random small acyclic joins
  (``workloads.estimator_workload``): features of every query with group-by
  attributes and the exact number of groups the run produced;
* training: the library's GPU kernels (``lmfao_mlp_train``), Adam on the mean
  squared error of the network's output against the shortfall of
  log2(1 + groups) below the bound feature (so the error is the log2
  q-error), with the best validation snapshot kept;
* margin: the 95th percentile of the validation under-estimate, added to the
  prediction so that few tables start too small;
* weights file: JSON with the feature names, network size, standardisation,
  margin and parameters; ``load`` turns it into the blob ``lmfao_options``
  takes.

Run ``python -m paper_2008_08657_amd.estimator --out weights.json`` on a GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "estimator_weights.json")
VERSION = 2     # the network predicts the shortfall below the bound feature
FEATURES = [
    "log2_root_rows", "log2_total_rows", "n_relations", "n_keys",
    "log2_distinct_0", "log2_distinct_1", "log2_distinct_2",
    "log2_domain_0", "log2_domain_1", "log2_domain_2",
    "distance_0", "distance_1", "distance_2",
    "log2_distinct_product", "log2_bound", "key_determined", "n_filter_conditions",
    "log2_holder_rows_0", "log2_holder_rows_1", "log2_holder_rows_2",
    "log2_join_distinct_parent_0", "log2_join_distinct_parent_1", "log2_join_distinct_parent_2",
    "log2_join_distinct_holder_0", "log2_join_distinct_holder_1", "log2_join_distinct_holder_2",
]
D = len(FEATURES)
BOUND = FEATURES.index("log2_bound")


def pack(mean, std, params, h: int, margin: float) -> np.ndarray:
    """The blob layout of ``lmfao_options.estimator``."""
    head = np.array([VERSION, D, h, margin], dtype=np.float32)
    return np.concatenate([head, np.asarray(mean, np.float32), np.asarray(std, np.float32),
                           np.asarray(params, np.float32)])


def save(path: str, mean, std, params, h: int, margin: float, meta: dict) -> None:
    doc = {"version": VERSION, "features": FEATURES, "hidden": int(h), "margin": float(margin),
           "mean": [float(x) for x in mean], "std": [float(x) for x in std],
           "params": [float(x) for x in np.asarray(params, np.float32)], "meta": meta}
    with open(path, "w") as f:
        json.dump(doc, f)


def load(path: str = WEIGHTS) -> np.ndarray:
    """Reads a weights file and returns the blob; rejects a file written for
    another feature layout."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("version") != VERSION or doc.get("features") != FEATURES:
        raise ValueError(f"{path}: estimator written for another feature layout")
    return pack(doc["mean"], doc["std"], doc["params"], doc["hidden"], doc["margin"])


def _predict_host(blob: np.ndarray, X: np.ndarray) -> np.ndarray:
    """The network on the host (FP32), as the library evaluates it."""
    h = int(blob[2])
    mean, std = blob[4:4 + D], blob[4 + D:4 + 2 * D]
    p = blob[4 + 2 * D:]
    o = 0
    W1 = p[o:o + D * h].reshape(D, h); o += D * h
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    w3 = p[o:o + h]; o += h
    b3 = p[o]
    X = np.asarray(X, np.float32)
    z = (X - mean) / np.where(std > 0, std, 1).astype(np.float32)
    a = np.maximum(z @ W1 + b1, 0)
    a = np.maximum(a @ W2 + b2, 0)
    return X[:, BOUND] - (a @ w3 + b3)


def corpus(problems, device="cuda:0", log=None, total=None):
    """Features and log2(1 + groups) of every query with group-by attributes
    of each problem, from one run of the engine per problem."""
    from . import binding
    X, t, tag = [], [], []
    skipped = 0
    for k, p in enumerate(problems):
        try:
            plan = binding.Plan(p, precision="f32", codegen=False, policy=p.get("policy"))
        except binding.LmfaoError as e:
            if e.status != 4:
                raise
            # keep the queries the engine plans on their own
            keep = []
            for q in p["batch"]:
                try:
                    binding.Plan(dict(p, batch=[q]), precision="f32", codegen=False, policy=p.get("policy"))
                    keep.append(q)
                except binding.LmfaoError as e1:
                    if e1.status != 4:
                        raise
                    skipped += 1
            if not keep:
                continue
            p = dict(p, batch=keep)
            plan = binding.Plan(p, precision="f32", codegen=False, policy=p.get("policy"))
        try:
            prep = binding.Prepared(plan, binding.device_columns(p, device))
        except binding.LmfaoError as e:
            if e.status != 4:
                raise
            skipped += len(p["batch"])
            continue
        prep.run(sync=True)
        res = prep.results()
        for q, query in enumerate(p["batch"]):
            if not query.get("groupby"):
                continue
            f = prep.features(q)
            if f is None:
                continue
            n_groups = len(res[q]["keys"])
            if n_groups == 0:
                continue   # empty join: no table to size
            X.append(f)
            t.append(np.log2(1.0 + n_groups))
            tag.append(p["name"])
        del prep, plan
        if log and (k + 1) % 20 == 0:
            log(f"corpus: {k + 1}/{total or '?'} workloads, {len(X)} outputs, {skipped} queries unsupported")
    return np.asarray(X, np.float32), np.asarray(t, np.float32), tag


def _he_init(h: int, seed: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(seed))
    parts = [g.standard_normal((D, h)) * np.sqrt(2.0 / D), np.zeros(h),
             g.standard_normal((h, h)) * np.sqrt(2.0 / h), np.zeros(h),
             g.standard_normal(h) * np.sqrt(2.0 / h), np.zeros(1)]
    return np.concatenate([np.ravel(x) for x in parts]).astype(np.float32)


def train(X, t, h: int = 64, rounds: int = 40, steps_per_round: int = 200, batch: int = 256, lr: float = 1e-3,
          val_frac: float = 0.15, seed: int = 0, groups=None, device="cuda:0"):
    """Trains on the GPU; the validation split is by workload (``groups``)
    when given.  Returns (blob, report)."""
    import torch
    from . import binding
    g = np.random.Generator(np.random.PCG64(seed))
    n = len(X)
    if groups is not None:
        names = sorted(set(groups))
        val_names = set(g.choice(names, max(1, int(len(names) * val_frac)), replace=False).tolist())
        val = np.array([x in val_names for x in groups])
    else:
        val = g.random(n) < val_frac
    tr = ~val
    mean = X[tr].mean(axis=0)
    std = X[tr].std(axis=0)
    std[std == 0] = 1
    Z = ((X - mean) / std).astype(np.float32)
    # target: how far below the bound the group count lies (never negative)
    short = np.maximum(X[:, BOUND] - t, 0).astype(np.float32)
    Xtr = torch.from_numpy(np.ascontiguousarray(Z[tr])).to(device)
    ttr = torch.from_numpy(np.ascontiguousarray(short[tr])).to(device)
    Xva = torch.from_numpy(np.ascontiguousarray(Z[val])).to(device)
    params = torch.from_numpy(_he_init(h, seed + 1)).to(device)
    ntr = int(tr.sum())
    bs = min(batch, ntr)
    best, best_err, trace = params.clone(), np.inf, []
    for r in range(rounds):
        order = torch.from_numpy(g.integers(0, ntr, steps_per_round * bs).astype(np.int32)).to(device)
        losses = binding.mlp_train(params, Xtr, ttr, order, bs, h, lr=lr)
        yv = X[val, BOUND] - binding.mlp_predict(params, Xva, h).cpu().numpy()
        err = float(np.mean((yv - t[val]) ** 2))
        trace.append((r, float(np.mean(losses[-20:])), err))
        if err < best_err:
            best_err, best = err, params.clone()
    yv = X[val, BOUND] - binding.mlp_predict(best, Xva, h).cpu().numpy()
    under = t[val] - yv
    margin = float(max(0.0, np.percentile(under, 95)))
    blob = pack(mean, std, best.cpu().numpy(), h, margin)
    report = {"train_outputs": ntr, "val_outputs": int(val.sum()), "val_mse": best_err, "margin": margin,
              "trace": trace}
    return blob, report


def qerror(pred_log2, true_log2) -> dict:
    """Percentiles of the q-error max(est/true, true/est) over (1 + groups)."""
    q = np.exp2(np.abs(np.asarray(pred_log2, np.float64) - np.asarray(true_log2, np.float64)))
    return {f"p{p}": float(np.percentile(q, p)) for p in (50, 90, 95, 99)} | {"max": float(q.max())}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--workloads", type=int, default=240)
    ap.add_argument("--max-rows", type=int, default=1_000_000)
    ap.add_argument("--hidden", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--corpus-out", default=None, help="also save the corpus (npz)")
    a = ap.parse_args(argv)
    import workloads as W
    log = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.time()
    probs = (W.estimator_workload(a.seed * 100_000 + s, a.max_rows) for s in range(a.workloads))
    X, t, tag = corpus(probs, log=log, total=a.workloads)
    log(f"corpus: {len(X)} outputs in {time.time() - t0:.1f} s")
    if a.corpus_out:
        np.savez(a.corpus_out, X=X, t=t, tag=np.asarray(tag))
    blob, rep = train(X, t, h=a.hidden, groups=tag, seed=a.seed)
    # held out: Rk-means chains (a generator the corpus never draws from)
    held = [W.rkmeans_chain(seed=s, n1=200_000, n2=20_000, n3=2_000, n_x=8, n_y=6, n_z=6, max_dom=1_000_000)
            for s in (101, 102)]
    Xh, th, _ = corpus(held)
    yh = _predict_host(blob, Xh)
    rep["held_out"] = {"outputs": len(Xh), "qerror": qerror(yh, th),
                       "qerror_with_margin": qerror(yh + blob[3], th),
                       "under_after_margin": float(np.mean(yh + blob[3] < th))}
    rep["corpus_seconds"] = time.time() - t0
    save(a.out, blob[4:4 + D], blob[4 + D:4 + 2 * D], blob[4 + 2 * D:], a.hidden, float(blob[3]),
         {k: v for k, v in rep.items() if k != "trace"} | {"workloads": a.workloads, "max_rows": a.max_rows,
                                                             "seed": a.seed})
    print(json.dumps({k: v for k, v in rep.items() if k != "trace"}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
