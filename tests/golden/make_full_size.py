"""Writes the full-size expected results of the measured workloads.

Runs the streaming tier-B oracle (``oracle.tierb``, the plain definition of
every query evaluated by enumerating the natural join on all host cores) on
the workloads ``workloads.bench_workload`` builds at full size, and stores
per query:

* queries with float aggregates, or with at most ``MAX_STORED`` groups: the
  keys, counts, sums and sums of |term| (``full_<config>.npz``);
* larger integer-only ones (the SUM(1) group-bys of the Rk-means chain, whose
  sums equal their counts): the group count, the total count and a SHA-256
  over the int64 keys (groups x |G|, C order) followed by the int64 counts,
  little-endian.

Every stored value comes from ``oracle/`` only.  The problem digest (SHA-256
of every generated column) is stored too, so that a test can tell when the
generator has changed and the file must be written again.

Usage: ``python tests/golden/make_full_size.py [config ...]`` (configs:
retail grocery cart chain; default all).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import tierb  # noqa: E402

MAX_STORED = 2_000


def result_digest(keys, count):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(keys, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(count, dtype="<i8").tobytes())
    return h.hexdigest()


def write(config):
    t0 = time.time()
    bw = W.bench_workload(config)
    p = bw["problem"]
    t_gen = time.time() - t0
    digest = W.problem_digest(p)
    st = {}
    res = tierb.evaluate(p, stats=st)
    arrays, meta = {}, {"config": config, "problem_digest": digest, "queries": [],
                        "oracle": "tier B (streaming enumeration, Neumaier FP64)",
                        "oracle_seconds": round(st["seconds"], 2), "threads": st["threads"],
                        "generate_seconds": round(t_gen, 2)}
    for qi, r in enumerate(res):
        n = int(r["keys"].shape[0])
        m = {"groups": n, "total_count": int(r["count"].sum())}
        int_only = all(not f for f in p["batch"][qi]["aggs"])
        if n <= MAX_STORED or not int_only:
            m["stored"] = True
            arrays[f"q{qi}_keys"] = r["keys"]
            arrays[f"q{qi}_count"] = r["count"]
            arrays[f"q{qi}_sum"] = r["sum"]
            arrays[f"q{qi}_abs"] = r["abs"]
        else:
            m["stored"] = False
            m["sha256"] = result_digest(r["keys"], r["count"])
        meta["queries"].append(m)
    arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    out = os.path.join(HERE, f"full_{config}.npz")
    np.savez_compressed(out, **arrays)
    print(f"{config}: {len(res)} queries, oracle {st['seconds']:.1f} s on {st['threads']} threads -> {out}",
          flush=True)


if __name__ == "__main__":
    for c in (sys.argv[1:] or ["retail", "grocery", "cart", "chain"]):
        write(c)
