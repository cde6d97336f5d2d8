"""Comparison of engine results with the oracle's.

Integers (group keys, counts) must be identical.  A float cell passes when

    |gpu - oracle| <= tol * max(|oracle|, 1e-3 * sum |terms|)

where ``sum |terms|`` is the oracle's sum of absolute product terms for that
cell.  The floor makes the test meaningful for cells whose exact value is a
near-cancelling sum of N(0,1) terms (plain relative error is ill-conditioned
there).  A form whose products carry a fixed relative error (the BF16x2
contraction, about 2^-16 per product) is held to ``floor=1``: its error bound
is relative to the sum of the terms' magnitudes.
"""
import numpy as np


def compare(gpu, ref, tol, where="", floor=1e-3):
    assert gpu["keys"].shape == ref["keys"].shape, f"{where}: group count {gpu['keys'].shape} != {ref['keys'].shape}"
    np.testing.assert_array_equal(gpu["keys"], ref["keys"], err_msg=f"{where}: keys")
    np.testing.assert_array_equal(gpu["count"], ref["count"], err_msg=f"{where}: counts")
    if ref["sum"].size == 0:
        return 0.0
    scale = np.maximum(np.abs(ref["sum"]), floor * ref["abs"])
    scale = np.where(scale == 0, 1.0, scale)
    err = np.abs(gpu["sum"] - ref["sum"]) / scale
    worst = float(err.max())
    assert worst <= tol, f"{where}: max scaled error {worst:.3e} > {tol:.1e} at {np.unravel_index(err.argmax(), err.shape)}"
    return worst


def compare_all(gpu_results, ref_results, tol, name="", floor=1e-3):
    worst = 0.0
    for i, (g, r) in enumerate(zip(gpu_results, ref_results)):
        worst = max(worst, compare(g, r, tol, f"{name} query {i}", floor))
    return worst
