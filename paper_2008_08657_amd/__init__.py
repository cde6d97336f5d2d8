"""MI355X (gfx950) engine for batches of group-by aggregates over joins.

The planner, runtime and HIP kernels live in the shared library
``liblmfao.so`` (C ABI: ``include/lmfao.h``); ``binding`` marshals Python
descriptions of a schema, join tree and aggregate batch into that ABI.
"""
import os as _os

# launch shapes chosen by lmfao_tune for the measured workloads on MI355X
# (JSON cache keyed by plan hash; a miss is tuned and added)
TUNED_SHAPES = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "tuned_shapes.json")

from .binding import (LmfaoError, Plan, Prepared, device_columns, kmeans_1d, load_library, ridge_bgd, tune,  # noqa: F401
                      marshal_problem, mlp_grad, mlp_grad_noalloc, mlp_predict, mlp_size, mlp_train)

__all__ = ["TUNED_SHAPES", "kmeans_1d", "LmfaoError", "Plan", "Prepared", "device_columns", "load_library", "marshal_problem", "mlp_grad", "tune",
           "mlp_grad_noalloc", "mlp_predict", "mlp_size", "mlp_train", "ridge_bgd"]
