"""MI355X (gfx950) engine for batches of group-by aggregates over joins.

The planner, runtime and HIP kernels live in the shared library
``liblmfao.so`` (C ABI: ``include/lmfao.h``); ``binding`` marshals Python
descriptions of a schema, join tree and aggregate batch into that ABI.
"""
from .binding import (LmfaoError, Plan, Prepared, device_columns, load_library, ridge_bgd,  # noqa: F401
                      marshal_problem, mlp_grad, mlp_grad_noalloc, mlp_predict, mlp_size, mlp_train)

__all__ = ["LmfaoError", "Plan", "Prepared", "device_columns", "load_library", "marshal_problem", "mlp_grad",
           "mlp_grad_noalloc", "mlp_predict", "mlp_size", "mlp_train", "ridge_bgd"]
