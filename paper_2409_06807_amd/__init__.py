"""MI355X (gfx950) Kino-PAX tree-growth planner: a C-ABI HIP library
(include/kp.h, csrc/) and its ctypes binding (kp.py)."""

from .kp import (  # noqa: F401
    OK, SOLVED, TIMEOUT, TREE_FULL, FRONTIER_EMPTY, E_ARG, E_DEVICE, E_WORKSPACE,
    E_START_INVALID, E_GOAL_INVALID, E_ORDER, EXPORTED, KPError, Planner, TRACE_DTYPE,
    load_library, make_desc, workspace_bytes, MLP_PARAMS, MLP_PACKED_BYTES, mlp_pack,
    mlp_forward, mlp_grad, mlp_adam, mlp_train, mlp_train_noalloc, mlp_partials, Batch,
    plan_adaptive,
)
