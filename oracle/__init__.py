"""Kino-PAX CPU oracle (FP64, sequential).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  The GPU library never calls it.
"""

from .kpo import (  # noqa: F401
    OK, SOLVED, TIMEOUT, TREE_FULL, FRONTIER_EMPTY, E_ARG, E_START_INVALID, E_GOAL_INVALID,
    RECORD_DTYPE, OraclePlanner, build, lib, philox4x32_10, control_map, deriv, step,
    state_ok, swept_hit, cell_of, region_score, estimates, replay, problem_struct, integrate_batch,
    segment_steps, near_cell_plane, set_threads, get_threads, AMB_TOL, COND_TILT,
    replay_trajectory,
)
