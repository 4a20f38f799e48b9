"""Seeded synthetic planning problems shared by the oracle, the tests and the bench.

This package only draws inputs: obstacle geometry, start and goal, dynamics
parameters and planner hyperparameters.  It holds none of the planner's
arithmetic, so both the GPU library and the CPU oracle can consume its output
without sharing any code with each other.
"""

from .scenes import (  # noqa: F401
    DI6,
    QUAD12,
    EULER,
    RK4,
    problem_c1,
    problem_c2,
    problem_c5,
    problem_small_di,
    problem_small_quad,
    problem_batch,
    random_boxes,
    forest,
    building,
)
