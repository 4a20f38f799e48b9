"""GPU parity: the HIP path against the FP64 oracle, iteration by iteration,
through the C ABI (kp_load_tree / kp_expand with a trace / kp_update_regions /
kp_update_tree / kp_copy_tree).  See lockstep.py for the protocol."""

import sys

import numpy as np
import pytest

import oracle
from workloads import (problem_small_di, problem_small_quad, problem_c1, problem_c2, problem_c5,
                       EULER, RK4)

import lockstep

pytestmark = pytest.mark.gpu


def _announce(name, p):
    print(f"[gpu-case] {name}: cap={p['node_cap']} obs={len(p['obstacles'])} "
          f"lam={p['lambda_max']} grid={p['grid']} sub={p['sub']} seed={p['seed']}", flush=True)
    sys.stdout.flush()


def _with_box(p, bounds):
    """The problem with some state-box coordinates replaced: {index: (lo, hi)}."""
    lo, hi = np.array(p["x_lo"], np.float32), np.array(p["x_hi"], np.float32)
    for i, (a, b) in bounds.items():
        lo[i], hi[i] = a, b
    return dict(p, x_lo=lo, x_hi=hi)


CASES = {
    "di-euler": lambda: problem_small_di(seed=1, cap=4096, n_obs=12),
    "di-euler-ragged": lambda: problem_small_di(seed=2, cap=3001, n_obs=7, lambda_max=7,
                                                grid=(5, 6, 7), sub=3),
    "di-rk4": lambda: problem_small_di(seed=3, cap=4096, n_obs=12, integrator=RK4),
    "di-sub1": lambda: problem_small_di(seed=4, cap=2500, n_obs=20, grid=(4, 4, 4), sub=1),
    "quad-rk4": lambda: problem_small_quad(seed=1, cap=8192, n_obs=60),
    # the c5 building (1200 boxes, 32^3 regions, lambda_max 8) at a small cap:
    # more regions than the region pass holds in registers
    "c5-building": lambda: problem_c5(seed=1, node_cap=12000),
    # Alg. 2's random segment duration (k uniform in 1..K steps)
    "di-duration": lambda: problem_small_di(seed=8, cap=4096, n_obs=12, duration_mode=1),
    "quad-duration": lambda: problem_small_quad(seed=4, cap=8192, n_obs=60, duration_mode=1),
    "quad-euler": lambda: problem_small_quad(seed=7, cap=8192, n_obs=60, integrator=EULER),
    # the kernel variant with the tilt range check and the two-sided state-box
    # test: a tilt bound too wide for the branch-free polynomials, and a box
    # that is not symmetric about zero
    "quad-wide-tilt": lambda: _with_box(problem_small_quad(seed=5, cap=8192, n_obs=60),
                                        {3: (-1.3, 1.3), 4: (-1.3, 1.3)}),
    "quad-asym-box": lambda: _with_box(problem_small_quad(seed=6, cap=8192, n_obs=60),
                                       {6: (-10.0, 8.0), 11: (-4.0, 5.0)}),
    # a velocity box not symmetric about zero: the double integrator's
    # two-sided state-box test
    "di-asym-box": lambda: _with_box(problem_small_di(seed=9, cap=4096, n_obs=12),
                                     {3: (-10.0, 9.0), 5: (-8.0, 10.0)}),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("reload", [True, False])
def test_lockstep(name, reload):
    p = CASES[name]()
    _announce(f"lockstep {name} reload={reload}", p)
    iters = 8 if name.startswith("quad") else 14
    rep = lockstep.run_lockstep(p, iterations=iters, reload=reload)
    print(rep.summary(), flush=True)
    assert rep.ok, rep.summary()
    assert rep.iterations >= 3 or rep.final_status in (oracle.TREE_FULL, oracle.SOLVED)


def test_lockstep_until_tree_full():
    p = problem_small_di(seed=9, cap=256, n_obs=5)
    _announce("tree-full", p)
    rep = lockstep.run_lockstep(p, iterations=50, reload=False)
    assert rep.ok, rep.summary()
    assert rep.final_status == oracle.TREE_FULL


def test_lockstep_until_goal():
    from test_oracle_planner import near_goal_problem
    p = near_goal_problem(1)
    _announce("goal", p)
    rep = lockstep.run_lockstep(p, iterations=60, reload=False)
    assert rep.ok, rep.summary()
    assert rep.final_status == oracle.SOLVED


# The planning loop itself (kp_plan, one iteration per call): the propagate
# launch and the fused commit / estimates / node-set launch that the bench
# times, at the workloads' own configurations.
PLAN_CASES = {
    # c1 as specified (32768-node cap, lambda_max 4) until its tree is full
    "c1": (lambda: problem_c1(seed=0), 40, None),
    # c2 as specified (4M cap, lambda_max 4): from iteration ~20 on a launch
    # has more than 16,384 lanes (several 256-tile chunks of the V_U commit)
    "c2": (lambda: problem_c2(seed=0), 24, None),
    # the c5 building at a reduced cap
    "c5": (lambda: problem_c5(seed=2, node_cap=40000), 30, None),
    # one node-pass block serving every 4096-node tile by ticket, two
    # propagate blocks serving every wave tile
    "di-few-blocks": (lambda: problem_small_di(seed=3, cap=20000, n_obs=20), 40, (2, 1)),
    "quad-few-blocks": (lambda: problem_small_quad(seed=2, cap=24000, n_obs=60, lambda_max=8),
                        14, (3, 2)),
    # a node-set cap of one block under a tree of more than 16 tiles: the
    # launcher raises the node-set grid to one block per 16-tile chunk
    "di-chunk-floor": (lambda: problem_small_di(seed=5, cap=100000, n_obs=20), 80, (4, 1)),
}


@pytest.mark.parametrize("name", list(PLAN_CASES))
@pytest.mark.parametrize("reload", [False, True])
def test_lockstep_plan(name, reload):
    make, iters, limits = PLAN_CASES[name]
    p = make()
    _announce(f"plan-lockstep {name} reload={reload} limits={limits}", p)
    rep = lockstep.run_lockstep_plan(p, iterations=iters, reload=reload, launch_limits=limits)
    print(rep.summary(), flush=True)
    assert rep.ok, rep.summary()
    assert rep.iterations >= 5 or rep.final_status in (oracle.TREE_FULL, oracle.SOLVED)
    if name == "c2":
        assert rep.max_lanes > 16384, rep.summary()
    if name in ("c1", "di-few-blocks"):
        assert rep.final_status == oracle.TREE_FULL, rep.summary()
    if name == "di-chunk-floor":
        assert rep.max_nodes > 16 * 4096, rep.summary()
