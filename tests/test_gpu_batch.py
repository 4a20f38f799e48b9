"""Batched planning on the GPU: every problem of a batch ends exactly as it
does when planned alone with kp_plan (status, goal, iterations, counters and
the whole tree), under every launch configuration, with and without graph
replay, with per-problem budgets, and the autotuner keeps results fixed."""

import sys

import numpy as np
import pytest

import oracle
from workloads import problem_batch, problem_small_di, problem_small_quad

pytestmark = pytest.mark.gpu

KEYS = ("status", "goal_id", "iterations", "n_nodes", "path_len", "lanes_total", "valid_total")
TREE_KEYS = ("x", "u", "parent", "cell", "flag", "birth", "sample", "nv", "ni", "visited", "avail",
             "thr")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def small_batch():
    # uneven: caps 1.5k .. 40k, 3 .. 60 boxes, different seeds and scenes
    specs = [(2000, 3, 0), (40000, 40, 1), (6000, 12, 2), (1500, 60, 3), (20000, 20, 4),
             (9000, 7, 5)]
    return [problem_small_di(seed=s, scene_seed=30 + s, n_obs=o, cap=c) for c, o, s in specs]


def alone(problems):
    from paper_2409_06807_amd import Planner
    out = []
    for p in problems:
        G = Planner(p)
        r = G.plan()
        out.append((r, G.copy_tree()))
        G.close()
    return out


def check_same(ref, planners, results):
    for (r0, t0), G, r in zip(ref, planners, results):
        for k in KEYS:
            assert r[k] == r0[k], (k, r[k], r0[k])
        t = G.copy_tree()
        assert t["N"] == t0["N"]
        for k in TREE_KEYS:
            assert np.array_equal(t[k], t0[k]), k


CONFIGS = [
    None,
    dict(use_graph=1),
    dict(iters_per_sync=3, prop_blocks=4, node_blocks=2),
    dict(iters_per_sync=16, use_graph=1, prop_blocks=16, node_blocks=8),
    dict(iters_per_sync=1),
]


@pytest.mark.parametrize("ci", range(len(CONFIGS)))
def test_batch_equals_single_planner(ci):
    from paper_2409_06807_amd import Planner, Batch
    cfg = CONFIGS[ci]
    _say(f"batch vs single, config {cfg}")
    ps = small_batch()
    ref = alone(ps)
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    if cfg:
        B.set_config(**cfg)
    res, ms = B.plan()
    assert ms > 0 and all(r["elapsed_ms"] <= ms for r in res)
    check_same(ref, planners, res)
    # the same batch again after a batch reset: identical again (graphs replay)
    B.reset([p["seed"] for p in ps])
    res2, _ = B.plan()
    check_same(ref, planners, res2)
    B.close()


def test_quad_batch_equals_single_planner():
    from paper_2409_06807_amd import Planner, Batch
    _say("quad batch")
    ps = [problem_small_quad(seed=s, scene_seed=40 + s, n_obs=o, cap=c)
          for c, o, s in [(8192, 60, 0), (3000, 20, 1), (12000, 90, 2)]]
    ref = alone(ps)
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    B.set_config(use_graph=1)
    res, _ = B.plan()
    check_same(ref, planners, res)
    B.close()


def test_batch_budget_stops_one_problem_and_it_resumes():
    from paper_2409_06807_amd import Planner, Batch
    _say("batch budget")
    ps = small_batch()[:3]
    ps[1] = dict(ps[1], max_iters=3)
    ref = alone(ps)
    assert ref[1][0]["status"] == oracle.TIMEOUT and ref[1][0]["iterations"] == 3
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    res, _ = B.plan()
    check_same(ref, planners, res)
    # the stopped problem continues afterwards exactly like its single twin
    G1 = Planner(ps[1])
    G1.plan()
    r_single = G1.plan()
    r_batch = planners[1].plan()
    for k in KEYS:
        assert r_single[k] == r_batch[k], k
    B.close()


def test_batch_argument_and_order_errors():
    from paper_2409_06807_amd import Planner, Batch, KPError, E_ARG, E_ORDER
    _say("batch errors")
    a = Planner(problem_small_di(seed=1))
    b = Planner(problem_small_quad(seed=1))
    with pytest.raises(KPError) as ei:
        Batch([a, b])
    assert ei.value.code == E_ARG
    c = Planner(problem_small_di(seed=2))
    B = Batch([a, c])
    c.expand()
    with pytest.raises(KPError) as ei:
        B.plan()
    assert ei.value.code == E_ORDER
    with pytest.raises(KPError) as ei:
        B.set_config(iters_per_sync=0)
    assert ei.value.code == E_ARG
    B.close()


def test_autotuner_keeps_results(tmp_path):
    from paper_2409_06807_amd import Planner, Batch, autotune
    _say("autotune small")
    ps = problem_batch(n=8, batch_seed=5, cap_range=(16384, 65536), obs_range=(10, 200))
    planners = [Planner(p) for p in ps]
    B = Batch(planners)

    def reset():
        for G, p in zip(planners, ps):
            G.reset(p["seed"])

    space = [dict(iters_per_sync=8, use_graph=0, prop_blocks=1024, node_blocks=512),
             dict(iters_per_sync=4, use_graph=1, prop_blocks=64, node_blocks=32),
             dict(iters_per_sync=16, use_graph=1, prop_blocks=256, node_blocks=128)]
    cfg, table = autotune.tune(B, reset, "test-sig", cache_path=str(tmp_path / "a.json"), space=space)
    assert cfg in space and len(table) == 3
    B.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_batch_with_learned_proposals_equals_single(graph):
    # problems with a learned proposal get their network pass inside the batch
    import paper_2409_06807_amd as kp
    from paper_2409_06807_amd import Planner, Batch
    import torch
    from workloads import mlp_inputs
    _say(f"batch with learned proposals, graph={graph}")
    ps = small_batch()[:4]
    params = torch.tensor(mlp_inputs.params(31, scale=1.0, out_scale=1.0), dtype=torch.float32,
                          device="cuda:0")
    packed = kp.mlp_pack(params)
    learned = [True, False, True, True]
    ref = []
    for p, l in zip(ps, learned):
        G = Planner(p)
        if l:
            G.set_proposal(packed, 0.7)
        r = G.plan()
        ref.append((r, G.copy_tree()))
        G.close()
    planners = [Planner(p) for p in ps]
    for G, l in zip(planners, learned):
        if l:
            G.set_proposal(packed, 0.7)
    B = Batch(planners)
    B.set_config(use_graph=graph)
    res, _ = B.plan()
    check_same(ref, planners, res)
    B.close()


def _batch_lockstep_problems(dyn):
    from workloads import DI6, QUAD12
    # obstacle counts up to 2000 (the batched workload's range): tables larger
    # than 64 KiB of LDS per propagate block
    ps = problem_batch(n=5, batch_seed=9, dynamics=DI6 if dyn == "di" else QUAD12,
                       cap_range=(16384, 40000), obs_range=(1200, 2000))
    ps += problem_batch(n=3, batch_seed=10, dynamics=DI6 if dyn == "di" else QUAD12,
                        cap_range=(16384, 40000), obs_range=(10, 100))
    return ps


@pytest.mark.parametrize("dyn,config", [
    ("di", None),
    ("di", dict(use_graph=1, prop_blocks=3, node_blocks=1)),
    ("quad", dict(prop_blocks=8, node_blocks=2)),
])
def test_batch_lockstep_against_oracle(dyn, config):
    """Batched planning against the oracle, iteration by iteration: every
    problem of the batch (one grid row each) must match its own FP64 oracle
    lane by lane and in every integer field of its tree."""
    import lockstep
    ps = _batch_lockstep_problems(dyn)
    _say(f"batch lock-step {dyn} config={config} obstacles={[len(p['obstacles']) for p in ps]}")
    assert max(len(p["obstacles"]) for p in ps) > 1536
    reps = lockstep.run_lockstep_batch(ps, iterations=12 if dyn == "di" else 8, config=config)
    for k, rep in enumerate(reps):
        print(f"problem {k}: {rep.summary()}", flush=True)
    assert all(rep.ok for rep in reps), [rep.summary() for rep in reps if not rep.ok][:3]
    assert all(rep.iterations >= 3 or rep.final_status in (oracle.TREE_FULL, oracle.SOLVED)
               for rep in reps)


# ---------------------------------------------------------------------------
# one persistent launch over a device work queue (kp_batch_plan_queue)
# ---------------------------------------------------------------------------
QUEUE_OFF = ("kp_batch_plan_queue is switched off: its first GPU run (the six small "
             "double-integrator problems below) did not finish and the cause is not yet known")


def test_queue_is_refused_while_switched_off():
    from paper_2409_06807_amd import Planner, Batch, KPError, E_ARG
    _say("queue refused while switched off")
    planners = [Planner(p) for p in small_batch()[:2]]
    B = Batch(planners)
    with pytest.raises(KPError) as ei:
        B.plan(queue=True)
    assert ei.value.code == E_ARG
    B.close()


@pytest.mark.skip(reason=QUEUE_OFF)
def test_queue_equals_single_planner():
    from paper_2409_06807_amd import Planner, Batch
    _say("queue vs single")
    ps = small_batch()
    ref = alone(ps)
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    res, ms = B.plan(queue=True)
    assert ms > 0 and all(0.0 <= r["elapsed_ms"] <= ms for r in res)
    check_same(ref, planners, res)
    # again after a batch reset, and then through the two-launch path
    B.reset([p["seed"] for p in ps])
    res2, _ = B.plan(queue=True)
    check_same(ref, planners, res2)
    B.reset([p["seed"] for p in ps])
    res3, _ = B.plan()
    check_same(ref, planners, res3)
    B.close()


@pytest.mark.skip(reason=QUEUE_OFF)
def test_queue_quad_and_grid_problems_equal_single():
    from paper_2409_06807_amd import Planner, Batch
    _say("queue quad batch")
    ps = [problem_small_quad(seed=s, scene_seed=40 + s, n_obs=o, cap=c)
          for c, o, s in [(8192, 60, 0), (3000, 20, 1), (12000, 90, 2)]]
    ref = alone(ps)
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    res, _ = B.plan(queue=True)
    check_same(ref, planners, res)
    B.close()
    _say("queue DI batch with obstacle grids")
    ps = problem_batch(n=6, batch_seed=9, cap_range=(16384, 40000), obs_range=(300, 2000))
    ref = alone(ps)
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    res, _ = B.plan(queue=True)
    check_same(ref, planners, res)
    B.close()


@pytest.mark.skip(reason=QUEUE_OFF)
def test_queue_budget_stops_one_problem_and_it_resumes():
    from paper_2409_06807_amd import Planner, Batch
    _say("queue budget")
    ps = small_batch()[:3]
    ps[1] = dict(ps[1], max_iters=3)
    ref = alone(ps)
    assert ref[1][0]["status"] == oracle.TIMEOUT and ref[1][0]["iterations"] == 3
    planners = [Planner(p) for p in ps]
    B = Batch(planners)
    res, _ = B.plan(queue=True)
    check_same(ref, planners, res)
    G1 = Planner(ps[1])
    G1.plan()
    r_single = G1.plan()
    r_batch = planners[1].plan()
    for k in KEYS:
        assert r_single[k] == r_batch[k], k
    B.close()


@pytest.mark.skip(reason=QUEUE_OFF)
def test_queue_refuses_learned_proposals():
    import paper_2409_06807_amd as kp
    from paper_2409_06807_amd import Planner, Batch, KPError, E_ARG
    import torch
    from workloads import mlp_inputs
    _say("queue refuses learned proposals")
    ps = small_batch()[:2]
    planners = [Planner(p) for p in ps]
    params = torch.tensor(mlp_inputs.params(31), dtype=torch.float32, device="cuda:0")
    planners[1].set_proposal(kp.mlp_pack(params), 0.5)
    B = Batch(planners)
    with pytest.raises(KPError) as ei:
        B.plan(queue=True)
    assert ei.value.code == E_ARG
    B.close()


@pytest.mark.skip(reason=QUEUE_OFF)
@pytest.mark.parametrize("dyn", ["di", "quad"])
def test_queue_lockstep_against_oracle(dyn):
    """The persistent queue kernel against the oracle, one iteration of every
    problem per call, lane by lane and in every integer field."""
    import lockstep
    ps = _batch_lockstep_problems(dyn)
    _say(f"queue lock-step {dyn} obstacles={[len(p['obstacles']) for p in ps]}")
    reps = lockstep.run_lockstep_batch(ps, iterations=12 if dyn == "di" else 8, queue=True)
    for k, rep in enumerate(reps):
        print(f"problem {k}: {rep.summary()}", flush=True)
    assert all(rep.ok for rep in reps), [rep.summary() for rep in reps if not rep.ok][:3]
    assert all(rep.iterations >= 3 or rep.final_status in (oracle.TREE_FULL, oracle.SOLVED)
               for rep in reps)
