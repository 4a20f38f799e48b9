"""Pins of the random segment duration (Alg. 2 samples dt in (0, T_prop]):
k ~ U{1..K} steps from Philox, the expansion integrates exactly k steps, the
double integrator's closed form over k steps, and planning with random
durations keeps the tree invariants and replays in FP64 edge by edge."""

import numpy as np
import scipy.stats

import oracle
from workloads import problem_small_di, problem_small_quad

from test_oracle_planner import check_invariants


def test_fixed_mode_is_k_steps():
    p = problem_small_di(seed=1)
    assert all(oracle.segment_steps(p, it, f, s) == 10 for it in range(3) for f in range(5)
               for s in range(4))


def test_random_duration_is_uniform_on_1_to_K():
    p = problem_small_di(seed=2, duration_mode=1)
    ks = np.array([oracle.segment_steps(p, it, f, s) for it in range(20) for f in range(100)
                   for s in range(4)])
    assert ks.min() == 1 and ks.max() == 10
    counts = np.bincount(ks, minlength=11)[1:]
    assert scipy.stats.chisquare(counts).pvalue > 1e-3
    # the duration word is word 1 of tag 1: independent of the control words
    p2 = dict(p, seed=3)
    ks2 = np.array([oracle.segment_steps(p2, it, f, s) for it in range(20) for f in range(100)
                    for s in range(4)])
    assert not np.array_equal(ks, ks2)


def test_expansion_integrates_k_steps_closed_form():
    """Double integrator, Euler: after k steps of h under u from (p0, v0),
    v = v0 + k h u and p = p0 + k h v0 + h^2 u k (k - 1) / 2."""
    p = problem_small_di(seed=4, n_obs=0, duration_mode=1)
    W = oracle.OraclePlanner(p)
    assert W.frontier() == oracle.OK
    recs = W.expand_all()
    x0 = W.state()["x"][0]
    h = float(np.float32(p["h"]))
    for r in recs:
        k = int(r["k_seg"])
        assert k == oracle.segment_steps(p, 0, int(r["parent"]), int(r["sample"]))
        u = r["u"][:3].astype(np.float64)
        # x' is the end of the whole k-step segment, valid or not (Alg. 2)
        assert r["steps"] == k
        v = x0[3:] + k * h * u
        pos = x0[:3] + k * h * x0[3:] + h * h * u * k * (k - 1) / 2
        assert np.allclose(r["x"][:6], np.concatenate([pos, v]), rtol=0, atol=1e-11)
        assert 1 <= r["fail"] <= k + 1 and (r["fail"] == k + 1) == bool(r["valid"])


def edge_steps(p, s, path):
    return [oracle.segment_steps(p, int(s["birth"][b]), int(s["parent"][b]), int(s["sample"][b]))
            for b in path[1:]]


def test_random_duration_plan_invariants_and_replay():
    p = problem_small_di(seed=5, duration_mode=1, cap=20000)
    W = oracle.OraclePlanner(p)
    st, goal, iters = W.plan(max_iters=200)
    s = W.state()
    check_invariants(p, s)
    # every stored edge re-integrates from its parent over its own duration
    N = s["N"]
    idx = np.arange(1, N)
    ks = np.array([oracle.segment_steps(p, int(s["birth"][i]), int(s["parent"][i]),
                                        int(s["sample"][i])) for i in idx], np.int32)
    ref = oracle.integrate_batch(p, s["x"][s["parent"][idx]], s["u"][idx], ks)
    assert np.allclose(ref, s["x"][idx], rtol=0, atol=1e-9)
    assert len(set(ks.tolist())) > 5
    if st == oracle.SOLVED:
        path = W.path(goal)
        valid, reached, _ = oracle.replay(p, s["x"][0], s["u"][path[1:]], 0.0, edge_steps(p, s, path))
        assert valid and reached


def test_random_duration_quad_runs():
    p = problem_small_quad(seed=2, cap=3000, duration_mode=1)
    W = oracle.OraclePlanner(p)
    for _ in range(4):
        if W.frontier() != oracle.OK:
            break
        recs = W.expand_all()
        assert np.array_equal(recs["steps"], recs["k_seg"])
        assert np.all((recs["fail"] >= 1) & (recs["fail"] <= recs["k_seg"] + 1))
        W.apply(recs)
        W.update_estimates()
        W.update_node_sets()
    s = W.state()
    s["sum_lanes"] = W.state(copy=False)["sum_lanes"]
    check_invariants(p, s)
