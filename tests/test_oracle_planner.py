"""Pins for the oracle planner (Alg. 1, 2, 4) on small problems.

* Tree invariants after free-run iterations: parent[i] < i and a single root
  (acyclic), V_E / V_O partition T, visited sub-regions = cells of the tree
  nodes, R_avail = regions of the tree nodes, sum(n_valid + n_invalid) =
  sum over iterations of |V_E| * lambda, sum(n_valid) >= |T| - 1, |T| <= t_e.
* Every stored control equals the FP32 control map of the numpy Philox words
  of its (iteration, parent, sample) counter (numpy Philox, not the C one).
* Double-integrator edges equal Euler's closed form from the parent.
* Node ids inside one iteration are ordered by (parent, sample).
* Statistical pins for Alg. 2's acceptance and Alg. 4's set moves.
* Forced failures: full tree, invalid start, invalid goal, start in goal,
  NaN dynamics parameter.
* FP64 replay of a found path.
"""

import numpy as np
import pytest

import oracle
from workloads import problem_small_di, problem_small_quad, EULER

from test_oracle_philox import philox_generic, PHILOX_4x32, _fma_f32_exact


def run_iters(P, k):
    sts = []
    for _ in range(k):
        st, g = P.iterate()
        sts.append(st)
        if st != oracle.OK:
            break
    return sts


def check_invariants(p, s):
    N = s["N"]
    assert 1 <= N <= p["node_cap"]
    par = s["parent"]
    assert par[0] == -1
    assert np.all(par[1:] >= 0) and np.all(par[1:] < np.arange(1, N))
    assert set(np.unique(s["flag"])) <= {0, 1}
    R = len(s["nv"])
    cells = s["cell"].astype(np.int64)
    vis = np.zeros(R, np.uint64)
    for c in cells:
        vis[c >> 6] |= np.uint64(1) << np.uint64(c & 63)
    assert np.array_equal(vis, s["visited"])
    av = np.zeros(R, np.uint8)
    av[cells >> 6] = 1
    assert np.array_equal(av, s["avail"])
    assert int(s["nv"].sum() + s["ni"].sum()) == s["sum_lanes"]
    assert int(s["nv"].sum()) >= N - 1
    # ids inside one iteration ordered by (parent, sample)
    b = s["birth"]
    for it in np.unique(b[b >= 0]):
        ids = np.nonzero(b == it)[0]
        key = list(zip(par[ids], s["sample"][ids]))
        assert key == sorted(key)
        assert np.all(np.diff(ids) == 1)


def expected_controls(p, it, f, s, m):
    seed = int(p["seed"])
    key = [seed & 0xFFFFFFFF, seed >> 32]
    w = philox_generic([it, f, s, 0], key, **PHILOX_4x32)
    out = []
    for j in range(m):
        lo, hi = np.float32(p["u_lo"][j]), np.float32(p["u_hi"][j])
        r = np.float32((w[j] >> 8) * 2.0**-24)
        out.append(_fma_f32_exact(np.float32(hi - lo), r, lo))
    return np.array(out, np.float32)


@pytest.mark.parametrize("make,iters", [(lambda: problem_small_di(seed=3), 12),
                                        (lambda: problem_small_di(seed=4, lambda_max=7, cap=3000,
                                                                  grid=(5, 6, 7), sub=3), 12),
                                        (lambda: problem_small_quad(seed=1, cap=3000), 6)])
def test_tree_invariants_and_controls(make, iters):
    p = make()
    P = oracle.OraclePlanner(p)
    run_iters(P, iters)
    s = P.state()
    check_invariants(p, s)
    m = P.m
    rng = np.random.default_rng(0)
    for i in rng.choice(np.arange(1, s["N"]), size=min(300, s["N"] - 1), replace=False):
        want = expected_controls(p, s["birth"][i], s["parent"][i], s["sample"][i], m)
        assert np.array_equal(s["u"][i], want)


def test_di_edges_closed_form():
    p = problem_small_di(seed=5)
    P = oracle.OraclePlanner(p)
    run_iters(P, 10)
    s = P.state()
    h = float(np.float32(p["h"]))
    K = int(p["steps"])
    for i in range(1, s["N"]):
        x0 = s["x"][s["parent"][i]]
        u = s["u"][i].astype(np.float64)
        v = x0[3:] + K * h * u
        q = x0[:3] + K * h * x0[3:] + h * h * u * K * (K - 1) / 2
        np.testing.assert_allclose(s["x"][i], np.concatenate([q, v]), atol=1e-9)


def test_acceptance_statistics():
    # Alg. 2 acceptance: a valid sample in a visited sub-region is accepted
    # with probability P_accept; in an unvisited one always.
    p = problem_small_di(cap=200000)
    P = oracle.OraclePlanner(p)
    v = P.state(copy=False)
    thr = v["thr"]
    visited = v["visited"]
    R = len(thr)
    thr[:] = int(0.3 * 2**32)
    visited[:] = 0
    visited[5] = 1  # sub-cell 0 of region 5 visited
    rng = np.random.default_rng(11)
    n = 40000
    recs = np.zeros(n, oracle.RECORD_DTYPE)
    recs["valid"] = 1
    recs["w_acc"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    recs["cell"] = np.where(np.arange(n) % 2 == 0, 5 * 64 + 0, 5 * 64 + 1)
    P.apply(recs)
    s = P.state(copy=False)
    nU = P.view().nU
    visited_acc = np.sum((recs["cell"] == 320) & (recs["w_acc"].astype(np.uint64) < thr[5]))
    assert nU == visited_acc + n // 2
    assert abs(visited_acc / (n // 2) - 0.3) < 0.015
    assert s["nv"][5] == n and s["ni"][5] == 0


def test_node_set_move_statistics():
    # Alg. 4: V_E -> V_O w.p. 1 - P; V_O -> V_E w.p. P (including just-demoted).
    p = problem_small_di(cap=200000)
    P = oracle.OraclePlanner(p)
    lib = oracle.lib()
    N = 100000
    lib.kpo_set_counters(P.h, N, 3)
    v = P.state(copy=False)
    v0 = P.view()
    cap = v0.cap
    flag = np.ctypeslib.as_array(v0.flag, (cap,))
    cell = np.ctypeslib.as_array(v0.cell, (cap,))
    thr = v["thr"]
    Pacc = 0.25
    thr[:] = int(Pacc * 2**32)
    cell[:N] = 7 * 64
    flag[:N] = 0
    flag[: N // 2] = 1
    P.update_node_sets()
    f = np.ctypeslib.as_array(P.view().flag, (cap,))[:N]
    stay_E = f[: N // 2].mean()
    to_E = f[N // 2:].mean()
    assert abs(to_E - Pacc) < 0.01
    assert abs(stay_E - (Pacc + (1 - Pacc) * Pacc)) < 0.01


def test_forced_tree_full():
    p = problem_small_di(cap=60, lambda_max=4)
    P = oracle.OraclePlanner(p)
    st, g, it = P.plan(max_iters=100)
    assert st == oracle.TREE_FULL
    assert P.state()["N"] <= 60


def test_forced_start_invalid():
    p = problem_small_di()
    p["obstacles"] = np.vstack([p["obstacles"], np.array([[4, 4, 4, 6, 6, 6]], np.float32)])
    with pytest.raises(ValueError):
        oracle.OraclePlanner(p)
    st = oracle.lib()
    s, keep = oracle.problem_struct(p)
    import ctypes
    code = ctypes.c_int32(0)
    h = st.kpo_create(ctypes.byref(s), ctypes.byref(code))
    assert not h and code.value == oracle.E_START_INVALID


def test_forced_goal_invalid():
    import ctypes
    p = problem_small_di()
    p["obstacles"] = np.vstack([p["obstacles"], np.array([[93, 93, 93, 97, 97, 97]], np.float32)])
    s, keep = oracle.problem_struct(p)
    code = ctypes.c_int32(0)
    assert not oracle.lib().kpo_create(ctypes.byref(s), ctypes.byref(code))
    assert code.value == oracle.E_GOAL_INVALID
    p = problem_small_di()
    p["goal_center"] = np.array([97, 50, 50], np.float32)  # ball leaves W
    s, keep = oracle.problem_struct(p)
    assert not oracle.lib().kpo_create(ctypes.byref(s), ctypes.byref(code))
    assert code.value == oracle.E_GOAL_INVALID


def test_start_in_goal():
    p = problem_small_di()
    p["goal_center"] = np.array([7, 7, 7], np.float32)
    p["goal_radius"] = np.float32(4.0)
    p["obstacles"] = np.zeros((0, 6), np.float32)
    P = oracle.OraclePlanner(p)
    st, g, it = P.plan(max_iters=10)
    assert st == oracle.SOLVED and g == 0 and it == 0
    assert list(P.path(0)) == [0]


def test_nan_dynamics_all_invalid():
    p = problem_small_quad(cap=2000)
    prm = np.array(p["dyn_params"], np.float32)
    prm[0] = np.nan  # mass
    p["dyn_params"] = prm
    P = oracle.OraclePlanner(p)
    st, g, it = P.plan(max_iters=5)
    s = P.state()
    assert st == oracle.TIMEOUT
    assert s["N"] == 1 and int(s["nv"].sum()) == 0 and int(s["ni"].sum()) == s["sum_lanes"] > 0


def test_ambiguity_band_ordering():
    p = problem_small_quad(seed=2, cap=3000)
    P = oracle.OraclePlanner(p)
    run_iters(P, 3)
    P.frontier()
    recs = P.expand_all()
    K = int(p["steps"])
    fail = recs["fail"]
    assert np.array_equal(recs["valid"] == 1, fail == K + 1)
    assert np.all(recs["fail_strict"] <= fail) and np.all(fail <= recs["fail_loose"])
    assert np.all(recs["steps"] == K)


def near_goal_problem(seed=0):
    """A goal four segments away behind two thin walls, so that small trees
    solve it before filling up."""
    p = problem_small_di(seed=seed, cap=20000, lambda_max=4)
    p["goal_center"] = np.array([13, 13, 7], np.float32)
    p["goal_radius"] = np.float32(4.0)
    p["obstacles"] = np.array([[9, 0, 0, 11, 8, 30], [0, 12, 0, 7, 14, 30]], np.float32)
    return p


@pytest.mark.parametrize("seed", range(3))
def test_found_path_replays_in_fp64(seed):
    p = near_goal_problem(seed)
    P = oracle.OraclePlanner(p)
    st, g, it = P.plan(max_iters=200)
    assert st == oracle.SOLVED
    s = P.state()
    path = P.path(g)
    assert path[0] == 0 and path[-1] == g
    ctl = s["u"][path[1:]]
    valid, reached, ends = oracle.replay(p, s["x"][0], ctl, margin=0.0)
    assert valid and reached
    np.testing.assert_allclose(ends, s["x"][path[1:]], atol=1e-9)
    # the exact (continuous) double-integrator trajectory also stays clear of
    # the un-inflated obstacles: Euler deviates from it by at most 0.0513 per
    # axis over a segment, below the 0.1 planning margin
    h = float(np.float32(p["h"]))
    K = int(p["steps"])
    obs = np.asarray(p["obstacles"], np.float64)
    x = s["x"][0].copy()
    t = np.linspace(0, K * h, 400)[:, None]
    for u in ctl.astype(np.float64):
        pts = x[:3] + x[3:] * t + 0.5 * u * t * t
        for o in obs:
            assert not np.any(np.all((pts >= o[:3]) & (pts <= o[3:]), axis=1))
        x = np.concatenate([x[:3] + x[3:] * K * h + 0.5 * u * (K * h) ** 2, x[3:] + u * K * h])


def test_threads_do_not_change_results():
    """The expansion loop may run on several OpenMP threads: every record, and
    so the whole planning run, is the same as on one thread."""
    p = problem_small_quad(seed=3, cap=6000)
    runs = []
    old = oracle.get_threads()
    try:
        for t in (1, 4):
            oracle.set_threads(t)
            W = oracle.OraclePlanner(p)
            recs = []
            for _ in range(4):
                if W.frontier() != oracle.OK:
                    break
                r = W.expand_all()
                recs.append(r.tobytes())
                W.apply(r)
                W.update_estimates()
                W.update_node_sets()
            s = W.state()
            runs.append((recs, {k: np.asarray(v).tobytes() for k, v in s.items()
                                if isinstance(v, np.ndarray)}))
    finally:
        oracle.set_threads(old)
    assert runs[0][0] == runs[1][0]
    assert runs[0][1] == runs[1][1]


def _traj_of(p, s, path):
    """The trajectory rows a GPU planner returns, from an oracle tree: FP32
    states, controls of the edge into each node, steps of each edge."""
    steps = [0] + [oracle.segment_steps(p, int(s["birth"][b]), int(s["parent"][b]),
                                        int(s["sample"][b])) for b in path[1:]]
    u = s["u"][path].copy()
    u[0] = 0.0
    return dict(x=s["x"][path].astype(np.float32), u=u, steps=np.asarray(steps, np.int32))


@pytest.mark.parametrize("dur", [0, 1])
def test_replay_trajectory_accepts_planned_paths(dur):
    p = near_goal_problem(1 if dur else 0)
    p["duration_mode"] = dur
    P = oracle.OraclePlanner(p)
    st, g, it = P.plan(max_iters=300)
    assert st == oracle.SOLVED
    s = P.state()
    path = P.path(g)
    r = oracle.replay_trajectory(p, _traj_of(p, s, path))
    assert r["valid"] and r["reached"] and r["first_bad"] == -1
    # FP32 storage of the states is the only difference from the FP64 tree
    assert r["worst"] < 1e-6


def test_replay_trajectory_quad_path_and_rejections():
    p = problem_small_quad(seed=4, cap=4000)
    P = oracle.OraclePlanner(p)
    run_iters(P, 5)
    s = P.state()
    node = int(s["N"]) - 1
    path = P.path(node)
    assert len(path) >= 4
    tr = _traj_of(p, s, path)
    r = oracle.replay_trajectory(p, tr)
    assert r["valid"] and not r["reached"] and r["worst"] < 1e-6
    # a changed control: the edge no longer ends at its stored child
    bad = dict(tr, u=tr["u"].copy())
    bad["u"][2, 0] = np.float32(bad["u"][2, 0] * 0.5 + 1.0)
    assert not oracle.replay_trajectory(p, bad)["valid"]
    # an obstacle around the end of the last edge: that edge is invalid
    e = len(path) - 2
    c = tr["x"][-1][:3].astype(np.float64)
    q = dict(p, obstacles=np.vstack([p["obstacles"], np.r_[c - 0.05, c + 0.05][None, :]]).astype(np.float32))
    r = oracle.replay_trajectory(q, tr)
    assert not r["valid"] and r["first_bad"] == e
