"""Pins for where an expansion's x' lies and which region its counter goes to.

Alg. 2 (Sec. III-A.2, Node Extension) propagates x' = PropagateODE(x, u, dt)
over the whole segment, maps x' to its sub-region, and only then tests the
trajectory's validity; an invalid sample increments n_invalid of x''s
region.  The validity test does not move x'.  These pins fix that against
closed forms that do not go through the oracle's own cell map:

* a double-integrator segment that first collides (or first leaves the
  velocity box) in region A and ends in region B counts n_invalid in B;
* over a whole iteration, the n_valid / n_invalid increments per region are
  the histogram of the closed-form Euler end points of the valid / invalid
  lanes;
* a quadcopter segment in pure pitch (theta = theta0 + q t exactly) is
  integrated through its failing step to the exact end state, and the step at
  which it comes near the Euler-angle singularity is recorded;
* a non-finite x' takes its parent's cell;
* the cell-plane ambiguity band agrees with a brute-force distance to the
  grid planes.
"""

import numpy as np
import pytest

import oracle
from workloads import problem_small_di, problem_small_quad


def region_of(p, pos):
    """Region id of a position by direct arithmetic (clamped to the grid)."""
    G = np.asarray(p["grid"], np.int64)
    lo = np.asarray(p["x_lo"], np.float32)[:3].astype(np.float64)
    hi = np.asarray(p["x_hi"], np.float32)[:3].astype(np.float64)
    r = np.floor((np.asarray(pos, np.float64) - lo) / (hi - lo) * G).astype(np.int64)
    r = np.clip(r, 0, G - 1)
    return int((r[2] * G[1] + r[1]) * G[0] + r[0])


def di_closed_form(x0, u, h, k):
    """Euler on p' = v, v' = u after k steps: v0 + k h u, p0 + k h v0 + h^2 u k (k-1) / 2."""
    x0 = np.asarray(x0, np.float64)
    u = np.asarray(u, np.float64)
    v = x0[3:] + k * h * u
    q = x0[:3] + k * h * x0[3:] + h * h * u * k * (k - 1) / 2
    return np.concatenate([q, v])


def single_lane(p, u):
    """Expand the root once with control u and apply it; returns the record
    and the counters before and after."""
    W = oracle.OraclePlanner(p)
    assert W.frontier() == oracle.OK
    before = {k: W.state()[k].copy() for k in ("nv", "ni")}
    rec = W.expand_one(0, 0, control=np.pad(np.asarray(u, np.float32), (0, 4 - len(u))))
    W.apply(np.array([rec], dtype=oracle.RECORD_DTYPE))
    after = {k: W.state()[k].copy() for k in ("nv", "ni")}
    return W, rec, before, after


def di_line_problem(x_init, obstacles):
    p = problem_small_di(seed=1, grid=(16, 16, 16), sub=4)
    p["x_init"] = np.asarray(x_init, np.float32)
    p["obstacles"] = np.asarray(obstacles, np.float32).reshape(-1, 6)
    return p


@pytest.mark.parametrize("case", ["obstacle", "velocity-box"])
def test_invalid_segment_counts_in_its_end_region(case):
    if case == "obstacle":
        # v0 = 9 along x, u = 0.5: positions 1 + 0.9 j + 0.0025 j (j - 1); the
        # swept box of step 3 (x in [2.805, 3.7075] grown by the 0.1 margin)
        # meets the wall x in [3, 3.5] first; the segment ends at x = 10.225
        p = di_line_problem([1, 47, 47, 9, 0, 0], [[3.0, 40, 40, 3.5, 55, 55]])
        u = [0.5, 0.0, 0.0]
        first_fail = 3
    else:
        # v0 = 9.95, u = 1: the velocity leaves |v| <= 10 at step 1 (x = 1.995);
        # the segment ends at x = 11.4
        p = di_line_problem([1, 47, 47, 9.95, 0, 0], np.zeros((0, 6)))
        u = [1.0, 0.0, 0.0]
        first_fail = 1
    h = float(np.float32(p["h"]))
    K = int(p["steps"])
    W, rec, before, after = single_lane(p, u)
    x0 = np.asarray(p["x_init"], np.float32).astype(np.float64)
    uf = np.asarray(u, np.float32).astype(np.float64)
    end = di_closed_form(x0, uf, h, K)
    at_fail = di_closed_form(x0, uf, h, first_fail)
    reg_end, reg_fail = region_of(p, end[:3]), region_of(p, at_fail[:3])
    assert reg_end != reg_fail  # the case separates the two readings
    assert rec["valid"] == 0 and rec["fail"] == first_fail
    assert rec["steps"] == K
    np.testing.assert_allclose(rec["x"][:6], end, rtol=0, atol=1e-12)
    assert rec["cell"] >> 6 == reg_end
    dni = after["ni"].astype(np.int64) - before["ni"].astype(np.int64)
    assert dni[reg_end] == 1 and dni.sum() == 1 and dni[reg_fail] == 0
    assert np.array_equal(after["nv"], before["nv"])


@pytest.mark.parametrize("seed,iters", [(3, 4), (6, 7)])
def test_iteration_counts_are_end_point_histograms(seed, iters):
    p = problem_small_di(seed=seed, n_obs=20, cap=20000)
    W = oracle.OraclePlanner(p)
    for _ in range(iters):
        assert W.iterate()[0] == oracle.OK
    assert W.frontier() == oracle.OK
    s = W.state()
    recs = W.expand_all()
    h = float(np.float32(p["h"]))
    K = int(p["steps"])
    R = len(s["nv"])
    want_v = np.zeros(R, np.int64)
    want_i = np.zeros(R, np.int64)
    G = np.asarray(p["grid"], np.float64)
    for r in recs:
        end = di_closed_form(s["x"][r["parent"]], r["u"][:3].astype(np.float64), h, K)
        # no end point may sit on a region plane (the two sides would differ)
        t = end[:3] / 100.0 * G
        assert np.all(np.abs(t - np.round(t)) > 1e-9)
        reg = region_of(p, end[:3])
        (want_v if r["valid"] else want_i)[reg] += 1
    assert np.sum(recs["valid"] == 0) > 20  # the case has invalid lanes
    W.apply(recs)
    a = W.state()
    assert np.array_equal(a["nv"].astype(np.int64) - s["nv"].astype(np.int64), want_v)
    assert np.array_equal(a["ni"].astype(np.int64) - s["ni"].astype(np.int64), want_i)


def test_invalid_quad_segment_integrates_through_failure():
    """Pure pitch: level, at rest, body rate q only, thrust T and no torque.
    Then p = r = 0 and q stay constant, phi = psi = 0, theta = theta0 + q t
    exactly, and the thrust direction is (sin theta, 0, cos theta), so
      vx = (T/m)(cos th0 - cos th)/q,  vz = (T/m)(sin th - sin th0)/q - g t,
      x  = x0 + (T/m)/q [t cos th0 - (sin th - sin th0)/q],
      z  = z0 + (T/m)/q [(cos th0 - cos th)/q - t sin th0] - g t^2 / 2.
    With theta0 = 0.9 and q = 4.5 the pitch leaves |theta| <= 1 at step 2,
    passes the conditioning bound 1.45 at step 7 and pi/2 near t = 0.15 s; the
    segment still runs its 20 steps to theta = 2.7."""
    p = problem_small_quad(seed=1, n_obs=0)
    p["obstacles"] = np.zeros((0, 6), np.float32)
    th0, q = 0.9, 4.5
    x0 = np.zeros(12, np.float32)
    x0[:3] = (50.0, 50.0, 60.0)
    x0[4] = th0
    x0[10] = q
    p["x_init"] = x0
    T = np.float32(12.0)
    W, rec, before, after = single_lane(p, [T, 0.0, 0.0, 0.0])
    x0 = x0.astype(np.float64)
    th0, q = x0[4], x0[10]
    h = float(np.float32(p["h"]))
    K = int(p["steps"])
    prm = np.asarray(p["dyn_params"], np.float32).astype(np.float64)
    a, g = float(T) / prm[0], prm[1]
    t = K * h
    th = th0 + q * t
    vx = a * (np.cos(th0) - np.cos(th)) / q
    vz = a * (np.sin(th) - np.sin(th0)) / q - g * t
    px = x0[0] + a / q * (t * np.cos(th0) - (np.sin(th) - np.sin(th0)) / q)
    pz = x0[2] + a / q * ((np.cos(th0) - np.cos(th)) / q - t * np.sin(th0)) - g * t * t / 2
    want = np.array([px, x0[1], pz, 0.0, th, 0.0, vx, 0.0, vz, 0.0, q, 0.0])
    assert rec["valid"] == 0 and rec["fail"] == 2 and rec["steps"] == K
    # RK4's truncation error on the thrust terms is far below 1e-6 at h = 0.02
    np.testing.assert_allclose(rec["x"][:12], want, rtol=0, atol=1e-6)
    assert rec["x"][4] == pytest.approx(th, abs=1e-12)
    assert rec["cond_step"] == 7
    reg = region_of(p, want[:3])
    assert rec["cell"] >> 6 == reg
    dni = after["ni"].astype(np.int64) - before["ni"].astype(np.int64)
    assert dni[reg] == 1 and dni.sum() == 1


def test_well_conditioned_records():
    """Double-integrator states are always well conditioned (finite, no
    singularity); a level quadcopter's first expansions are too."""
    p = problem_small_di(seed=2)
    W = oracle.OraclePlanner(p)
    for _ in range(3):
        W.iterate()
    W.frontier()
    recs = W.expand_all()
    assert np.all(recs["cond_step"] == recs["k_seg"] + 1)
    assert np.all((recs["fail"] >= 1) & (recs["fail"] <= recs["k_seg"] + 1))
    assert np.array_equal(recs["valid"] == 1, recs["fail"] == recs["k_seg"] + 1)


def test_non_finite_end_takes_parent_cell():
    p = problem_small_quad(cap=2000)
    prm = np.array(p["dyn_params"], np.float32)
    prm[0] = np.nan  # mass: every end state is NaN
    p["dyn_params"] = prm
    W = oracle.OraclePlanner(p)
    st, g, it = W.plan(max_iters=3)
    s = W.state()
    assert s["N"] == 1
    root_region = int(s["cell"][0]) >> 6
    assert int(s["ni"][root_region]) == s["sum_lanes"] > 0
    assert int(s["ni"].sum()) == s["sum_lanes"]


def test_cell_plane_band_brute_force():
    """kpo_near_cell_plane(p, tol) against the distance to the nearest interior
    plane lo + k (hi - lo) / na, k = 1 .. na - 1, per axis.  Points are drawn
    either well inside the band (< tol / 2) or well outside it (> 2 tol)."""
    p = problem_small_di(grid=(5, 6, 7), sub=3)
    tol = 1e-4
    na = np.asarray(p["grid"]) * int(p["sub"])
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(3000):
        pos = rng.uniform(0.0, 100.0, 3)
        if rng.random() < 0.5:  # move one axis next to a plane
            a = rng.integers(3)
            k = rng.integers(0, na[a] + 1)  # includes the outer faces
            pos[a] = 100.0 * k / na[a] + rng.uniform(-3 * tol, 3 * tol)
        d = np.inf
        for a in range(3):
            planes = 100.0 * np.arange(1, na[a]) / na[a]
            d = min(d, float(np.min(np.abs(pos[a] - planes))))
        if tol / 2 <= d <= 2 * tol:
            continue
        assert oracle.near_cell_plane(p, pos, tol) == (d < tol), (pos, d)
        checked += 1
    assert checked > 2000
