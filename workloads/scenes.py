"""Scene and problem generators (numpy PCG64, seeded).

Every floating-point value is rounded to float32 here, so that the GPU
library (which takes float32 geometry) and the FP64 oracle (which widens the
same float32 numbers exactly) see bit-identical inputs.

A problem is a plain dict:

    dynamics      DI6 (6D double integrator) or QUAD12 (12D quadcopter)
    integrator    EULER or RK4
    h, steps      integration step and steps per segment (segment time = h*steps)
    dyn_params    float32[8]; quadcopter: mass, gravity, Ixx, Iyy, Izz
    u_lo, u_hi    control box U
    x_lo, x_hi    valid state box; its first three components are the workspace W
    obstacles     float32[n, 6] closed boxes (lo xyz, hi xyz)
    margin        collision inflation
    x_init        initial state
    goal_center, goal_radius   X_goal, a closed ball in position
    grid, sub     regions per axis (workspace grid), sub-regions per region axis
    node_cap      t_e, the maximum tree size
    lambda_max    maximum branching factor
    delta, epsilon  constants of the region score and acceptance probability
    seed          planner seed (Philox key)
    t_max_ms, max_iters  time and iteration budget

Paper context: the problem objects follow Problem 1 and the experiments
section (systems, three 3D environments, t_e and lambda_max settings).  The
paper's Forest / Narrow Passage / Building scene data are not available; the
scenes here are synthetic stand-ins with the sizes of the workloads.
"""

from __future__ import annotations

import numpy as np

DI6 = 0
QUAD12 = 1
EULER = 0
RK4 = 1

W_LO = 0.0
W_HI = 100.0

f32 = np.float32


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def _point_box_dist(p, box):
    """Euclidean distance from point p to a closed box (lo3, hi3)."""
    lo, hi = box[:3], box[3:]
    d = np.maximum(np.maximum(lo - p, 0.0), p - hi)
    return float(np.sqrt(np.sum(d * d)))


def random_boxes(seed, n, side_lo, side_hi, start, goal_c, goal_r,
                 start_clear=1.0, goal_clear=1.0):
    """n axis-aligned boxes with per-axis sides U[side_lo, side_hi] and min
    corner U[0, 100 - side], redrawn while within start_clear of the start or
    within goal_r + goal_clear of the goal centre."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    start = np.asarray(start, np.float64)
    goal_c = np.asarray(goal_c, np.float64)
    while len(out) < n:
        side = rng.uniform(side_lo, side_hi, size=3)
        lo = rng.uniform(0.0, W_HI - side)
        box = _f32(np.concatenate([lo, lo + side])).astype(np.float64)
        if _point_box_dist(start, box) < start_clear:
            continue
        if _point_box_dist(goal_c, box) < goal_r + goal_clear:
            continue
        out.append(box)
    return _f32(np.array(out).reshape(-1, 6))


def forest(seed, n, start, goal_c, goal_r, foot=2.0, h_lo=20.0, h_hi=100.0,
           clear=2.0):
    """n vertical pillars: footprint foot x foot with corner U[0, 100-foot]^2,
    from z = 0 up to a height U[h_lo, h_hi]; redrawn while within `clear` of
    the start or of the goal ball."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    start = np.asarray(start, np.float64)
    goal_c = np.asarray(goal_c, np.float64)
    while len(out) < n:
        xy = rng.uniform(0.0, W_HI - foot, size=2)
        top = rng.uniform(h_lo, h_hi)
        box = _f32([xy[0], xy[1], 0.0, xy[0] + foot, xy[1] + foot, top]).astype(np.float64)
        if _point_box_dist(start, box) < clear:
            continue
        if _point_box_dist(goal_c, box) < goal_r + clear:
            continue
        out.append(box)
    return _f32(np.array(out).reshape(-1, 6))


def building(seed, n_total=1200, floors=3, rooms=4, wall=0.5, slab=1.0,
             door_w=2.0, door_h=2.0, hatch=2.0, clutter_side=(1.0, 4.0)):
    """A multi-floor building inside [0,100]^3 made of exactly n_total boxes.

    Floors are separated by slabs of thickness `slab`, each with one square
    hatch of side `hatch` (cut by splitting the slab into four boxes).  Every
    floor is a rooms x rooms grid of rooms separated by walls of thickness
    `wall`; every wall between two adjacent rooms has one doorway door_w wide
    and door_h high at floor level (cut by splitting the wall into three boxes).
    The remainder up to n_total is seeded clutter inside rooms, kept clear of
    doorways, hatches, the start room corner and the goal room corner.
    Returns (boxes, start_pos, goal_center).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    H = W_HI / floors
    cell = W_HI / rooms
    boxes = []
    keepout = []  # boxes (lo, hi) that clutter must avoid
    # slabs between floors, each with a hatch
    for f in range(1, floors):
        z0 = f * H - slab / 2
        z1 = z0 + slab
        # hatch position alternates corners so that the path must cross floors
        if f % 2 == 1:
            hx, hy = W_HI - cell / 2, W_HI - cell / 2
        else:
            hx, hy = cell / 2, cell / 2
        hx0, hx1 = hx - hatch / 2, hx + hatch / 2
        hy0, hy1 = hy - hatch / 2, hy + hatch / 2
        boxes.append([0, 0, z0, hx0, W_HI, z1])
        boxes.append([hx1, 0, z0, W_HI, W_HI, z1])
        boxes.append([hx0, 0, z0, hx1, hy0, z1])
        boxes.append([hx0, hy1, z0, hx1, W_HI, z1])
        keepout.append([hx0 - 3, hy0 - 3, z0 - H / 2, hx1 + 3, hy1 + 3, z1 + H / 2])
    # interior walls per floor with doorways
    for f in range(floors):
        zf0 = f * H + (slab / 2 if f > 0 else 0.0)
        zf1 = (f + 1) * H - (slab / 2 if f < floors - 1 else 0.0)
        for k in range(1, rooms):
            c = k * cell
            for j in range(rooms):
                a0, a1 = j * cell, (j + 1) * cell
                # doorway centre along the wall, away from the corners
                dc = rng.uniform(a0 + 4.0, a1 - 4.0)
                d0, d1 = dc - door_w / 2, dc + door_w / 2
                # wall normal to x at x = c spanning y in [a0, a1]
                boxes.append([c - wall / 2, a0, zf0, c + wall / 2, d0, zf1])
                boxes.append([c - wall / 2, d1, zf0, c + wall / 2, a1, zf1])
                boxes.append([c - wall / 2, d0, zf0 + door_h, c + wall / 2, d1, zf1])
                keepout.append([c - 3, d0 - 1, zf0, c + 3, d1 + 1, zf0 + door_h + 2])
                # wall normal to y at y = c spanning x in [a0, a1]
                dc = rng.uniform(a0 + 4.0, a1 - 4.0)
                d0, d1 = dc - door_w / 2, dc + door_w / 2
                boxes.append([a0, c - wall / 2, zf0, d0, c + wall / 2, zf1])
                boxes.append([d1, c - wall / 2, zf0, a1, c + wall / 2, zf1])
                boxes.append([d0, c - wall / 2, zf0 + door_h, d1, c + wall / 2, zf1])
                keepout.append([d0 - 1, c - 3, zf0, d1 + 1, c + 3, zf0 + door_h + 2])
    start = np.array([5.0, 5.0, 2.0])
    goal_c = np.array([W_HI - 8.0, W_HI - 8.0, (floors - 1) * H + 6.0])
    keepout.append([0, 0, 0, 12, 12, 12])
    keepout.append([goal_c[0] - 9, goal_c[1] - 9, goal_c[2] - 9,
                    goal_c[0] + 9, goal_c[1] + 9, goal_c[2] + 9])
    keepout = np.array(keepout, np.float64)
    if len(boxes) > n_total:
        raise ValueError("building skeleton has more boxes than n_total")
    while len(boxes) < n_total:
        side = rng.uniform(clutter_side[0], clutter_side[1], size=3)
        lo = rng.uniform(0.0, W_HI - side)
        hi = lo + side
        ok = True
        for ko in keepout:
            if np.all(lo <= ko[3:]) and np.all(ko[:3] <= hi):
                ok = False
                break
        if ok:
            boxes.append([lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]])
    return _f32(np.array(boxes, np.float64)), start, goal_c


def _base(dynamics, integrator, h, steps):
    return dict(dynamics=dynamics, integrator=integrator, h=f32(h), steps=int(steps))


def _di_fields(x_init, v_max=10.0, u_max=1.0):
    return dict(
        dyn_params=_f32(np.zeros(8)),
        u_lo=_f32([-u_max] * 3),
        u_hi=_f32([u_max] * 3),
        x_lo=_f32([W_LO] * 3 + [-v_max] * 3),
        x_hi=_f32([W_HI] * 3 + [v_max] * 3),
        x_init=_f32(x_init),
    )


QUAD_PARAMS = (1.0, 9.81, 0.02, 0.02, 0.04)  # mass, gravity, Ixx, Iyy, Izz


def _quad_fields(x_init, v_max=10.0, w_max=5.0, tilt_max=1.0):
    m, g = QUAD_PARAMS[0], QUAD_PARAMS[1]
    prm = np.zeros(8)
    prm[:5] = QUAD_PARAMS
    return dict(
        dyn_params=_f32(prm),
        u_lo=_f32([0.0, -0.1, -0.1, -0.1]),
        u_hi=_f32([2.0 * m * g, 0.1, 0.1, 0.1]),
        x_lo=_f32([W_LO] * 3 + [-tilt_max, -tilt_max, -1000.0] + [-v_max] * 3 + [-w_max] * 3),
        x_hi=_f32([W_HI] * 3 + [tilt_max, tilt_max, 1000.0] + [v_max] * 3 + [w_max] * 3),
        x_init=_f32(x_init),
    )


def _planner_fields(grid, sub, cap, lambda_max, seed, margin=0.1,
                    delta=1e-3, epsilon=1e-2, t_max_ms=60000.0, max_iters=100000):
    return dict(grid=[int(g) for g in grid], sub=int(sub), node_cap=int(cap),
                lambda_max=int(lambda_max), seed=int(seed), margin=f32(margin),
                delta=float(delta), epsilon=float(epsilon),
                t_max_ms=float(t_max_ms), max_iters=int(max_iters))


def problem_c1(seed=0, scene_seed=1, **kw):
    """6D double integrator, Euler h=0.1 x 10, 20 random boxes side U[5,15],
    start (5,5,5,0,0,0), goal ball r=5 at (95,95,95), 8^3 regions,
    32768-node cap, 4 samples per frontier node."""
    start = [5.0, 5.0, 5.0]
    goal = [95.0, 95.0, 95.0]
    p = _base(DI6, EULER, 0.1, 10)
    p.update(_di_fields(start + [0.0, 0.0, 0.0]))
    p.update(obstacles=random_boxes(scene_seed, 20, 5.0, 15.0, start, goal, 5.0),
             goal_center=_f32(goal), goal_radius=f32(5.0))
    p.update(_planner_fields((8, 8, 8), 4, 32768, 4, seed))
    p["name"] = "c1-di6-boxes20"
    p.update(kw)
    return p


def problem_c2(seed=0, scene_seed=2, **kw):
    """12D quadcopter, RK4 h=0.02 x 20, forest of 300 pillars 2x2x[20,100],
    start (5,5,10) at rest, goal ball r=5 at (95,95,10), 16^3 regions,
    4,194,304-node cap.  The workload does not fix the samples per frontier
    node; lambda_max = 4 is the value that solved every query of a 12-seed
    sweep over {4, 6, 8, 12, 16, 32} with the lowest median time."""
    start = [5.0, 5.0, 10.0]
    goal = [95.0, 95.0, 10.0]
    p = _base(QUAD12, RK4, 0.02, 20)
    p.update(_quad_fields(start + [0.0] * 9))
    p.update(obstacles=forest(scene_seed, 300, start, goal, 5.0),
             goal_center=_f32(goal), goal_radius=f32(5.0))
    p.update(_planner_fields((16, 16, 16), 4, 4194304, 4, seed))
    p["name"] = "c2-quad12-forest300"
    p.update(kw)
    return p


def problem_c5(seed=0, scene_seed=5, **kw):
    """6D double integrator, Euler h=0.1 x 10, 3-floor building of 1200 boxes
    with 2-unit doorways, 32^3 regions, 8,388,608-node cap, lambda_max 8."""
    boxes, start, goal = building(scene_seed)
    p = _base(DI6, EULER, 0.1, 10)
    p.update(_di_fields(list(start) + [0.0, 0.0, 0.0]))
    p.update(obstacles=boxes, goal_center=_f32(goal), goal_radius=f32(5.0))
    p.update(_planner_fields((32, 32, 32), 4, 8388608, 8, seed))
    p["name"] = "c5-di6-building1200"
    p.update(kw)
    return p


def problem_small_di(seed=0, scene_seed=11, n_obs=12, cap=4096, lambda_max=4,
                     grid=(8, 8, 8), sub=4, integrator=EULER, **kw):
    """A scaled-down c1: same dynamics and workspace, fewer boxes, small cap."""
    start = [5.0, 5.0, 5.0]
    goal = [95.0, 95.0, 95.0]
    p = _base(DI6, integrator, 0.1, 10)
    p.update(_di_fields(start + [0.0, 0.0, 0.0]))
    p.update(obstacles=random_boxes(scene_seed, n_obs, 5.0, 15.0, start, goal, 5.0),
             goal_center=_f32(goal), goal_radius=f32(5.0))
    p.update(_planner_fields(grid, sub, cap, lambda_max, seed))
    p["name"] = "small-di6"
    p.update(kw)
    return p


def problem_small_quad(seed=0, scene_seed=12, n_obs=60, cap=8192, lambda_max=32,
                       grid=(16, 16, 16), sub=4, **kw):
    """A scaled-down c2: same quadcopter and forest statistics, small cap."""
    start = [5.0, 5.0, 10.0]
    goal = [95.0, 95.0, 10.0]
    p = _base(QUAD12, RK4, 0.02, 20)
    p.update(_quad_fields(start + [0.0] * 9))
    p.update(obstacles=forest(scene_seed, n_obs, start, goal, 5.0),
             goal_center=_f32(goal), goal_radius=f32(5.0))
    p.update(_planner_fields(grid, sub, cap, lambda_max, seed))
    p["name"] = "small-quad12"
    p.update(kw)
    return p


def problem_batch(n=256, batch_seed=3, dynamics=DI6, obs_range=(10, 2000),
                  cap_range=(16384, 1048576), min_sep=50.0, occupancy=0.03, **kw):
    """Independent queries of uneven size for batched planning.  Query k has
    its own generator PCG64([batch_seed, k]): an obstacle count and a node cap
    drawn log-uniformly from obs_range and cap_range, box sides around
    s = (occupancy * 100^3 / count)^(1/3) (per axis U[s/2, 3s/2], so the
    occupied volume stays near `occupancy` whatever the count), and a start
    and a goal centre uniform in [5, 95]^3 at least min_sep apart, the start
    at rest.  Double integrator (c1 dynamics, 8^3 regions) or quadcopter (c2
    dynamics, 16^3 regions); lambda_max 4; planner seed k."""
    out = []
    for k in range(n):
        rng = np.random.Generator(np.random.PCG64([batch_seed, k]))
        n_obs = int(round(np.exp(rng.uniform(np.log(obs_range[0]), np.log(obs_range[1])))))
        cap = int(round(np.exp(rng.uniform(np.log(cap_range[0]), np.log(cap_range[1])))))
        while True:
            start = rng.uniform(5.0, 95.0, size=3)
            goal = rng.uniform(5.0, 95.0, size=3)
            if np.linalg.norm(goal - start) >= min_sep:
                break
        s = (occupancy * W_HI ** 3 / n_obs) ** (1.0 / 3.0)
        start = [float(v) for v in _f32(start)]
        goal = [float(v) for v in _f32(goal)]
        obs = random_boxes(int(rng.integers(1 << 31)), n_obs, 0.5 * s, 1.5 * s, start, goal, 5.0)
        if dynamics == DI6:
            p = _base(DI6, EULER, 0.1, 10)
            p.update(_di_fields(start + [0.0] * 3))
            grid = (8, 8, 8)
        else:
            p = _base(QUAD12, RK4, 0.02, 20)
            p.update(_quad_fields(start + [0.0] * 9))
            grid = (16, 16, 16)
        p.update(obstacles=obs, goal_center=_f32(goal), goal_radius=f32(5.0))
        p.update(_planner_fields(grid, 4, cap, 4, k))
        p["name"] = f"c3-batch-{'di6' if dynamics == DI6 else 'quad12'}-q{k}"
        p.update(kw)
        out.append(p)
    return out
