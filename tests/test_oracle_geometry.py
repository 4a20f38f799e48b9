"""Pins for validity (state box, swept-box collision) and the cell map.

Collision: the swept axis-aligned box of two consecutive positions, grown by
the margin, is tested against closed obstacle boxes.  Brute force: a dense
lattice over the grown box (faces included) must contain a point inside an
obstacle exactly when the test reports a hit, on random configurations kept
away from touching (within the lattice spacing); and dense sampling of the
straight segment never finds a hit the box test misses (superset).

Cell map: the returned (region, sub-cell) pair is decoded back into a box,
which must contain the point; points outside W clamp to the border cells.
"""

import numpy as np
import pytest

import oracle
from workloads import problem_small_di


def scene(obstacles, margin=0.1):
    p = problem_small_di()
    p["obstacles"] = np.asarray(obstacles, np.float32).reshape(-1, 6)
    p["margin"] = np.float32(margin)
    return p


def lattice_hit(lo, hi, obs, n=24):
    axes = [np.linspace(lo[a], hi[a], n) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    for o in obs:
        inside = np.all((P >= o[:3]) & (P <= o[3:]), axis=1)
        if inside.any():
            return True
    return False


def gap_or_overlap(lo, hi, o):
    # smallest |distance| between a face of the grown box and the facing face
    # of the obstacle along each axis
    d = []
    for a in range(3):
        d.append(abs(lo[a] - o[3 + a]))
        d.append(abs(o[a] - hi[a]))
    return min(d)


@pytest.mark.parametrize("seed", range(6))
def test_swept_box_equals_lattice_bruteforce(seed):
    rng = np.random.default_rng(seed)
    checked = 0
    while checked < 150:
        o_lo = rng.uniform(0, 20, 3)
        o = np.concatenate([o_lo, o_lo + rng.uniform(1, 6, 3)]).astype(np.float32).astype(np.float64)
        p0 = rng.uniform(-2, 28, 3)
        p1 = p0 + rng.uniform(-3, 3, 3)
        margin = 0.1
        lo = np.minimum(p0, p1) - margin
        hi = np.maximum(p0, p1) + margin
        spacing = np.max(hi - lo) / 23
        if gap_or_overlap(lo, hi, o) < 2 * spacing:
            continue
        p = scene([o], margin)
        got = oracle.swept_hit(p, p0, p1)
        assert got == lattice_hit(lo, hi, [o])
        checked += 1


@pytest.mark.parametrize("seed", range(4))
def test_swept_box_is_superset_of_segment(seed):
    rng = np.random.default_rng(100 + seed)
    obs = []
    for _ in range(3):
        lo = rng.uniform(0, 20, 3)
        obs.append(np.concatenate([lo, lo + rng.uniform(1, 5, 3)]))
    obs = np.asarray(obs, np.float32).astype(np.float64)
    p = scene(obs, 0.0)
    t = np.linspace(0, 1, 2001)[:, None]
    for _ in range(300):
        p0 = rng.uniform(-2, 25, 3)
        p1 = p0 + rng.uniform(-4, 4, 3)
        pts = p0 + t * (p1 - p0)
        seg_hit = any(np.all((pts >= o[:3]) & (pts <= o[3:]), axis=1).any() for o in obs)
        if seg_hit:
            assert oracle.swept_hit(p, p0, p1, 0.0)


def test_swept_box_touching_counts():
    o = [10, 10, 10, 12, 12, 12]
    p = scene([o], 0.0)
    assert oracle.swept_hit(p, [9, 11, 11], [10, 11, 11], 0.0)          # touches the face
    assert not oracle.swept_hit(p, [9, 11, 11], [9.999, 11, 11], 0.0)   # short of it
    assert oracle.swept_hit(p, [9, 11, 11], [9.95, 11, 11], 0.05)       # margin closes the gap


def test_state_box_and_finiteness():
    p = problem_small_di()
    x = np.array([50, 50, 50, 0, 0, 0], np.float64)
    assert oracle.state_ok(p, x)
    for i, bad in [(0, -1e-9), (2, 100.0 + 1e-9), (3, 10.0 + 1e-9), (5, -10.0 - 1e-9)]:
        y = x.copy()
        y[i] = bad
        assert not oracle.state_ok(p, y)
        assert oracle.state_ok(p, y, relax=1e-6)
    y = x.copy()
    y[1] = np.nan
    assert not oracle.state_ok(p, y, relax=1e9)
    y[1] = np.inf
    assert not oracle.state_ok(p, y, relax=1e300)
    y = x.copy()
    y[4] = 10.0  # closed box: the bound itself is valid
    assert oracle.state_ok(p, y)


def decode_cell(p, cell):
    G = p["grid"]
    S = p["sub"]
    region, local = cell >> 6, cell & 63
    rx = region % G[0]
    ry = (region // G[0]) % G[1]
    rz = region // (G[0] * G[1])
    sx = local % S
    sy = (local // S) % S
    sz = local // (S * S)
    return np.array([rx * S + sx, ry * S + sy, rz * S + sz]), region


@pytest.mark.parametrize("grid,sub", [((8, 8, 8), 4), ((16, 16, 16), 4), ((5, 7, 3), 3),
                                      ((4, 4, 4), 1), ((32, 32, 32), 2)])
def test_cell_map_enumeration(grid, sub):
    p = problem_small_di(grid=grid, sub=sub)
    lo = np.asarray(p["x_lo"][:3], np.float64)
    hi = np.asarray(p["x_hi"][:3], np.float64)
    na = np.array(grid) * sub
    w = (hi - lo) / na
    rng = np.random.default_rng(1)
    pts = rng.uniform(lo, hi, size=(3000, 3))
    for q in pts:
        c = oracle.cell_of(p, q)
        idx, region = decode_cell(p, c)
        assert np.all(idx >= 0) and np.all(idx < na)
        cl = lo + idx * w
        # containment up to rounding at the plane itself
        assert np.all(q >= cl - 1e-9) and np.all(q <= cl + w + 1e-9)
        assert (c & 63) < sub ** 3
        rbox_lo = lo + (idx // sub) * sub * w
        assert np.all(q >= rbox_lo - 1e-9) and np.all(q <= rbox_lo + sub * w + 1e-9)
        assert region < grid[0] * grid[1] * grid[2]
    # outside W clamps to the border cells
    c = oracle.cell_of(p, [-5.0, 150.0, 50.0])
    idx, _ = decode_cell(p, c)
    assert idx[0] == 0 and idx[1] == na[1] - 1
