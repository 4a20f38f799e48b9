"""Pins for UpdateEstimates (Alg. 3, eqs. 3-5), Lemma 1 and eq. (6).

The oracle drops the common factor vol(R_i)^4 (equal for every region of a
uniform grid) and sums scores exactly as integers.  These tests evaluate the
paper's formulas literally -- FreeVol with the region volume, Score, then
P_accept with an exact rational sum -- and compare.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import problem_small_di

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def literal_score(delta, nv, ni, cov, vol):
    """Eqs. (3) and (4) in exact rational arithmetic, volume included."""
    d = Fraction(str(delta))
    free_vol = (d + nv) * vol / (d + nv + ni)
    return free_vol ** 4 / ((1 + cov) * (1 + (nv + ni) ** 2))


def test_hand_cases():
    with open(os.path.join(GOLDEN, "region_score_cases.json")) as f:
        cases = json.load(f)["cases"]
    vol = Fraction(125, 64) * 1000  # (100 / 8)^3, the c1 region volume
    for c in cases:
        want = literal_score(c["delta"], c["nv"], c["ni"], c["cov"], vol) / vol ** 4
        if "score_exact" in c:
            assert want == Fraction(c["score_exact"])
        got = oracle.region_score(c["delta"], c["nv"], c["ni"], c["cov"])
        assert got == pytest.approx(float(want), rel=1e-14)


def test_single_available_region_has_p_one():
    R = 8
    avail = np.zeros(R, np.uint8)
    avail[3] = 1
    e = oracle.estimates(avail, np.full(R, 7), np.full(R, 9), np.full(R, 3), 1e-3, 1e-2)
    assert np.all(e["P"] == 1.0)
    assert np.all(e["thr"] == 2**32)


@pytest.mark.parametrize("k", [2, 3, 7, 100, 1000])
def test_equal_scores(k):
    R = k + 5
    avail = np.zeros(R, np.uint8)
    avail[:k] = 1
    nv = np.full(R, 11)
    ni = np.full(R, 4)
    vis = np.full(R, 0b1011)
    e = oracle.estimates(avail, nv, ni, vis, 1e-3, 1e-2)
    want = 1.0 / k + 1e-2
    assert np.all(e["P"][:k] == min(1.0, want))
    assert np.all(e["P"][k:] == 1.0)  # regions outside R_avail keep P_accept = 1


@pytest.mark.parametrize("seed", range(8))
def test_p_accept_matches_literal_eq5(seed):
    rng = np.random.default_rng(seed)
    R = int(rng.integers(20, 600))
    avail = (rng.random(R) < 0.7).astype(np.uint8)
    avail[0] = 1
    scale = 10 ** rng.uniform(0, 5, R)
    nv = (rng.random(R) * scale).astype(np.uint64)
    ni = (rng.random(R) * scale).astype(np.uint64)
    vis = rng.integers(0, 2**63, R, dtype=np.uint64) & rng.integers(0, 2**63, R, dtype=np.uint64)
    delta, eps = 1e-3, 1e-2
    e = oracle.estimates(avail, nv, ni, vis, delta, eps)
    vol = Fraction(15625, 8)
    S = {r: literal_score(delta, int(nv[r]), int(ni[r]), bin(int(vis[r])).count("1"), vol)
         for r in range(R) if avail[r]}
    total = sum(S.values())
    unclamped = 0.0
    for r in range(R):
        P = e["P"][r]
        assert eps <= P <= 1.0  # Lemma 1
        if not avail[r]:
            assert P == 1.0 and e["thr"][r] == 2**32
            continue
        lit = min(Fraction(1), S[r] / total + Fraction(eps))
        # deviation bounded by the integer quantisation of the sum (2^-46 relative per region)
        assert abs(P - float(lit)) <= 1e-9
        if P < 1.0:
            assert e["thr"][r] == int(np.floor(P * 2.0**32))
            unclamped += P - eps
        else:
            assert e["thr"][r] == 2**32
    if all(e["P"][avail == 1] < 1.0):
        assert unclamped == pytest.approx(1.0, abs=1e-9)


def small_planner():
    return oracle.OraclePlanner(problem_small_di(cap=1000, lambda_max=6))


@pytest.mark.parametrize("N,nE,lam_max,cap,want", [
    (1, 1, 6, 1000, 6),          # early: lambda_max
    (900, 30, 6, 1000, 3),       # floor(100 / 30) = 3
    (990, 11, 6, 1000, 0),       # floor(10 / 11) = 0 -> tree full
    (999, 1, 6, 1000, 1),
])
def test_branching_factor_eq6(N, nE, lam_max, cap, want):
    p = problem_small_di(cap=cap, lambda_max=lam_max)
    P = oracle.OraclePlanner(p)
    lib = oracle.lib()
    lib.kpo_set_counters(P.h, N, 0)
    v = P.view()
    flag = np.ctypeslib.as_array(v.flag, (cap,))
    flag[:] = 0
    idx = np.linspace(0, N - 1, nE).astype(int)
    flag[idx] = 1
    st = P.frontier()
    s = P.state()
    assert s["lam"] == want
    assert list(s["F"]) == sorted(set(idx.tolist()))
    assert st == (oracle.TREE_FULL if want == 0 else oracle.OK)


def test_frontier_empty():
    P = small_planner()
    v = P.view()
    np.ctypeslib.as_array(v.flag, (v.cap,))[:] = 0
    assert P.frontier() == oracle.FRONTIER_EMPTY
