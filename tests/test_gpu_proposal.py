"""GPU parity of the learned control proposal: the MFMA network (forward,
gradient, Adam step) against the FP64 reference on seeded inputs, the
planner's per-frontier Gaussian and mixture draws in lock-step with the
oracle, training rows logged from a path, and learned-proposal plans that
replay in FP64."""

import sys

import ctypes as C

import numpy as np
import pytest

import oracle
from oracle import proposal as P
from workloads import mlp_inputs, problem_small_di, problem_small_quad, problem_c2

import lockstep
from test_gpu_plan import replay_path_edgewise

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device="cuda:0")


def packed(params):
    import paper_2409_06807_amd as kp
    return kp.mlp_pack(dev(params))


# Tolerance of a network output (derived): each BF16 rounding of an input or
# hidden activation that lands on the neighbouring BF16 value because the two
# sides' sums differ in the last bits moves an output by at most 2^-8 of the
# absolute-value network (P.abs_scale); 2^-6 allows four such roundings in one
# row.  FP32 accumulation over at most 128 terms adds < 1e-6 of the same scale.
def out_tol(params, X):
    return 2.0 ** -6 * P.abs_scale(params, X) + 1e-6


@pytest.mark.parametrize("rows", [0, 1, 37, 1000, 4099])
def test_forward_matches_reference(rows):
    import paper_2409_06807_amd as kp
    _say(f"mlp forward rows={rows}")
    params = mlp_inputs.params(1, scale=1.0, out_scale=1.0)
    X = mlp_inputs.features(2, rows)
    out = kp.mlp_forward(packed(params), dev(X)).cpu().numpy().astype(np.float64)
    assert out.shape == (rows, 8)
    if rows == 0:
        return
    ref, _ = P.forward(params, X)
    err = np.abs(out - ref)
    tol = out_tol(params, X)
    assert np.all(err <= tol), float(np.max(err / tol))
    # almost every row sees no rounding flip at all: FP32 sums only
    assert np.median(err / P.abs_scale(params, X)) < 1e-5


def test_forward_special_network():
    """Identity-like network on BF16-exact inputs: the output is relu(x) exactly."""
    import paper_2409_06807_amd as kp
    _say("mlp forward identity network")
    W1 = np.zeros((128, 16))
    W1[:16, :16] = np.eye(16)
    W3 = np.zeros((8, 128))
    W3[:, :8] = np.eye(8)
    params = P.pack(W1, np.zeros(128), np.eye(128), np.zeros(128), W3, np.zeros(8))
    X = np.round(mlp_inputs.features(3, 70) * 64.0) / 64.0
    out = kp.mlp_forward(packed(params), dev(X)).cpu().numpy()
    assert np.array_equal(out, np.maximum(X[:, :8], 0.0).astype(np.float32))


def grad_tol(params, X, T, m):
    # each product term carries at most a few BF16 roundings (2^-8 relative
    # each) plus the occasional activation flip of the forward pass
    return 2.0 ** -5 * P.loss_grad_abs(params, X, T, m) + 1e-7


@pytest.mark.parametrize("m,batch,key", [(4, 64 * 3 + 17, 0), (3, 64, 0), (4, 128, 77)])
def test_gradient_matches_reference(m, batch, key):
    import paper_2409_06807_amd as kp
    _say(f"mlp grad m={m} batch={batch} key={key}")
    params = mlp_inputs.params(4, scale=1.0, out_scale=1.0)
    n_rows = batch if key == 0 else 500
    X = mlp_inputs.features(5, n_rows)
    T = mlp_inputs.targets(6, n_rows)
    step = 3
    partials, loss = kp.mlp_grad(packed(params), dev(X), dev(T), m, batch, key, step)
    g = partials.cpu().numpy().astype(np.float64).sum(axis=0)
    rows = np.arange(batch) if key == 0 else P.batch_rows(key, step, batch, n_rows)
    L, ref = P.loss_grad(params, X[rows], T[rows], m)
    assert abs(float(loss.sum()) - L) <= 1e-3 * abs(L) + 1e-5
    tol = grad_tol(params, X[rows], T[rows], m)
    assert np.all(np.abs(g - ref) <= tol), float(np.max(np.abs(g - ref) / tol))
    assert np.linalg.norm(g - ref) <= 1e-2 * np.linalg.norm(ref)
    # unused control slots get exactly zero
    if m == 3:
        W3g = g[P.OFF_W3:P.OFF_B3].reshape(8, 128)
        assert not W3g[3].any() and not W3g[7].any()


def test_adam_matches_reference():
    import paper_2409_06807_amd as kp
    _say("mlp adam")
    params = mlp_inputs.params(7)
    m1, m2 = mlp_inputs.moments(8)
    parts = mlp_inputs.partials(9, 5)
    t = 7
    # the entry point takes FP32 hyperparameters: the reference gets the same values
    lr, b1, b2, eps = (float(np.float32(v)) for v in (2e-3, 0.9, 0.999, 1e-8))
    tp, t1, t2 = dev(params), dev(m1), dev(m2)
    kp.mlp_adam(tp, t1, t2, dev(parts), t, lr, b1, b2, eps)
    ref, r1, r2 = P.adam(params, m1, m2, parts.sum(axis=0), t, lr, b1, b2, eps)
    got = tp.cpu().numpy().astype(np.float64)
    # Derived FP32 bounds: each sum of a few products carries at most a few
    # roundings (2^-24 relative) of the magnitudes summed; the FP32 sum of the
    # partial gradients is the first of them.
    u = 2.0 ** -24
    gabs = np.abs(parts).sum(axis=0)
    g = parts.sum(axis=0)
    e1 = 4 * u * (b1 * np.abs(m1) + (1 - b1) * gabs * 5)
    e2 = 4 * u * (b2 * m2 + (1 - b2) * gabs * (np.abs(g) + gabs) * 5)
    assert np.all(np.abs(t1.cpu().numpy() - r1) <= e1)
    assert np.all(np.abs(t2.cpu().numpy() - r2) <= e2)
    ibc1, ibc2 = 1 / (1 - b1 ** t), 1 / (1 - b2 ** t)
    den = np.sqrt(r2 * ibc2) + eps
    ratio = np.abs(r1) * ibc1 / den
    e_step = lr * (e1 * ibc1 / den + ratio * (0.5 * e2 / r2 + 8 * u))
    assert np.all(np.abs(got - ref) <= e_step + 2 * np.spacing(np.abs(ref).astype(np.float32)))


LOCK_CASES = {
    "di": lambda: problem_small_di(seed=5, cap=4096, n_obs=12),
    "quad": lambda: problem_small_quad(seed=3, cap=8192, n_obs=60),
}


@pytest.mark.parametrize("name", list(LOCK_CASES))
@pytest.mark.parametrize("reload", [True, False])
def test_learned_lockstep(name, reload):
    p = LOCK_CASES[name]()
    _say(f"learned lock-step {name} reload={reload}")
    params = mlp_inputs.params(11, scale=1.0, out_scale=1.0)
    prop = dict(params=params, packed=packed(params), mix=0.7)
    rep = lockstep.run_lockstep(p, 12, reload=reload, proposal=prop)
    print(rep.summary(), f"learned={rep.learned_lanes}", flush=True)
    assert rep.ok, rep.summary()
    assert rep.iterations >= 3 and rep.learned_lanes > 100


def test_mix_zero_is_uniform_and_mix_one_is_refused():
    """mix = 0 gives the uniform planner's tree bit for bit; mix = 1 (no
    uniform share) is refused; with mix = 0.99 a node's stored control is
    Alg. 2's uniform draw exactly when its mixture word says uniform, and
    every control lies in U."""
    from paper_2409_06807_amd import Planner, KPError, E_ARG
    from test_oracle_planner import expected_controls
    from oracle import proposal as PR
    _say("mix 0 / mix 1 / mix 0.99")
    p = problem_small_di(seed=6, cap=4096, n_obs=12)
    params = mlp_inputs.params(12, scale=1.0, out_scale=1.0)
    pk = packed(params)
    G = Planner(p)
    for bad in (1.0, 1.5, -0.1):
        with pytest.raises(KPError) as ei:
            G.set_proposal(pk, bad)
        assert ei.value.code == E_ARG
        assert G.lib.kp_set_proposal(G.h, C.c_void_p(pk.data_ptr()), None, 0,
                                     C.c_float(bad)) == E_ARG
    G.close()
    trees = {}
    for mix in (None, 0.0, 0.99):
        G = Planner(p)
        if mix is not None:
            G.set_proposal(pk, mix)
        G.plan()
        trees[mix] = G.copy_tree()
        G.close()
    a, b = trees[None], trees[0.0]
    assert a["N"] == b["N"]
    for k in ("x", "u", "parent", "cell", "flag", "thr"):
        assert np.array_equal(a[k], b[k]), k
    g = trees[0.99]
    lo = np.asarray(p["u_lo"], np.float32)
    hi = np.asarray(p["u_hi"], np.float32)
    assert np.all(g["u"][1:] >= lo) and np.all(g["u"][1:] <= hi)
    thr = PR.mix_threshold(0.99)
    n_uniform = 0
    for i in range(1, min(g["N"], 2000)):
        it, f, s = int(g["birth"][i]), int(g["parent"][i]), int(g["sample"][i])
        uni = expected_controls(p, it, f, s, 3)
        learned = PR.is_learned(int(p["seed"]), it, f, s, thr)
        assert np.array_equal(g["u"][i], uni) == (not learned), i
        n_uniform += int(not learned)
    assert 0 < n_uniform < 100


def test_log_path_rows_match_reference():
    """Training rows from an oracle-grown tree loaded into the GPU."""
    from paper_2409_06807_amd import Planner
    import torch
    _say("log path")
    p = problem_small_di(seed=7, cap=4096, n_obs=12)
    W = oracle.OraclePlanner(p)
    W.plan(max_iters=60)
    s = W.state()
    node = s["goal_id"] if s["goal_id"] >= 0 else s["N"] - 1
    path = W.path(node)
    G = Planner(p)
    G.load_tree(lockstep.gpu_state_from_oracle(s))
    cap = 64
    X = torch.zeros((cap, 16), dtype=torch.float32, device="cuda:0")
    T = torch.zeros((cap, 4), dtype=torch.float32, device="cuda:0")
    n = G.log_path(int(node), X, T, row0=3)
    assert n == min(len(path) - 1, cap - 3)
    Xg = X.cpu().numpy()
    Tg = T.cpu().numpy()
    assert not Xg[:3].any() and not Xg[3 + n:].any()
    par = np.asarray(path[:-1])[:n]
    ch = np.asarray(path[1:])[:n]
    Xr = P.features(p, s["x"][par], s["thr"][s["cell"][par] >> 6])
    assert np.allclose(Xg[3:3 + n], Xr, rtol=1e-5, atol=1e-6)
    c, rr = P.control_box(p, 3)
    Tr = (s["u"][ch][:, :3].astype(np.float64) - c) / rr
    assert np.allclose(Tg[3:3 + n, :3], Tr, rtol=1e-5, atol=1e-6) and not Tg[3:3 + n, 3].any()
    G.close()


def test_trained_proposal_plans_replay_in_fp64():
    """End to end on the full-size forest: log solution paths of uniform plans
    (training seeds), train, plan evaluation seeds with the learned proposal;
    each solution replays in FP64 edge by edge."""
    import torch
    import paper_2409_06807_amd as kp
    from paper_2409_06807_amd import Planner
    _say("trained proposal on c2")
    p = problem_c2(seed=0)
    G = Planner(p)
    cap = 4096
    X = torch.zeros((cap, 16), dtype=torch.float32, device="cuda:0")
    T = torch.zeros((cap, 4), dtype=torch.float32, device="cuda:0")
    rows = 0
    for seed in range(1000, 1012):
        G.reset(seed)
        r = G.plan()
        if r["status"] == oracle.SOLVED:
            rows += G.log_path(r["goal_id"], X, T, rows)
    assert rows > 100
    params = dev(mlp_inputs.params(13))
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    pk = torch.empty(kp.MLP_PACKED_BYTES, dtype=torch.uint8, device="cuda:0")
    losses = kp.mlp_train(params, m1, m2, pk, X[:rows], T[:rows], 4, 256, 300, 3e-3, key=5)
    lv = losses.cpu().numpy()
    assert np.all(np.isfinite(lv)) and lv[-20:].mean() < lv[:20].mean()
    G.set_proposal(pk, 0.7)
    for seed in (0, 1):
        G.reset(seed)
        r = G.plan()
        assert r["status"] == oracle.SOLVED, r
        path = G.path(r["goal_id"])
        g = G.copy_tree()
        valid, reached, worst = replay_path_edgewise(p, g, path)
        assert valid and reached and worst <= 1e-5, (seed, valid, reached, worst)
    G.close()


@pytest.mark.parametrize("make", [lambda: problem_small_di(seed=6, cap=12000, n_obs=12),
                                  lambda: problem_small_quad(seed=3, cap=16000, n_obs=40, lambda_max=8)])
def test_tree_edge_rows(make):
    """kp_log_tree_edges: one row per tree edge whose child is strictly closer
    to the goal centre than its parent, in node id order; features of the
    parent as the FP64 reference defines them, the edge's control in
    normalised units.  The distance test is an FP32 decision: the reference
    takes it in FP32 too, summing the squared offsets with one rounding per
    term (a fused multiply-add; the exact product fits FP64)."""
    import torch
    from paper_2409_06807_amd import Planner
    p = make()
    _say(f"tree edge rows {p['name']} cap={p['node_cap']}")
    G = Planner(p)
    G.plan()
    g = G.copy_tree()
    N = int(g["N"])
    x32 = g["x"][:N]
    x = x32.astype(np.float64)
    c32 = np.asarray(p["goal_center"], np.float32)
    par = g["parent"][:N]

    def dist2(rows):
        d = np.zeros(len(rows), np.float32)
        for k in range(3):
            e = (x32[rows, k] - c32[k]).astype(np.float32)
            d = (e.astype(np.float64) * e.astype(np.float64) + d.astype(np.float64)).astype(np.float32)
        return d

    ids = np.arange(1, N)
    dc, da = dist2(ids), dist2(par[ids])
    child = 1 + np.nonzero(dc < da)[0]
    assert 100 < len(child) < N - 1
    X = torch.zeros((N, 16), dtype=torch.float32, device="cuda:0")
    T = torch.zeros((N, 4), dtype=torch.float32, device="cuda:0")
    rows = G.log_tree_edges(X, T, 3)
    assert rows == len(child)
    m = G.m
    Xh = X.cpu().numpy()
    Th = T.cpu().numpy()
    assert np.all(Xh[:3] == 0) and np.all(Xh[3 + rows:] == 0)
    ref = P.features(p, x[par[child]], g["thr"][g["cell"][par[child]] >> 6])
    np.testing.assert_allclose(Xh[3:3 + rows], ref, rtol=0, atol=1e-5)
    lo = np.asarray(p["u_lo"], np.float32)[:m].astype(np.float64)
    hi = np.asarray(p["u_hi"], np.float32)[:m].astype(np.float64)
    want_t = (g["u"][child].astype(np.float64) - 0.5 * (lo + hi)) / (0.5 * (hi - lo))
    np.testing.assert_allclose(Th[3:3 + rows, :m], want_t, rtol=0, atol=1e-6)
    # a short buffer takes the first rows only
    rows2 = G.log_tree_edges(X[:10], T[:10], 4)
    assert rows2 == 6
    G.close()
