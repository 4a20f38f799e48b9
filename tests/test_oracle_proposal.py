"""Pins of the FP64 learned-proposal reference (oracle/proposal.py) against
library routines, closed forms and finite differences."""

import math

import numpy as np
import pytest
import scipy.stats
import torch

import oracle
from oracle import proposal as P
from workloads import mlp_inputs, problem_c2, problem_small_di

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-20, 20, 20000)
    # exact ties at the BF16 rounding point, odd and even upper halves
    ties = (rng.integers(0x3F800000, 0x43000000, 2000, dtype=np.uint32) & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32), np.float32([0.0, -0.0, 1.0, -3.5e38])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(P.bf16(x), ref)


def test_forward_is_three_dense_layers():
    """Unquantised forward equals torch.nn.Linear/ReLU layers holding the same
    weights (row-major [out][in] with the bias after each matrix)."""
    params = mlp_inputs.params(3, scale=0.3)
    X = mlp_inputs.features(4, 37)
    W1, b1, W2, b2, W3, b3 = P.unpack(params)
    net = torch.nn.Sequential(torch.nn.Linear(16, 128), torch.nn.ReLU(), torch.nn.Linear(128, 128),
                              torch.nn.ReLU(), torch.nn.Linear(128, 8)).double()
    with torch.no_grad():
        for lin, (W, b) in zip([net[0], net[2], net[4]], [(W1, b1), (W2, b2), (W3, b3)]):
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        ref = net(torch.from_numpy(X)).numpy()
    o, _ = P.forward(params, X, quant=False)
    assert np.allclose(o, ref, rtol=1e-12, atol=1e-12)


def test_forward_quantised_closed_form():
    """Identity-like network on BF16-exact inputs: every rounding is exact, so
    the quantised output is relu(x) in the first 8 outputs."""
    W1 = np.zeros((128, 16))
    W1[:16, :16] = np.eye(16)
    W2 = np.eye(128)
    W3 = np.zeros((8, 128))
    W3[:, :8] = np.eye(8)
    params = P.pack(W1, np.zeros(128), W2, np.zeros(128), W3, np.zeros(8))
    X = np.array([[0.5, -1.0, 2.0, 0.25, -0.125, 3.0, 1.5, 4.0] + [1.0] * 8,
                  [-2.0, 0.75, 0.0, 8.0, 1.0, -1.0, 0.375, 0.0] + [0.0] * 8])
    o, _ = P.forward(params, X, quant=True)
    assert np.array_equal(o, np.maximum(X[:, :8], 0.0))
    # a value that is not BF16-exact is rounded on input
    o2, _ = P.forward(params, np.array([[1.0 + 2.0 ** -12] + [0.0] * 15]), quant=True)
    assert o2[0, 0] == 1.0


def test_head_at_zero_and_bounds():
    p = problem_c2()
    m = 4
    c, r = P.control_box(p, m)
    mean, std = P.head(np.zeros((1, 8)), p, m)
    assert np.allclose(mean[0], c) and np.allclose(std[0], r)
    o = np.array([[50.0, -50.0, 0.3, -0.2, 9.0, -9.0, -1.0, 0.0]])
    mean, std = P.head(o, p, m)
    lo = np.asarray(p["u_lo"], np.float64)
    hi = np.asarray(p["u_hi"], np.float64)
    assert np.all(mean[0] >= lo - 1e-9) and np.all(mean[0] <= hi + 1e-9)
    assert np.isclose(std[0, 0], r[0]) and np.isclose(std[0, 1], r[1] * math.exp(P.LS_MIN))


def test_loss_is_gaussian_nll():
    rng = np.random.default_rng(5)
    B, m = 50, 4
    o = rng.standard_normal((B, 8))
    T = rng.uniform(-1, 1, (B, 4))
    ls = np.clip(o[:, 4:8], P.LS_MIN, P.LS_MAX)
    lp = scipy.stats.norm.logpdf(T, loc=np.tanh(o[:, :4]), scale=np.exp(ls))
    ref = float(np.mean(np.sum(-lp - 0.5 * math.log(2 * math.pi), axis=1)))
    assert math.isclose(P.loss(o, T, m), ref, rel_tol=1e-12)


@pytest.mark.parametrize("m", [3, 4])
def test_gradient_matches_finite_differences(m):
    params = mlp_inputs.params(7 + m, scale=0.5)
    X = mlp_inputs.features(8 + m, 12)
    T = mlp_inputs.targets(9 + m, 12)
    L, g = P.loss_grad(params, X, T, m, quant=False)
    o, _ = P.forward(params, X, quant=False)
    assert math.isclose(L, P.loss(o, T, m), rel_tol=1e-12)
    rng = np.random.default_rng(m)
    idx = np.concatenate([rng.integers(a, b, 12) for a, b in
                          [(P.OFF_W1, P.OFF_B1), (P.OFF_B1, P.OFF_W2), (P.OFF_W2, P.OFF_B2),
                           (P.OFF_B2, P.OFF_W3), (P.OFF_W3, P.OFF_B3), (P.OFF_B3, P.N_PARAMS)]])
    h = 1e-6
    for i in idx:
        a = params.copy()
        b = params.copy()
        a[i] += h
        b[i] -= h
        fd = (P.loss_grad(a, X, T, m, quant=False)[0] - P.loss_grad(b, X, T, m, quant=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
    # the unused control slot of the double integrator gets no gradient
    if m == 3:
        W3g = g[P.OFF_W3:P.OFF_B3].reshape(8, 128)
        assert not W3g[3].any() and not W3g[7].any()


def test_log_std_clip_blocks_gradient():
    params = mlp_inputs.params(21, scale=0.3)
    W1, b1, W2, b2, W3, b3 = P.unpack(params)
    b3 = b3.copy()
    b3[4] = 50.0     # log-std of control 0 far above LS_MAX
    b3[5] = -50.0    # control 1 far below LS_MIN
    q = P.pack(W1, b1, W2, b2, W3, b3)
    X = mlp_inputs.features(22, 10)
    T = mlp_inputs.targets(23, 10)
    _, g = P.loss_grad(q, X, T, 4, quant=False)
    assert g[P.OFF_B3 + 4] == 0.0 and g[P.OFF_B3 + 5] == 0.0
    assert g[P.OFF_B3 + 6] != 0.0


def test_adam_matches_torch_and_first_step():
    rng = np.random.default_rng(11)
    theta0 = rng.standard_normal(300)
    grads = [rng.standard_normal(300) for _ in range(6)]
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    t = torch.tensor(theta0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=lr, betas=(b1, b2), eps=eps)
    th, m1, m2 = theta0.copy(), np.zeros(300), np.zeros(300)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad()
        t.grad = torch.from_numpy(g.copy())
        opt.step()
        th, m1, m2 = P.adam(th, m1, m2, g, k, lr, b1, b2, eps)
        if k == 1:
            assert np.allclose(th, theta0 - lr * grads[0] / (np.abs(grads[0]) + eps), rtol=0, atol=1e-15)
    assert np.allclose(th, t.detach().numpy(), rtol=0, atol=1e-13)


def test_box_muller_special_values_and_distribution():
    z0, z1 = P.box_muller(0xFFFFFFFF, 0)   # u1 = 1 -> radius 0
    assert z0 == 0.0 and z1 == 0.0
    z0, z1 = P.box_muller(0, 1 << 30)      # u2 = 1/4 -> all on the sine
    rad = math.sqrt(-2.0 * math.log(2.0 ** -24))
    assert abs(z0) < 1e-12 and math.isclose(z1, rad, rel_tol=1e-12)
    zs = []
    for k in range(6000):
        w = oracle.philox4x32_10((k, 7, 0, P.TAG_GAUSS), (1, 2))
        zs.extend(P.box_muller(w[0], w[1]))
        zs.extend(P.box_muller(w[2], w[3]))
    zs = np.array(zs)
    assert scipy.stats.kstest(zs, "norm").pvalue > 1e-3
    assert abs(zs.mean()) < 0.03 and abs(zs.var() - 1.0) < 0.04


def test_mixture_threshold_and_frequency():
    assert P.mix_threshold(0.0) == 0 and P.mix_threshold(1.0) == 2 ** 32
    p = problem_small_di()
    mean = np.zeros(3)
    std = np.ones(3)
    n_learned = 0
    N = 4000
    for k in range(N):
        learned, u = P.draw(p["seed"], 3, k, 1, mean, std, p, 3, P.mix_threshold(0.7))
        if learned:
            n_learned += 1
            assert np.all(u >= np.asarray(p["u_lo"], np.float64)) and np.all(u <= np.asarray(p["u_hi"], np.float64))
    # binomial(4000, 0.7): sd ~ 29
    assert abs(n_learned - 0.7 * N) < 5 * math.sqrt(N * 0.21)
    assert not P.draw(p["seed"], 3, 0, 0, mean, std, p, 3, 0)[0]
    assert P.draw(p["seed"], 3, 0, 0, mean, std, p, 3, 2 ** 32)[0]


def test_draw_narrow_gaussian_is_the_mean():
    p = problem_c2()
    mean = np.array([9.0, 0.01, -0.02, 0.05])
    std = np.full(4, 1e-12)
    learned, u = P.draw(0, 1, 2, 3, mean, std, p, 4, 2 ** 32)
    assert learned and np.allclose(u, mean, atol=1e-9)
    # a mean outside U is clipped to the box
    learned, u = P.draw(0, 1, 2, 3, np.array([99.0, 1.0, -1.0, 0.0]), std, p, 4, 2 ** 32)
    assert np.allclose(u, [p["u_hi"][0], p["u_hi"][1], p["u_lo"][2], 0.0], atol=1e-7)


def test_batch_rows_range_and_uniformity():
    rows = P.batch_rows(99, 4, 8000, 10)
    assert rows.min() >= 0 and rows.max() < 10
    counts = np.bincount(rows, minlength=10)
    assert scipy.stats.chisquare(counts).pvalue > 1e-3


def test_features_closed_form():
    p = problem_c2()
    lo = np.asarray(p["x_lo"], np.float64)
    hi = np.asarray(p["x_hi"], np.float64)
    x = 0.5 * (lo + hi)
    f = P.features(p, x, 2 ** 31)[0]
    assert np.allclose(f[:13], 0.0)
    g = np.asarray(p["goal_center"], np.float64)
    assert np.allclose(f[13:16], (g - x[:3]) * 2.0 / (hi[:3] - lo[:3]))
    f = P.features(p, x, 2 ** 40)[0]      # P_accept is at most 1
    assert f[12] == 1.0
    pd = problem_small_di()
    fd = P.features(pd, np.zeros(6), 0)[0]
    assert fd[6] == -1.0 and not fd[10:].any()


def test_training_reduces_loss():
    """A few hundred Adam steps of the reference fit a smooth synthetic policy."""
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (256, 16))
    X[:, 10:] = 0.0
    T = np.tanh(X[:, :4] @ rng.standard_normal((4, 4)) * 0.7)
    params = mlp_inputs.params(5, scale=1.0)
    m1 = np.zeros_like(params)
    m2 = np.zeros_like(params)
    L0 = P.loss_grad(params, X, T, 4)[0]
    for t in range(1, 301):
        L, g = P.loss_grad(params, X, T, 4)
        params, m1, m2 = P.adam(params, m1, m2, g, t, 3e-3)
    assert L < L0 - 1.0


def test_expansion_with_given_control():
    """A given control replaces only the control: with the uniform draw's own
    control the record is unchanged; with another one the end state is the
    re-integration under it, and the acceptance word stays the same."""
    p = problem_small_di()
    W = oracle.OraclePlanner(p)
    assert W.frontier() == oracle.OK
    base = W.expand_all()
    same = W.expand_all(controls=np.stack([np.pad(r["u"][:3], (0, 1)) for r in base]))
    assert base.tobytes() == same.tobytes()
    u = np.array([[0.5, -0.25, 1.0, 0.0]], np.float32)
    rec = W.expand_one(base["parent"][0], base["sample"][0], control=u[0])
    assert rec["w_acc"] == base["w_acc"][0]
    assert np.array_equal(rec["u"][:3], u[0, :3])
    ref = oracle.integrate_batch(p, W.state()["x"][rec["parent"]][None, :], u[:, :3],
                                 np.array([rec["steps"]], np.int32))
    assert np.allclose(rec["x"][:6], ref[0], rtol=0, atol=1e-12)
