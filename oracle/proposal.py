"""Learned control proposal, FP64 reference.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this module; the GPU library never calls it.

Alg. 2 draws each expansion's control uniformly from U.  The learned
proposal keeps that draw with probability 1 - mix and otherwise takes the
control from a Gaussian whose mean and spread a small network predicts from
the parent node.  Because the uniform part keeps a positive density on all
of U, the completeness argument of Sec. V (Theorem 1, through the
probabilistic completeness of tree planners with random controls) still
applies.

Network (three dense layers, BF16 operands, exact sums):
    x  = bf16(features)                         16 inputs
    h1 = bf16(relu(W1 x + b1))                  128
    h2 = bf16(relu(W2 h1 + b2))                 128
    o  = W3 h2 + b3                             8 = (mean part, log-std part)
The weights used are the BF16 roundings of the FP32 parameters.  Every BF16
rounding is round-to-nearest-even of the FP32 value nearest to the operand.
Parameters are one flat FP32 vector: W1 [128][16], b1 [128], W2 [128][128],
b2 [128], W3 [8][128], b3 [8] (row-major, output index first).

Head, for control j < m (c_j, r_j: centre and half-width of U):
    mean_j = c_j + r_j * tanh(o_j)
    std_j  = r_j * exp(clip(o_{4+j}, LS_MIN, LS_MAX))
Draw of expansion (it, f, s), from Philox words (tag 4 and tag 5 of the
counter (it, f, s, tag), key = seed):
    learned  iff  word 0 of tag 4 < floor(mix * 2^32)
    z_0, z_1 = Box-Muller(tag-5 words 0, 1); z_2, z_3 = Box-Muller(words 2, 3)
    u_j = clip(mean_j + std_j * z_j, lo_j, hi_j)
with Box-Muller(a, b): u1 = ((a >> 8) + 1) 2^-24, u2 = (b >> 8) 2^-24,
rad = sqrt(-2 ln u1), (rad cos 2 pi u2, rad sin 2 pi u2)  (Box & Muller, 1958).

Training objective: the mean over a minibatch of the Gaussian negative
log-likelihood of a logged control, in the normalised units t_j = (u_j - c_j) / r_j
(constant terms dropped):
    L = mean_rows sum_{j<m} [ (t_j - tanh o_j)^2 exp(-2 ls_j) / 2 + ls_j ]
Its gradient treats each BF16 rounding as the identity (the rounded value is
what the next layer consumes; the derivative passes through unchanged).
Optimiser: Adam with bias correction (Kingma & Ba, 2015).
"""

from __future__ import annotations

import math

import numpy as np

from .kpo import philox4x32_10

IN, HID, OUT = 16, 128, 8
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * IN
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + OUT * HID
N_PARAMS = OFF_B3 + OUT
LS_MIN, LS_MAX = -4.0, 0.0
TAG_MIX, TAG_GAUSS, TAG_BATCH = 4, 5, 6


def bf16(a):
    """Round to the nearest BF16 value (ties to even) through FP32; returns FP64."""
    a32 = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    b = a32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    q = np.asarray(params, np.float64)
    if q.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    W1 = q[OFF_W1:OFF_B1].reshape(HID, IN)
    b1 = q[OFF_B1:OFF_W2]
    W2 = q[OFF_W2:OFF_B2].reshape(HID, HID)
    b2 = q[OFF_B2:OFF_W3]
    W3 = q[OFF_W3:OFF_B3].reshape(OUT, HID)
    b3 = q[OFF_B3:]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), b3]).astype(np.float64)


# ---------------------------------------------------------------------------
# input features of a node
# ---------------------------------------------------------------------------
def feature_affine(p):
    """Centre and scale of each raw feature, fixed by the problem: the state box
    maps to [-1, 1]; P_accept in [0, 1] maps to [-1, 1]; the goal offset is
    scaled by the workspace half-extent.  Unused inputs have scale 0."""
    n = 6 if int(p["dynamics"]) == 0 else 12
    lo = np.asarray(p["x_lo"], np.float64)
    hi = np.asarray(p["x_hi"], np.float64)
    c = np.zeros(IN)
    s = np.zeros(IN)
    c[:n] = 0.5 * (lo[:n] + hi[:n])
    s[:n] = 2.0 / (hi[:n] - lo[:n])
    c[n], s[n] = 0.5, 2.0
    s[n + 1:n + 4] = 2.0 / (hi[:3] - lo[:3])
    return c, s


def features(p, x, thr):
    """Network inputs of nodes with states x (rows) whose regions have the
    acceptance thresholds thr (P_accept * 2^32, eq. 5): raw features are the
    state, P_accept and the goal centre minus the position."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    n = 6 if int(p["dynamics"]) == 0 else 12
    raw = np.zeros((x.shape[0], IN))
    raw[:, :n] = x[:, :n]
    raw[:, n] = np.minimum(np.asarray(thr, np.float64), 2.0 ** 32) / 2.0 ** 32
    raw[:, n + 1:n + 4] = np.asarray(p["goal_center"], np.float64)[None, :] - x[:, :3]
    c, s = feature_affine(p)
    return (raw - c[None, :]) * s[None, :]


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def forward(params, X, quant=True):
    """Raw outputs o (rows x 8) and the intermediate values the gradient needs."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    q = bf16 if quant else (lambda a: np.asarray(a, np.float64))
    x = q(np.atleast_2d(np.asarray(X, np.float64)))
    V1, V2, V3 = q(W1), q(W2), q(W3)
    z1 = x @ V1.T + b1
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ V2.T + b2
    h2 = q(np.maximum(z2, 0.0))
    o = h2 @ V3.T + b3
    cache = dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, V2=V2, V3=V3)
    return o, cache


def control_box(p, m):
    lo = np.asarray(p["u_lo"], np.float32)[:m].astype(np.float64)
    hi = np.asarray(p["u_hi"], np.float32)[:m].astype(np.float64)
    return 0.5 * (lo + hi), 0.5 * (hi - lo)


def head(o, p, m):
    """Gaussian mean and standard deviation in control units (rows x m each)."""
    c, r = control_box(p, m)
    o = np.atleast_2d(o)
    mean = c[None, :] + r[None, :] * np.tanh(o[:, :m])
    std = r[None, :] * np.exp(np.clip(o[:, 4:4 + m], LS_MIN, LS_MAX))
    return mean, std


def loss(o, T, m):
    """Mean negative log-likelihood (constants dropped) of normalised targets T."""
    o = np.atleast_2d(o)
    a = np.tanh(o[:, :m])
    ls = np.clip(o[:, 4:4 + m], LS_MIN, LS_MAX)
    r = np.asarray(T, np.float64)[:, :m] - a
    return float(np.mean(np.sum(0.5 * r * r * np.exp(-2.0 * ls) + ls, axis=1)))


def loss_grad(params, X, T, m, quant=True):
    """Loss and its gradient with respect to the FP32 parameters (flat)."""
    o, k = forward(params, X, quant)
    B = o.shape[0]
    T = np.asarray(T, np.float64)
    a = np.tanh(o[:, :m])
    raw_ls = o[:, 4:4 + m]
    ls = np.clip(raw_ls, LS_MIN, LS_MAX)
    e2 = np.exp(-2.0 * ls)
    r = T[:, :m] - a
    L = float(np.mean(np.sum(0.5 * r * r * e2 + ls, axis=1)))
    do = np.zeros((B, OUT))
    do[:, :m] = -r * (1.0 - a * a) * e2 / B
    inside = (raw_ls > LS_MIN) & (raw_ls < LS_MAX)
    do[:, 4:4 + m] = np.where(inside, (1.0 - r * r * e2) / B, 0.0)
    gW3 = do.T @ k["h2"]
    gb3 = do.sum(axis=0)
    dz2 = (do @ k["V3"]) * (k["z2"] > 0.0)
    gW2 = dz2.T @ k["h1"]
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ k["V2"]) * (k["z1"] > 0.0)
    gW1 = dz1.T @ k["x"]
    gb1 = dz1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def abs_scale(params, X):
    """The network's outputs evaluated with |.| on every weight, bias and
    input and relu dropped: a bound on how far any one rounding of an input
    or activation to a neighbouring BF16 value can move each output (times
    the relative size of that rounding, 2^-8)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    x = np.abs(bf16(np.atleast_2d(np.asarray(X, np.float64))))
    a1 = x @ np.abs(bf16(W1)).T + np.abs(b1)
    a2 = a1 @ np.abs(bf16(W2)).T + np.abs(b2)
    return a2 @ np.abs(bf16(W3)).T + np.abs(b3)


def loss_grad_abs(params, X, T, m):
    """The gradient's terms summed in absolute value (same contractions with
    |.| on every factor): a scale for the rounding error of any evaluation."""
    o, k = forward(params, X, True)
    B = o.shape[0]
    T = np.asarray(T, np.float64)
    a = np.tanh(o[:, :m])
    raw_ls = o[:, 4:4 + m]
    ls = np.clip(raw_ls, LS_MIN, LS_MAX)
    e2 = np.exp(-2.0 * ls)
    r = T[:, :m] - a
    do = np.zeros((B, OUT))
    do[:, :m] = np.abs(r * (1.0 - a * a) * e2) / B
    do[:, 4:4 + m] = (1.0 + r * r * e2) / B
    dz2 = (do @ np.abs(k["V3"])) * (k["z2"] > 0.0)
    dz1 = (dz2 @ np.abs(k["V2"])) * (k["z1"] > 0.0)
    return pack(dz1.T @ np.abs(k["x"]), dz1.sum(0), dz2.T @ np.abs(k["h1"]), dz2.sum(0),
                do.T @ np.abs(k["h2"]), do.sum(0))


def adam(theta, m1, m2, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam step t (1-based) with bias correction; returns new (theta, m1, m2)."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m1 = beta1 * np.asarray(m1, np.float64) + (1.0 - beta1) * g
    m2 = beta2 * np.asarray(m2, np.float64) + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** t)
    vh = m2 / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2


# ---------------------------------------------------------------------------
# sampling
# ---------------------------------------------------------------------------
def box_muller(wa, wb):
    u1 = (((int(wa) >> 8) + 1)) * 2.0 ** -24
    u2 = (int(wb) >> 8) * 2.0 ** -24
    rad = math.sqrt(-2.0 * math.log(u1))
    return rad * math.cos(2.0 * math.pi * u2), rad * math.sin(2.0 * math.pi * u2)


def mix_threshold(mix):
    """Integer threshold on a Philox word: the learned branch is taken iff
    word < threshold, so its probability is threshold / 2^32."""
    return min(int(math.floor(float(np.float32(mix)) * 2.0 ** 32)), 2 ** 32)


def _key(seed):
    return (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)


def is_learned(seed, it, f, s, mix_thr):
    """Mixture choice of expansion (it, f, s): an exact integer comparison."""
    return int(philox4x32_10((it, f, s, TAG_MIX), _key(seed))[0]) < mix_thr


def gaussians(seed, it, f, s):
    """The four standard normal draws of expansion (it, f, s)."""
    g = philox4x32_10((it, f, s, TAG_GAUSS), _key(seed))
    z0, z1 = box_muller(g[0], g[1])
    z2, z3 = box_muller(g[2], g[3])
    return np.array([z0, z1, z2, z3])


def uniform_control(seed, it, f, s, p, m):
    """Alg. 2's uniform control of expansion (it, f, s) (FP32 values)."""
    from .kpo import control_map
    w = philox4x32_10((it, f, s, 0), _key(seed))
    return np.array([control_map(w[j], np.float32(p["u_lo"][j]), np.float32(p["u_hi"][j]))
                     for j in range(m)], np.float32)


def draw(seed, it, f, s, mean, std, p, m, mix_thr):
    """Mixture draw of one expansion.  Returns (learned, u) with u in FP64 for
    a learned draw; None for a uniform draw (Alg. 2's own control map)."""
    if not is_learned(seed, it, f, s, mix_thr):
        return False, None
    z = gaussians(seed, it, f, s)
    lo = np.asarray(p["u_lo"], np.float32).astype(np.float64)
    hi = np.asarray(p["u_hi"], np.float32).astype(np.float64)
    u = np.array([min(max(mean[j] + std[j] * z[j], lo[j]), hi[j]) for j in range(m)])
    return True, u


def batch_rows(key, step, batch, n_rows):
    """Minibatch row indices of training step `step`: row k is the high word
    of (Philox word 0 of counter (step, k, 0, 6)) * n_rows."""
    kk = (int(key) & 0xFFFFFFFF, (int(key) >> 32) & 0xFFFFFFFF)
    out = np.empty(batch, np.int64)
    for k in range(batch):
        w = int(philox4x32_10((step, k, 0, TAG_BATCH), kk)[0])
        out[k] = (w * int(n_rows)) >> 32
    return out
