"""Seeded inputs for the learned control proposal: network parameters,
feature rows, normalised control targets and partial gradients.

Only random draws live here, with the shapes of the proposal's interface
(a flat FP32 vector of W1 [128][16], b1 [128], W2 [128][128], b2 [128],
W3 [8][128], b3 [8]); none of the network's arithmetic.
"""

from __future__ import annotations

import numpy as np

LAYERS = ((128, 16), (128, 128), (8, 128))   # (outputs, inputs) of each dense layer
N_PARAMS = sum(o * i + o for o, i in LAYERS)


def params(seed: int, scale: float = 1.0, out_scale: float = 0.1) -> np.ndarray:
    """Glorot-uniform weights times `scale` (the last layer also times
    `out_scale`, so a fresh network starts near a zero output), small biases.
    Returned as FP64 holding FP32 values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, (o, i) in enumerate(LAYERS):
        a = scale * np.sqrt(6.0 / (i + o)) * (out_scale if k == len(LAYERS) - 1 else 1.0)
        parts.append(rng.uniform(-a, a, o * i))
        parts.append(rng.uniform(-0.05, 0.05, o) * scale)
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def features(seed: int, rows: int, used: int = 16) -> np.ndarray:
    """Feature rows in [-1.5, 1.5] (FP32 values); inputs past `used` are zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1.5, 1.5, (rows, 16))
    x[:, used:] = 0.0
    return x.astype(np.float32).astype(np.float64)


def targets(seed: int, rows: int) -> np.ndarray:
    """Normalised control targets in [-1, 1] (FP32 values), 4 per row."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, (rows, 4)).astype(np.float32).astype(np.float64)


def partials(seed: int, n: int, scale: float = 1e-2) -> np.ndarray:
    """n rows of partial gradients (FP32 values)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal((n, N_PARAMS)) * scale).astype(np.float32).astype(np.float64)


def moments(seed: int) -> tuple:
    """Adam moment vectors of an optimiser some steps in: m1 ~ N(0, 1e-2^2),
    m2 ~ m1^2 + |N(0, 1e-4)|."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m1 = rng.standard_normal(N_PARAMS) * 1e-2
    m2 = m1 * m1 + np.abs(rng.standard_normal(N_PARAMS)) * 1e-4
    return m1.astype(np.float32).astype(np.float64), m2.astype(np.float32).astype(np.float64)
