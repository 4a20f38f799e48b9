"""kp_mlp_train_noalloc (partial gradients in the library's static device
array) against kp_mlp_train (partial gradients in a caller workspace): the
same parameters, Adam moments, packed network and partial losses, bit for
bit, on two calls in a row -- the second one smaller than the first, so that
it runs over what the first left in the shared array -- and the size limit
refused with a message."""

import ctypes as C
import sys

import numpy as np
import pytest

from workloads import mlp_inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def _state(seed):
    import torch
    import paper_2409_06807_amd as kp
    params = _dev(mlp_inputs.params(seed))
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    packed = torch.empty(kp.MLP_PACKED_BYTES, dtype=torch.uint8, device="cuda:0")
    return params, m1, m2, packed


def _same(a, b, what):
    assert a.shape == b.shape, what
    assert np.array_equal(a.cpu().numpy().view(np.uint8), b.cpu().numpy().view(np.uint8)), what


# (rows of training data, minibatch rows, Adam steps, first step, data seed):
# the first call fills the whole static array (2048 rows = 32 partial
# gradients); the second, smaller one leaves most of it as the first call
# wrote it, and starts from the first call's parameters and moments.
CALLS = [(5000, 2048, 6, 0, 11), (900, 200, 4, 6, 12)]


def test_noalloc_training_matches_workspace_training():
    import torch
    import paper_2409_06807_amd as kp
    ref = _state(21)
    new = tuple(t.clone() for t in ref)
    torch.cuda.synchronize()
    for rows, batch, steps, step0, seed in CALLS:
        _say(f"no-alloc training: rows={rows} batch={batch} steps={steps} step0={step0}")
        X = _dev(mlp_inputs.features(seed, rows, used=14))
        T = _dev(mlp_inputs.targets(seed + 100, rows))
        nb = kp.mlp_partials(batch)
        loss_ref = kp.mlp_train(*ref, X, T, 4, batch, steps, 2e-3, key=0x5EED + seed, step0=step0)
        loss_new = torch.full((steps, nb), float("nan"), dtype=torch.float32, device="cuda:0")
        kp.mlp_train_noalloc(*new, X, T, 4, batch, steps, 2e-3, 0x5EED + seed, loss_new,
                             step0=step0)
        torch.cuda.synchronize()
        for a, b, what in zip(ref, new, ("params", "m1", "m2", "packed")):
            _same(a, b, f"{what} after rows={rows} batch={batch}")
        _same(loss_ref, loss_new.sum(dim=1), f"losses after rows={rows} batch={batch}")
        assert np.all(np.isfinite(loss_new.cpu().numpy()))


def test_noalloc_training_refuses_oversized_batch():
    import torch
    import paper_2409_06807_amd as kp
    _say("no-alloc training: batch above the static limit")
    params, m1, m2, packed = _state(22)
    X = _dev(mlp_inputs.features(13, 3000))
    T = _dev(mlp_inputs.targets(14, 3000))
    loss = torch.zeros((1, kp.mlp_partials(kp.kp.MLP_STATIC_MAX_BATCH + 64)), dtype=torch.float32,
                       device="cuda:0")
    before = params.clone()
    lib = kp.load_library()
    st = lib.kp_mlp_train_noalloc(
        C.c_void_p(params.data_ptr()), C.c_void_p(m1.data_ptr()), C.c_void_p(m2.data_ptr()),
        C.c_void_p(packed.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
        3000, 4, kp.kp.MLP_STATIC_MAX_BATCH + 64, 1, 0, C.c_float(1e-3), 7,
        C.c_void_p(loss.data_ptr()), None)
    assert st == kp.E_ARG
    msg = lib.kp_last_error(None).decode()
    assert "batch" in msg and str(kp.kp.MLP_STATIC_MAX_BATCH) in msg, msg
    torch.cuda.synchronize()
    _same(params, before, "parameters untouched by a refused call")
