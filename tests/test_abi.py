"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/kp.h, sizes workspaces, and rejects bad arguments before
any device work."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from workloads import problem_c1, problem_c2, problem_c5, problem_small_di

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "kp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2409_06807_amd as kp
    from paper_2409_06807_amd import build
    if not os.path.exists(kp.kp.LIB_PATH):
        build.build()
    return kp.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_entry_points()
    assert len(names) >= 15
    import paper_2409_06807_amd as kp
    assert sorted(kp.EXPORTED) == names
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_bytes(lib):
    import paper_2409_06807_amd as kp
    small = kp.workspace_bytes(problem_small_di(cap=1000))
    c1 = kp.workspace_bytes(problem_c1())
    c2 = kp.workspace_bytes(problem_c2())
    c5 = kp.workspace_bytes(problem_c5())
    assert 0 < small < c1 < c2
    # node arrays dominate: 12 + 4 floats + 14 bytes of ids / flags per node, plus
    # the staging area for accepted samples (c2)
    assert c2 > 4194304 * (16 * 4 + 14)
    assert c2 < 4194304 * 200
    assert c5 > 8388608 * (9 * 4 + 14)
    assert c2 % 256 == 0


def test_bad_descriptions_rejected(lib):
    import paper_2409_06807_amd as kp
    p = problem_small_di()
    d, keep = kp.make_desc(p)
    assert lib.kp_workspace_bytes(None) == 0
    for field, bad in [("abi_version", 7), ("dynamics", 9), ("steps", 0), ("sub", 5),
                       ("lambda_max", 0), ("lambda_max", 256), ("node_cap", 0),
                       ("n_obstacles", 5000), ("delta", 0.0), ("epsilon", 0.0)]:
        d2, keep2 = kp.make_desc(p)
        setattr(d2, field, bad)
        assert lib.kp_workspace_bytes(C.byref(d2)) == 0, field
        h = C.c_void_p()
        st = lib.kp_create_problem(C.byref(d2), C.c_void_p(256), 1 << 30, None, C.byref(h))
        assert st == kp.E_ARG and not h.value, field
    d.grid[0] = 1000
    d.grid[1] = 1000
    assert lib.kp_workspace_bytes(C.byref(d)) == 0


def test_null_and_workspace_errors(lib):
    import paper_2409_06807_amd as kp
    p = problem_small_di()
    d, keep = kp.make_desc(p)
    h = C.c_void_p()
    assert lib.kp_create_problem(None, C.c_void_p(256), 1 << 30, None, C.byref(h)) == kp.E_ARG
    assert lib.kp_create_problem(C.byref(d), None, 1 << 30, None, C.byref(h)) == kp.E_ARG
    need = lib.kp_workspace_bytes(C.byref(d))
    assert lib.kp_create_problem(C.byref(d), C.c_void_p(256), need - 1, None,
                                 C.byref(h)) == kp.E_WORKSPACE
    assert lib.kp_create_problem(C.byref(d), C.c_void_p(257), need, None,
                                 C.byref(h)) == kp.E_WORKSPACE
    for fn in ("kp_destroy_problem", "kp_update_regions"):
        assert getattr(lib, fn)(None) == kp.E_ARG
    assert lib.kp_expand(None, None) == kp.E_ARG
    assert lib.kp_update_tree(None, None) == kp.E_ARG
    assert lib.kp_plan(None, None) == kp.E_ARG
    assert lib.kp_trace_bytes(None) == 0
    assert lib.kp_status_str(kp.SOLVED) == b"solved"
    assert lib.kp_last_error(None) == b""


def test_invalid_start_and_goal_detected_on_host(lib):
    import paper_2409_06807_amd as kp
    p = problem_small_di()
    p["obstacles"] = np.vstack([p["obstacles"], np.array([[4, 4, 4, 6, 6, 6]], np.float32)])
    d, keep = kp.make_desc(p)
    h = C.c_void_p()
    need = lib.kp_workspace_bytes(C.byref(d))
    assert lib.kp_create_problem(C.byref(d), C.c_void_p(256), need, None,
                                 C.byref(h)) == kp.E_START_INVALID
    p = problem_small_di()
    p["goal_center"] = np.array([97, 50, 50], np.float32)
    d, keep = kp.make_desc(p)
    assert lib.kp_create_problem(C.byref(d), C.c_void_p(256), need, None,
                                 C.byref(h)) == kp.E_GOAL_INVALID


def test_struct_layouts_match_header(lib):
    import paper_2409_06807_amd as kp
    assert C.sizeof(kp.kp.TreeHost) == 8 + 12 * 8
    assert kp.TRACE_DTYPE.itemsize == 100
    src = open(os.path.join(ROOT, "include", "kp.h")).read()
    assert f"KP_ABI_VERSION {kp.kp.KP_ABI_VERSION}u" in src
    assert f"#define KP_MLP_STATIC_MAX_BATCH {kp.kp.MLP_STATIC_MAX_BATCH}\n" in src
    # the description's last fields: duration mode and a zero reserved word
    assert kp.kp.Desc.duration_mode.offset + 8 == C.sizeof(kp.kp.Desc)
    p = problem_small_di()
    d, keep = kp.make_desc(p)
    assert lib.kp_workspace_bytes(C.byref(d)) > 0
    d.duration_mode = 2
    assert lib.kp_workspace_bytes(C.byref(d)) == 0
    d.duration_mode = 1
    d.reserved = 5
    assert lib.kp_workspace_bytes(C.byref(d)) == 0


def test_binding_refuses_bad_network_tensors():
    # shapes, dtypes and devices are checked before anything reaches the library
    import torch
    import paper_2409_06807_amd as kp
    X = torch.zeros((4, 16))
    with pytest.raises(kp.KPError):
        kp.mlp_forward(torch.zeros(kp.MLP_PACKED_BYTES, dtype=torch.uint8), X)
    with pytest.raises(kp.KPError):
        kp.mlp_pack(torch.zeros(kp.MLP_PARAMS))
    with pytest.raises(kp.KPError):
        kp.mlp_grad(None, X, torch.zeros((4, 4)), 4, 4)
