"""ctypes binding of libkinopax.so (include/kp.h).

Argument marshalling only: every step of the planning iteration runs in the
library's HIP kernels.  PyTorch provides the device workspace and the stream.
Importing this module never falls back to anything: if the library is
missing, it raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkinopax.so")

KP_ABI_VERSION = 3
OK, SOLVED, TIMEOUT, TREE_FULL, FRONTIER_EMPTY = 0, 1, 2, 3, 4
E_ARG, E_DEVICE, E_WORKSPACE, E_START_INVALID, E_GOAL_INVALID, E_ORDER = -1, -2, -3, -4, -5, -6
KERNELS = {"propagate": 0, "region": 1, "nodesets": 2, "frontier": 3, "commit": 4, "post": 5,
           "proposal": 6}
MLP_INPUTS, MLP_HIDDEN, MLP_OUTPUTS = 16, 128, 8
MLP_PARAMS = 19720
MLP_PACKED_BYTES = 87072
MLP_BLOCK_ROWS = 64

EXPORTED = [
    "kp_workspace_bytes", "kp_trace_bytes", "kp_create_problem", "kp_destroy_problem",
    "kp_reset", "kp_expand", "kp_update_regions", "kp_update_tree", "kp_plan", "kp_get_stats",
    "kp_copy_tree", "kp_load_tree", "kp_get_path", "kp_set_profiling", "kp_kernel_times",
    "kp_status_str", "kp_last_error", "kp_mlp_pack", "kp_mlp_forward", "kp_mlp_grad",
    "kp_mlp_adam", "kp_mlp_train", "kp_set_proposal", "kp_log_path",
    "kp_batch_workspace_bytes", "kp_batch_create", "kp_batch_set_config", "kp_batch_get_config",
    "kp_batch_plan", "kp_batch_destroy", "kp_batch_last_error", "kp_batch_reset",
    "kp_transfer_tree", "kp_set_trace", "kp_set_launch_limits", "kp_get_trajectory",
    "kp_log_tree_edges", "kp_mlp_train_noalloc", "kp_batch_plan_queue",
]


class Desc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("dynamics", C.c_int32), ("integrator", C.c_int32),
        ("steps", C.c_int32), ("h", C.c_float), ("dyn_params", C.c_float * 8),
        ("u_lo", C.c_float * 4), ("u_hi", C.c_float * 4),
        ("x_lo", C.c_float * 12), ("x_hi", C.c_float * 12),
        ("obstacles", C.POINTER(C.c_float)), ("n_obstacles", C.c_int32), ("margin", C.c_float),
        ("x_init", C.c_float * 12), ("goal_center", C.c_float * 3), ("goal_radius", C.c_float),
        ("grid", C.c_int32 * 3), ("sub", C.c_int32), ("node_cap", C.c_int32),
        ("lambda_max", C.c_int32), ("delta", C.c_double), ("epsilon", C.c_double),
        ("seed", C.c_uint64), ("t_max_ms", C.c_double), ("max_iters", C.c_int32),
        ("iters_per_sync", C.c_int32), ("duration_mode", C.c_int32), ("reserved", C.c_int32),
    ]


class PlanResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("goal_id", C.c_int32), ("iterations", C.c_int32),
        ("n_nodes", C.c_int32), ("path_len", C.c_int32), ("pad", C.c_int32),
        ("elapsed_ms", C.c_double), ("lanes_total", C.c_uint64), ("valid_total", C.c_uint64),
    ]


class BatchConfig(C.Structure):
    _fields_ = [("iters_per_sync", C.c_int32), ("use_graph", C.c_int32),
                ("prop_blocks", C.c_int32), ("node_blocks", C.c_int32)]


class IterStats(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_frontier", C.c_int32), ("lam", C.c_int32),
        ("iteration", C.c_int32), ("goal_id", C.c_int32), ("done_code", C.c_int32),
        ("n_new", C.c_int32), ("device_error", C.c_int32),
        ("lanes_total", C.c_uint64), ("valid_total", C.c_uint64), ("invalid_total", C.c_uint64),
        ("steps_total", C.c_uint64), ("box_tests_total", C.c_uint64),
        ("checked_steps_total", C.c_uint64),
        ("grid_propagate", C.c_int32), ("grid_nodes", C.c_int32),
    ]


class TreeHost(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("iteration", C.c_int32),
        ("x", C.POINTER(C.c_float)), ("u", C.POINTER(C.c_float)),
        ("parent", C.POINTER(C.c_int32)), ("cell", C.POINTER(C.c_uint32)),
        ("flag", C.POINTER(C.c_uint8)), ("birth", C.POINTER(C.c_int32)),
        ("sample", C.POINTER(C.c_uint8)), ("nv", C.POINTER(C.c_uint64)),
        ("ni", C.POINTER(C.c_uint64)), ("visited", C.POINTER(C.c_uint64)),
        ("avail", C.POINTER(C.c_uint8)), ("thr", C.POINTER(C.c_uint64)),
    ]


TRACE_DTYPE = np.dtype({
    "names": ["parent", "sample", "u", "x", "steps", "fail_step", "valid", "cell", "goal",
              "accept", "new_id"],
    "formats": [np.int32, np.int32, (np.float32, 4), (np.float32, 12), np.int32, np.int32,
                np.int32, np.uint32, np.int32, np.int32, np.int32],
    "offsets": [0, 4, 8, 24, 72, 76, 80, 84, 88, 92, 96],
    "itemsize": 100,
})

_lib = None


def load_library():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2409_06807_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.kp_workspace_bytes.argtypes = [C.POINTER(Desc)]
    L.kp_workspace_bytes.restype = C.c_size_t
    L.kp_trace_bytes.argtypes = [P]
    L.kp_trace_bytes.restype = C.c_size_t
    L.kp_create_problem.argtypes = [C.POINTER(Desc), P, C.c_size_t, P, C.POINTER(P)]
    L.kp_create_problem.restype = C.c_int
    for name in ("kp_destroy_problem",):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = C.c_int
    L.kp_reset.argtypes = [P, C.c_uint64]
    L.kp_reset.restype = C.c_int
    L.kp_expand.argtypes = [P, P]
    L.kp_expand.restype = C.c_int
    L.kp_update_regions.argtypes = [P]
    L.kp_update_regions.restype = C.c_int
    L.kp_update_tree.argtypes = [P, C.POINTER(C.c_int32)]
    L.kp_update_tree.restype = C.c_int
    L.kp_plan.argtypes = [P, C.POINTER(PlanResult)]
    L.kp_plan.restype = C.c_int
    L.kp_get_stats.argtypes = [P, C.POINTER(IterStats)]
    L.kp_get_stats.restype = C.c_int
    L.kp_copy_tree.argtypes = [P, C.POINTER(TreeHost)]
    L.kp_copy_tree.restype = C.c_int
    L.kp_load_tree.argtypes = [P, C.POINTER(TreeHost)]
    L.kp_load_tree.restype = C.c_int
    L.kp_get_path.argtypes = [P, C.c_int32, P, C.c_int32, C.POINTER(C.c_int32)]
    L.kp_get_path.restype = C.c_int
    L.kp_set_profiling.argtypes = [P, C.c_int32]
    L.kp_set_profiling.restype = C.c_int
    L.kp_kernel_times.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.kp_kernel_times.restype = C.c_int
    L.kp_log_tree_edges.argtypes = [P, P, P, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.kp_log_tree_edges.restype = C.c_int
    L.kp_get_trajectory.argtypes = [P, C.c_int32, P, P, P, C.c_int32, C.POINTER(C.c_int32)]
    L.kp_get_trajectory.restype = C.c_int
    L.kp_set_trace.argtypes = [P, P]
    L.kp_set_trace.restype = C.c_int
    L.kp_set_launch_limits.argtypes = [P, C.c_int32, C.c_int32]
    L.kp_set_launch_limits.restype = C.c_int
    L.kp_status_str.argtypes = [C.c_int]
    L.kp_status_str.restype = C.c_char_p
    L.kp_last_error.argtypes = [P]
    L.kp_last_error.restype = C.c_char_p
    L.kp_mlp_pack.argtypes = [P, P, P]
    L.kp_mlp_forward.argtypes = [P, P, C.c_int32, P, P]
    L.kp_mlp_grad.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_int32,
                              P, P, P]
    L.kp_mlp_adam.argtypes = [P, P, P, P, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                              C.c_float, P]
    L.kp_mlp_train.argtypes = [P, P, P, P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               C.c_int32, C.c_float, C.c_uint64, P, P, P]
    L.kp_mlp_train_noalloc.argtypes = [P, P, P, P, P, P, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int32, C.c_int32, C.c_float, C.c_uint64, P, P]
    L.kp_set_proposal.argtypes = [P, P, P, C.c_int64, C.c_float]
    L.kp_log_path.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    for name in ("kp_mlp_pack", "kp_mlp_forward", "kp_mlp_grad", "kp_mlp_adam", "kp_mlp_train",
                 "kp_mlp_train_noalloc", "kp_set_proposal", "kp_log_path"):
        getattr(L, name).restype = C.c_int
    L.kp_batch_workspace_bytes.argtypes = [C.c_int32]
    L.kp_batch_workspace_bytes.restype = C.c_size_t
    L.kp_batch_create.argtypes = [P, C.c_int32, P, C.c_size_t, C.POINTER(P)]
    L.kp_batch_set_config.argtypes = [P, C.POINTER(BatchConfig)]
    L.kp_batch_get_config.argtypes = [P, C.POINTER(BatchConfig)]
    L.kp_batch_plan.argtypes = [P, P, C.POINTER(C.c_double)]
    L.kp_batch_plan_queue.argtypes = [P, P, C.POINTER(C.c_double)]
    L.kp_batch_destroy.argtypes = [P]
    L.kp_batch_reset.argtypes = [P, P]
    L.kp_transfer_tree.argtypes = [P, P]
    L.kp_transfer_tree.restype = C.c_int
    for name in ("kp_batch_create", "kp_batch_set_config", "kp_batch_get_config", "kp_batch_plan",
                 "kp_batch_plan_queue", "kp_batch_destroy", "kp_batch_reset"):
        getattr(L, name).restype = C.c_int
    L.kp_batch_last_error.argtypes = [P]
    L.kp_batch_last_error.restype = C.c_char_p
    _lib = L
    return L


def make_desc(p: dict, iters_per_sync: int = 0):
    """Fill kp_problem_desc from a workload dict.  Returns (desc, keepalive)."""
    d = Desc()
    dyn = int(p["dynamics"])
    n = 6 if dyn == 0 else 12
    m = 3 if dyn == 0 else 4
    d.abi_version = KP_ABI_VERSION
    d.dynamics = dyn
    d.integrator = int(p["integrator"])
    d.steps = int(p["steps"])
    d.h = float(np.float32(p["h"]))
    for i, v in enumerate(np.asarray(p["dyn_params"], np.float32)[:8]):
        d.dyn_params[i] = float(v)
    for j in range(m):
        d.u_lo[j] = float(np.float32(p["u_lo"][j]))
        d.u_hi[j] = float(np.float32(p["u_hi"][j]))
    for i in range(n):
        d.x_lo[i] = float(np.float32(p["x_lo"][i]))
        d.x_hi[i] = float(np.float32(p["x_hi"][i]))
        d.x_init[i] = float(np.float32(p["x_init"][i]))
    obs = np.ascontiguousarray(np.asarray(p["obstacles"], np.float32).reshape(-1, 6))
    d.obstacles = obs.ctypes.data_as(C.POINTER(C.c_float))
    d.n_obstacles = obs.shape[0]
    d.margin = float(np.float32(p["margin"]))
    for a in range(3):
        d.goal_center[a] = float(np.float32(p["goal_center"][a]))
        d.grid[a] = int(p["grid"][a])
    d.goal_radius = float(np.float32(p["goal_radius"]))
    d.sub = int(p["sub"])
    d.node_cap = int(p["node_cap"])
    d.lambda_max = int(p["lambda_max"])
    d.delta = float(p["delta"])
    d.epsilon = float(p["epsilon"])
    d.seed = int(p["seed"]) & ((1 << 64) - 1)
    d.t_max_ms = float(p["t_max_ms"])
    d.max_iters = int(p["max_iters"])
    d.iters_per_sync = int(iters_per_sync)
    d.duration_mode = int(p.get("duration_mode", 0))
    return d, obs


def workspace_bytes(p: dict) -> int:
    d, keep = make_desc(p)
    return int(load_library().kp_workspace_bytes(C.byref(d)))


class KPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kp status {code}: {msg}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Planner:
    """One planning problem on one GPU.  The workspace is a torch uint8 CUDA
    tensor owned by this object; kernels run on the given (or current) torch
    stream."""

    def __init__(self, p: dict, device="cuda:0", stream=None, iters_per_sync: int = 0):
        import torch
        self.lib = load_library()
        self.problem = p
        self.n = 6 if int(p["dynamics"]) == 0 else 12
        self.m = 3 if int(p["dynamics"]) == 0 else 4
        self.R = int(np.prod(p["grid"]))
        self.cap = int(p["node_cap"])
        self.device = torch.device(device)
        self._desc, self._keep = make_desc(p, iters_per_sync)
        nbytes = int(self.lib.kp_workspace_bytes(C.byref(self._desc)))
        if nbytes == 0:
            raise KPError(E_ARG, "invalid problem description")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            st = self.lib.kp_create_problem(C.byref(self._desc), C.c_void_p(self.workspace.data_ptr()),
                                            nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise KPError(st, self.lib.kp_status_str(st).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.kp_destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            msg = self.lib.kp_last_error(self.h).decode() if self.h else ""
            raise KPError(st, f"{self.lib.kp_status_str(st).decode()} {msg}")
        return st

    # --- Alg. 1 steps ---
    def reset(self, seed: int):
        self._check(self.lib.kp_reset(self.h, int(seed) & ((1 << 64) - 1)))

    def trace_buffer(self):
        import torch
        nb = int(self.lib.kp_trace_bytes(self.h))
        return torch.zeros(nb, dtype=torch.uint8, device=self.device)

    def expand(self, trace=None):
        ptr = C.c_void_p(trace.data_ptr()) if trace is not None else None
        self._check(self.lib.kp_expand(self.h, ptr))

    def update_regions(self):
        self._check(self.lib.kp_update_regions(self.h))

    def update_tree(self, want_goal=False):
        if want_goal:
            g = C.c_int32(-1)
            self._check(self.lib.kp_update_tree(self.h, C.byref(g)))
            return g.value
        self._check(self.lib.kp_update_tree(self.h, None))
        return None

    def plan(self) -> dict:
        r = PlanResult()
        st = self.lib.kp_plan(self.h, C.byref(r))
        self._check(st, allow=(SOLVED, TIMEOUT, TREE_FULL, FRONTIER_EMPTY))
        return dict(status=r.status, goal_id=r.goal_id, iterations=r.iterations,
                    n_nodes=r.n_nodes, path_len=r.path_len, elapsed_ms=r.elapsed_ms,
                    lanes_total=int(r.lanes_total), valid_total=int(r.valid_total))

    def stats(self) -> dict:
        s = IterStats()
        self._check(self.lib.kp_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in IterStats._fields_}

    def trace(self, buf, lanes: int):
        a = buf[: lanes * TRACE_DTYPE.itemsize].cpu().numpy()
        return a.view(TRACE_DTYPE)

    # --- state ---
    def _host_arrays(self):
        cap, R = self.cap, self.R
        return dict(
            x=np.zeros(self.n * cap, np.float32), u=np.zeros(self.m * cap, np.float32),
            parent=np.zeros(cap, np.int32), cell=np.zeros(cap, np.uint32),
            flag=np.zeros(cap, np.uint8), birth=np.zeros(cap, np.int32),
            sample=np.zeros(cap, np.uint8), nv=np.zeros(R, np.uint64), ni=np.zeros(R, np.uint64),
            visited=np.zeros(R, np.uint64), avail=np.zeros(R, np.uint8), thr=np.zeros(R, np.uint64))

    @staticmethod
    def _tree_struct(a, N, it):
        t = TreeHost()
        t.n_nodes = N
        t.iteration = it
        for k in ("x", "u", "parent", "cell", "flag", "birth", "sample", "nv", "ni", "visited",
                  "avail", "thr"):
            setattr(t, k, a[k].ctypes.data_as(dict(TreeHost._fields_)[k]))
        return t

    def copy_tree(self) -> dict:
        a = self._host_arrays()
        t = self._tree_struct(a, 0, 0)
        self._check(self.lib.kp_copy_tree(self.h, C.byref(t)))
        N = t.n_nodes
        return dict(
            N=N, it=t.iteration,
            x=a["x"][: self.n * N].reshape(self.n, N).T.copy(),
            u=a["u"][: self.m * N].reshape(self.m, N).T.copy(),
            parent=a["parent"][:N].copy(), cell=a["cell"][:N].copy(), flag=a["flag"][:N].copy(),
            birth=a["birth"][:N].copy(), sample=a["sample"][:N].copy(),
            nv=a["nv"], ni=a["ni"], visited=a["visited"], avail=a["avail"], thr=a["thr"])

    def load_tree(self, s: dict):
        """s: N, it, x [N, n], u [N, m], parent, cell, flag, birth, sample, nv, ni,
        visited, avail, thr (numpy)."""
        N = int(s["N"])
        a = dict(
            x=np.ascontiguousarray(np.asarray(s["x"], np.float32)[:N].T).ravel(),
            u=np.ascontiguousarray(np.asarray(s["u"], np.float32)[:N].T).ravel(),
            parent=np.ascontiguousarray(s["parent"][:N], np.int32),
            cell=np.ascontiguousarray(s["cell"][:N], np.uint32),
            flag=np.ascontiguousarray(s["flag"][:N], np.uint8),
            birth=np.ascontiguousarray(s["birth"][:N], np.int32),
            sample=np.ascontiguousarray(np.maximum(s["sample"][:N], 0), np.uint8),
            nv=np.ascontiguousarray(s["nv"], np.uint64), ni=np.ascontiguousarray(s["ni"], np.uint64),
            visited=np.ascontiguousarray(s["visited"], np.uint64),
            avail=np.ascontiguousarray(s["avail"], np.uint8),
            thr=np.ascontiguousarray(s["thr"], np.uint64))
        t = self._tree_struct(a, N, int(s["it"]))
        self._check(self.lib.kp_load_tree(self.h, C.byref(t)))

    # --- learned proposal ---
    def set_proposal(self, packed=None, mix: float = 0.7):
        """Draw controls from the packed network (kp_mlp_pack output) with
        probability mix; packed=None returns to the uniform draw."""
        import torch
        if not (0.0 <= float(mix) < 1.0):
            raise KPError(E_ARG, "mix must be in [0, 1): the uniform share keeps every control reachable")
        if packed is None or mix == 0.0:
            self._check(self.lib.kp_set_proposal(self.h, None, None, 0, C.c_float(0.0)))
            self._proposal = None
            return
        head = torch.empty((self.cap, 8), dtype=torch.float32, device=self.device)
        self._check(self.lib.kp_set_proposal(self.h, C.c_void_p(packed.data_ptr()),
                                             C.c_void_p(head.data_ptr()), self.cap,
                                             C.c_float(float(mix))))
        self._proposal = (packed, head)   # borrowed by the library

    def head_rows(self, rows: int):
        """Gaussian mean and std per frontier entry from the last network pass."""
        if getattr(self, "_proposal", None) is None:
            raise KPError(E_ARG, "no learned proposal set")
        return self._proposal[1][:rows].cpu().numpy()

    def log_path(self, node: int, X, T, row0: int) -> int:
        _need(X, MLP_INPUTS, "X")
        _need(T, 4, "T", rows=int(X.shape[0]))
        n = C.c_int32(0)
        self._check(self.lib.kp_log_path(self.h, int(node), C.c_void_p(X.data_ptr()),
                                         C.c_void_p(T.data_ptr()), int(X.shape[0]), int(row0),
                                         C.byref(n)))
        return n.value

    def log_tree_edges(self, X, T, row0: int) -> int:
        """Training rows from every tree edge that moves towards the goal
        (kp_log_tree_edges); returns the rows written."""
        _need(X, MLP_INPUTS, "X")
        _need(T, 4, "T", rows=int(X.shape[0]))
        n = C.c_int32(0)
        self._check(self.lib.kp_log_tree_edges(self.h, C.c_void_p(X.data_ptr()),
                                               C.c_void_p(T.data_ptr()), int(X.shape[0]),
                                               int(row0), C.byref(n)))
        return n.value

    def transfer_from(self, other: "Planner"):
        """Take over `other`'s tree (same problem and seed, capacity >= its |T|)."""
        self._check(self.lib.kp_transfer_tree(other.h, self.h))

    def path(self, node: int):
        n = C.c_int32(0)
        ids = np.zeros(1 << 16, np.int32)
        self._check(self.lib.kp_get_path(self.h, int(node), _ptr(ids), len(ids), C.byref(n)))
        return ids[: n.value].copy()

    def set_trace(self, buf):
        """kp_plan writes per-lane records of its expansions into buf (a
        trace_buffer()); None turns it off.  The buffer must stay alive."""
        self._plan_trace = buf
        ptr = C.c_void_p(buf.data_ptr()) if buf is not None else None
        self._check(self.lib.kp_set_trace(self.h, ptr))

    def set_launch_limits(self, prop_blocks: int = 0, node_blocks: int = 0):
        """Cap the workgroups per launch (0: occupancy maximum); results do
        not depend on it."""
        self._check(self.lib.kp_set_launch_limits(self.h, int(prop_blocks), int(node_blocks)))

    def trajectory(self, node: int) -> dict:
        """Root-to-node trajectory: states x [len][n], edge controls u [len][m]
        (zero for the root), integration steps per edge (0 for the root)."""
        n = C.c_int32(0)
        self._check(self.lib.kp_get_trajectory(self.h, int(node), None, None, None, 0, C.byref(n)))
        L = int(n.value)
        x = np.zeros((L, self.n), np.float32)
        u = np.zeros((L, self.m), np.float32)
        k = np.zeros(L, np.int32)
        self._check(self.lib.kp_get_trajectory(self.h, int(node), _ptr(x), _ptr(u), _ptr(k), L,
                                               C.byref(n)))
        return dict(x=x, u=u, steps=k)

    # --- timing ---
    def set_profiling(self, on: bool):
        self._check(self.lib.kp_set_profiling(self.h, 1 if on else 0))

    def kernel_times(self) -> dict:
        out = {}
        for name, k in KERNELS.items():
            n = C.c_int64(0)
            ms = C.c_double(0.0)
            self._check(self.lib.kp_kernel_times(self.h, k, C.byref(n), C.byref(ms)))
            out[name] = (int(n.value), float(ms.value))
        return out


# ---------------------------------------------------------------------------
# learned proposal: network kernels without a planner handle
# ---------------------------------------------------------------------------
def _need(t, cols, name, rows=None):
    """A contiguous FP32 CUDA tensor of shape (rows, cols): the kernels index
    it by these sizes, so anything else is refused before any launch."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and t.dim() == 2 and t.shape[1] == cols
            and (rows is None or t.shape[0] >= rows)):
        raise KPError(E_ARG, f"{name}: need a contiguous float32 CUDA tensor of shape "
                             f"({'>= ' + str(rows) if rows is not None else 'rows'}, {cols})")


def _stream_ptr(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _mlp_check(st, what):
    if st != OK:
        raise KPError(st, what)


def mlp_pack(params, packed=None):
    """FP32 parameters (device tensor of MLP_PARAMS floats) -> packed tensor."""
    import torch
    if not (params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()
            and params.numel() == MLP_PARAMS):
        raise KPError(E_ARG, f"params: need {MLP_PARAMS} contiguous float32 CUDA values")
    if packed is not None and packed.numel() * packed.element_size() < MLP_PACKED_BYTES:
        raise KPError(E_ARG, "packed: too small")
    if packed is None:
        packed = torch.empty(MLP_PACKED_BYTES, dtype=torch.uint8, device=params.device)
    _mlp_check(load_library().kp_mlp_pack(C.c_void_p(params.data_ptr()), C.c_void_p(packed.data_ptr()),
                                          _stream_ptr(params)), "kp_mlp_pack")
    return packed


def mlp_forward(packed, X):
    """Raw outputs (rows x 8) of the rows of X (rows x 16, FP32 device tensor)."""
    import torch
    _need(X, MLP_INPUTS, "X")
    rows = int(X.shape[0])
    out = torch.zeros((rows, MLP_OUTPUTS), dtype=torch.float32, device=X.device)
    _mlp_check(load_library().kp_mlp_forward(C.c_void_p(packed.data_ptr()), C.c_void_p(X.data_ptr()),
                                             rows, C.c_void_p(out.data_ptr()), _stream_ptr(X)),
               "kp_mlp_forward")
    return out


def mlp_partials(batch: int) -> int:
    return (int(batch) + MLP_BLOCK_ROWS - 1) // MLP_BLOCK_ROWS


def mlp_grad(packed, X, T, n_ctrl: int, batch: int, key: int = 0, step: int = 0):
    """Partial gradients (ceil(batch/64) x MLP_PARAMS) and partial losses."""
    import torch
    _need(X, MLP_INPUTS, "X")
    _need(T, 4, "T", rows=int(X.shape[0]))
    nb = mlp_partials(batch)
    partials = torch.empty((nb, MLP_PARAMS), dtype=torch.float32, device=X.device)
    loss = torch.empty(nb, dtype=torch.float32, device=X.device)
    _mlp_check(load_library().kp_mlp_grad(
        C.c_void_p(packed.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
        int(X.shape[0]), int(n_ctrl), int(batch), int(key) & ((1 << 64) - 1), int(step),
        C.c_void_p(partials.data_ptr()), C.c_void_p(loss.data_ptr()), _stream_ptr(X)), "kp_mlp_grad")
    return partials, loss


def mlp_adam(params, m1, m2, partials, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on params, m1, m2 in place."""
    _need(partials, MLP_PARAMS, "partials")
    for t, name in ((params, "params"), (m1, "m1"), (m2, "m2")):
        if not (t.is_cuda and t.is_contiguous() and t.numel() == MLP_PARAMS):
            raise KPError(E_ARG, f"{name}: need {MLP_PARAMS} contiguous float32 CUDA values")
    _mlp_check(load_library().kp_mlp_adam(
        C.c_void_p(params.data_ptr()), C.c_void_p(m1.data_ptr()), C.c_void_p(m2.data_ptr()),
        C.c_void_p(partials.data_ptr()), int(partials.shape[0]), int(step), C.c_float(lr),
        C.c_float(beta1), C.c_float(beta2), C.c_float(eps), _stream_ptr(params)), "kp_mlp_adam")


def mlp_train(params, m1, m2, packed, X, T, n_ctrl: int, batch: int, steps: int, lr: float,
              key: int, step0: int = 0):
    """`steps` minibatch Adam steps; returns the per-step losses (device tensor)."""
    import torch
    _need(X, MLP_INPUTS, "X")
    _need(T, 4, "T", rows=int(X.shape[0]))
    for t, name in ((params, "params"), (m1, "m1"), (m2, "m2")):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == MLP_PARAMS):
            raise KPError(E_ARG, f"{name}: need {MLP_PARAMS} contiguous float32 CUDA values")
    nb = mlp_partials(batch)
    partials = torch.empty((nb, MLP_PARAMS), dtype=torch.float32, device=X.device)
    loss = torch.empty((max(steps, 1), nb), dtype=torch.float32, device=X.device)
    _mlp_check(load_library().kp_mlp_train(
        C.c_void_p(params.data_ptr()), C.c_void_p(m1.data_ptr()), C.c_void_p(m2.data_ptr()),
        C.c_void_p(packed.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
        int(X.shape[0]), int(n_ctrl), int(batch), int(steps), int(step0), C.c_float(lr),
        int(key) & ((1 << 64) - 1), C.c_void_p(partials.data_ptr()), C.c_void_p(loss.data_ptr()),
        _stream_ptr(X)), "kp_mlp_train")
    return loss[:steps].sum(dim=1)


MLP_STATIC_MAX_BATCH = 2048


def mlp_train_noalloc(params, m1, m2, packed, X, T, n_ctrl: int, batch: int, steps: int,
                      lr: float, key: int, loss, step0: int = 0):
    """kp_mlp_train_noalloc: mlp_train with the partial gradients in the
    library's static device array; loss (steps x ceil(batch/64) float32,
    caller-owned) receives the partial losses.  Allocates nothing."""
    import torch
    _need(X, MLP_INPUTS, "X")
    _need(T, 4, "T", rows=int(X.shape[0]))
    for t, name in ((params, "params"), (m1, "m1"), (m2, "m2")):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == MLP_PARAMS):
            raise KPError(E_ARG, f"{name}: need {MLP_PARAMS} contiguous float32 CUDA values")
    if not (loss.is_cuda and loss.dtype == torch.float32 and loss.is_contiguous() and
            loss.numel() >= max(int(steps), 1) * mlp_partials(max(int(batch), 1))):
        raise KPError(E_ARG, "loss: need steps x ceil(batch/64) contiguous float32 CUDA values")
    lib = load_library()
    st = lib.kp_mlp_train_noalloc(
        C.c_void_p(params.data_ptr()), C.c_void_p(m1.data_ptr()), C.c_void_p(m2.data_ptr()),
        C.c_void_p(packed.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
        int(X.shape[0]), int(n_ctrl), int(batch), int(steps), int(step0), C.c_float(lr),
        int(key) & ((1 << 64) - 1), C.c_void_p(loss.data_ptr()), _stream_ptr(X))
    if st != OK:
        raise KPError(st, "kp_mlp_train_noalloc: " + (lib.kp_last_error(None) or b"").decode())


# ---------------------------------------------------------------------------
# batched planning
# ---------------------------------------------------------------------------
class Batch:
    """Planners advanced together by kp_batch_plan (one launch per kernel and
    iteration for the whole batch).  The planners stay usable on their own."""

    def __init__(self, planners):
        import torch
        self.lib = load_library()
        self.planners = list(planners)
        n = len(self.planners)
        nbytes = int(self.lib.kp_batch_workspace_bytes(n))
        if nbytes == 0:
            raise KPError(E_ARG, "empty batch")
        dev = self.planners[0].device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        hs = (C.c_void_p * n)(*[p.h for p in self.planners])
        h = C.c_void_p()
        st = self.lib.kp_batch_create(hs, n, C.c_void_p(self.workspace.data_ptr()), nbytes, C.byref(h))
        if st != OK:
            raise KPError(st, self.lib.kp_status_str(st).decode())
        self.h = h

    def _check(self, st):
        if st != OK:
            msg = self.lib.kp_batch_last_error(self.h).decode() if self.h else ""
            raise KPError(st, f"{self.lib.kp_status_str(st).decode()} {msg}")

    def config(self) -> dict:
        c = BatchConfig()
        self._check(self.lib.kp_batch_get_config(self.h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in BatchConfig._fields_}

    def set_config(self, **kw):
        cur = self.config()
        cur.update(kw)
        c = BatchConfig(**{k: int(v) for k, v in cur.items()})
        self._check(self.lib.kp_batch_set_config(self.h, C.byref(c)))

    def reset(self, seeds):
        """kp_reset of every problem with its seed, one wait for all."""
        a = np.ascontiguousarray(np.asarray(seeds, np.uint64))
        if a.shape != (len(self.planners),):
            raise KPError(E_ARG, "one seed per problem")
        self._check(self.lib.kp_batch_reset(self.h, _ptr(a)))

    def plan(self, queue: bool = False):
        """Returns (per-problem result dicts, batch wall time in ms).
        queue=True: one persistent launch over a device work queue
        (kp_batch_plan_queue); otherwise kp_batch_plan."""
        n = len(self.planners)
        res = (PlanResult * n)()
        ms = C.c_double(0.0)
        fn = self.lib.kp_batch_plan_queue if queue else self.lib.kp_batch_plan
        self._check(fn(self.h, res, C.byref(ms)))
        out = [dict(status=r.status, goal_id=r.goal_id, iterations=r.iterations, n_nodes=r.n_nodes,
                    path_len=r.path_len, elapsed_ms=r.elapsed_ms, lanes_total=int(r.lanes_total),
                    valid_total=int(r.valid_total)) for r in res]
        return out, ms.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.kp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_adaptive(p: dict, growth: int = 2, cap_max: int = 1 << 26, device="cuda:0"):
    """Remark 1's adaptive tree capacity: plan, and whenever eq. (6) stops
    the query on a full tree, move the tree into a planner `growth` times
    larger and go on.  Returns (final result, planner, list of
    (capacity, transfer ms))."""
    import time
    import torch
    G = Planner(p, device=device)
    r = G.plan()
    resizes = []
    cap = int(p["node_cap"])
    while r["status"] == TREE_FULL and cap * growth <= cap_max:
        cap *= growth
        H = Planner(dict(p, node_cap=cap), device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.transfer_from(G)
        resizes.append((cap, (time.perf_counter() - t0) * 1e3))
        G.close()
        G = H
        r = G.plan()
    return r, G, resizes
