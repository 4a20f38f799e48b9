"""ctypes binding of the C oracle (kpo.c).  TEST INFRASTRUCTURE ONLY."""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kpo.c")
LIB = os.path.join(HERE, "libkpo.so")

OK, SOLVED, TIMEOUT, TREE_FULL, FRONTIER_EMPTY = 0, 1, 2, 3, 4
E_ARG, E_START_INVALID, E_GOAL_INVALID = -1, -4, -5

AMB_TOL = 1e-4  # ambiguity band for FP-decided outcomes (workspace / state units)
# Quadcopter states with |pitch| above this are too close to the Euler-angle
# singularity (|pitch| = pi/2) for their FP64 values to serve as a reference
# of a lower-precision trajectory; see kpo.c well_conditioned.
COND_TILT = 1.45


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", SRC, "-o", tmp, "-lm"], cwd=HERE)
        os.replace(tmp, LIB)
    return LIB


class Problem(C.Structure):
    _fields_ = [
        ("dyn", C.c_int32), ("integ", C.c_int32), ("steps", C.c_int32), ("n_obs", C.c_int32),
        ("h", C.c_double), ("prm", C.c_double * 8),
        ("u_lo", C.c_float * 4), ("u_hi", C.c_float * 4),
        ("x_lo", C.c_double * 12), ("x_hi", C.c_double * 12),
        ("obs", C.POINTER(C.c_double)), ("margin", C.c_double),
        ("x_init", C.c_double * 12), ("goal_c", C.c_double * 3), ("goal_r", C.c_double),
        ("grid", C.c_int32 * 3), ("sub", C.c_int32), ("cap", C.c_int32),
        ("lambda_max", C.c_int32), ("delta", C.c_double), ("eps", C.c_double),
        ("seed", C.c_uint64), ("amb_tol", C.c_double), ("dur_mode", C.c_int32),
        ("pad_", C.c_int32), ("cond_tilt", C.c_double),
    ]


class View(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("m", C.c_int32), ("R", C.c_int32), ("cap", C.c_int32),
        ("N", C.c_int32), ("it", C.c_int32), ("nF", C.c_int32), ("lam", C.c_int32),
        ("nU", C.c_int32), ("goal_id", C.c_int32),
        ("x", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_float)),
        ("parent", C.POINTER(C.c_int32)), ("cell", C.POINTER(C.c_uint32)),
        ("flag", C.POINTER(C.c_uint8)), ("birth", C.POINTER(C.c_int32)),
        ("sample", C.POINTER(C.c_int32)), ("nv", C.POINTER(C.c_uint64)),
        ("ni", C.POINTER(C.c_uint64)), ("visited", C.POINTER(C.c_uint64)),
        ("avail", C.POINTER(C.c_uint8)), ("thr", C.POINTER(C.c_uint64)),
        ("F", C.POINTER(C.c_int32)), ("sum_lanes", C.c_uint64),
    ]


RECORD_DTYPE = np.dtype({
    "names": ["parent", "sample", "u", "x", "steps", "valid", "cell", "goal", "w_acc",
              "fail_strict", "fail_loose", "amb_cell", "amb_goal", "k_seg", "fail", "cond_step"],
    "formats": [np.int32, np.int32, (np.float32, 4), (np.float64, 12), np.int32, np.int32,
                np.uint32, np.int32, np.uint32, np.int32, np.int32, np.int32, np.int32, np.int32,
                np.int32, np.int32],
    "offsets": [0, 4, 8, 24, 120, 124, 128, 132, 136, 140, 144, 148, 152, 156, 160, 164],
    "itemsize": 168,
})

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        vp = C.c_void_p
        L.kpo_philox4x32_10.argtypes = [vp, vp, vp]
        L.kpo_control_map.argtypes = [C.c_uint32, C.c_float, C.c_float]
        L.kpo_control_map.restype = C.c_float
        L.kpo_deriv.argtypes = [C.POINTER(Problem), vp, vp, vp]
        L.kpo_step.argtypes = [C.POINTER(Problem), vp, vp, vp]
        L.kpo_state_ok.argtypes = [C.POINTER(Problem), vp, C.c_double]
        L.kpo_swept_hit.argtypes = [C.POINTER(Problem), vp, vp, C.c_double]
        L.kpo_cell_of.argtypes = [C.POINTER(Problem), vp]
        L.kpo_cell_of.restype = C.c_uint32
        L.kpo_near_cell_plane.argtypes = [C.POINTER(Problem), vp, C.c_double]
        L.kpo_near_cell_plane.restype = C.c_int
        L.kpo_set_threads.argtypes = [C.c_int32]
        L.kpo_get_threads.restype = C.c_int32
        L.kpo_region_score.argtypes = [C.c_double, C.c_uint64, C.c_uint64, C.c_int]
        L.kpo_region_score.restype = C.c_double
        L.kpo_estimates.argtypes = [C.c_int, vp, vp, vp, vp, C.c_double, C.c_double, vp, vp, vp, vp]
        L.kpo_create.argtypes = [C.POINTER(Problem), C.POINTER(C.c_int32)]
        L.kpo_create.restype = P
        L.kpo_clone.argtypes = [P]
        L.kpo_clone.restype = P
        L.kpo_destroy.argtypes = [P]
        L.kpo_frontier.argtypes = [P]
        L.kpo_frontier.restype = C.c_int32
        L.kpo_num_lanes.argtypes = [P]
        L.kpo_num_lanes.restype = C.c_int64
        L.kpo_expand_one.argtypes = [P, C.c_int32, C.c_int32, vp, vp]
        L.kpo_expand_all.argtypes = [P, vp]
        L.kpo_expand_all.restype = C.c_int64
        L.kpo_expand_one_u.argtypes = [P, C.c_int32, C.c_int32, vp, vp, vp]
        L.kpo_segment_steps.argtypes = [C.POINTER(Problem), C.c_uint32, C.c_uint32, C.c_uint32]
        L.kpo_segment_steps.restype = C.c_int32
        L.kpo_expand_all_u.argtypes = [P, vp, vp]
        L.kpo_expand_all_u.restype = C.c_int64
        L.kpo_apply.argtypes = [P, vp, C.c_int64]
        L.kpo_update_estimates.argtypes = [P]
        L.kpo_update_node_sets.argtypes = [P]
        L.kpo_update_node_sets.restype = C.c_int32
        L.kpo_iterate.argtypes = [P, C.POINTER(C.c_int32)]
        L.kpo_iterate.restype = C.c_int32
        L.kpo_plan.argtypes = [P, C.c_int32, C.c_double, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32)]
        L.kpo_plan.restype = C.c_int32
        L.kpo_path.argtypes = [P, C.c_int32, vp, C.c_int32]
        L.kpo_path.restype = C.c_int32
        L.kpo_replay.argtypes = [C.POINTER(Problem), vp, C.c_int32, vp, C.c_double, vp,
                                 C.POINTER(C.c_int32)]
        L.kpo_replay.restype = C.c_int32
        L.kpo_replay_k.argtypes = [C.POINTER(Problem), vp, C.c_int32, vp, vp, C.c_double, vp,
                                   C.POINTER(C.c_int32)]
        L.kpo_replay_k.restype = C.c_int32
        L.kpo_replay_edges.argtypes = [C.POINTER(Problem), C.c_int32, vp, vp, vp, C.c_double,
                                        C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                        vp]
        L.kpo_replay_edges.restype = C.c_int32
        L.kpo_integrate_batch.argtypes = [C.POINTER(Problem), C.c_int64, vp, vp, vp, vp]
        L.kpo_get_view.argtypes = [P, C.POINTER(View)]
        L.kpo_set_counters.argtypes = [P, C.c_int32, C.c_int32]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def problem_struct(p: dict, amb_tol: float = AMB_TOL, cond_tilt: float = COND_TILT):
    """Build the oracle's problem struct from a workload dict.  Returns
    (struct, keepalive) -- keep the second item alive as long as the first."""
    s = Problem()
    dyn = int(p["dynamics"])
    n = 6 if dyn == 0 else 12
    m = 3 if dyn == 0 else 4
    s.dyn = dyn
    s.integ = int(p["integrator"])
    s.steps = int(p["steps"])
    s.h = float(np.float32(p["h"]))
    for i, v in enumerate(np.asarray(p["dyn_params"], np.float32)[:8]):
        s.prm[i] = float(v)
    for j in range(m):
        s.u_lo[j] = float(np.float32(p["u_lo"][j]))
        s.u_hi[j] = float(np.float32(p["u_hi"][j]))
    for i in range(n):
        s.x_lo[i] = float(np.float32(p["x_lo"][i]))
        s.x_hi[i] = float(np.float32(p["x_hi"][i]))
        s.x_init[i] = float(np.float32(p["x_init"][i]))
    obs = np.ascontiguousarray(np.asarray(p["obstacles"], np.float32).astype(np.float64).reshape(-1, 6))
    s.n_obs = obs.shape[0]
    s.obs = obs.ctypes.data_as(C.POINTER(C.c_double))
    s.margin = float(np.float32(p["margin"]))
    for a in range(3):
        s.goal_c[a] = float(np.float32(p["goal_center"][a]))
        s.grid[a] = int(p["grid"][a])
    s.goal_r = float(np.float32(p["goal_radius"]))
    s.sub = int(p["sub"])
    s.cap = int(p["node_cap"])
    s.lambda_max = int(p["lambda_max"])
    s.delta = float(p["delta"])
    s.eps = float(p["epsilon"])
    s.seed = int(p["seed"]) & ((1 << 64) - 1)
    s.amb_tol = float(amb_tol)
    s.dur_mode = int(p.get("duration_mode", 0))
    s.cond_tilt = float(cond_tilt)
    return s, obs


# ---------------------------------------------------------------------------
# primitive wrappers (used by the pins)
# ---------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, np.uint32))
    k = np.ascontiguousarray(np.asarray(key, np.uint32))
    out = np.zeros(4, np.uint32)
    lib().kpo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's expansion loop (OpenMP; results do not depend on it)."""
    lib().kpo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().kpo_get_threads())


def segment_steps(p, it, f, s):
    """Integration steps of expansion (it, f, s) (random duration when the
    problem's duration_mode is 1)."""
    pb = _PB(p)
    return int(lib().kpo_segment_steps(C.byref(pb.s), int(it), int(f), int(s)))


def control_map(w, lo, hi):
    return np.float32(lib().kpo_control_map(int(w), float(lo), float(hi)))


class _PB:
    def __init__(self, p):
        self.s, self.keep = problem_struct(p)
        self.n = 6 if int(p["dynamics"]) == 0 else 12
        self.m = 3 if int(p["dynamics"]) == 0 else 4


def deriv(p, x, u):
    pb = _PB(p)
    x = np.ascontiguousarray(np.asarray(x, np.float64))
    u = np.ascontiguousarray(np.asarray(u, np.float64))
    dx = np.zeros(pb.n)
    lib().kpo_deriv(C.byref(pb.s), _ptr(x), _ptr(u), _ptr(dx))
    return dx


def step(p, x, u):
    pb = _PB(p)
    x = np.ascontiguousarray(np.asarray(x, np.float64))
    u = np.ascontiguousarray(np.asarray(u, np.float64))
    xn = np.zeros(pb.n)
    lib().kpo_step(C.byref(pb.s), _ptr(x), _ptr(u), _ptr(xn))
    return xn


def state_ok(p, x, relax=0.0):
    pb = _PB(p)
    x = np.ascontiguousarray(np.asarray(x, np.float64))
    return bool(lib().kpo_state_ok(C.byref(pb.s), _ptr(x), float(relax)))


def swept_hit(p, p0, p1, inflate=None):
    pb = _PB(p)
    a = np.ascontiguousarray(np.asarray(p0, np.float64))
    b = np.ascontiguousarray(np.asarray(p1, np.float64))
    if inflate is None:
        inflate = pb.s.margin
    return bool(lib().kpo_swept_hit(C.byref(pb.s), _ptr(a), _ptr(b), float(inflate)))


def cell_of(p, pos):
    pb = _PB(p)
    a = np.ascontiguousarray(np.asarray(pos, np.float64))
    return int(lib().kpo_cell_of(C.byref(pb.s), _ptr(a)))


def near_cell_plane(p, pos, tol=AMB_TOL):
    pb = _PB(p)
    a = np.ascontiguousarray(np.asarray(pos, np.float64))
    return bool(lib().kpo_near_cell_plane(C.byref(pb.s), _ptr(a), float(tol)))


def region_score(delta, nv, ni, cov):
    return float(lib().kpo_region_score(float(delta), int(nv), int(ni), int(cov)))


def estimates(avail, nv, ni, visited, delta, eps):
    R = len(avail)
    avail = np.ascontiguousarray(np.asarray(avail, np.uint8))
    nv = np.ascontiguousarray(np.asarray(nv, np.uint64))
    ni = np.ascontiguousarray(np.asarray(ni, np.uint64))
    visited = np.ascontiguousarray(np.asarray(visited, np.uint64))
    score = np.zeros(R)
    q = np.zeros(R, np.uint64)
    P = np.zeros(R)
    thr = np.zeros(R, np.uint64)
    lib().kpo_estimates(R, _ptr(avail), _ptr(nv), _ptr(ni), _ptr(visited), float(delta),
                        float(eps), _ptr(score), _ptr(q), _ptr(P), _ptr(thr))
    return dict(score=score, q=q, P=P, thr=thr)


def integrate_batch(p, x0, u, steps):
    """FP64 end states of segments (x0[i], u[i], steps[i])."""
    pb = _PB(p)
    x0 = np.ascontiguousarray(np.asarray(x0, np.float64).reshape(-1, pb.n))
    u = np.ascontiguousarray(np.asarray(u, np.float32).reshape(-1, pb.m))
    steps = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, np.int32), (len(x0),)))
    out = np.zeros_like(x0)
    lib().kpo_integrate_batch(C.byref(pb.s), len(x0), _ptr(x0), _ptr(u), _ptr(steps), _ptr(out))
    return out


def replay(p, x0, controls, margin=0.0, edge_steps=None):
    """FP64 replay of a path; returns (valid, reached_goal, end_states).
    edge_steps: integration steps per edge (default: the problem's steps)."""
    pb = _PB(p)
    x0 = np.ascontiguousarray(np.asarray(x0, np.float64))
    ctl = np.ascontiguousarray(np.asarray(controls, np.float32).reshape(-1, pb.m))
    ends = np.zeros((max(len(ctl), 1), pb.n))
    g = C.c_int32(0)
    ks = None if edge_steps is None else np.ascontiguousarray(np.asarray(edge_steps, np.int32))
    v = lib().kpo_replay_k(C.byref(pb.s), _ptr(x0), len(ctl), _ptr(ctl),
                           _ptr(ks) if ks is not None else None, float(margin), _ptr(ends),
                           C.byref(g))
    return bool(v), bool(g.value), ends[:len(ctl)]


def replay_trajectory(p, traj, margin=0.0, tol=AMB_TOL, rel_tol=1e-5):
    """FP64 replay of a returned trajectory (dict of x [L][n], u [L][m] and
    steps [L] for the L nodes from the root, as the GPU library returns it),
    edge by edge from each stored parent, against the un-inflated obstacles
    less the ambiguity band.  Returns dict(valid, reached, worst, first_bad):
    valid = every edge stays valid and ends within rel_tol of its stored child;
    reached = the last edge's FP64 end lies in the goal ball (within tol)."""
    pb = _PB(p)
    x = np.ascontiguousarray(np.asarray(traj["x"], np.float32).reshape(-1, pb.n))
    u = np.ascontiguousarray(np.asarray(traj["u"], np.float32).reshape(-1, pb.m))
    k = np.ascontiguousarray(np.asarray(traj["steps"], np.int32))
    L = len(x)
    worst = C.c_double(0.0)
    bad = C.c_int32(-1)
    end = np.zeros(pb.n)
    if L < 2:
        end[:] = x[0] if L else 0.0
        ok = True
    else:
        ok = bool(lib().kpo_replay_edges(C.byref(pb.s), L - 1, _ptr(x), _ptr(u), _ptr(k),
                                         float(margin), float(tol), C.byref(worst), C.byref(bad),
                                         _ptr(end)))
    c = np.asarray(p["goal_center"], np.float32).astype(np.float64)
    reached = float(np.sqrt(np.sum((end[:3] - c) ** 2))) <= float(np.float32(p["goal_radius"])) + tol
    valid = ok and worst.value <= rel_tol
    return dict(valid=valid, reached=reached, worst=float(worst.value), first_bad=int(bad.value))


# ---------------------------------------------------------------------------
# planner
# ---------------------------------------------------------------------------
class OraclePlanner:
    """The FP64 sequential planner.  Array views are numpy views of the
    planner's own memory, valid until the planner is destroyed."""

    def __init__(self, p: dict, amb_tol: float = AMB_TOL, _handle=None, _keep=None):
        self.problem = p
        if _handle is not None:
            self.h = _handle
            self._keep = _keep
            self.status = OK
        else:
            self._struct, self._keep = problem_struct(p, amb_tol)
            st = C.c_int32(0)
            self.h = lib().kpo_create(C.byref(self._struct), C.byref(st))
            self.status = st.value
            if not self.h:
                raise ValueError(f"oracle create failed with status {st.value}")
        self.n = 6 if int(p["dynamics"]) == 0 else 12
        self.m = 3 if int(p["dynamics"]) == 0 else 4

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().kpo_destroy(h)
            self.h = None

    def clone(self) -> "OraclePlanner":
        h = lib().kpo_clone(self.h)
        if not h:
            raise RuntimeError("clone failed")
        return OraclePlanner(self.problem, _handle=h, _keep=self._keep)

    # --- state ---
    def view(self):
        v = View()
        lib().kpo_get_view(self.h, C.byref(v))
        return v

    def state(self, copy=True):
        v = self.view()
        N, cap, R = v.N, v.cap, v.R
        as_np = np.ctypeslib.as_array
        d = dict(
            N=N, it=v.it, nF=v.nF, lam=v.lam, goal_id=v.goal_id, sum_lanes=int(v.sum_lanes),
            x=as_np(v.x, (cap, v.n))[:N], u=as_np(v.u, (cap, v.m))[:N],
            parent=as_np(v.parent, (cap,))[:N], cell=as_np(v.cell, (cap,))[:N],
            flag=as_np(v.flag, (cap,))[:N], birth=as_np(v.birth, (cap,))[:N],
            sample=as_np(v.sample, (cap,))[:N],
            nv=as_np(v.nv, (R,)), ni=as_np(v.ni, (R,)), visited=as_np(v.visited, (R,)),
            avail=as_np(v.avail, (R,)), thr=as_np(v.thr, (R,)),
            F=as_np(v.F, (cap,))[:v.nF],
        )
        if copy:
            d = {k: (np.array(a) if isinstance(a, np.ndarray) else a) for k, a in d.items()}
        return d

    # --- Alg. 1-4 steps ---
    def frontier(self) -> int:
        return lib().kpo_frontier(self.h)

    def num_lanes(self) -> int:
        return lib().kpo_num_lanes(self.h)

    def expand_all(self, controls=None):
        """Every lane of Alg. 2; controls (lanes x 4 FP32) replaces the
        uniform draws when given."""
        n = self.num_lanes()
        recs = np.zeros(max(n, 1), RECORD_DTYPE)
        if controls is None:
            lib().kpo_expand_all(self.h, _ptr(recs))
        else:
            U = np.zeros((max(n, 1), 4), np.float32)
            U[:n] = np.asarray(controls, np.float32)[:n, :4] if n else U[:0]
            lib().kpo_expand_all_u(self.h, _ptr(U), _ptr(recs))
        return recs[:n]

    def expand_one(self, f, s, want_traj=False, control=None):
        rec = np.zeros(1, RECORD_DTYPE)
        K = int(self.problem["steps"])
        traj = np.zeros((K + 1, self.n)) if want_traj else None
        u = None
        if control is not None:
            u = np.zeros(4, np.float32)
            u[:self.m] = np.asarray(control, np.float32)[:self.m]
        lib().kpo_expand_one_u(self.h, int(f), int(s), _ptr(u) if u is not None else None,
                               _ptr(rec), _ptr(traj) if traj is not None else None)
        return (rec[0], traj) if want_traj else rec[0]

    def apply(self, recs):
        recs = np.ascontiguousarray(recs, dtype=RECORD_DTYPE)
        lib().kpo_apply(self.h, _ptr(recs), len(recs))

    def update_estimates(self):
        lib().kpo_update_estimates(self.h)

    def update_node_sets(self) -> int:
        return lib().kpo_update_node_sets(self.h)

    def iterate(self):
        g = C.c_int32(-1)
        st = lib().kpo_iterate(self.h, C.byref(g))
        return st, g.value

    def plan(self, max_iters=None, t_max_ms=None):
        p = self.problem
        mi = int(p["max_iters"] if max_iters is None else max_iters)
        tm = float(p["t_max_ms"] if t_max_ms is None else t_max_ms)
        g = C.c_int32(-1)
        iters = C.c_int32(0)
        st = lib().kpo_plan(self.h, mi, tm, C.byref(g), C.byref(iters))
        return st, g.value, iters.value

    def path(self, node):
        ids = np.zeros(1 << 16, np.int32)
        n = lib().kpo_path(self.h, int(node), _ptr(ids), len(ids))
        if n < 0:
            raise RuntimeError("path longer than buffer")
        return ids[:n].copy()
