"""Bench: Kino-PAX planning on one MI355X.

A step is one full planning query (Alg. 1 from initialisation to a goal node,
a full tree or the time budget) on the 12D quadcopter forest workload, with a
different planner seed per step.  The timed region covers K queries back to
back; inputs (problem, obstacles, workspace) are resident on the GPU before it
starts.

Prints one JSON line: value = valid expansions per second over the whole
timed region (sum of n_valid increments / wall time), plus the median
time-to-solution over solved queries, a roofline entry for the dominant
kernel (propagation, ALU-bound) from HIP-event kernel durations, and the CPU
oracle's throughput on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "median time-to-solution (ms) + valid expansions/s; learned vs uniform proposal"

# Algorithmic work model of the propagation kernel (counted from the
# formulas, not from the compiled code): FP32 operations per integration step
# (a fused multiply-add counts 2, a sin or cos 1, a compare 1), per checked
# step (the state-box test and the swept box; a lane checks its steps up to
# its first failing one and integrates on to the end of its segment), per
# swept-box test against one obstacle, and integer operations per
# Philox4x32-10 block.
INTEG_OPS = {
    (1, 1): 4 * 43 + 156,     # quadcopter RK4: 4 derivatives x 43 + stages / combination 156
    (0, 0): 12,               # double integrator Euler: 6 FMA
    (0, 1): 36 + 24 + 36,     # double integrator RK4: 3 stages x 12 + 12 x 2 accum + 12 x 3 final
    (1, 0): 43 + 24,          # quadcopter Euler
}
CHECK_OPS = {
    (1, 1): 24 + 12,          # state box 12 x 2 compares + swept box 6 min/max + 6 margin adds
    (0, 0): 12 + 12,
    (0, 1): 12 + 12,
    (1, 0): 24 + 12,
}
BOX_TEST_OPS = 6


def prop_ops(dyn, integ, steps, checked, boxes, lanes):
    """Algorithmic operations of a set of propagate launches."""
    philox_per_lane = 2 if dyn == 1 else 1
    return (steps * INTEG_OPS[(dyn, integ)] + checked * CHECK_OPS[(dyn, integ)] +
            boxes * BOX_TEST_OPS + lanes * philox_per_lane * PHILOX_OPS)
PHILOX_OPS = 100
PEAK_FP32_TFLOPS = 157.3

# HBM bytes per propagate launch from two rocprofv3 counter passes (FETCH_SIZE,
# WRITE_SIZE), already scaled by the copy-kernel calibration; only used while
# the kernel sources and the build flags still hash to what was profiled.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_propagate_traffic.json")
KERNEL_SOURCES = ("paper_2409_06807_amd/csrc/kp_kernels.hip",
                  "paper_2409_06807_amd/csrc/kp_internal.h",
                  "paper_2409_06807_amd/csrc/kp_device.h",
                  "paper_2409_06807_amd/build.py")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str = "k_propagate"):
    """Scaled HBM bytes per launch of `kernel` on `workload` from the counter
    record, or None when the record is missing or the kernel sources changed."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    entry = rec.get("workloads", {}).get(workload)
    if entry is None:
        return None
    if kernel != "k_propagate":
        entry = entry.get("other_kernels", {}).get(kernel)
        if entry is None:
            return None
    return entry["bytes_per_launch"]


PEAK_HBM_GBS = 8000.0


def post_hbm(workload: str, kt):
    """HBM entry of k_post (commit, estimates and node sets: the region and
    tree phases): counter bytes per launch over the live average launch."""
    n, ms = kt["post"]
    b = measured_traffic(workload, "k_post")
    if not n or b is None:
        return {"kernel": "k_post", "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": None, "traffic": b,
                "avg_launch_ms": ms / n if n else None}
    gbs = b / (ms / n * 1e-3) / 1e9
    return {"kernel": "k_post", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": b, "avg_launch_ms": ms / n}


def gpu_workload(name: str, seed: int = 0):
    from workloads import problem_c1, problem_c2, problem_c5
    return {"c1": problem_c1, "c2": problem_c2, "c5": problem_c5}[name](seed=seed)


def host_cores() -> int:
    """Threads the oracle may use: the CPUs this process may run on, bounded
    by OMP_NUM_THREADS when it is set (a host may set it to its CPU share)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def oracle_throughput(P, budget_s: float):
    """The oracle's valid expansions per second on the leading iterations of
    the planner P: it stops before the first iteration whose predicted time
    (its expansion count times the time per expansion so far) would overrun
    the budget."""
    import oracle
    t0 = time.perf_counter()
    done = 0
    while True:
        if P.frontier() != oracle.OK:
            break
        lanes_next = P.num_lanes()
        spent = time.perf_counter() - t0
        lanes_so_far = P.state(copy=False)["sum_lanes"]
        per_lane = spent / lanes_so_far if lanes_so_far else 0.0
        if done > 0 and spent + lanes_next * per_lane > budget_s:
            break
        st, g = P.iterate()
        done += 1
        if st != oracle.OK:
            break
    dt = time.perf_counter() - t0
    s = P.state(copy=False)
    return done, int(s["sum_lanes"]), int(s["nv"].sum()), int(s["N"]), dt


def oracle_leg(name: str, budget_s: float, tts_seeds: int, tts_budget_s: float, replays):
    """The CPU oracle (FP64, plain C, unchanged for this) on the host cores:
      * single-threaded throughput on the leading iterations of seed 0;
      * planning queries of seeds 0, 1, ... to their end on every host core
        (OpenMP over the expansion loop; the results are those of one
        thread), until tts_seeds queries or the budget: its time-to-solution;
      * FP64 replay of every trajectory the GPU legs returned, edge by edge
        from each stored parent, against the obstacles without the margin.
    replays: {leg: [(problem, trajectory), ...]}.  Returns the cpu_baseline
    entry and {leg: replay summary}."""
    import oracle
    cores = host_cores()
    oracle.set_threads(1)
    p = gpu_workload(name, 0)
    done, lanes1, nv1, n1, dt1 = oracle_throughput(oracle.OraclePlanner(p), budget_s)
    single = {"value": nv1 / dt1, "unit": "valid expansions/s", "cores": 1,
              "sample": f"{p['name']} seed 0, first {done} iterations: {lanes1} expansions, "
                        f"{nv1} valid, |T| = {n1}, {dt1:.1f} s"}
    oracle.set_threads(cores)
    tts, runs = [], []
    t_all = time.perf_counter()
    nv_all = lanes_all = 0
    for s in range(tts_seeds):
        if s > 0 and time.perf_counter() - t_all > tts_budget_s:
            break
        P = oracle.OraclePlanner(gpu_workload(name, s))
        a = time.perf_counter()
        st, g, it = P.plan(max_iters=100000, t_max_ms=60000.0)
        ms = (time.perf_counter() - a) * 1e3
        v = P.state(copy=False)
        nv_all += int(v["nv"].sum())
        lanes_all += int(v["sum_lanes"])
        runs.append({"seed": s, "status": int(st), "ms": ms, "iterations": int(it), "nodes": int(v["N"])})
        if st == oracle.SOLVED:
            tts.append(ms)
        del P
    wall = time.perf_counter() - t_all
    oracle.set_threads(1)
    entry = {
        "value": nv_all / wall if wall > 0 else 0.0, "unit": "valid expansions/s", "cores": cores,
        "kind": "oracle",
        "sample": f"{p['name']} seeds 0..{len(runs) - 1} planned to their end on {cores} threads "
                  f"(OpenMP over the expansion loop): {lanes_all} expansions, {nv_all} valid, "
                  f"{wall:.1f} s",
        "single_thread": single,
        "median_tts_ms": statistics.median(tts) if tts else None,
        "mean_tts_ms": statistics.mean(tts) if tts else None,
        "success_rate": len(tts) / len(runs) if runs else None,
        "queries": runs,
    }
    rep = {}
    for leg, items in replays.items():
        ok = reached = 0
        worst = 0.0
        for prob, tr in items:
            r = oracle.replay_trajectory(prob, tr)
            ok += int(r["valid"] and r["reached"])
            reached += int(r["reached"])
            worst = max(worst, r["worst"])
        rep[leg] = {"replay_valid_rate": ok / len(items) if items else None,
                    "replayed_paths": len(items), "worst_edge_rel_dev": worst}
    return entry, rep


def percentile(v, q):
    if not v:
        return None
    s = sorted(v)
    k = (len(s) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def expand_only(G, p, dyn, integ, reps):
    """Propagation at full occupancy: grow seed 0's tree step by step and stop
    before the first expansion whose lane count would stop growing (the
    largest iteration of the query), then time that expansion `reps` times,
    reloading the tree before each one."""
    import torch
    G.reset(0)
    best = None
    while True:
        st = G.stats()
        if st["done_code"]:
            break
        lanes = st["n_frontier"] * st["lam"]
        if best is not None and lanes < best[0]:
            break
        if best is None or lanes >= max(best[0], 1 << 16):
            best = (lanes, G.copy_tree())
        G.expand()
        G.update_regions()
        G.update_tree()
    lanes, tree = best
    times = []
    steps = boxes = checked = 0
    for _ in range(reps):
        G.load_tree(tree)
        s0 = G.stats()
        G.set_profiling(True)
        G.expand()
        torch.cuda.synchronize()
        kt = G.kernel_times()
        G.set_profiling(False)
        s1 = G.stats()
        times.append(kt["propagate"][1])
        steps = s1["steps_total"] - s0["steps_total"]
        checked = s1["checked_steps_total"] - s0["checked_steps_total"]
        boxes = s1["box_tests_total"] - s0["box_tests_total"]
        G.update_regions()
        G.update_tree()
    ms = statistics.median(times)
    ops = prop_ops(dyn, integ, steps, checked, boxes, lanes)
    tf = ops / (ms * 1e-3) / 1e12
    print(json.dumps({
        "mode": "expand-only", "workload": p["name"], "iteration": int(tree["it"]),
        "tree_nodes": int(tree["N"]), "lanes": int(lanes), "repetitions": reps,
        "propagate_ms_median": ms, "propagate_ms_all": times,
        "lanes_per_us": lanes / (ms * 1e3), "steps_per_lane": steps / lanes,
        "checked_steps_per_lane": checked / lanes,
        "box_tests_per_checked_step": boxes / checked if checked else None,
        "algorithmic_tflops": tf, "peak_tflops": PEAK_FP32_TFLOPS,
        "frac": tf / PEAK_FP32_TFLOPS}))


TRAIN_SEED0 = 1000  # training queries use planner seeds disjoint from the evaluated ones


def learned_leg(G, p, steps, warmup, n_paths, rows_target, train_steps, batch, lr, mix):
    """Learned proposal against the uniform planner: log training rows from
    uniform queries on training seeds (the solution paths of n_paths queries,
    then, up to rows_target rows, every tree edge of those queries that moves
    towards the goal: valid expansions that made progress), train the network
    on the GPU, then time the same evaluation seeds with the learned proposal
    mixed in."""
    import torch
    import paper_2409_06807_amd as kp
    from paper_2409_06807_amd import SOLVED
    from workloads import mlp_inputs
    m = 3 if int(p["dynamics"]) == 0 else 4
    cap = max(64 * n_paths, rows_target)
    X = torch.zeros((cap, 16), dtype=torch.float32, device="cuda:0")
    T = torch.zeros((cap, 4), dtype=torch.float32, device="cuda:0")
    rows = solved_paths = 0
    t0 = time.perf_counter()
    for s in range(TRAIN_SEED0, TRAIN_SEED0 + n_paths):
        G.reset(s)
        r = G.plan()
        if r["status"] == SOLVED:
            rows += G.log_path(r["goal_id"], X, T, rows)
            solved_paths += 1
    path_rows = rows
    edge_trees = 0
    for s in range(TRAIN_SEED0, TRAIN_SEED0 + n_paths):
        if rows >= rows_target:
            break
        G.reset(s)
        G.plan()
        rows += G.log_tree_edges(X, T, rows)
        edge_trees += 1
    collect_s = time.perf_counter() - t0
    params = torch.tensor(mlp_inputs.params(13), dtype=torch.float32, device="cuda:0")
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    pk = torch.empty(kp.MLP_PACKED_BYTES, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = kp.mlp_train(params, m1, m2, pk, X[:rows], T[:rows], m, batch, train_steps, lr, key=5)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3
    lv = losses.cpu().numpy()
    G.set_proposal(pk, mix)
    for s in range(warmup):
        G.reset(s % max(steps, 1))
        G.plan()
    torch.cuda.synchronize()
    results, per_ms = [], []
    t0 = time.perf_counter()
    for s in range(steps):
        a = time.perf_counter()
        G.reset(s)
        results.append(G.plan())
        per_ms.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    G.set_profiling(True)
    paths = []
    for s in range(steps):
        G.reset(s)
        r = G.plan()
        if r["status"] == SOLVED:
            paths.append((dict(p, seed=s), G.trajectory(r["goal_id"])))
    kt = G.kernel_times()
    G.set_profiling(False)
    G.set_proposal(None)
    solved = [ms for ms, r in zip(per_ms, results) if r["status"] == SOLVED]
    n_head, head_ms = kt["proposal"]
    return paths, {
        "mix": mix,
        "median_tts_ms": statistics.median(solved) if solved else None,
        "mean_tts_ms": statistics.mean(solved) if solved else None,
        "p10_tts_ms": percentile(solved, 10),
        "p90_tts_ms": percentile(solved, 90),
        "success_rate": len(solved) / len(results),
        "valid_expansions_per_s": sum(r["valid_total"] for r in results) / elapsed,
        "iterations": [r["iterations"] for r in results],
        "tree_nodes": [r["n_nodes"] for r in results],
        "kernel_ms_per_query": {k: v[1] / max(steps, 1) for k, v in kt.items()},
        "proposal_launches": n_head,
        "proposal_ms_per_launch": head_ms / n_head if n_head else None,
        "training": {
            "seeds": f"{TRAIN_SEED0}..{TRAIN_SEED0 + n_paths - 1} (uniform planner)",
            "solved_paths": solved_paths, "path_rows": path_rows,
            "progress_edge_rows": rows - path_rows, "progress_edge_trees": edge_trees,
            "rows": rows, "steps": train_steps, "batch": batch,
            "lr": lr, "loss_first10": float(lv[:10].mean()), "loss_last10": float(lv[-10:].mean()),
            "collect_s": collect_s, "train_ms": train_ms,
        },
    }


def batched_leg(n_queries, batch_seed=3):
    """Batched planning of uneven queries against planning them one by one:
    the same queries and seeds, identical per-query results required."""
    import tempfile
    from paper_2409_06807_amd import Planner, Batch, SOLVED, TREE_FULL, autotune
    from workloads import problem_batch
    ps = problem_batch(n=n_queries, batch_seed=batch_seed)
    planners = [Planner(p) for p in ps]

    seeds = [p["seed"] for p in ps]
    B = None

    def reset():
        B.reset(seeds)

    seq_ms, seq = [], []
    for rep in range(2):   # the first pass warms every handle up
        seq_ms, seq = [], []
        t0 = time.perf_counter()
        for G, p in zip(planners, ps):
            a = time.perf_counter()
            G.reset(p["seed"])
            seq.append(G.plan())
            seq_ms.append((time.perf_counter() - a) * 1e3)
        seq_total = (time.perf_counter() - t0) * 1e3
    B = Batch(planners)
    keys = ("status", "goal_id", "iterations", "n_nodes", "lanes_total", "valid_total")

    def run(queue=False):
        t0 = time.perf_counter()
        reset()
        res, bms = B.plan(queue=queue)
        total = (time.perf_counter() - t0) * 1e3
        same = all(r[k] == s[k] for s, r in zip(seq, res) for k in keys)
        return dict(total_ms=total, batch_ms=bms,
                    median_completion_ms=statistics.median(r["elapsed_ms"] for r in res),
                    identical_to_sequential=same)

    run()
    default = dict(config=B.config(), **run())
    cfg, table = autotune.tune(B, reset, autotune.signature(ps, "mi355x"),
                               cache_path=os.path.join(tempfile.mkdtemp(), "autotune.json"))
    tuned = dict(config=cfg, **run())
    B.close()
    paths = [(pq, G.trajectory(r["goal_id"])) for pq, G, r in zip(ps, planners, seq)
             if r["status"] == SOLVED]
    st = [r["status"] for r in seq]
    return paths, {
        "workload": f"c3-batch-di6: {n_queries} double-integrator queries, boxes log-uniform in "
                    "[10, 2000], caps log-uniform in [16k, 1M], start/goal >= 50 apart",
        "queries": n_queries, "solved": st.count(SOLVED), "tree_full": st.count(TREE_FULL),
        "sequential": {"total_ms": seq_total, "median_query_ms": statistics.median(seq_ms),
                       "queries_per_s": n_queries / (seq_total * 1e-3)},
        "batched_default": default,
        "batched_tuned": dict(tuned, queries_per_s=n_queries / (tuned["total_ms"] * 1e-3),
                              candidates=len(table)),
        "speedup_total_tuned": seq_total / tuned["total_ms"],
    }


def sweep(workload, seeds, caps, eps_delta, lambdas=(), only_lambda=False):
    """Time-to-solution and failures against the tree capacity t_e (the
    paper's only scaling experiment, Sec. VI), then against epsilon and delta
    at the workload's own capacity, and against the branching bound lambda_max
    of eq. (6).  One JSON line per setting."""
    from paper_2409_06807_amd import Planner, SOLVED

    def run(p):
        G = Planner(p)
        G.reset(0)
        G.plan()   # warm-up
        ms, st, it = [], [], []
        for s in seeds:
            a = time.perf_counter()
            G.reset(s)
            r = G.plan()
            ms.append((time.perf_counter() - a) * 1e3)
            st.append(r["status"])
            it.append(r["iterations"])
        G.close()
        solved = [m for m, s in zip(ms, st) if s == SOLVED]
        return {"success_rate": len(solved) / len(st),
                "median_tts_ms": statistics.median(solved) if solved else None,
                "mean_tts_ms": statistics.mean(solved) if solved else None,
                "median_iterations": statistics.median(it), "statuses": st}

    for lam in lambdas:
        p = gpu_workload(workload, 0)
        p["lambda_max"] = int(lam)
        print(json.dumps({"mode": "lambda_max sweep", "workload": p["name"], "lambda_max": int(lam),
                          "node_cap": int(p["node_cap"]), "seeds": len(seeds), **run(p)}),
              flush=True)
    if only_lambda:
        return
    for cap in caps:
        p = gpu_workload(workload, 0)
        p["node_cap"] = int(cap)
        print(json.dumps({"mode": "t_e sweep", "workload": p["name"], "node_cap": int(cap),
                          "seeds": len(seeds), **run(p)}), flush=True)
    # Alg. 2's random segment duration (k uniform in 1..K steps) at the workload's capacity
    p = gpu_workload(workload, 0)
    p["duration_mode"] = 1
    print(json.dumps({"mode": "random segment duration", "workload": p["name"],
                      "node_cap": int(p["node_cap"]), "seeds": len(seeds), **run(p)}), flush=True)
    # Remark 1: start small and grow the capacity by 2x whenever the tree fills
    from paper_2409_06807_amd import plan_adaptive
    p0 = gpu_workload(workload, 0)
    start = int(p0["node_cap"]) // 8
    ms, st, rs = [], [], []
    for s in seeds:
        p = dict(p0, node_cap=start, seed=s)
        a = time.perf_counter()
        r, G, resizes = plan_adaptive(p, growth=2, cap_max=int(p0["node_cap"]) * 2)
        ms.append((time.perf_counter() - a) * 1e3)
        st.append(r["status"])
        rs.extend(resizes)
        G.close()
    solved = [m for m, s_ in zip(ms, st) if s_ == SOLVED]
    print(json.dumps({"mode": "adaptive t_e", "workload": p0["name"], "start_cap": start,
                      "growth": 2, "seeds": len(seeds), "success_rate": len(solved) / len(st),
                      "median_ms_with_resizes": statistics.median(solved) if solved else None,
                      "resizes": len(rs),
                      "mean_transfer_ms": statistics.mean(t for _, t in rs) if rs else None,
                      "note": "wall time includes creating each larger planner",
                      "statuses": st}), flush=True)
    for eps, delta in eps_delta:
        p = gpu_workload(workload, 0)
        p["epsilon"], p["delta"] = float(eps), float(delta)
        print(json.dumps({"mode": "epsilon/delta sweep", "workload": p["name"], "epsilon": eps,
                          "delta": delta, "seeds": len(seeds), **run(p)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50,
                    help="queries timed (planner seeds 0 .. steps-1; the paper plans 50 queries per scene)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c5"])
    ap.add_argument("--profile-steps", type=int, default=-1,
                    help="queries in the HIP-event pass (default: the same seeds as the timed steps)")
    ap.add_argument("--cpu-budget-s", type=float, default=10.0,
                    help="single-threaded oracle sample (s)")
    ap.add_argument("--cpu-tts-seeds", type=int, default=5,
                    help="queries the oracle plans to their end on all host cores")
    ap.add_argument("--cpu-tts-budget-s", type=float, default=60.0,
                    help="no further oracle query starts after this many seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters-per-sync", type=int, default=0)
    ap.add_argument("--expand-only", action="store_true",
                    help="instead of whole queries, time the propagate kernel on the largest "
                         "iteration of one query (the tree reloaded before each repetition) and "
                         "print that measurement")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal leg")
    ap.add_argument("--learned-paths", type=int, default=256,
                    help="uniform training queries whose solution paths are logged")
    ap.add_argument("--learned-rows", type=int, default=2_000_000,
                    help="training rows: solution paths, then progress edges of the training trees")
    ap.add_argument("--learned-train-steps", type=int, default=3000)
    ap.add_argument("--learned-batch", type=int, default=2048)
    ap.add_argument("--learned-mix", type=float, default=0.7)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the bench line, sweep the tree capacity t_e and then epsilon "
                         "and delta on the workload (one JSON line per setting)")
    ap.add_argument("--lambda-sweep", action="store_true",
                    help="instead of the bench line, sweep lambda_max (eq. 6) on the workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-planning leg")
    ap.add_argument("--batch-queries", type=int, default=256)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (a kernel of known "
                         "traffic, used to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; run it with --gpus 1 (the planner does not "
              "shard a query over several GPUs).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_06807_amd import Planner, SOLVED

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.sweep or args.lambda_sweep:
        seeds = list(range(max(args.steps, 1)))
        base = int(gpu_workload(args.workload, 0)["node_cap"])
        caps = [base // 8, base // 4, base // 2, base, base * 2]
        eps_delta = [(1e-2, 1e-3), (1e-3, 1e-3), (1e-1, 1e-3), (1e-2, 1e-1), (1e-2, 1e-5)]
        lambdas = (2, 4, 6, 8, 12, 16, 32)
        sweep(args.workload, seeds, caps, eps_delta, lambdas=lambdas,
              only_lambda=args.lambda_sweep)
        return

    p = gpu_workload(args.workload, 0)
    G = Planner(p, device="cuda:0", iters_per_sync=args.iters_per_sync)
    dyn, integ = int(p["dynamics"]), int(p["integrator"])
    if args.expand_only:
        expand_only(G, p, dyn, integ, max(args.steps, 1))
        return

    # warm-up and profiled queries reuse the timed seeds, so that a profiler's
    # per-kernel average over the whole run describes the same launch mix
    for s in range(args.warmup):
        G.reset(s % max(args.steps, 1))
        G.plan()
    torch.cuda.synchronize()

    results = []
    per_ms = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        a = time.perf_counter()
        G.reset(s)
        r = G.plan()
        per_ms.append((time.perf_counter() - a) * 1e3)
        results.append(r)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    valid = sum(r["valid_total"] for r in results)
    lanes = sum(r["lanes_total"] for r in results)
    solved = [ms for ms, r in zip(per_ms, results) if r["status"] == SOLVED]

    # per-kernel HIP-event durations on the planner's stream (separate pass)
    G.set_profiling(True)
    steps_tot = box_tot = lanes_prof = checked_tot = 0
    profile_steps = args.steps if args.profile_steps < 0 else args.profile_steps
    paths = []
    for s in range(profile_steps):
        G.reset(s)
        r = G.plan()
        if r["status"] == SOLVED:
            paths.append((gpu_workload(args.workload, s), G.trajectory(r["goal_id"])))
        st = G.stats()
        steps_tot += st["steps_total"]
        checked_tot += st["checked_steps_total"]
        box_tot += st["box_tests_total"]
        lanes_prof += st["lanes_total"]
    kt = G.kernel_times()
    G.set_profiling(False)
    n_launch, prop_ms = kt["propagate"]
    ops = prop_ops(dyn, integ, steps_tot, checked_tot, box_tot, lanes_prof)
    achieved = ops / (prop_ms * 1e-3) / 1e12 if prop_ms > 0 else 0.0

    line = {
        "metric": METRIC,
        "value": valid / elapsed,
        "unit": "valid expansions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": p["name"],
            "dynamics": "12D quadcopter RK4 h=0.02 x 20" if dyn == 1 else "6D double integrator",
            "obstacles": int(len(p["obstacles"])),
            "regions": list(p["grid"]),
            "node_cap": int(p["node_cap"]),
            "lambda_max": int(p["lambda_max"]),
            "query": "one planning query per step, planner seeds 0..steps-1",
        },
        "median_tts_ms": statistics.median(solved) if solved else None,
        "mean_tts_ms": statistics.mean(solved) if solved else None,
        "p10_tts_ms": percentile(solved, 10),
        "p90_tts_ms": percentile(solved, 90),
        "success_rate": len(solved) / len(results),
        "attempted_expansions_per_s": lanes / elapsed,
        "statuses": [r["status"] for r in results],
        "iterations": [r["iterations"] for r in results],
        "roofline": {
            "kernel": "k_propagate",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": measured_traffic(p["name"]),
            "launches": n_launch,
            "avg_launch_ms": prop_ms / n_launch if n_launch else None,
            "ops_per_launch": ops / n_launch if n_launch else None,
            "steps_per_lane": steps_tot / lanes_prof if lanes_prof else None,
            "checked_steps_per_lane": checked_tot / lanes_prof if lanes_prof else None,
            "box_tests_per_checked_step": box_tot / checked_tot if checked_tot else None,
        },
        "post_hbm": post_hbm(p["name"], kt),
        "grid": {"propagate": G.stats()["grid_propagate"], "nodes": G.stats()["grid_nodes"]},
        "kernel_ms": {k: v[1] for k, v in kt.items()},
        "kernel_launches": {k: v[0] for k, v in kt.items()},
    }
    replays = {"uniform": paths}
    if not args.no_learned:
        lpaths, lrn = learned_leg(G, p, args.steps, args.warmup, args.learned_paths,
                                  args.learned_rows, args.learned_train_steps, args.learned_batch,
                                  3e-3, args.learned_mix)
        replays["learned"] = lpaths
        um, lm = line["median_tts_ms"], lrn["median_tts_ms"]
        lrn["median_tts_ratio_learned_over_uniform"] = lm / um if (um and lm) else None
        line["learned"] = lrn
    if not args.no_batched:
        bpaths, line["batched"] = batched_leg(args.batch_queries)
        replays["batched"] = bpaths
    if not args.no_cpu_baseline:
        # the oracle leg: CPU baseline timings, then the FP64 replay of every
        # trajectory the legs above returned (outside every timed region)
        entry, rep = oracle_leg(args.workload, args.cpu_budget_s, args.cpu_tts_seeds,
                                args.cpu_tts_budget_s, replays)
        line["cpu_baseline"] = entry
        line.update(rep["uniform"])
        if "learned" in rep:
            line["learned"].update(rep["learned"])
        if "batched" in rep:
            line["batched"].update(rep["batched"])
    print(json.dumps(line))


if __name__ == "__main__":
    main()
