"""Launch-shape autotuner for batched planning.

A candidate is a kp_batch_config: iterations between status reads, HIP-graph
replay on or off, and the per-problem caps on propagate and node-pass
workgroups.  Every candidate plans the same batch from the same seeds; the
kernels' results do not depend on launch shapes, so every candidate must
return identical per-problem results, and a candidate that does not is an
error, not a choice.  The fastest candidate (median batch wall time over
`reps` runs) is cached in a JSON file under the batch's signature.
"""

from __future__ import annotations

import json
import os
import statistics

RESULT_KEYS = ("status", "goal_id", "iterations", "n_nodes", "path_len", "lanes_total",
               "valid_total")


def default_cache_path() -> str:
    return os.environ.get("KP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "kinopax", "autotune.json"))


def signature(problems, device_name: str = "") -> str:
    """Dynamics, problem count, and the total node capacity and obstacle
    count rounded to powers of two: batches with the same signature get the
    same configuration."""
    dyn = int(problems[0]["dynamics"])
    cap = sum(int(p["node_cap"]) for p in problems)
    obs = sum(len(p["obstacles"]) for p in problems)
    return (f"dyn{dyn}-n{len(problems)}-cap2^{max(cap, 1).bit_length()}"
            f"-obs2^{max(obs, 1).bit_length()}-{device_name}")


def candidates(default: dict) -> list:
    """The search space around the library's default configuration."""
    out = []
    for ips in (4, 8, 16):
        for graph in (0, 1):
            for div in (1, 4, 16, 64):
                out.append(dict(iters_per_sync=ips, use_graph=graph,
                                prop_blocks=max(1, default["prop_blocks"] // div),
                                node_blocks=max(1, default["node_blocks"] // div)))
    return out


def _key(results):
    return [tuple(r[k] for k in RESULT_KEYS) for r in results]


def load_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, cache: dict):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(batch, reset, sig: str, cache_path: str | None = None, space=None, reps: int = 1,
         use_cache: bool = True):
    """Pick a configuration for `batch` (an object with config(), set_config(**cfg)
    and plan() -> (results, ms)); reset() must put every problem back at the
    start of its query.  Returns (config, table) where table lists every
    candidate's median time; the chosen configuration is left set on the batch."""
    path = cache_path or default_cache_path()
    cache = load_cache(path) if use_cache else {}
    if sig in cache:
        cfg = cache[sig]["config"]
        batch.set_config(**cfg)
        return cfg, cache[sig].get("table", [])
    default = batch.config()
    space = space if space is not None else candidates(default)
    ref = None
    table = []
    for cfg in space:
        batch.set_config(**cfg)
        times = []
        for _ in range(max(1, reps)):
            reset()
            res, ms = batch.plan()
            if ref is None:
                ref = _key(res)
            elif _key(res) != ref:
                raise RuntimeError(f"configuration {cfg} changed the planning results")
            times.append(ms)
        table.append(dict(config=cfg, ms=statistics.median(times)))
    best = min(table, key=lambda t: t["ms"])
    batch.set_config(**best["config"])
    cache[sig] = dict(config=best["config"], table=table)
    save_cache(path, cache)
    return best["config"], table
