"""Host logic of the batched-planning autotuner (no GPU): it keeps the
fastest configuration, refuses one that changes results, and caches."""

import pytest

from paper_2409_06807_amd import autotune
from workloads import problem_batch


class FakeBatch:
    """Stands in for a kp_batch: time depends on the configuration, results
    do not (unless told to)."""

    def __init__(self, bad=None):
        self.cfg = dict(iters_per_sync=8, use_graph=0, prop_blocks=1024, node_blocks=512)
        self.bad = bad
        self.runs = 0

    def config(self):
        return dict(self.cfg)

    def set_config(self, **kw):
        self.cfg.update(kw)

    def plan(self):
        self.runs += 1
        c = self.cfg
        ms = 10.0 - 2.0 * c["use_graph"] + abs(c["iters_per_sync"] - 8) * 0.5 + c["prop_blocks"] / 1024
        res = [dict(status=1, goal_id=7, iterations=12, n_nodes=100, path_len=5, lanes_total=400,
                    valid_total=200)]
        if self.bad is not None and c == self.bad:
            res[0]["n_nodes"] = 101
        return res, ms


def test_tune_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    b = FakeBatch()
    cfg, table = autotune.tune(b, lambda: None, "sig-a", cache_path=path)
    assert cfg == dict(iters_per_sync=8, use_graph=1, prop_blocks=16, node_blocks=8)
    assert b.config() == cfg and len(table) == 24
    # a second tuning of the same signature reads the cache and plans nothing
    b2 = FakeBatch()
    cfg2, _ = autotune.tune(b2, lambda: None, "sig-a", cache_path=path)
    assert cfg2 == cfg and b2.runs == 0 and b2.config() == cfg
    assert "sig-a" in autotune.load_cache(path)


def test_tune_rejects_result_changes(tmp_path):
    bad = dict(iters_per_sync=16, use_graph=1, prop_blocks=256, node_blocks=128)
    with pytest.raises(RuntimeError):
        autotune.tune(FakeBatch(bad=bad), lambda: None, "sig-b", cache_path=str(tmp_path / "c.json"))


def test_signature_and_batch_workload():
    ps = problem_batch(n=12, batch_seed=3)
    s = autotune.signature(ps, "gfx950")
    assert s.startswith("dyn0-n12-") and s.endswith("gfx950")
    caps = [p["node_cap"] for p in ps]
    obs = [len(p["obstacles"]) for p in ps]
    assert min(caps) >= 16384 and max(caps) <= 1048576 and min(obs) >= 10 and max(obs) <= 2000
    for p in ps:
        d = sum((float(a) - float(b)) ** 2 for a, b in zip(p["x_init"][:3], p["goal_center"])) ** 0.5
        assert d >= 50.0
    # deterministic
    assert [len(p["obstacles"]) for p in problem_batch(n=12, batch_seed=3)] == obs
