"""The autotuner's host logic on the CPU: the Eq. (1) prior, the coordinate
descent (with a stand-in for the timed measurement), the cache, the per-box
buckets and the per-box parameter table of a batch."""
import ctypes as C
import math
import os

import numpy as np
import pytest

from paper_1810_09898_amd import autotune as AT
from paper_1810_09898_amd import sfcngb as S
from paper_1810_09898_amd.pipeline import StepConfig
from paper_1810_09898_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _W:
    """The few attributes of a workload that the prior and the cache read."""

    def __init__(self, n_ngb, n=1 << 20, n_active=1 << 18, kernel=1):
        self.n_ngb, self.n, self.n_active, self.kernel = n_ngb, n, n_active, kernel
        self.box_L = np.ones(1)
        self.hydro = True


@pytest.mark.parametrize("n_ngb", [32, 64, 128, 295, 512])
def test_prior_follows_eq1(n_ngb):
    """Eq. (1): a group within R = f h_0 holds ~f^3 N_ngb particles and its
    superset (1 + f)^3 N_ngb; the prior aims at N_group = N_ngb / 8 (the
    paper's f = 1/2) within the wave's 64 lanes."""
    cfg = AT.prior(_W(n_ngb))
    ng = min(64, max(4, n_ngb // 8))
    f_exact = (ng / n_ngb) ** (1.0 / 3.0)
    assert cfg.f in AT.F_GRID
    assert abs(cfg.f - f_exact) <= min(abs(g - f_exact) for g in AT.F_GRID) + 1e-12
    assert cfg.n_group_max == min(64, max(8, ng))
    assert cfg.policy == S.POLICY_PAPER
    sup = (1 + cfg.f) ** 3 * n_ngb
    assert cfg.t_cand >= min(1.3 * sup, AT.T_GRID[-1])
    assert cfg.t_cand in AT.T_GRID


def test_prior_at_the_paper_point():
    # N_ngb = 291 (the paper's test case) gives its own f = 1/2 and a
    # superset of 3.375 N_ngb candidates
    cfg = AT.prior(_W(291))
    assert cfg.f == 0.5
    assert abs((1 + cfg.f) ** 3 - 3.375) < 1e-15


def _stub_cost(best):
    """A separable cost with its minimum at `best` (and one infeasible point)."""
    calls = []

    def fn(w, cfg):
        calls.append(cfg)
        c = 1.0
        c += 0.3 * abs(math.log(cfg.n_group_max / best.n_group_max))
        c += 0.2 * (cfg.policy != best.policy) + 0.5 * abs(cfg.f - best.f)
        c += 0.1 * abs(math.log2(cfg.t_cand / best.t_cand))
        c += 0.05 * abs(math.log2(cfg.n_leaf / best.n_leaf)) + 2.0 * abs(cfg.skin - best.skin)
        flags = S.ST_GUARD if cfg.n_group_max == 64 else 0
        return {"step_ms": c, "flags": flags}
    return fn, calls


def test_coordinate_descent_finds_the_optimum():
    best = StepConfig(policy=S.POLICY_PAPER, f=0.7, n_group_max=24, t_cand=2048, n_leaf=64,
                      skin=1.05)
    fn, calls = _stub_cost(best)
    got, cost, seen = AT.tune(_W(295), rounds=3, log=lambda s: None, measure_fn=fn)
    assert (got.policy, got.f, got.n_group_max, got.t_cand, got.n_leaf, got.skin) == \
        (best.policy, best.f, best.n_group_max, best.t_cand, best.n_leaf, best.skin)
    assert abs(cost - 1.0) < 1e-12
    # every configuration is measured once; flagged ones are never chosen
    keys = [AT._key(c) for c in calls]
    assert len(keys) == len(set(keys))
    assert all(r["flags"] == 0 for k, r in seen.items() if k == AT._key(got))


def test_tuned_config_is_cached(tmp_path):
    best = StepConfig(policy=S.POLICY_COUNT, f=0.0, n_group_max=16, t_cand=1024, n_leaf=32)
    fn, calls = _stub_cost(best)
    path = str(tmp_path / "cache.json")
    w = _W(64)
    a = AT.tuned_config(w, log=lambda s: None, path=path, measure_fn=fn)
    n = len(calls)
    b = AT.tuned_config(w, log=lambda s: None, path=path, measure_fn=fn)
    assert a == b and len(calls) == n  # the second call reads the cache
    assert a.policy == S.POLICY_COUNT and a.n_group_max == 16


def test_per_box_tuning_and_table():
    w = W.plummer_batch(n_boxes=6, seed0=1000, n_range=(2000, 30000))
    buckets = AT.box_buckets(w)
    assert sum(len(v) for v in buckets.values()) == 6
    for sig, boxes in buckets.items():
        for b in boxes:
            n_b = int(w.box_off[b + 1] - w.box_off[b])
            frac = float(w.state["active"][w.box_off[b]:w.box_off[b + 1]].mean())
            assert AT.box_signature(n_b, frac) == sig
    # a stand-in cost that prefers a larger cap for boxes with more actives
    seen_boxes = []

    def fn(sw, cfg):
        seen_boxes.append(sw.n)
        want = 32 if sw.n_active > 3000 else 8
        return {"step_ms": 1.0 + abs(math.log(cfg.n_group_max / want))
                + 0.1 * (cfg.policy != S.POLICY_PAPER) + abs(cfg.f - 0.5), "flags": 0}
    cfg_for_box, res = AT.tune_boxes(w, AT.prior(w), log=lambda s: None, measure_fn=fn)
    assert set(res) == set(buckets)
    table = AT.per_box_params(w, cfg_for_box)
    arr = (S.GroupParams * 6).from_buffer_copy(table.tobytes())
    assert table.nbytes == 6 * C.sizeof(S.GroupParams)
    for b in range(6):
        a0, a1 = int(w.box_off[b]), int(w.box_off[b + 1])
        want = 32 if int(w.state["active"][a0:a1].sum()) > 3000 else 8
        sig = AT.box_signature(a1 - a0, float(w.state["active"][a0:a1].mean()))
        rep = max(buckets[sig], key=lambda q: int(w.box_off[q + 1] - w.box_off[q]))
        rep_act = int(w.state["active"][w.box_off[rep]:w.box_off[rep + 1]].sum())
        assert arr[b].n_group_max == (32 if rep_act > 3000 else 8)
        assert arr[b].policy == S.POLICY_PAPER and arr[b].f == 0.5
        assert arr[b].t_cand == AT.prior(w).t_cand  # the stand-in cost ignores the tile
    # the sub-workload of a box is that box alone
    sw = AT.sub_workload(w, 2)
    assert sw.n == int(w.box_off[3] - w.box_off[2])
    assert np.array_equal(sw.state["x"], w.state["x"][w.box_off[2]:w.box_off[3]])
