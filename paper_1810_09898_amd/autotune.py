"""Autotuner for the grouping and tile parameters.

The paper finds its grouping factor f by hand, from a few full runs (section
"Results": f = 0.45, 0.50, 0.55 tried, 0.50 best).  Here the search is
automatic: a coordinate descent over

    policy/f  - paper policy with f in F_GRID, count policy, tree policy by depth
    n_group_max, t_cand (candidate tile), n_leaf (tree), skin (walk radius)

timing the whole step (sort, tree, groups, density, hydro) captured once as
a HIP graph and replayed through the C-ABI, on the actual workload, starting
from the prior of Eq. (1): a group within R = f h holds about f^3 N_ngb
particles, so f = (N_group / N_ngb)^(1/3) for the target group size, while
the superset grows as (1 + f)^3 N_ngb.  Results are cached in a JSON file
keyed by a workload signature (N bucket, active fraction bucket, N_ngb,
kernel).

A batch of boxes is tuned per box: boxes are bucketed by their own
signature (particle count and active fraction), the largest box of each
bucket is tuned on its own for the group parameters (policy, f,
n_group_max), and the per-box parameter table of the batch gives every box
its bucket's result; the launch-wide parameters (tile, leaf size) are then
tuned on the whole batch with that table.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict

import numpy as np

from . import sfcngb as S
from .pipeline import Pipeline, StepConfig

F_GRID = (0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 1.0)
NG_GRID = (4, 8, 16, 24, 32, 48, 64)
T_GRID = (256, 512, 1024, 2048, 4096)
LEAF_GRID = (8, 16, 32, 64, 128, 256)
SKIN_GRID = (1.0, 1.05, 1.1)
LEVEL_GRID = (3, 4, 5, 6, 7, 8)  # tree policy: depth of the grouping nodes

CACHE = os.environ.get("SFCNGB_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib",
                                    "tune_cache.json"))


def signature(w) -> str:
    n_bucket = int(round(math.log2(max(w.n, 1))))
    a_bucket = int(round(10 * w.n_active / max(w.n, 1)))
    return f"n2^{n_bucket}-act{a_bucket}-ngb{w.n_ngb}-k{w.kernel}-b{len(w.box_L)}-h{int(w.hydro)}"


def box_signature(n_b: int, frac: float) -> tuple:
    """Bucket of one box of a batch: particle count to the nearest power of
    two, active fraction on a log scale (eight buckets per decade)."""
    return (int(round(math.log2(max(n_b, 1)))),
            int(round(8 * math.log10(max(frac, 1e-3)))) if frac > 0 else -99)


def prior(w) -> StepConfig:
    """Eq. (1): f = (N_group / N_ngb)^(1/3); aim at N_group ~ N_ngb/8 (f = 0.5,
    the paper's choice), capped by the 64 lanes of a wave; the tile holds the
    expected superset (1 + f)^3 N_ngb with a margin."""
    ng = min(64, max(4, w.n_ngb // 8))
    f = (ng / w.n_ngb) ** (1.0 / 3.0)
    f = min(F_GRID, key=lambda v: abs(v - f))
    sup = (1 + f) ** 3 * w.n_ngb
    t = next((t for t in T_GRID if t >= 1.3 * sup), T_GRID[-1])
    return StepConfig(n_leaf=16, policy=S.POLICY_PAPER, n_group_max=min(64, max(8, ng)), f=f,
                      t_cand=t, hydro_t_cand=t, skin=1.0)


def measure(w, cfg: StepConfig, reps: int = 5, gp_box=None) -> dict:
    """Device time (ms) of the whole step as the median of `reps` replays of
    its HIP graph, and of density and hydro from one eager step with events;
    the status flags of the step (a configuration that overflows a device
    capacity or hits a loop limit is not a candidate)."""
    import torch
    side = torch.cuda.Stream()
    gpb = None if gp_box is None else torch.as_tensor(gp_box, device="cuda")
    with torch.cuda.stream(side):
        pl = Pipeline(w, cfg, gp_box=gpb)
    pl.step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(side)
    pl.sort()
    pl.tree()
    pl.groups()
    pl.density()
    ev[1].record(side)
    if pl.hydro:
        pl.hydro_force()
    ev[2].record(side)
    torch.cuda.synchronize()
    st = pl.ctx.status(raise_on_overflow=False)
    pl.ctx.graph_begin()
    pl.step()
    g = pl.ctx.graph_end()
    times = []
    try:
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(side)
            pl.ctx.graph_launch(g)
            b.record(side)
            side.synchronize()
            times.append(a.elapsed_time(b))
    finally:
        pl.ctx.graph_destroy(g)
    del pl
    return {"step_ms": float(np.median(times)), "search_ms": ev[0].elapsed_time(ev[2]),
            "hydro_ms": ev[1].elapsed_time(ev[2]), "flags": st["flags"]}


def _key(cfg):
    return (cfg.policy, cfg.n_group_max, round(cfg.f, 3), cfg.t_cand, cfg.n_leaf, cfg.skin,
            cfg.level if cfg.policy == S.POLICY_TREE else -1)


def tune(w, base: StepConfig | None = None, rounds: int = 2, log=print, objective="step_ms",
         measure_fn=None, axes=("group", "cap", "tile", "leaf", "skin"), gp_box=None):
    """Coordinate descent from `base` (default: the Eq. (1) prior) over the
    named axes; measure_fn(w, cfg) -> {objective: ms, "flags": ...} (default:
    graph replays of the step on the GPU)."""
    measure_fn = measure_fn or (lambda ww, c: measure(ww, c, gp_box=gp_box))
    best = base or prior(w)
    seen = {}

    def cost(cfg):
        k = _key(cfg)
        if k not in seen:
            t0 = time.time()
            r = measure_fn(w, cfg)
            seen[k] = r
            log(f"  {asdict(cfg)} -> {r} ({time.time() - t0:.1f} s)")
        r = seen[k]
        return r[objective] if r["flags"] == 0 else float("inf")

    def candidates(axis, b):
        if axis == "group":
            return ([b.with_(policy=S.POLICY_PAPER, f=f) for f in F_GRID]
                    + [b.with_(policy=S.POLICY_COUNT, f=0.0)]
                    + [b.with_(policy=S.POLICY_TREE, level=lv) for lv in LEVEL_GRID])
        if axis == "cap":
            return [b.with_(n_group_max=g) for g in NG_GRID]
        if axis == "tile":
            return [b.with_(t_cand=t, hydro_t_cand=t) for t in T_GRID]
        if axis == "leaf":
            return [b.with_(n_leaf=l) for l in LEAF_GRID]
        if axis == "skin":
            return [b.with_(skin=s) for s in SKIN_GRID]
        raise ValueError(axis)

    best_cost = cost(best)
    for _ in range(rounds):
        improved = False
        for axis in axes:
            for c in candidates(axis, best):
                v = cost(c)
                if v < best_cost * 0.995:
                    best, best_cost, improved = c, v, True
        if not improved:
            break
    return best, best_cost, seen


def load_cache(path=None) -> dict:
    path = path or CACHE
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def tuned_config(w, retune=False, log=print, path=None, measure_fn=None) -> StepConfig:
    """Cached tuned configuration for this workload's signature."""
    path = path or CACHE
    cache = load_cache(path)
    sig = signature(w)
    if sig in cache and not retune:
        return StepConfig(**cache[sig]["config"])
    best, c, _ = tune(w, log=log, measure_fn=measure_fn)
    cache[sig] = {"config": asdict(best), "cost_ms": c}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1)
    return best


def per_box_params(w, cfg_for_box) -> np.ndarray:
    """Per-box group parameter table (device layout of sfc_group_params) for a
    batch of boxes: cfg_for_box(b, n_b, active_fraction) -> (policy, cap, f[, level
    [, t_cand]]) (t_cand 0: the call's)."""
    nb = len(w.box_L)
    arr = (S.GroupParams * nb)()
    for b in range(nb):
        a0, a1 = int(w.box_off[b]), int(w.box_off[b + 1])
        frac = float(w.state["active"][a0:a1].mean()) if a1 > a0 else 0.0
        pol, cap, f, *rest = cfg_for_box(b, a1 - a0, frac)
        lev = int(rest[0]) if len(rest) > 0 else 0
        tc = int(rest[1]) if len(rest) > 1 else 0
        arr[b] = S.GroupParams(int(pol), int(cap), float(f), lev, tc)
    return np.frombuffer(bytes(arr), dtype=np.uint8).copy()


def sub_workload(w, b):
    """Box b of a batch as a workload of its own."""
    from .workloads import Workload
    a0, a1 = int(w.box_off[b]), int(w.box_off[b + 1])
    st = {k: np.ascontiguousarray(v[a0:a1]) for k, v in w.state.items()}
    st["orig"] = np.arange(a1 - a0, dtype=np.uint32)
    return Workload(f"{w.name}[{b}]", st, np.array([0, a1 - a0], np.int64),
                    np.array([w.box_L[b]]), w.kernel, w.n_ngb, w.dn, w.fixed_h, w.hydro,
                    w.n_group_max, w.f)


def box_buckets(w) -> dict:
    """box_signature -> the boxes of the batch in that bucket (boxes with at
    least one active particle)."""
    out = {}
    for b in range(len(w.box_L)):
        a0, a1 = int(w.box_off[b]), int(w.box_off[b + 1])
        if a1 <= a0:
            continue
        frac = float(w.state["active"][a0:a1].mean())
        if frac <= 0:
            continue
        out.setdefault(box_signature(a1 - a0, frac), []).append(b)
    return out


def tune_boxes(w, base: StepConfig, log=print, rounds=1, measure_fn=None):
    """Per-box group parameters for a batch: each bucket's largest box tuned
    on its own over the group policy/f, the cap and the superset tile
    (launch-wide parameters from `base`; a bucket's tile becomes its boxes'
    t_cand, under the launch's).  Returns (cfg_for_box for per_box_params,
    per-bucket results)."""
    res = {}
    for sig, boxes in sorted(box_buckets(w).items()):
        rep = max(boxes, key=lambda b: int(w.box_off[b + 1] - w.box_off[b]))
        sw = sub_workload(w, rep)
        log(f"bucket {sig}: {len(boxes)} boxes, tuning box {rep} ({sw.n} particles, "
            f"{sw.n_active} active)")
        best, c, _ = tune(sw, base, rounds=rounds, log=log, measure_fn=measure_fn,
                          axes=("group", "cap", "tile"))
        res[sig] = (best.policy, best.n_group_max, best.f, best.level, best.t_cand)

    def cfg_for_box(b, n_b, frac):
        if n_b == 0 or frac <= 0:
            return (S.POLICY_COUNT, 1, 0.0, 0)
        sig = box_signature(n_b, frac)
        if sig in res:
            return res[sig]
        # a bucket with no tuned box: the nearest tuned one
        near = min(res, key=lambda s: (s[0] - sig[0]) ** 2 + (s[1] - sig[1]) ** 2)
        return res[near]

    return cfg_for_box, res


def batch_rule(b, n_b, frac):
    """Hand rule for batches (the reference point of the per-box tuner):
    dense active sets group well (paper policy, f = 0.5); sparse ones group
    poorly, so cap by count of the few actives."""
    if frac < 0.05:
        return (S.POLICY_PAPER, 8, 0.5)
    return (S.POLICY_PAPER, 32, 0.5)


if __name__ == "__main__":
    import argparse

    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lognormal_hydro")
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--start", default="",
                    help="start of the descent instead of the Eq. (1) prior: comma-separated "
                         "StepConfig fields, e.g. n_leaf=128,n_group_max=24,f=0.5,t_cand=2048")
    ap.add_argument("--bins", default="0",
                    help="timestep bins to tune one after the other (workloads with state['bin']: "
                         "bin b = the particles whose deepest bin is >= b are active)")
    args = ap.parse_args()
    W.VERBOSE = True
    w = W.WORKLOADS[args.workload]()
    if len(w.box_L) > 1:
        base = prior(w)
        cfg_for_box, res = tune_boxes(w, base, log=lambda s: print(s, flush=True))
        print("per-box", {str(k): v for k, v in res.items()}, flush=True)
        table = per_box_params(w, cfg_for_box)
        best, c, _ = tune(w, base, rounds=1, axes=("tile", "leaf"), gp_box=table,
                          log=lambda s: print(s, flush=True))
        print("best launch-wide", asdict(best), c, flush=True)
    else:
        base = dict(w.state)
        for b in [int(v) for v in args.bins.split(",")]:
            if "bin" in base:
                w.state = dict(base)
                w.state["active"] = (base["bin"] >= b).astype(np.uint8)
            print(f"workload {args.workload} bin {b}: {w.n_active} active", flush=True)
            start = prior(w)
            if args.start:
                kw = {}
                for item in args.start.split(","):
                    key, val = item.split("=")
                    kw[key] = type(getattr(start, key))(float(val) if "." in val else int(val))
                start = start.with_(**kw)
                if "t_cand" in kw:
                    start = start.with_(hydro_t_cand=kw["t_cand"])
            print("start", asdict(start), flush=True)
            best, c, seen = tune(w, start, rounds=args.rounds, log=lambda s: print(s, flush=True))
            print("best", asdict(best), c, flush=True)
