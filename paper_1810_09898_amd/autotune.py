"""Autotuner for the grouping and tile parameters.

The paper finds its grouping factor f by hand, from a few full runs (section
"Results": f = 0.45, 0.50, 0.55 tried, 0.50 best).  Here the search is
automatic: a coordinate descent over

    policy/f  - paper policy with f in F_GRID, or count policy
    n_group_max, t_cand (LDS candidate tile), n_leaf (tree), skin (walk radius)

timing density + hydro (HIP events through the C-ABI) on the actual
workload, starting from the prior of Eq. (1): a group within R = f h holds
about f^3 N_ngb particles, so f = (N_group / N_ngb)^(1/3) for the target
group size, while the superset grows as (1 + f)^3 N_ngb.  Results are cached
in a JSON file keyed by a workload signature (N bucket, active fraction
bucket, N_ngb, kernel).
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
T_GRID = (1024, 2048, 4096)
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


def prior(w) -> StepConfig:
    """Eq. (1): f = (N_group / N_ngb)^(1/3); aim at N_group ~ N_ngb/8 (f = 0.5,
    the paper's choice), capped by the 64 lanes of a wave."""
    ng = min(64, max(4, w.n_ngb // 8))
    f = (ng / w.n_ngb) ** (1.0 / 3.0)
    f = min(F_GRID, key=lambda v: abs(v - f))
    sup = (1 + f) ** 3 * w.n_ngb
    t = next((t for t in T_GRID if t >= 1.3 * sup), T_GRID[-1])
    return StepConfig(n_leaf=16, policy=S.POLICY_PAPER, n_group_max=min(64, max(8, ng)), f=f,
                      chunk=1024, t_cand=t, hydro_t_cand=t, skin=1.0)


def measure(w, cfg: StepConfig, reps: int = 3) -> dict:
    """Median device time (ms) of density (+ hydro) and of the whole step."""
    import torch
    pl = Pipeline(w, cfg)
    pl.step()
    torch.cuda.synchronize()
    dens, hyd, step = [], [], []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        pl.sort()
        pl.tree()
        pl.groups()
        ev[1].record()
        pl.density()
        ev[2].record()
        if pl.hydro:
            pl.hydro_force()
        ev[3].record()
        torch.cuda.synchronize()
        dens.append(ev[1].elapsed_time(ev[2]))
        hyd.append(ev[2].elapsed_time(ev[3]))
        step.append(ev[0].elapsed_time(ev[3]))
    st = pl.ctx.status(raise_on_overflow=False)
    del pl
    return {"density_ms": float(np.median(dens)), "hydro_ms": float(np.median(hyd)),
            "step_ms": float(np.median(step)), "flags": st["flags"]}


def _key(cfg):
    return (cfg.policy, cfg.n_group_max, round(cfg.f, 3), cfg.t_cand, cfg.n_leaf, cfg.skin,
            cfg.level if cfg.policy == S.POLICY_TREE else -1)


def tune(w, base: StepConfig | None = None, rounds: int = 2, log=print, objective="step_ms"):
    """Coordinate descent from `base` (default: the Eq. (1) prior)."""
    best = base or prior(w)
    seen = {}

    def cost(cfg):
        k = _key(cfg)
        if k not in seen:
            t0 = time.time()
            r = measure(w, cfg)
            seen[k] = r
            log(f"  {asdict(cfg)} -> {r} ({time.time() - t0:.1f} s)")
        r = seen[k]
        return r[objective] if r["flags"] == 0 else float("inf")

    best_cost = cost(best)
    for _ in range(rounds):
        improved = False
        axes = [
            [best.with_(policy=S.POLICY_PAPER, f=f) for f in F_GRID]
            + [best.with_(policy=S.POLICY_COUNT, f=0.0)]
            + [best.with_(policy=S.POLICY_TREE, level=lv) for lv in LEVEL_GRID],
            [best.with_(n_group_max=g) for g in NG_GRID],
            [best.with_(t_cand=t, hydro_t_cand=t) for t in T_GRID],
            [best.with_(n_leaf=l) for l in LEAF_GRID],
            [best.with_(skin=s) for s in SKIN_GRID],
        ]
        for cands in axes:
            for c in cands:
                v = cost(c)
                if v < best_cost * 0.995:
                    best, best_cost, improved = c, v, True
        if not improved:
            break
    return best, best_cost, seen


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def tuned_config(w, retune=False, log=print) -> StepConfig:
    """Cached tuned configuration for this workload's signature."""
    cache = load_cache()
    sig = signature(w)
    if sig in cache and not retune:
        return StepConfig(**cache[sig]["config"])
    best, c, _ = tune(w, log=log)
    cache[sig] = {"config": asdict(best), "cost_ms": c}
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    with open(CACHE, "w") as fh:
        json.dump(cache, fh, indent=1)
    return best


def per_box_params(w, cfg_for_box) -> np.ndarray:
    """Per-box group parameter table (device layout of sfc_group_params) for a
    batch of boxes: cfg_for_box(b, n_b, active_fraction) -> (policy, cap, f, chunk[,
    level])."""
    nb = len(w.box_L)
    arr = (S.GroupParams * nb)()
    for b in range(nb):
        a0, a1 = int(w.box_off[b]), int(w.box_off[b + 1])
        frac = float(w.state["active"][a0:a1].mean()) if a1 > a0 else 0.0
        pol, cap, f, chunk, *lev = cfg_for_box(b, a1 - a0, frac)
        arr[b] = S.GroupParams(int(pol), int(cap), float(f), int(chunk), int(lev[0]) if lev else 0)
    return np.frombuffer(bytes(arr), dtype=np.uint8).copy()


def batch_rule(b, n_b, frac):
    """Per-box rule for batches: dense active sets group well (paper policy,
    f = 0.5); sparse ones group poorly, so cap by count of the few actives."""
    if frac < 0.05:
        return (S.POLICY_PAPER, 8, 0.5, 1024)
    return (S.POLICY_PAPER, 32, 0.5, 1024)


if __name__ == "__main__":
    import argparse

    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lognormal_hydro")
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--bins", default="0",
                    help="timestep bins to tune one after the other (workloads with state['bin']: "
                         "bin b = the particles whose deepest bin is >= b are active)")
    args = ap.parse_args()
    W.VERBOSE = True
    w = W.WORKLOADS[args.workload]()
    base = dict(w.state)
    for b in [int(v) for v in args.bins.split(",")]:
        if "bin" in base:
            w.state = dict(base)
            w.state["active"] = (base["bin"] >= b).astype(np.uint8)
        print(f"workload {args.workload} bin {b}: {w.n_active} active", flush=True)
        print("prior", asdict(prior(w)), flush=True)
        best, c, seen = tune(w, rounds=args.rounds, log=lambda s: print(s, flush=True))
        print("best", asdict(best), c, flush=True)
