"""Timing of one step on any of the synthetic workloads.

    python -m paper_1810_09898_amd.measure --workload plummer_batch [--steps K]

One JSON line per measured step kind: per-phase device times (HIP events on
the library's stream), active updates per second of the whole step and of
density + hydro, and the status counters of one step.

- plummer_batch: the 64-box batch in one launch per phase, with a per-box
  group parameter table (dense boxes: cap 32, sparse ones: cap 8).
- lognormal_bins: three nested timestep bins (all, 10 %, 1 % active) of the
  large lognormal box; one line per bin.
- the other workloads: one line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _phases(pl, reps):
    import torch
    names = ["sort", "tree", "groups", "density", "hydro"]
    calls = [pl.sort, pl.tree, pl.groups, pl.density, pl.hydro_force if pl.hydro else None]
    out = {k: [] for k in names}
    for _ in range(reps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in names]
        for (a, b), f in zip(ev, calls):
            a.record()
            if f is not None:
                f()
            b.record()
        torch.cuda.synchronize()
        for k, (a, b) in zip(names, ev):
            out[k].append(a.elapsed_time(b))
    return {k: float(np.median(v)) for k, v in out.items()}


def run(w, cfg, label, steps, gp_box=None):
    import torch
    from .pipeline import Pipeline
    gpb = None if gp_box is None else torch.as_tensor(gp_box, device="cuda")
    pl = Pipeline(w, cfg, gp_box=gpb)
    pl.step()
    torch.cuda.synchronize()
    pl.ctx.status_clear()
    pl.step()
    st = pl.ctx.status(raise_on_overflow=False)
    ph = _phases(pl, steps)
    A = int(w.state["active"].sum())
    t = sum(ph.values())
    line = {"workload": label, "n": w.n, "boxes": len(w.box_L), "n_active": A,
            "phases_ms": {k: round(v, 4) for k, v in ph.items()}, "step_ms": round(t, 4),
            "active_updates_per_s": round(A / (t * 1e-3), 1),
            "density_plus_hydro_updates_per_s": round(A / ((ph["density"] + ph["hydro"]) * 1e-3), 1),
            "status": st, "config": {k: getattr(cfg, k) for k in
                                     ("n_leaf", "policy", "n_group_max", "f", "t_cand", "skin")}}
    print(json.dumps(line), flush=True)
    del pl
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lognormal_hydro")
    ap.add_argument("--steps", type=int, default=5)
    args = ap.parse_args()
    from . import workloads as W
    from . import autotune
    from .pipeline import StepConfig
    W.VERBOSE = True
    t0 = time.time()
    w = W.WORKLOADS[args.workload]()
    print(f"# {args.workload}: generated in {time.time() - t0:.1f} s, n={w.n}", file=sys.stderr,
          flush=True)
    if args.workload == "plummer_batch":
        cfg = StepConfig(n_leaf=16, n_group_max=32, f=0.5, t_cand=1024, hydro_t_cand=1024)
        run(w, cfg, "plummer_batch (per-box parameters)", args.steps,
            gp_box=autotune.per_box_params(w, autotune.batch_rule))
    elif args.workload == "lognormal_bins":
        cfg = StepConfig(n_leaf=32, n_group_max=36, f=0.6, t_cand=2048, hydro_t_cand=2048)
        base = dict(w.state)
        for b, frac in ((0, "100%"), (1, "10%"), (2, "1%")):
            w.state = dict(base)
            w.state["active"] = (base["bin"] >= b).astype(np.uint8)
            run(w, cfg, f"lognormal_bins bin {b} ({frac} active)", args.steps)
    else:
        cfg = StepConfig(n_leaf=32, n_group_max=36, f=0.6, t_cand=2048, hydro_t_cand=2048)
        if w.n_ngb < 100:
            cfg = cfg.with_(n_leaf=16, f=0.5, t_cand=1024, hydro_t_cand=1024)
        run(w, cfg, args.workload, args.steps)


if __name__ == "__main__":
    main()
