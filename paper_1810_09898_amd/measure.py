"""Timing of one step on any of the synthetic workloads.

    python -m paper_1810_09898_amd.measure --workload plummer_batch [--steps K]

One JSON line per measured step kind: per-phase device times (HIP events on
the library's stream), active updates per second of the whole step and of
density + hydro, and the status counters of one step.

- plummer_batch: the 64-box batch in one launch per phase, with a per-box
  group parameter table (dense boxes: cap 32, sparse ones: cap 8).
- lognormal_bins: three nested timestep bins (all, 10 %, 1 % active) of the
  large lognormal box; one line per bin, each with the step also captured in
  a HIP graph and replayed, and the FP32-compensated results compared with
  the FP64-accumulator variant on the GPU (relative errors per field).
- the other workloads: one line.
- --workload lognormal_bins --reuse-bins SKIN: bins 1 and 2 on the
  supersets kept by the full step (all active) after a drift (the first of
  FRACS), beside the ordinary bin steps.
- --reuse SKINS: superset reuse after a drift.  Per skin, a walking step that
  keeps its supersets, then per drift (the fastest particle moving FRACS times
  the smallest h, as in a global step limited by the Courant condition;
  positions advanced in place along v) the step on the kept
  supersets (tree refit, density, hydro; h reset to the walking step's input
  before each repetition), beside the ordinary step (skin 1, nothing kept).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _phases(pl, reps):
    import torch
    torch.cuda.synchronize()
    names = ["sort", "tree", "groups", "density", "hydro"]
    calls = [pl.sort, pl.tree, pl.groups, pl.density, pl.hydro_force if pl.hydro else None]
    out = {k: [] for k in names}
    st = pl.ctx.stream
    for _ in range(reps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in names]
        for (a, b), f in zip(ev, calls):
            a.record(st)
            if f is not None:
                f()
            b.record(st)
        torch.cuda.synchronize()
        for k, (a, b) in zip(names, ev):
            out[k].append(a.elapsed_time(b))
    return {k: float(np.median(v)) for k, v in out.items()}


def _graph_ms(pl, reps):
    """the whole step captured once as a HIP graph, median of `reps` replays"""
    import torch
    s = pl.ctx.stream
    pl.ctx.graph_begin()
    pl.step()
    g = pl.ctx.graph_end()
    out = []
    try:
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            pl.ctx.graph_launch(g)
            b.record(s)
            s.synchronize()
            out.append(a.elapsed_time(b))
    finally:
        pl.ctx.graph_destroy(g)
    return float(np.median(out))


def _precision(w, cfg, pl32):
    """FP32-compensated sums of `pl32` against the FP64-accumulator variant
    of the same step (same neighbour sets and h): per field, the largest and
    the 99.9th percentile relative error over the active particles (vectors:
    |a32 - a64| / |a64|; du/dt: |du32 - du64| / rms du64)."""
    import torch
    from . import sfcngb as S
    from .pipeline import Pipeline
    r32 = {**pl32.sorted_numpy(("h", "rho", "active")), **pl32.outputs_numpy()}
    pl = Pipeline(w, cfg.with_(accum=S.ACCUM_F64), hydro=pl32.hydro)
    pl.step()
    torch.cuda.synchronize()
    r64 = {**pl.sorted_numpy(("h", "active")), **pl.outputs_numpy()}
    del pl
    act = r32["active"] != 0
    out = {"same_h": bool(np.array_equal(r32["h"], r64["h"]))}

    def stats(e):
        e = e[act]
        return {"max": float(e.max()), "p999": float(np.quantile(e, 0.999))}

    with np.errstate(divide="ignore", invalid="ignore"):  # inactive particles hold zeros
        out["rho"] = stats(np.abs(r32["rho"].astype(np.float64) / r64["rho64"] - 1.0))
        if pl32.hydro:
            a32 = np.stack([r32[k].astype(np.float64) for k in ("ax", "ay", "az")])
            a64 = np.stack([r64[k + "64"] for k in ("ax", "ay", "az")])
            out["acc"] = stats(np.linalg.norm(a32 - a64, axis=0) / np.linalg.norm(a64, axis=0))
            du = r64["dudt64"]
            out["dudt"] = stats(np.abs(r32["dudt"] - du) / np.sqrt(np.mean(du[act] ** 2)))
    return out


def run(w, cfg, label, steps, gp_box=None, graph=False, precision=False):
    import torch
    from .pipeline import Pipeline
    gpb = None if gp_box is None else torch.as_tensor(gp_box, device="cuda")
    side = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    with torch.cuda.stream(side):
        pl = Pipeline(w, cfg, gp_box=gpb)
    pl.step()
    torch.cuda.synchronize()
    pl.ctx.status_clear()
    pl.ctx.set_trace(True)  # the schedule's tail, on this one step only
    pl.step()
    st = pl.ctx.status(raise_on_overflow=False)
    pl.ctx.set_trace(False)
    ph = _phases(pl, steps)
    A = int(w.state["active"].sum())
    t = sum(ph.values())
    line = {"workload": label, "n": w.n, "boxes": len(w.box_L), "n_active": A,
            "phases_ms": {k: round(v, 4) for k, v in ph.items()}, "step_ms": round(t, 4),
            "active_updates_per_s": round(A / (t * 1e-3), 1),
            "density_plus_hydro_updates_per_s": round(A / ((ph["density"] + ph["hydro"]) * 1e-3), 1),
            "status": st, "config": {k: getattr(cfg, k) for k in
                                     ("n_leaf", "policy", "n_group_max", "f", "t_cand", "skin")}}
    if graph:
        line["graph_step_ms"] = round(_graph_ms(pl, steps), 4)
    if precision:
        line["fp32_vs_fp64"] = _precision(w, cfg, pl)
    print(json.dumps(line), flush=True)
    del pl
    return line


def _reuse_phases(pl, h0, reps):
    import torch
    names = ["refit", "density", "hydro"]
    calls = [pl.refit, lambda: pl.density(reuse=True), lambda: pl.hydro_force(reuse=True)]
    out = {k: [] for k in names}
    st = pl.ctx.stream
    for _ in range(reps):
        with torch.cuda.stream(st):
            pl.ps.t["h"].copy_(h0)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in names]
        for (a, b), f in zip(ev, calls):
            a.record(st)
            f()
            b.record(st)
        torch.cuda.synchronize()
        for k, (a, b) in zip(names, ev):
            out[k].append(a.elapsed_time(b))
    return {k: float(np.median(v)) for k, v in out.items()}


def reuse_scan(w, cfg, steps, skins, fracs):
    import torch
    from .pipeline import Pipeline
    A = int(w.state["active"].sum())
    base = Pipeline(w, cfg)
    base.step()
    ph = _phases(base, steps)
    t_base = sum(ph.values())
    del base
    print(json.dumps({"workload": w.name, "kind": "ordinary step", "phases_ms": ph,
                      "step_ms": round(t_base, 4)}), flush=True)
    for skin in skins:
        # a skin makes the supersets larger: a larger tile keeps them whole
        T = cfg.t_cand if skin == 1.0 else 2 * cfg.t_cand
        c = cfg.with_(skin=skin, hydro_skin=skin, keep_supersets=True, t_cand=T, hydro_t_cand=T)
        pl = Pipeline(w, c)
        pl.step()
        torch.cuda.synchronize()
        ph_keep = _phases(pl, steps)  # walking steps that keep (the last one stays kept)
        t = pl.ps.t
        x0, y0, z0, h0 = (t[k].clone() for k in ("x", "y", "z", "h"))
        L = torch.as_tensor(w.box_L, dtype=torch.float64, device="cuda")
        Lp = L[0] if len(w.box_L) == 1 else None
        v = torch.sqrt(t["vx"].double() ** 2 + t["vy"].double() ** 2 + t["vz"].double() ** 2)
        hmin = float(torch.min(h0))
        for frac in fracs:
            dt = frac * hmin / float(v.max())
            for k, k0, vk in (("x", x0, "vx"), ("y", y0, "vy"), ("z", z0, "vz")):
                a = torch.remainder(k0 + dt * t[vk].double(), Lp)
                t[k].copy_(torch.where(a >= Lp, a - Lp, a))
            pl.ctx.status_clear()
            t["h"].copy_(h0)
            pl.reuse_step()
            torch.cuda.synchronize()
            st = pl.ctx.status(raise_on_overflow=False)
            ph_r = _reuse_phases(pl, h0, steps)
            tr = sum(ph_r.values())
            print(json.dumps({
                "workload": w.name, "kind": "reuse", "skin": skin, "drift_frac_min_h": frac,
                "walking_keep_step_ms": round(sum(ph_keep.values()), 4),
                "walking_keep_phases_ms": ph_keep, "reuse_step_ms": round(tr, 4),
                "reuse_phases_ms": ph_r, "ordinary_step_ms": round(t_base, 4),
                "reuse_updates_per_s": round(A / (tr * 1e-3), 1),
                "deferred_frac": round(st["n_deferred"] / max(A, 1) / 2, 5),
                "status": st}), flush=True)
        del pl


def reuse_bins(w, steps, skin, frac):
    """The finer bins of lognormal_bins on the supersets kept by the full
    step (all active, skin), after a drift of frac times the smallest h,
    beside the ordinary bin steps (sort, tree, groups, walks)."""
    import torch
    from .pipeline import Pipeline
    base = dict(w.state)
    ordinary = {}
    for b in (1, 2):
        w.state = dict(base)
        w.state["active"] = (base["bin"] >= b).astype(np.uint8)
        pl = Pipeline(w, BIN_CONFIGS[b])
        pl.step()
        ph = _phases(pl, steps)
        ordinary[b] = (sum(ph.values()), ph)
        del pl
        torch.cuda.empty_cache()
    w.state = dict(base)
    w.state["active"] = np.ones(w.n, np.uint8)
    c = BIN_CONFIGS[0]
    c = c.with_(skin=skin, hydro_skin=skin, keep_supersets=True, t_cand=2 * c.t_cand,
                hydro_t_cand=2 * c.hydro_t_cand)
    pl = Pipeline(w, c)
    pl.step()
    ph_keep = _phases(pl, steps)
    t = pl.ps.t
    x0, y0, z0, h0 = (t[k].clone() for k in ("x", "y", "z", "h"))
    Lp = float(w.box_L[0])
    v = torch.sqrt(t["vx"].double() ** 2 + t["vy"].double() ** 2 + t["vz"].double() ** 2)
    dt = frac * float(torch.min(h0)) / float(v.max())
    for k, k0, vk in (("x", x0, "vx"), ("y", y0, "vy"), ("z", z0, "vz")):
        a = torch.remainder(k0 + dt * t[vk].double(), Lp)
        t[k].copy_(torch.where(a >= Lp, a - Lp, a))
    bins = torch.as_tensor(base["bin"], device="cuda")[t["orig"].long()]
    print(json.dumps({"workload": w.name, "kind": "full step keeping its supersets", "skin": skin,
                      "step_ms": round(sum(ph_keep.values()), 4), "phases_ms": ph_keep}), flush=True)
    for b in (1, 2):
        t["active"].copy_((bins >= b).to(torch.uint8))
        A = int((bins >= b).sum())
        pl.ctx.status_clear()
        t["h"].copy_(h0)
        pl.reuse_step()
        torch.cuda.synchronize()
        st = pl.ctx.status(raise_on_overflow=False)
        ph_r = _reuse_phases(pl, h0, steps)
        tr = sum(ph_r.values())
        print(json.dumps({
            "workload": w.name, "kind": "bin reuse", "bin": b, "n_active": A, "skin": skin,
            "drift_frac_min_h": frac, "reuse_step_ms": round(tr, 4), "reuse_phases_ms": ph_r,
            "ordinary_step_ms": round(ordinary[b][0], 4), "ordinary_phases_ms": ordinary[b][1],
            "speedup": round(ordinary[b][0] / tr, 3), "status": st}), flush=True)
    del pl


def _bin_configs():
    from .pipeline import StepConfig
    # chosen by autotune.py (`--workload lognormal_bins --bins 0,1,2`)
    c = StepConfig(n_leaf=128, n_group_max=36, f=0.5, t_cand=2048, hydro_t_cand=2048)
    return {0: c, 1: c, 2: c}


def ngroup_sweep(w, steps, caps=(1, 8, 16, 32, 64)):
    """The density pass on the 262 144-particle clustered workload (N_ngb =
    64, 10 % active) for group caps N_group in `caps`, count policy and the
    paper's policy with f = 0.5 (the analogue of the paper's hand sweep of f,
    section "Results"): per case the density call's device time, the whole
    step's, mean group size, candidates per active and tests per active."""
    import torch
    from . import sfcngb as S
    from .pipeline import Pipeline, StepConfig
    A = int(w.state["active"].sum())
    base = None
    for pol, name in ((S.POLICY_COUNT, "count"), (S.POLICY_PAPER, "paper f=0.5")):
        for cap in caps:
            cfg = StepConfig(n_leaf=16, policy=pol, n_group_max=cap, f=0.5, t_cand=1024,
                             hydro_t_cand=1024)
            pl = Pipeline(w, cfg)
            pl.step()
            torch.cuda.synchronize()
            pl.ctx.status_clear()
            pl.step()
            st = pl.ctx.status(raise_on_overflow=False)
            ph = _phases(pl, steps)
            if base is None:
                base = ph["density"]
            line = {"sweep": "N_group", "workload": w.name, "policy": name, "n_group_max": cap,
                    "density_ms": round(ph["density"], 4), "step_ms": round(sum(ph.values()), 4),
                    "speedup_vs_ungrouped": round(base / ph["density"], 3),
                    "groups": st["n_groups"], "mean_group_size": round(A / max(st["n_groups"], 1), 2),
                    "cand_per_active": round(st["sum_cand"] / A, 1),
                    "tests_per_active": round(st["sum_tests"] / A, 1), "flags": st["flags"]}
            print(json.dumps(line), flush=True)
            del pl


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lognormal_hydro")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--reuse", default="", help="comma-separated skins: superset reuse scan")
    ap.add_argument("--fracs", default="0.05,0.1,0.3")
    ap.add_argument("--reuse-bins", type=float, default=0.0,
                    help="skin: finer bins of lognormal_bins on the full step's supersets")
    ap.add_argument("--sweep", action="store_true",
                    help="plummer_clustered: the N_group sweep {1, 8, 16, 32, 64}")
    ap.add_argument("--tune-boxes", action="store_true",
                    help="plummer_batch: also tune the per-box group parameters (graph replays of "
                         "each size/activity bucket's largest box) and time the batch with them")
    args = ap.parse_args()
    from . import workloads as W
    from . import autotune
    from .pipeline import StepConfig
    W.VERBOSE = True
    global BIN_CONFIGS
    BIN_CONFIGS = _bin_configs()
    t0 = time.time()
    w = W.WORKLOADS[args.workload]()
    print(f"# {args.workload}: generated in {time.time() - t0:.1f} s, n={w.n}", file=sys.stderr,
          flush=True)
    if args.sweep:
        ngroup_sweep(w, args.steps)
    elif args.reuse_bins:
        reuse_bins(w, args.steps, args.reuse_bins, float(args.fracs.split(",")[0]))
    elif args.reuse:
        cfg = StepConfig(n_leaf=128, n_group_max=24, f=0.5, t_cand=2048, hydro_t_cand=2048)
        reuse_scan(w, cfg, args.steps, [float(v) for v in args.reuse.split(",")],
                   [float(v) for v in args.fracs.split(",")])
    elif args.workload == "plummer_batch":
        cfg = StepConfig(n_leaf=16, n_group_max=32, f=0.5, t_cand=1024, hydro_t_cand=1024)
        run(w, cfg, "plummer_batch (hand rule per box)", args.steps,
            gp_box=autotune.per_box_params(w, autotune.batch_rule))
        if args.tune_boxes:
            t1 = time.time()
            cfg_for_box, res = autotune.tune_boxes(
                w, cfg, log=lambda m: print(f"# {m}", file=sys.stderr, flush=True))
            print(json.dumps({"workload": "plummer_batch", "kind": "per-box tuning",
                              "seconds": round(time.time() - t1, 1),
                              "buckets": {str(k): v for k, v in res.items()}}), flush=True)
            run(w, cfg, "plummer_batch (tuned per box)", args.steps,
                gp_box=autotune.per_box_params(w, cfg_for_box))
    elif args.workload == "lognormal_bins":
        base = dict(w.state)
        for b, frac in ((0, "100%"), (1, "10%"), (2, "1%")):
            w.state = dict(base)
            w.state["active"] = (base["bin"] >= b).astype(np.uint8)
            run(w, BIN_CONFIGS[b], f"lognormal_bins bin {b} ({frac} active)", args.steps,
                graph=True, precision=True)
    else:
        cfg = StepConfig(n_leaf=32, n_group_max=36, f=0.6, t_cand=2048, hydro_t_cand=2048)
        if w.n_ngb < 100:
            cfg = cfg.with_(n_leaf=16, f=0.5, t_cand=1024, hydro_t_cand=1024)
        run(w, cfg, args.workload, args.steps)


if __name__ == "__main__":
    main()
