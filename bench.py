"""Benchmark of the grouped SPH neighbour search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = one pass of the whole hot path over the 2,097,152-particle
lognormal workload (128^3 particles, sigma_lnrho = 1.5, P(k) ~ k^-2,
Wendland C6, N_ngb = 295, 25% active in curve-contiguous runs): Hilbert keys
+ radix sort + gather, octree, active list + groups, density with the
smoothing-length loop, hydro force.  Inputs are resident in HBM before the
timed region; every step starts from the same unsorted inputs.

Prints one JSON line: active-particle density+hydro updates per second for
the whole step, plus the grouped/ungrouped speedup, per-phase times, the
HBM-roofline fraction of the dominant kernel and the oracle's rate on the
host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# wave64 VALU instructions per second: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
# the same in lane instructions (16 lanes per SIMD per cycle): 39.3e12/s, the
# non-packed FP32 / FP64 vector rate (78.6 TFLOP/s counting an FMA as two)
ALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic lane instructions per unit of work: a member x candidate test
# of the filter, a density pair sum, a hydro pair sum
TEST_OPS, DENS_PAIR_OPS, HYD_PAIR_OPS = 10, 30, 80
# algorithmic bytes per candidate record and per active (x, y, z FP64 + m FP32;
# hydro adds h FP64 and v, rho, P f/rho^2, c FP32) and per active particle of
# inputs read plus outputs written
DENS_BC, DENS_BIO = 28, 52
HYD_BC, HYD_BIO = 60, 84
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_lognormal_2m.json")


def bench_config():
    """Launch configuration timed by the benchmark (chosen by autotune.py on
    the 2M lognormal workload)."""
    from paper_1810_09898_amd.pipeline import StepConfig
    from paper_1810_09898_amd import sfcngb as S
    return StepConfig(n_leaf=128, policy=S.POLICY_PAPER, n_group_max=24, f=0.5,
                      t_cand=2048, hydro_t_cand=2048, skin=1.0)


def _src_hash():
    from paper_1810_09898_amd.profsum import src_hash
    return src_hash()


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_phases(pl, reps=3):
    """Per-call device time (ms) of one step, median over reps, via HIP events
    recorded on the stream the library launches on."""
    import torch
    names = ["sort", "tree", "groups", "density", "hydro"]
    calls = [pl.sort, pl.tree, pl.groups, pl.density, pl.hydro_force]
    out = {k: [] for k in names}
    for _ in range(reps):
        ev = [_events() for _ in names]
        for (a, b), f in zip(ev, calls):
            a.record()
            f()
            b.record()
        torch.cuda.synchronize()
        for k, (a, b) in zip(names, ev):
            out[k].append(a.elapsed_time(b))
    return {k: float(np.median(v)) for k, v in out.items()}


def _oracle_rate(w, s, ob, act, budget_s, seed):
    """Active updates/s of the oracle on seeded samples of `act` (density with
    the h loop, then hydro), growing the sample until `budget_s` is used."""
    import oracle
    rng = np.random.default_rng(seed)
    S = 64
    t_used = 0.0
    done = 0
    while t_used < budget_s and done < len(act):
        samp = np.sort(rng.choice(act, min(S, len(act)), replace=False))
        t0 = time.perf_counter()
        r = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, samp, w.kernel, w.n_ngb,
                           w.dn, use_grid=True)
        h = s["h"].copy()
        h[samp] = r.h
        oracle.hydro(s["x"], s["y"], s["z"], h, s["m"], s["vx"], s["vy"], s["vz"], s["u"],
                     s["rho"], s["fgrad"], ob, samp, w.kernel, use_grid=True)
        dt = time.perf_counter() - t0
        t_used += dt
        done += len(samp)
        if dt < budget_s / 8:
            S *= 2
    return done, t_used


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s=15.0, single_s=5.0):
    """The oracle (FP64, OpenMP over targets, cell-grid pruning) on a seeded
    sample of the same workload: density with the h loop, then hydro; on
    every host thread, and on one."""
    import oracle
    ob = oracle.Boxes(w.box_off, w.box_L)
    keys, perm, s = oracle.sorted_state(w.state, ob)
    act = np.nonzero(s["active"])[0]
    cores = oracle.get_threads()
    done, t_used = _oracle_rate(w, s, ob, act, budget_s, 0)
    oracle.set_threads(1)
    try:
        d1, t1 = _oracle_rate(w, s, ob, act, single_s, 1)
    finally:
        oracle.set_threads(cores)
    return {"value": done / t_used, "unit": "active updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "single_core_value": d1 / t1,
            "sample": f"{done} seeded actives of the 2M lognormal workload, density "
                      f"(h loop) + hydro, FP64 cell-grid oracle, {t_used:.1f} s on {cores} "
                      f"threads; {d1} actives in {t1:.1f} s on one"}


def _stats(e):
    e = np.asarray(e, np.float64)
    return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)),
            "median": float(np.median(e))}


def error_table(w, pl32, pl64, n_samp=2048, seed=7):
    """Error per field of the GPU step against the FP64 oracle on seeded
    sampled actives, for the FP32-compensated and the FP64-accumulator
    variants of the kernels.  Density fields against the oracle's h loop and
    sums (h must be bit-exact); hydro sums against the oracle's sums on the
    h, rho and f that the GPU's hydro pass consumed (rho, f stored in FP32).
    rho and f: relative error; drho/dh, a (each component), du/dt: |error|
    over the sum of the per-pair term magnitudes; v_sig: relative error."""
    import oracle
    ob = oracle.Boxes(w.box_off, w.box_L)
    keys, perm, s = oracle.sorted_state(w.state, ob)
    act = np.nonzero(s["active"])[0]
    rng = np.random.default_rng(seed)
    samp = np.sort(rng.choice(act, min(n_samp, len(act)), replace=False))
    r = oracle.density(s["x"], s["y"], s["z"], s["h"], s["m"], ob, samp, w.kernel, w.n_ngb, w.dn,
                       use_grid=True)
    out = {"samples": int(len(samp)), "fields": {}}
    for name, pl, suf in (("fp32_kahan", pl32, ""), ("fp64_accum", pl64, "64")):
        sn = pl.sorted_numpy(("h", "rho", "fgrad", "orig"))
        o = pl.outputs_numpy()
        assert np.array_equal(sn["orig"], s["orig"]), "GPU sort differs from the oracle's"
        tab = {"h_bit_exact": bool(np.array_equal(sn["h"][samp], r.h))}
        rho = o["rho64"] if suf else sn["rho"]
        drho = o["drhodh64"] if suf else o["drhodh"]
        fg = o["fgrad64"] if suf else sn["fgrad"]
        tab["rho"] = _stats(np.abs(rho[samp] / r.rho - 1))
        tab["drhodh"] = _stats(np.abs(drho[samp] - r.drhodh) / r.abs_drhodh)
        tab["fgrad"] = _stats(np.abs(fg[samp] / r.fgrad - 1))
        hr = oracle.hydro(s["x"], s["y"], s["z"], sn["h"], s["m"], s["vx"], s["vy"], s["vz"],
                          s["u"], sn["rho"].astype(np.float64), sn["fgrad"].astype(np.float64),
                          ob, samp, w.kernel, use_grid=True)
        ea = np.max([np.abs(o[k + suf][samp] - ref) / hr.abs_a
                     for k, ref in (("ax", hr.ax), ("ay", hr.ay), ("az", hr.az))], axis=0)
        tab["acc"] = _stats(ea)
        tab["dudt"] = _stats(np.abs(o["dudt" + suf][samp] - hr.dudt) / hr.abs_du)
        tab["vsigmax"] = _stats(np.abs(o["vsigmax"][samp] / hr.vsigmax - 1))
        out["fields"][name] = tab
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ungrouped", action="store_true")
    ap.add_argument("--no-errors", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_09898_amd import sfcngb as S
    from paper_1810_09898_amd import workloads as W
    from paper_1810_09898_amd.pipeline import Pipeline

    t0 = time.time()
    w = W.lognormal_hydro()
    print(f"# workload generated in {time.time() - t0:.1f} s: n={w.n} active={w.n_active}",
          file=sys.stderr, flush=True)
    cfg = bench_config()
    pl = Pipeline(w, cfg)
    A = w.n_active

    for _ in range(args.warmup):
        pl.step()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    a, b = _events()
    torch.cuda.synchronize()
    a.record()
    for _ in range(args.steps):
        pl.step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    print(f"# timed {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # per-phase times and candidate counts of one step
    pl.ctx.status_clear()
    ph = time_phases(pl, reps=1)
    st = pl.ctx.status()
    ph = time_phases(pl, reps=3)
    dens_hyd_ms = ph["density"] + ph["hydro"]
    # sum_cand of one step covers the density and the hydro supersets
    pl.ctx.status_clear()
    pl.sort(); pl.tree(); pl.groups(); pl.density()
    st_d = pl.ctx.status()
    pl.ctx.status_clear()
    pl.hydro_force()
    st_h = pl.ctx.status()
    # the schedule of one traced step (untimed): how long the device runs
    # for the slowest workgroup / wave after the average one is done
    pl.ctx.set_trace(True)
    pl.step()
    st_tr = pl.ctx.status()
    pl.ctx.set_trace(False)
    sched = {name: {"units": st_tr["sched_units"][k], "span_us": round(st_tr["sched_span_us"][k], 1),
                    "tail_us": round(st_tr["sched_tail_us"][k], 1)}
             for k, name in enumerate(("k_dgrp_workgroups", "k_hmem_waves"))}

    speed = None
    if not args.no_ungrouped:
        ung = Pipeline(w, cfg.with_(policy=S.POLICY_COUNT, n_group_max=1))
        ung.step()
        torch.cuda.synchronize()
        ph_u = time_phases(ung, reps=3)
        speed = {
            "density": ph_u["density"] / ph["density"],
            "hydro": ph_u["hydro"] / ph["hydro"],
            "density_plus_hydro": (ph_u["density"] + ph_u["hydro"]) / dens_hyd_ms,
            "step": sum(ph_u.values()) / sum(ph.values()),
            "ungrouped_ms": ph_u,
        }
        del ung

    # roofline of the dominant call (its kernels run back to back on the
    # library's stream; the events bracket them all): density = record
    # kernel + walk + group filter rounds + solo members + per-member sums;
    # hydro = max-h refit + record kernel + walk + group filter + solo
    # members + per-member sums.  The calls are bound by vector ALU issue and
    # latency, not by HBM bandwidth, so the roofline is the ALU one:
    # algorithmic lane instructions (tests and pairs counted by the kernels x
    # the per-unit costs) / the call's time, against the chip's
    # lane-instruction rate.  The HBM view (algorithmic bytes) rides along.
    dens_bytes = st_d["sum_cand"] * DENS_BC + A * DENS_BIO
    hyd_bytes = st_h["sum_cand"] * HYD_BC + A * HYD_BIO
    dens_ops = st_d["sum_tests"] * TEST_OPS + st_d["sum_pairs"] * DENS_PAIR_OPS
    hyd_ops = st_h["sum_tests"] * TEST_OPS + st_h["sum_pairs"] * HYD_PAIR_OPS
    if ph["hydro"] >= ph["density"]:
        kname, kbytes, kops, kms = "hydro_force", hyd_bytes, hyd_ops, ph["hydro"]
    else:
        kname, kbytes, kops, kms = "density", dens_bytes, dens_ops, ph["density"]
    achieved = kbytes / (kms * 1e-3) / 1e9
    ach_ops = kops / (kms * 1e-3) / 1e12
    traffic, valu = None, None
    if os.path.exists(PMC_FILE):
        pm = json.load(open(PMC_FILE))
        call = pm.get("calls", {}).get(kname)
        if pm.get("src_hash") == _src_hash() and call:
            traffic = call.get("hbm_bytes")
            insts = call.get("valu_insts")
            if insts:
                valu = {"insts": insts, "achieved": round(insts / (kms * 1e-3), 1),
                        "peak": VALU_PEAK_WAVE_INSTS, "unit": "wave64 VALU insts/s",
                        "frac": round(insts / (kms * 1e-3) / VALU_PEAK_WAVE_INSTS, 4)}
    peak_t = ALU_PEAK_LANE_OPS / 1e12
    roof = {"bound": "alu", "achieved": round(ach_ops, 3), "peak": round(peak_t, 2),
            "unit": "T lane-instructions/s", "frac": round(ach_ops / peak_t, 4),
            "traffic": traffic, "kernel": kname,
            "kernels": ("k_dens_prep + k_walk + k_gcount + k_gorder + k_dgrp + k_dens_solo"
                        if kname == "density"
                        else "refit + k_hydro_prep + k_walk + k_hmem + k_hydro_solo"),
            "algorithmic_ops": int(kops),
            "ops_model": f"{TEST_OPS} per member x candidate test, {DENS_PAIR_OPS} per density "
                         f"pair, {HYD_PAIR_OPS} per hydro pair",
            "launch_ms": round(kms, 4),
            "hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(kbytes)},
            "other_call": {"name": "hydro_force" if kname == "density" else "density",
                           "launch_ms": round(ph["hydro"] if kname == "density" else ph["density"], 4),
                           "alu_frac": round((hyd_ops if kname == "density" else dens_ops)
                                             / ((ph["hydro"] if kname == "density" else ph["density"])
                                                * 1e-3) / ALU_PEAK_LANE_OPS, 4)},
            "valu": valu}

    # error per field against the FP64 oracle (both accumulators)
    err = None
    if not args.no_errors:
        pl64 = Pipeline(w, cfg.with_(accum=S.ACCUM_F64))
        pl.step()
        pl64.step()
        torch.cuda.synchronize()
        err = error_table(w, pl, pl64)
        del pl64
        print(f"# error table done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)

    value = A / (ms * 1e-3)
    line = {
        "metric": "active-particle density+hydro updates/s on 1 GPU (whole step: sort, tree, "
                  "groups, density with h loop, hydro)",
        "value": round(value, 1),
        "unit": "active updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 positions/membership, f32 compensated sums",
        "data": "synthetic (seeded lognormal field)",
        "config": {"workload": "lognormal_2m: 128^3=2097152 particles, sigma_lnrho=1.5, "
                               "P(k)~k^-2, Wendland C6, N_ngb=295+-6, 25% active runs, "
                               "density (h loop) then hydro",
                   "n_active": A, "n_leaf": cfg.n_leaf, "policy": "paper", "f": cfg.f,
                   "n_group_max": cfg.n_group_max, "t_cand": cfg.t_cand,
                   "parallelism": "single GPU"},
        "density_plus_hydro_updates_per_s": round(A / (dens_hyd_ms * 1e-3), 1),
        "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "grouped_vs_ungrouped": speed,
        "groups": st_d["n_groups"],
        "mean_group_size": round(A / max(st_d["n_groups"], 1), 2),
        "cand_per_active_density": round(st_d["sum_cand"] / A, 1),
        "cand_per_active_hydro": round(st_h["sum_cand"] / A, 1),
        "h_evaluations_per_active": round(st_d["sum_iters"] / A, 3),
        "solo_members": st_d["n_deferred"] + st_h["n_deferred"],
        "schedule": sched,
        "roofline": roof,
        "error_vs_fp64_oracle": err,
        "cpu_baseline": cpu,
        "paper_speedups_context": {"density": 1.65, "hydro": 1.30, "total": 1.34,
                                   "hardware": "Gadget3 on 8 MPI ranks x 2 threads (CPU)"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
