"""Summaries of rocprofv3 output for the benchmark's kernels.

    python -m paper_1810_09898_amd.profsum trace DB OUT.txt --cmd "..."
        kernel-trace statistics (rocpd database, top_kernels view) as text.

    python -m paper_1810_09898_amd.profsum pmc OUT.json --cmd "..." \\
        --calib-fetch DIR --calib-write DIR RUN_DIR [RUN_DIR ...]
        per-call counter totals from `rocprofv3 --pmc ... --output-format csv`
        runs of bench.py, as JSON and as a text table (OUT with .txt).  FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are
        scaled by the reading of a plain copy of known size (calib.py) to give
        HBM bytes; TCC_HIT / TCC_MISS give the L2 hit rate.  A "call" is one
        library entry point: density = the record kernel, the walk, the group
        kernel and the solo kernel; hydro_force = the max-h refit, the record
        kernel, the walk, the group and solo kernels.  The source hash of the
        search kernels is stored so that the numbers are dropped once the
        kernels change.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def src_hash() -> str:
    h = hashlib.sha256()
    for f in ("search.hip", "internal.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace(db: str, out: str, cmd: str) -> str:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels"))
    lines = [f"# command: {cmd}",
             "# rocprofv3 kernel trace (top_kernels view of the rocpd database); microseconds",
             f"{'calls':>6} {'total_us':>12} {'avg_us':>10} {'pct':>6}  kernel"]
    for name, calls, tot, avg, pct in rows:
        if pct < 0.01:
            continue
        lines.append(f"{calls:6d} {tot:12.1f} {avg:10.1f} {pct:6.2f}  {name[:110]}")
    txt = "\n".join(lines) + "\n"
    with open(out, "w") as fh:
        fh.write(txt)
    return txt


def _csv(d: str):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(f[0])))


def _dispatches(rows):
    """dispatch id -> (kernel short name, {counter: value})"""
    out = collections.OrderedDict()
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        d = int(r["Dispatch_Id"])
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").split("<")[0]
        out.setdefault(d, (name, {}))[1][r["Counter_Name"]] = float(r["Counter_Value"])
    return out


DENS_CALL = ("k_dens_prep", "k_reset_pass", "k_walk", "k_gcount", "k_gorder", "k_dgrp")
HYDRO_CALL = ("k_tree_leaves", "k_tree_up3", "k_tree_nchild", "k_hydro_prep", "k_reset_pass",
              "k_walk", "k_hmem")


def _calls(disp):
    """split the dispatch sequence into density and hydro_force calls: each
    call ends with its solo-member kernel; the kernels before it back to
    the call's first one belong to it"""
    items = list(disp.items())
    calls = {"density": [], "hydro_force": []}
    for k, (_, (name, _cs)) in enumerate(items):
        for last, before, call in (("k_dens_solo", DENS_CALL, "density"),
                                   ("k_hydro_solo", HYDRO_CALL, "hydro_force")):
            if name != last:
                continue
            seg = [items[k]]
            j = k - 1
            while j >= 0 and items[j][1][0] in before and len(seg) < 16:
                seg.insert(0, items[j])
                j -= 1
            calls[call].append(seg)
    return calls


def _derived(m, f_fetch, f_write):
    """HBM bytes from the copy-calibrated FETCH_SIZE / WRITE_SIZE (KiB), the L2
    hit rate from TCC_HIT / TCC_MISS"""
    e = dict(m)
    if "FETCH_SIZE" in m and "WRITE_SIZE" in m:
        e["hbm_bytes"] = m["FETCH_SIZE"] * 1024 * f_fetch + m["WRITE_SIZE"] * 1024 * f_write
    hit = m.get("TCC_HIT_sum", m.get("TCC_HIT"))
    miss = m.get("TCC_MISS_sum", m.get("TCC_MISS"))
    if hit is not None and miss is not None and hit + miss > 0:
        e["l2_hit_rate"] = hit / (hit + miss)
    if "SQ_INSTS_VALU" in m:
        e["valu_insts"] = m["SQ_INSTS_VALU"]
    return e


def pmc(out: str, cmd: str, calib_fetch: str, calib_write: str, runs) -> dict:
    def copy_reading(d, counter):
        v = [float(r["Counter_Value"]) for r in _csv(d)
             if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter]
        return sum(v) / len(v)

    f_fetch = COPY_BYTES / (copy_reading(calib_fetch, "FETCH_SIZE") * 1024)
    f_write = COPY_BYTES / (copy_reading(calib_write, "WRITE_SIZE") * 1024)
    per_call = collections.defaultdict(lambda: collections.defaultdict(list))
    per_kernel = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in runs:
        disp = _dispatches(_csv(d))
        for name, cs in disp.values():
            for c, v in cs.items():
                per_kernel[name][c].append(v)
        for call, segs in _calls(disp).items():
            for seg in segs:
                tot = collections.Counter()
                for _, (_, cs) in seg:
                    tot.update(cs)
                for c, v in tot.items():
                    per_call[call][c].append(v)
    res = {"src_hash": src_hash(), "command": cmd, "copy_factor_fetch": f_fetch,
           "copy_factor_write": f_write, "calls": {}, "kernels": {}}
    for call, cs in per_call.items():
        m = {c: sum(v) / len(v) for c, v in sorted(cs.items())}
        res["calls"][call] = _derived(m, f_fetch, f_write)
    for k, cs in per_kernel.items():
        m = {c: sum(v) / len(v) for c, v in sorted(cs.items())}
        res["kernels"][k] = _derived(m, f_fetch, f_write)
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    with open(os.path.splitext(out)[0] + ".txt", "w") as fh:
        fh.write(_table(res))
    return res


def _table(res) -> str:
    cols = (("hbm_bytes", "HBM GB", 1e9), ("l2_hit_rate", "L2 hit", 1.0),
            ("SQ_INSTS_VALU", "VALU M", 1e6), ("SQ_INSTS_SALU", "SALU M", 1e6),
            ("SQ_INSTS_LDS", "LDS M", 1e6), ("SQ_INSTS_VMEM_RD", "VMEM M", 1e6))
    lines = ["# PMC counters per call and per kernel, 2M lognormal step (benchmark configuration)",
             f"# {res['command']}",
             f"# copy-kernel calibration: FETCH_SIZE x {res['copy_factor_fetch']:.4f}, "
             f"WRITE_SIZE x {res['copy_factor_write']:.4f} -> bytes",
             "# values are per dispatch (per call for the calls), averaged over the dispatches "
             "of the runs", "",
             f"{'call/kernel':30s} " + " ".join(f"{h:>9s}" for _, h, _ in cols)]
    rows = [(f"call {k}", v) for k, v in res["calls"].items()]
    rows += sorted(res["kernels"].items(), key=lambda kv: -kv[1].get("hbm_bytes", 0.0))
    for name, v in rows:
        if v.get("hbm_bytes", 0.0) < 1e7 and not name.startswith("call"):
            continue
        lines.append(f"{name[:30]:30s} " + " ".join(
            f"{v.get(c, 0.0) / sc:9.3f}" if c in ("hbm_bytes", "l2_hit_rate")
            else f"{v.get(c, 0.0) / sc:9.1f}" for c, _, sc in cols))
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("out")
    p.add_argument("--cmd", required=True)
    p.add_argument("--calib-fetch", required=True)
    p.add_argument("--calib-write", required=True)
    p.add_argument("runs", nargs="+")
    a = ap.parse_args()
    if a.what == "trace":
        print(trace(a.db, a.out, a.cmd))
    else:
        print(json.dumps(pmc(a.out, a.cmd, a.calib_fetch, a.calib_write, a.runs), indent=1))


if __name__ == "__main__":
    main()
