"""HBM traffic of the benchmark's dominant kernel from two rocprofv3 counter runs, and the kernel
time summary of a rocprofv3 kernel trace.

    cd /tmp && export TMPDIR=/tmp   # (R: the repository root, OUT: any output folder)
    rocprofv3 --pmc FETCH_SIZE -d $OUT/pmc_fetch -o f -- \\
        python3 -u $R/bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-secondary --calibrate
    rocprofv3 --pmc WRITE_SIZE -d $OUT/pmc_write -o w -- \\
        python3 -u $R/bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-secondary --calibrate
    python3 $R/traffic.py --fetch $OUT/pmc_fetch --write $OUT/pmc_write

`--calibrate` makes the benchmark first copy 1 GiB with the library's plain copy kernel; the ratio
of 1 GiB to what each counter reads for that copy scales the counter values of the other kernels
(FETCH_SIZE and WRITE_SIZE count in KiB per dispatch).  The result goes to profiles/traffic.json
together with the hash of the kernel sources it was taken on; bench.py reports it only while that
hash matches.

    rocprofv3 --kernel-trace --stats -d $OUT/prof_step -o step -- \
        python3 -u $R/bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-secondary
    python3 $R/traffic.py --trace $OUT/prof_step > profiles/step256_fp64_kernel_trace.md

prints per-kernel launch counts and durations, and for the dominant kernel the average launch
duration over one step's launch mix (the figure bench.py measures with HIP events).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GIB = float(1 << 30)
# The kernels that can dominate the 256^3 FP64 step: their HIP symbols and how one step's launches
# are averaged.  conv_z_fused runs over 3 components once (Vor2Vel) and over 1 component three times
# (pressure); its dispatches are grouped by grid size (a launch over c components has c times the
# grid) and weighted by that mix.  if_xy runs four different launches per step (and nowhere else), so
# its dispatches are averaged as they come.
KERNELS = {"conv_z_fused": "nslgf::k_col<double, 512, 2, 2,", "if_xy": "nslgf::k_if_xy<double,"}
STEP_MIX = {"conv_z_fused": {3: 1, 1: 3}, "if_xy": None}


def step_average(key, grids_values):
    """(average per launch over one step, details) from [(grid size, value)] of one kernel."""
    mix = STEP_MIX[key]
    if mix is None:
        vals = [v for _, v in grids_values]
        return sum(vals) / len(vals), {"launches": len(vals)}
    groups = collections.defaultdict(list)
    for g, v in grids_values:
        groups[g].append(v)
    g1 = min(groups)
    by_comp = {g // g1: sum(v) / len(v) for g, v in groups.items()}
    if not all(c in by_comp for c in mix):
        raise SystemExit(f"{key}: launches over {sorted(by_comp)} components, expected {sorted(mix)}")
    avg = sum(mix[c] * by_comp[c] for c in mix) / sum(mix.values())
    return avg, {"by_components": {str(c): by_comp[c] for c in sorted(by_comp)},
                 "launches_by_components": {str(c): len(groups[c * g1]) for c in sorted(by_comp)},
                 "step_mix_components": {str(c): m for c, m in mix.items()}}


def per_dispatch(run_dir: str, counter: str):
    """{dispatch: (kernel name, grid size, value)} of one counter from a rocprofv3 --pmc output folder
    (the rocpd SQLite database, or counter_collection.csv files)."""
    vals = collections.OrderedDict()

    def add(key, name, grid, v):
        old = vals.get(key, (name, int(grid), 0.0))
        vals[key] = (old[0], old[1], old[2] + float(v))

    for f in glob.glob(os.path.join(run_dir, "**", "*_results.db"), recursive=True):
        con = sqlite3.connect(f)
        for did, name, grid, v in con.execute(
                "select dispatch_id, kernel_name, grid_size, value from counters_collection where counter_name = ?",
                (counter,)):
            add((f, did), name, grid, v)
        con.close()
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    add((f, r["Dispatch_Id"]), r["Kernel_Name"], r["Grid_Size"], r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} values under {run_dir}")
    return vals


def summarize(run_dir: str, counter: str):
    """Calibration factor, and per kernel the counter in bytes per launch averaged over one step's
    launch mix (dispatches grouped by grid size: a launch over c components has c times the grid)."""
    vals = per_dispatch(run_dir, counter)
    copies = [v for name, _, v in vals.values() if "k_copy" in name]
    if not copies:
        raise SystemExit(f"{run_dir}: no calibration copy (run bench.py with --calibrate)")
    factor = GIB / (max(copies) * 1024.0)
    out = {}
    for key, sym in KERNELS.items():
        gv = [(grid, v * 1024.0 * factor) for name, grid, v in vals.values() if sym in name]
        if not gv:
            continue
        avg, det = step_average(key, gv)
        out[key] = {"dispatches": len(gv), "bytes_avg": avg, "detail": det}
    return factor, out


def trace_summary(run_dir: str, last: int) -> str:
    """Markdown summary of a rocprofv3 --kernel-trace database; the dominant kernel's launch-mix
    average is taken over its last `last` launches (the timed steps)."""
    dbs = glob.glob(os.path.join(run_dir, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no *_results.db under {run_dir}")
    rows = []
    for f in dbs:
        con = sqlite3.connect(f)
        rows += con.execute("select name, duration, grid_x * grid_y * grid_z, dispatch_id from kernels "
                            "order by dispatch_id").fetchall()
        con.close()
    per = collections.defaultdict(list)
    for name, dur, grid, _ in rows:
        per[name].append((float(dur), int(grid)))
    total = sum(d for v in per.values() for d, _ in v)
    out = ["| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(d for d, _ in kv[1])):
        t = sum(d for d, _ in v)
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {len(v)} | {t / 1e6:.3f} | {t / len(v) / 1e6:.4f} | {100 * t / total:.1f} |")
    for key, sym in KERNELS.items():
        mine = [(g, d) for name, v in per.items() if sym in name for d, g in v]
        if not mine:
            continue
        avg, det = step_average(key, mine[-last:])
        parts = ""
        if "by_components" in det:
            parts = ", ".join(f"{c} component(s): {t / 1e6:.4f} ms ({det['launches_by_components'][c]} launches)"
                              for c, t in det["by_components"].items()) + "; "
        out.append("")
        out.append(f"`{key}` (`{sym}`), last {last} launches (the timed steps): {parts}"
                   f"average over one step's launches: {avg / 1e6:.4f} ms per launch.")
    return "\n".join(out)


def surrogate_summary(run_dir: str, n: int, iters: int) -> str:
    """Markdown per-layer summary of the surrogate's convolutions from a rocprofv3 --kernel-trace of
    `python -m paper_1601_00035_amd.surrogate_run --time-iters K --n n`: the last `iters` training
    iterations, each layer's forward, data-gradient and weight-gradient launches (the weight gradient
    with its layout copies and chunk sums), against the layer's roofline max(FLOP / 2.5 PFLOP/s BF16
    dense, algorithmic bytes / 8 TB/s)."""
    from paper_1601_00035_amd.surrogate import LAYERS, LEVEL

    dbs = glob.glob(os.path.join(run_dir, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no *_results.db under {run_dir}")
    rows = []
    for f in dbs:
        con = sqlite3.connect(f)
        rows += con.execute("select name, duration from kernels order by dispatch_id").fetchall()
        con.close()

    def kind(name):
        short = name.split("(")[0]
        if "k_conv_lds<" in short or "k_conv_mfma<" in short:
            return "dgrad" if short.rstrip(">").endswith("-1") else "fwd"
        if "k_conv_wgrad" in short:
            return "wgrad"
        if "k_to_blocked8" in short:
            return "pre"
        if "k_sum_chunk" in short:
            return "post"
        return None

    # training iterations: 10 forward convolutions, then the weight gradients 9 .. 0 and data gradients
    # 9 .. 1 interleaved; walk the dispatches, attributing the layout copies to the next weight gradient
    # and the chunk sums to the previous one
    seq, pre = [], 0.0
    for name, dur in rows:
        k = kind(name)
        if k in ("fwd", "dgrad"):
            seq.append([k, float(dur)])
        elif k == "pre":
            pre += float(dur)
        elif k == "wgrad":
            seq.append(["wgrad", float(dur) + pre])
            pre = 0.0
        elif k == "post" and seq and seq[-1][0] == "wgrad":
            seq[-1][1] += float(dur)
    per_iter = 10 + 9 + 10
    seq = seq[-iters * per_iter:]
    if len(seq) < iters * per_iter:
        raise SystemExit("fewer convolution launches than the iterations need")
    order = [("fwd", li) for li in range(10)]
    for li in range(9, -1, -1):
        order.append(("wgrad", li))
        if li >= 1:
            order.append(("dgrad", li))
    times = collections.defaultdict(list)
    for i in range(iters):
        chunk = seq[i * per_iter:(i + 1) * per_iter]
        for (k, li), (k2, d) in zip(order, chunk):
            if k != k2:
                raise SystemExit(f"launch order differs from a training iteration: {k} vs {k2}")
            times[(k, li)].append(d)
    out = ["| layer | grid | cin -> cout | op | avg us | TFLOP/s | GB/s | roofline us (bound) | frac |",
           "|---:|---:|---|---|---:|---:|---:|---:|---:|"]
    total = 0.0
    for li, (ci, co) in enumerate(LAYERS):
        r = n >> LEVEL[li]
        nv = r ** 3
        flop = 2.0 * nv * 27 * ci * co
        for k in ("fwd", "dgrad", "wgrad"):
            if (k, li) not in times:
                continue
            t = sum(times[(k, li)]) / len(times[(k, li)]) / 1e3  # us
            total += t
            if k == "fwd":
                byt = nv * ci * 2 + nv * co * 4 + 27 * ci * co * 2
            elif k == "dgrad":
                byt = nv * co * 2 + nv * ci * 4 + 27 * ci * co * 2
            else:
                byt = nv * (ci + co) * 2 + 27 * ci * co * 4
            tm, tb = flop / 2.5e15 * 1e6, byt / 8e12 * 1e6
            roof = max(tm, tb)
            out.append(f"| {li} | {r}^3 | {ci} -> {co} | {k} | {t:.1f} | {flop / t / 1e6:.0f} | {byt / t / 1e3:.0f} | "
                       f"{roof:.1f} ({'mfma' if tm >= tb else 'hbm'}) | {roof / t:.2f} |")
    out.append("")
    out.append(f"Convolutions: {total / 1e3:.3f} ms of each training iteration (average of the last {iters}).")
    return "\n".join(out)


def sq_summary(run_dirs: list) -> str:
    """Markdown summary of SQ counter runs (rocprofv3 --pmc over the benchmark) for the dominant
    kernels: per launch (dispatches grouped like the traffic figures) the raw counters and the derived
    rates of rocprofv3's own definitions (GRBM_GUI_ACTIVE summed over the 8 XCDs, so one XCD's clock
    is a eighth of it; 256 CUs, 32 wave slots per CU)."""
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    meta = {}
    for d in run_dirs:
        for f in glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True):
            con = sqlite3.connect(f)
            for did, name, grid, c, v in con.execute(
                    "select dispatch_id, kernel_name, grid_size, counter_name, value from counters_collection"):
                vals[(name, grid, f, did)][c] += float(v)
                meta[(name, grid, f, did)] = (name, int(grid))
            con.close()
    out = []
    for key, sym in KERNELS.items():
        groups = collections.defaultdict(list)
        for k, cv in vals.items():
            if sym in k[0]:
                # conv_z_fused: by grid (components); others: by instantiation and grid
                gk = k[1] if key == "conv_z_fused" else (k[0].split("(")[0].replace("void ", ""), k[1])
                groups[gk].append(cv)
        if not groups:
            continue
        g1 = min(groups) if key == "conv_z_fused" else None
        out.append(f"### `{key}` (`{sym}`)")
        out.append("")
        out.append("| launch | n | waves | VALU instr / wave | LDS instr / wave | occupancy % | VALU busy % | "
                   "LDS active % | LDS bank-conflict % | XCD clock us |")
        out.append("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
        for grid in sorted(groups):
            runs = groups[grid]
            avg = collections.defaultdict(float)
            cnt = collections.Counter()
            for cv in runs:
                for c, v in cv.items():
                    avg[c] += v
                    cnt[c] += 1
            a = {c: avg[c] / cnt[c] for c in avg}
            gclk = a.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
            waves = a.get("SQ_WAVES", float("nan"))

            def pct(c, scale):
                return f"{100.0 * a[c] / scale:.1f}" if c in a and scale else "-"

            label = f"{grid // g1} component(s)" if key == "conv_z_fused" else f"`{grid[0]}`, grid {grid[1]}"
            vi = f"{a['SQ_INSTS_VALU'] / waves:.0f}" if "SQ_INSTS_VALU" in a and waves == waves else "-"
            li = f"{a['SQ_INSTS_LDS'] / waves:.0f}" if "SQ_INSTS_LDS" in a and waves == waves else "-"
            occ = f"{400.0 * a['SQ_WAVE_CYCLES'] / gclk / 256 / 32:.1f}" if "SQ_WAVE_CYCLES" in a and gclk else "-"
            out.append(f"| {label} | {len(runs)} | {waves:.0f} | {vi} | {li} | {occ} | "
                       f"{pct('SQ_ACTIVE_INST_VALU', gclk * 256)} | {pct('SQ_ACTIVE_INST_LDS', gclk * 256)} | "
                       f"{pct('SQ_LDS_BANK_CONFLICT', gclk * 256)} | {gclk / 2.4e3:.1f} |")
        out.append("")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--trace", help="rocprofv3 --kernel-trace output folder: print the time summary instead")
    ap.add_argument("--surrogate-trace", help="rocprofv3 --kernel-trace folder of surrogate_run --time-iters: "
                                              "print the per-layer summary")
    ap.add_argument("--sq", nargs="+", help="rocprofv3 --pmc folders of SQ counter runs over the benchmark: print "
                                            "the counter summary of the dominant kernels")
    ap.add_argument("--n", type=int, default=128, help="grid of the surrogate run")
    ap.add_argument("--iters", type=int, default=3, help="timed iterations of the surrogate run")
    ap.add_argument("--last", type=int, default=12, help="launches of the dominant kernel in the timed steps")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    a = ap.parse_args()
    if a.trace:
        print(trace_summary(a.trace, a.last))
        return
    if a.sq:
        print(sq_summary(a.sq))
        return
    if a.surrogate_trace:
        print(surrogate_summary(a.surrogate_trace, a.n, a.iters))
        return
    if not (a.fetch and a.write):
        ap.error("--fetch and --write are required without --trace")
    import bench

    ff, fk = summarize(a.fetch, "FETCH_SIZE")
    wf, wk = summarize(a.write, "WRITE_SIZE")
    kernels = {}
    for key in KERNELS:
        if key in fk and key in wk:
            kernels[key] = {"bytes_per_launch": int(fk[key]["bytes_avg"] + wk[key]["bytes_avg"]),
                            "read_bytes_per_launch": int(fk[key]["bytes_avg"]),
                            "write_bytes_per_launch": int(wk[key]["bytes_avg"]),
                            "read_detail": fk[key]["detail"], "write_detail": wk[key]["detail"],
                            "dispatches": fk[key]["dispatches"]}
    rec = {"workload": "ns_lgf_step_256_ring_fp64", "source_hash": bench.kernel_source_hash(),
           "calibration": {"FETCH_SIZE_factor": round(ff, 4), "WRITE_SIZE_factor": round(wf, 4),
                           "copy_bytes": int(GIB)},
           "kernels": kernels,
           "command": ["rocprofv3 --pmc FETCH_SIZE -- python3 -u bench.py --steps 2 --warmup 1 --no-cpu-baseline "
                       "--no-secondary --calibrate",
                       "rocprofv3 --pmc WRITE_SIZE -- python3 -u bench.py --steps 2 --warmup 1 --no-cpu-baseline "
                       "--no-secondary --calibrate"]}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
