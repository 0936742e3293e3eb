#!/usr/bin/env python3
"""Benchmark of the fast-LGF Navier-Stokes hot path on one MI355X.

Workload: the vortex ring of the 256^3 LGF-solve case (R = 1, sigma = 0.1 R, dx = R/48, Gamma = 1,
Re = 500, CFL 0.5), FP64.  One timed step is one pass of the whole hot path:
  Vor2Vel (the three-component LGF solve of the edge vorticity, then Cbar) followed by one
  Scheme A IF-HERK step (three scalar LGF pressure solves, five vector integrating factors, three
  nonlinear terms, divergence, gradient and bookkeeping).
The LGF spectrum is built once before timing (preprocessing).  `value` is the LGF-solve throughput
of the step: 6 scalar 256^3 solves per step, in points per second.

Also reported (outside the timed steps): the three-component LGF solve alone in FP64 and FP32 with
the FP32 error against FP64, per-kernel event times with algorithmic bytes, the roofline of the
dominant kernel, and the oracle (plain C direct lattice sum) timed on a bounded sample of the same
solve on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_per_step(N: int, P: int, es: int) -> dict:
    """Algorithmic HBM bytes per timed step for each kernel name (FP64 es = 8): every kernel counted
    as reading its inputs once and writing its outputs once."""
    n3 = N ** 3
    nh = P // 2 + 1
    ce = 2 * es
    C = 6  # scalar LGF solves per step: 3 (Vor2Vel) + 3 (pressure)
    CL = 4  # convolution launches per step (one of three components, three of one); the spectrum is read once per launch
    return {
        # the three pressure solves read their source as the divergence of r (3 fields) in this pass
        "conv_x_r2c": C * (n3 * es + N * N * nh * ce) + 3 * 2 * n3 * es,
        "conv_y_fwd": C * (N * N * nh * ce + N * P * nh * ce),
        "conv_z_fused": C * 2 * N * P * nh * ce + CL * nh ** 3 * es,
        "conv_y_inv": C * (N * P * nh * ce + N * N * nh * ce),
        "conv_x_c2r": C * (N * N * nh * ce + n3 * es),
        # 15 component-applications of the IF (fused x-y pass, then z pass); the x-y pass of the last
        # stage also reads w^{2,1} and w^{2,2}, those of stages 1 and 2 project on the way (reading
        # dhat per component, q, and w^{2,1} in stage 2; writing w^{1,1} and w^{2,2})
        "if_xy": (15 * 2 + 6 + 9 + 12) * n3 * es,
        "if_z": 15 * 2 * n3 * es,
        "curl_bar": 6 * n3 * es,
        "stage_rhs": 30 * n3 * es,
        "stage_project": 7 * n3 * es,  # the last stage only (H^3 = I): reads r, dhat, writes u
        "axpby": 2 * n3 * es,
    }


def kernel_source_hash() -> str:
    """Hash of the sources of the LGF path's kernels (every HIP source and header of the library but
    the surrogate's, which holds none of them): counter figures taken on other sources are not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1601_00035_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")) and f != "surrogate.hip":
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(w, dx, seconds: float):
    """The oracle's direct lattice sum on a bounded sample of target points of the same solve."""
    import numpy as np

    import workloads
    from oracle import lgf as olgf
    from oracle import native

    n = w.shape[-1]
    t0 = time.perf_counter()
    olgf.lgf_cube(n - 1)
    table_s = time.perf_counter() - t0
    native.load()
    comps = [q for q in range(3) if w[q].any()]
    # grow the sample until it takes about `seconds` (each call also scans the source box once)
    count = 64
    while True:
        tg = workloads.sample_targets(n, count, seed=12)
        t0 = time.perf_counter()
        for q in comps:
            native.lgf_direct_targets(w[q], dx, tg)
        el = time.perf_counter() - t0
        if el >= 0.5 * seconds or count >= 200000:
            break
        count = int(count * min(8.0, max(1.5, seconds / max(el, 1e-3))))
    pts = len(tg) * len(comps)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": pts / el / 1e6,
        "unit": "Mpts/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{len(tg)} seeded target points x {len(comps)} nonzero vorticity components of the 256^3 "
                  f"LGF solve, direct O(N_src N_tgt) sum in FP64 ({el:.1f} s; table build {table_s:.1f} s not included)",
    }


def cpu_oracle_sizes(nslgf, torch, cores: int):
    """The oracle's direct sum against the GPU convolution on the compact random source (radius 12 n / 32
    cells, seed 0) at 32^3 and 64^3 (full grids) and 128^3 (a seeded sample of 4096 targets, the full
    time extrapolated and labelled so), on all host threads and, at 32^3, on one thread."""
    import ctypes

    import numpy as np

    import workloads
    from oracle import native

    native.load()
    out = {"cores": cores}
    for n in (32, 64, 128):
        s = workloads.compact_random_source(n, 12.0 * n / 32, seed=0)
        t = torch.from_numpy(s).to("cuda:0")
        y = nslgf.lgf_convolve(t, 1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            nslgf.lgf_convolve(t, 1.0, y)
        e1.record()
        torch.cuda.synchronize()
        gpu_ms = e0.elapsed_time(e1) / 10
        rec = {"sources": int(np.count_nonzero(s)), "gpu_ms": round(gpu_ms, 4)}
        if n <= 64:
            t0 = time.perf_counter()
            native.lgf_direct(s, 1.0)
            el = time.perf_counter() - t0
            rec.update({"oracle_s": round(el, 3), "oracle_full": True})
        else:
            tg = workloads.sample_targets(n, 4096, seed=12)
            t0 = time.perf_counter()
            native.lgf_direct_targets(s, 1.0, tg)
            el = time.perf_counter() - t0
            rec.update({"oracle_s": round(el * n ** 3 / len(tg), 1), "oracle_full": False,
                        "oracle_sample": f"{len(tg)} targets in {el:.2f} s, full grid extrapolated"})
        rec["gpu_speedup"] = round(rec["oracle_s"] * 1e3 / gpu_ms, 1)
        out[f"{n}^3"] = rec
    # one thread (the OpenMP runtime the oracle's library uses), 32^3 full
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        s = workloads.compact_random_source(32, 12.0, seed=0)
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        native.lgf_direct(s, 1.0)
        out["32^3_one_thread_s"] = round(time.perf_counter() - t0, 3)
        gomp.omp_set_num_threads(cores)
    except OSError:
        out["32^3_one_thread_s"] = None
    return out


def batched_measure(nslgf, torch, dtype, reps=3, sizes=None):
    """32 uneven Scheme A steps (n ~ U{48..192}, seeded rings): the same steps issued one state after
    another on one stream, against one captured graph per batch in both of its forms (batched passes: one
    launch per kernel over every group of equal boxes; per problem: each problem on a branch stream)."""
    import workloads

    dev = torch.device("cuda:0")
    specs = workloads.batch_specs(32, seed=0, sizes=sizes)
    solo, batch = [], []
    cells = 0
    for (n, dx, ring, re, cfl) in specs:
        w = torch.from_numpy(workloads.ring_edge_vorticity(n, dx, ring, quad=2)).to(dev)
        u = nslgf.vor2vel(w, dx)
        dt = cfl * dx / nslgf.max_cell_speed(u)
        u = u.to(dtype)
        a = nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=8)
        b = nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=8)
        b.work = a.work  # the two sets never run at the same time
        b.c.work = a.work.data_ptr()
        solo.append(a)
        batch.append(b)
        cells += n ** 3
        del w
    stream = torch.cuda.current_stream()
    # correctness: one step each way from identical states, per form of the batch graph
    modes = (("per_problem", nslgf.BATCH_PER_PROBLEM), ("batched_passes", nslgf.BATCH_PASSES))
    equal, info = {}, {}
    for name, mode in modes:
        for a, b in zip(solo, batch):
            b.u.copy_(a.u)
            b.c.t = a.c.t
        nslgf.set_batch_mode(mode)
        for st in solo:
            st.step()
        nslgf.herk_step_batched(batch)
        torch.cuda.synchronize()
        equal[name] = all(torch.equal(a.u, b.u) and torch.equal(a.d, b.d) for a, b in zip(solo, batch))
        info[name] = nslgf.batch_info()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_solo = timed(lambda: [st.step() for st in solo])
    ms = {}
    for name, mode in modes:
        nslgf.set_batch_mode(mode)
        nslgf.herk_step_batched(batch)  # (captures the form's graph)
        ms[name] = timed(lambda: nslgf.herk_step_batched(batch))
    nslgf.set_batch_mode(nslgf.BATCH_PASSES)
    best = min(ms, key=ms.get)
    sizes = sorted(set(sp[0] for sp in specs))
    return {"problems": len(specs), "sizes": sizes, "cells": cells, "ms_one_by_one": round(ms_solo, 3),
            "ms_graph_per_problem": round(ms["per_problem"], 3),
            "ms_graph_batched_passes": round(ms["batched_passes"], 3),
            "batched_passes_groups_launches": list(info["batched_passes"]),
            "speedup_best_vs_one_by_one": round(ms_solo / ms[best], 3), "best_form": best,
            "Mcells_per_s": round(cells / (ms[best] * 1e-3) / 1e6, 1),
            "bitwise_equal_to_one_by_one": equal}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--fft-plan", type=int, default=-1, choices=(-1, 0, 1, 2),
                    help="column-pass FFT radix plan: -1 default, 0 narrow, 1 wide, 2 narrow on fewer elements")
    ap.add_argument("--calibrate", action="store_true",
                    help="first copy 1 GiB with the library's plain copy kernel (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 (multi-GPU sharding is design-only)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1601_00035_amd as nslgf
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nslgf.set_fft_plan(args.fft_plan)
    if args.calibrate:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        nslgf.copy(a, b)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 1 GiB read + 1 GiB written")
    n, dx, ring, re, cfl = workloads.ring_case("conv256")
    t0 = time.perf_counter()
    w_np = workloads.ring_edge_vorticity(n, dx, ring)
    log(f"input: ring vorticity {n}^3 generated in {time.perf_counter() - t0:.1f} s")
    w = torch.from_numpy(w_np).to(dev)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    nslgf.lgf_table(n, n, n, torch.float64)
    torch.cuda.synchronize()
    table_s = time.perf_counter() - t0
    log(f"LGF table + spectrum (FP64) built in {table_s:.2f} s")

    u = nslgf.vor2vel(w, dx)
    dt = cfl * dx / nslgf.max_cell_speed(u)
    st = nslgf.HerkState(u, dx, dt, re, "A", n_buf=16)

    def step():
        nslgf.vor2vel(w, dx, out=u)
        st.step()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done (dt = {dt:.4e})")

    # headline: K steps with no per-kernel events, bracketed by synchronisation
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    assert torch.isfinite(u).all().item(), "non-finite velocity"
    log(f"timed {args.steps} steps: {ms:.3f} ms/step (wall {wall:.2f} s)")
    # per-kernel durations: the same K steps again with HIP events around every launch, recorded on the
    # stream each kernel is launched on (the library's profiler)
    nslgf.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = nslgf.profile_read()
    nslgf.profile_enable(False)

    N, P = n, 512
    lgf_pts = 6 * N ** 3
    value = lgf_pts / (ms * 1e-3) / 1e6

    # per-kernel achieved bandwidth from the event timings and the algorithmic bytes
    alg = alg_bytes_per_step(N, P, 8)
    kern = {}
    for name, (calls, tot) in prof.items():
        per_step_ms = tot / args.steps
        b = alg.get(name)
        kern[name] = {"launches_per_step": calls / args.steps, "ms_per_step": round(per_step_ms, 4)}
        if b is not None and tot > 0:
            kern[name]["alg_GBps"] = round(b / (per_step_ms * 1e-3) / 1e9, 1)
    dom = max((k for k in prof if k in alg), key=lambda k: prof[k][1])
    calls, tot = prof[dom]
    launches = calls / args.steps
    avg_ms = tot / calls
    bytes_per_launch = alg[dom] / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    workload = "ns_lgf_step_256_ring_fp64"
    traffic = load_traffic(dom, workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_ms, 5)}

    secondary = {}
    if not args.no_secondary:
        # the three-component LGF solve alone, FP64 and FP32, with the FP32 error against FP64
        def time_conv(src, reps=10):
            out = nslgf.lgf_convolve(src, dx)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                nslgf.lgf_convolve(src, dx, out=out)
            b.record(stream)
            torch.cuda.synchronize()
            return out, a.elapsed_time(b) / reps

        y64, ms64 = time_conv(w)
        w32 = w.float()
        nslgf.lgf_table(n, n, n, torch.float32)
        y32, ms32 = time_conv(w32)
        d = (y32.double() - y64)
        rel_l2 = (d.norm() / y64.norm()).item()
        rel_linf = (d.abs().max() / y64.abs().max()).item()
        def solve_bytes(es):
            # algorithmic bytes of one three-component solve: the five passes per component, the
            # spectrum once
            nh, ce, n3 = P // 2 + 1, 2 * es, N ** 3
            per_comp = 2 * (n3 * es + N * N * nh * ce) + 2 * (N * N * nh * ce + N * P * nh * ce)
            per_comp += 2 * N * P * nh * ce
            return 3 * per_comp + nh ** 3 * es

        def rate(ms, es):
            gbs = solve_bytes(es) / (ms * 1e-3) / 1e9
            return {"alg_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}

        secondary["lgf_solve_3comp"] = {
            "fp64": {"ms": round(ms64, 4), "Mpts_per_s": round(3 * N ** 3 / (ms64 * 1e-3) / 1e6, 1), **rate(ms64, 8)},
            "fp32": {"ms": round(ms32, 4), "Mpts_per_s": round(3 * N ** 3 / (ms32 * 1e-3) / 1e6, 1), **rate(ms32, 4),
                     "rel_l2_vs_fp64": rel_l2, "rel_linf_vs_fp64": rel_linf},
        }
        del w32, y32, y64
        torch.cuda.empty_cache()
        # the whole step in FP32 (Vor2Vel + IF-HERK step from the same start as an FP64 step), its
        # time and its deviation from the FP64 step
        u0 = nslgf.vor2vel(w, dx)
        s64 = nslgf.HerkState(u0.clone(), dx, dt, re, "A", n_buf=16)
        s64.step()
        w32 = w.float()
        s32 = nslgf.HerkState(u0.float(), dx, dt, re, "A", n_buf=16)
        s32.step()
        diff = (s32.u.double() - s64.u)
        step_err = {"rel_l2_vs_fp64": float(diff.norm() / s64.u.norm()),
                    "rel_linf_vs_fp64": float(diff.abs().max() / s64.u.abs().max())}
        # the projection's divergence check, in FP64 for both forms (guarded steps from the same start)
        div = {}
        for name, dtp in (("fp64", torch.float64), ("fp32", torch.float32)):
            sg = nslgf.HerkState(u0.to(dtp).clone(), dx, dt, re, "A", n_buf=16, guard=True)
            sg.step()
            div[name] = sg.div_max * dx / float(u0.abs().max())
        step_err["fp64_divergence_check"] = {"max_abs_Dbar_u_times_dx_over_umax": div,
                                             "cells": "at least n_buf + r_i + 1 from every face, every stage"}
        # cost of the guard: FP64 steps (no Vor2Vel) with and without it, from the same state
        def steps_ms(guard):
            st = nslgf.HerkState(u0.clone(), dx, dt, re, "A", n_buf=16, guard=guard)
            st.step()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(5):
                st.step()
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / 5

        step_err["fp64_divergence_check"]["fp64_step_ms"] = {"plain": round(steps_ms(False), 4),
                                                             "guarded": round(steps_ms(True), 4)}

        def step32():
            nslgf.vor2vel(w32, dx, out=s32.u)
            s32.step()

        step32()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            step32()
        e1.record(stream)
        torch.cuda.synchronize()
        ms32s = e0.elapsed_time(e1) / 5
        secondary["step_fp32"] = {"ms_per_step": round(ms32s, 4),
                                  "Mpts_per_s": round(6 * N ** 3 / (ms32s * 1e-3) / 1e6, 1),
                                  "speedup_vs_fp64": round(ms / ms32s, 3), **step_err}
        del u0, s64, s32, w32, diff
        torch.cuda.empty_cache()
        # velocity refresh (Sec. 4.4) at 256^3 FP64 and its cadence for this step (Appendix D estimate)
        ur = u.clone()
        nslgf.velocity_refresh(ur, dx, 16)
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        r0.record(stream)
        for _ in range(5):
            nslgf.velocity_refresh(ur, dx, 16)
        r1.record(stream)
        torch.cuda.synchronize()
        ms_ref = r0.elapsed_time(r1) / 5
        umax = nslgf.max_component_abs(u, 16)
        beta = dt / (dx * dx * re)
        cadence = {}
        for rel_eps in (1e-10, 1e-8, 1e-6):
            q = nslgf.refresh_interval(beta, 16, umax, rel_eps * umax)
            cadence[f"{rel_eps:g}"] = {"q_max": q, "refresh_ms_per_step": round(ms_ref / q, 4) if q else None}
        secondary["velocity_refresh"] = {"ms": round(ms_ref, 4), "n_buf": 16, "beta": beta, "umax": umax,
                                         "cadence_by_eps_over_umax": cadence}
        del ur
        torch.cuda.empty_cache()
        # vortex-ring integrals (Sec. 6.2) and the ring speed over the first step against Saffman's
        # thin-ring formula (Sec. 6.3): U = Gamma / (4 pi R) (log(8 R / sigma) - beta_0)
        origin = (-(n - 1) / 2.0 * dx,) * 3
        ud = nslgf.vor2vel(w, dx)
        d0 = nslgf.flow_diagnostics(ud, dx, origin, 16)
        sd = nslgf.HerkState(ud, dx, dt, re, "A", n_buf=16)
        sd.step()
        d1 = nslgf.flow_diagnostics(ud, dx, origin, 16)
        t0 = time.perf_counter()
        for _ in range(5):
            nslgf.flow_diagnostics(ud, dx, origin, 16)
        ms_diag = (time.perf_counter() - t0) / 5 * 1e3
        uz = (d1["X"][2] - d0["X"][2]) / dt
        beta0 = 0.5 * (1.0 - 0.5772156649015329 + math.log(2.0))
        us = ring.gamma / (4 * math.pi * ring.R) * (math.log(8 * ring.R / ring.sigma) - beta0)
        secondary["ring_diagnostics"] = {"ms_incl_sync": round(ms_diag, 4), "I_z": d0["I"][2], "K": d0["K"],
                                         "E": d0["E"], "J": d0["J"], "U_z_first_step": uz, "U_saffman": us,
                                         "rel_diff": (uz - us) / us,
                                         "I_z_change_first_step": d1["I"][2] / d0["I"][2] - 1}
        del ud, sd
        torch.cuda.empty_cache()
        # active-domain block weights (Sec. 4.3) of the 256^3 ring: how much of the box the support,
        # solution and expanded-solution blocks keep (blocks of 16^3 cells, one buffer block)
        mu, nu = nslgf.block_weights(u, dx, 16, 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            nslgf.block_weights(u, dx, 16, 16)
        ms_bw = (time.perf_counter() - t0) / 5 * 1e3
        frac = {}
        for eps in (1e-2, 1e-4, 1e-6):
            _, sp, so, xs = nslgf.classify_blocks(mu, nu, eps, eps, 1)
            frac[f"{eps:g}"] = {"supp": round(float(sp.mean()), 4), "xsoln": round(float(xs.mean()), 4)}
        # steps on that active domain, re-classified every step with re-initialisation on a change
        # (Sec. 4.3), against plain steps of the same state
        ua = u.clone()
        sa = nslgf.HerkState(ua, dx, dt, re, "A", n_buf=16)
        sa.run_adaptive(1, 16, 1e-6, 1e-3, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nre, nedge = sa.run_adaptive(3, 16, 1e-6, 1e-3, 1)
        torch.cuda.synchronize()
        ms_ad = (time.perf_counter() - t0) / 3 * 1e3
        sp = nslgf.HerkState(ua.clone(), dx, dt, re, "A", n_buf=16)
        sp.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            sp.step()
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) / 3 * 1e3
        secondary["active_domain"] = {"block": 16, "blocks": int(mu.size), "ms_incl_sync": round(ms_bw, 4),
                                      "fraction_of_box_by_eps": frac,
                                      "adaptive_steps": {"eps_supp": 1e-6, "eps_soln": 1e-3, "n_xb": 1, "steps": 3,
                                                         "ms_per_step": round(ms_ad, 4), "reinits": nre,
                                                         "edge_steps": nedge,
                                                         "plain_step_ms": round(ms_plain, 4)}}
        del ua, sa, sp
        torch.cuda.empty_cache()
        # steps on an active box that follows the flow (the bounding box of the expanded solution domain,
        # Sec. 4.2, 4.3 and the grid update of Sec. 5), 20 steps in one call, against 20 plain steps:
        # time per step (block weights and their host round trip included) and the difference on the
        # box less its outer block layer
        nact = 20
        uref = u.clone()
        sref = nslgf.HerkState(uref, dx, dt, re, "A", n_buf=16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nact):
            sref.step()
        torch.cuda.synchronize()
        ms_ref = (time.perf_counter() - t0) / nact * 1e3
        active = {"block": 16, "n_xb": 1, "steps": nact, "plain_step_ms": round(ms_ref, 4), "by_eps": {}}
        for es, eo in ((1e-8, 1e-3), (1e-6, 1e-3), (1e-4, 1e-3)):
            for rep in range(2):  # the first run builds the plans of the boxes it meets
                ub = u.clone()
                sb = nslgf.HerkState(ub, dx, dt, re, "A", n_buf=16)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                nre, nrg, org, size = sb.run_active(nact, 16, es, eo, 1)
                torch.cuda.synchronize()
                ms_b = (time.perf_counter() - t0) / nact * 1e3
            inner = (slice(None),) + tuple(slice(o + 16, o + n_ - 16) for o, n_ in zip(reversed(org), reversed(size)))
            err = float((ub - uref)[inner].abs().max() / uref.abs().max())
            active["by_eps"][f"{es:g}"] = {"eps_soln": eo, "ms_per_step": round(ms_b, 4),
                                           "speedup_vs_plain": round(ms_ref / ms_b, 3), "reinits": nre,
                                           "box_changes": nrg, "box_first_cell_xyz": list(org),
                                           "box_size_xyz": list(size),
                                           "box_fraction_of_grid": round(size[0] * size[1] * size[2] / N ** 3, 4),
                                           "rel_diff_vs_plain_on_box_less_one_block": err}
            del ub, sb
        secondary["active_box"] = active
        del uref, sref
        torch.cuda.empty_cache()
        # launch tuner: the 256^3 FP64 step with the choices timed on the device against the defaults
        ut = u.clone()
        st_t = nslgf.HerkState(ut, dx, dt, re, "A", n_buf=16)

        def time_steps(k=10):
            st_t.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                st_t.step()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / k * 1e3

        ms_default = time_steps()
        default_cfg = nslgf.tuning_info(N, N, N)
        nslgf.set_tuning(nslgf.TUNE_AUTO)
        nslgf.lgf_table(N, N, N, torch.float64)  # rebuilt with the column plans timed
        tuned_cfg = nslgf.tuning_info(N, N, N)
        ms_tuned = time_steps()
        nslgf.set_tuning(nslgf.TUNE_DEFAULT)
        secondary["tuning"] = {"default": {**default_cfg, "step_ms": round(ms_default, 4)},
                               "tuned": {**tuned_cfg, "step_ms": round(ms_tuned, 4)},
                               "cell_shapes": nslgf.CELL_SHAPES}
        del ut, st_t
        torch.cuda.empty_cache()
        log("batched form: 32 uneven steps, FP64 and FP32 ...")
        secondary["batched"] = {"fp64": batched_measure(nslgf, torch, torch.float64),
                                "fp32": batched_measure(nslgf, torch, torch.float32),
                                "ensemble_64cubed_fp64": batched_measure(nslgf, torch, torch.float64, sizes=(64,))}
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores ...")
        cpu = cpu_baseline(w_np, dx, args.cpu_seconds)
        if not args.no_secondary:
            log("oracle against the GPU convolution at 32^3, 64^3, 128^3 ...")
            secondary["cpu_oracle"] = cpu_oracle_sizes(nslgf, torch, cpu["cores"])

    line = {
        "metric": "LGF solve Mpts/s & %HBM peak at 256^3; FP32/batched vs FP64 at stated rel err",
        "value": round(value, 2),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "grid": [N, N, N],
            "step": "Vor2Vel (3-component LGF solve + Cbar) + one Scheme A IF-HERK step",
            "lgf_points_per_step": lgf_pts,
            "ring": {"R": 1.0, "sigma_over_R": 0.1, "dx_over_R": 1 / 48, "Re": re, "cfl": cfl, "dt": dt},
            "n_buf": 16,
            "padded": [P, P, P],
            "table_build_s": round(table_s, 3),
            "fft_plan": args.fft_plan,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kern,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
