"""Generate data with the plain FP64 step, train the surrogate U-Net and run the judged roll-out.

  python -m paper_1601_00035_amd.surrogate_run --n 128 --trajectories 20 --steps 100 --iters 3000 \
      --out report.json

Data: `trajectories` perturbed rings (sigma/R ~ U[0.1, 0.3], Re ~ U[250, 1000], seeded) at n^3 with
dx = R/24 (n = 128) or dx = 2 (R + 5 sigma)/(n - 16) (smaller boxes), `steps` Scheme A steps each,
every step's vorticity kept (trajectories x (steps + 1) snapshots).  Training: Adam on random
(w_k, w_{k+h}) pairs (--mode correct: on (w_k, w_{k+1}, w_{k+h}) triples, the network correcting the
linear extrapolation of one plain step).  Evaluation: judged roll-out on a held-out ring, against the persistence
baseline w_{k+h} ~ w_k and the linear extrapolation of one plain step, with the plain FP64 step as
judge and fallback.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import torch


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--trajectories", type=int, default=20)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--horizon", type=int, default=4)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=3e-4,
                    help="peak Adam step size (1e-3 let the loss spike and, in some runs, the ReLUs die)")
    ap.add_argument("--lr-min", type=float, default=1e-5,
                    help="cosine decay of the Adam step size from --lr to this over the iterations (negative: constant)")
    ap.add_argument("--eval-blocks", type=int, default=6)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=["persist", "correct"], default="persist",
                    help="persist: the network maps w_k to w_{k+h} - w_k; correct: it maps (w_k, w_{k+1} - w_k) "
                         "to the error of the linear extrapolation of one plain step")
    ap.add_argument("--gain", type=float, default=None, help="target scale (default 5 persist, 30 correct)")
    ap.add_argument("--out", default="")
    ap.add_argument("--time-iters", type=int, default=0,
                    help="only time this many training iterations (after one warm-up) on a seeded random field "
                         "at n^3, and print the time per iteration (no data, no roll-out)")
    a = ap.parse_args(argv)
    if a.time_iters:
        return time_iterations(a.n, a.time_iters, a.seed)

    import workloads
    from . import surrogate as S

    torch.cuda.set_device(0)
    n = a.n
    specs = workloads.surrogate_specs(a.trajectories + 1, seed=a.seed)
    train_specs, eval_spec = specs[:-1], specs[-1]

    def dx_of(sigma):
        return 1.0 / 24.0 if n == 128 else 2.0 * (1.0 + 5.0 * sigma) / (n - 16)

    t0 = time.perf_counter()
    trajs, res = [], []
    for (sig, re, seed) in train_specs:
        snaps, dt = S.make_trajectory(n, dx_of(sig), sig, re, seed, a.steps)
        trajs.append(snaps)
        res.append(re)
        print(f"trajectory sigma={sig:.3f} Re={re:.0f}: {snaps.shape[0]} snapshots, dt={dt:.4f}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    snapshots = sum(t.shape[0] for t in trajs)

    gain = a.gain if a.gain is not None else (30.0 if a.mode == "correct" else 5.0)
    net = S.UNet("cuda:0", seed=a.seed, in_real=7 if a.mode == "correct" else 4)
    t0 = time.perf_counter()
    losses = S.train(net, trajs, res, a.horizon, a.iters, lr=a.lr, seed=a.seed, log_every=max(1, a.iters // 20),
                     mode=a.mode, gain=gain, lr_min=a.lr_min if a.lr_min >= 0 else None)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    for it, l in losses:
        print(f"iter {it}: loss {l:.4e}", file=sys.stderr, flush=True)
    del trajs
    torch.cuda.empty_cache()

    sig, re, seed = eval_spec
    ro = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, a.eval_blocks, a.horizon, a.tol, gain=gain, mode=a.mode)
    reduction = [p / e for e, p in zip(ro["err"], ro["persistence_err"])]
    report = {
        "mode": a.mode, "gain": gain, "lr": a.lr, "lr_min": a.lr_min, "grid": n, "trajectories": len(train_specs), "snapshots": snapshots, "steps_per_trajectory": a.steps,
        "horizon": a.horizon, "train_iters": a.iters, "data_gen_s": round(gen_s, 2), "train_s": round(train_s, 2),
        "ms_per_train_iter": round(1e3 * train_s / max(1, a.iters), 3),
        "loss_first": losses[0][1], "loss_last": losses[-1][1],
        "eval": {"sigma": sig, "Re": re, "tol": a.tol, "rel_err": ro["err"], "persistence_rel_err": ro["persistence_err"],
                 "error_reduction_vs_persistence": reduction, "extrapolation_rel_err": ro["extrapolation_err"],
                 "accepted": ro["accepted"],
                 "accept_rate": sum(ro["accepted"]) / len(ro["accepted"]),
                 "ms_surrogate_proposal": ro["ms_surrogate"], "ms_plain_horizon": ro["ms_plain"]},
    }
    line = json.dumps(report)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


def time_iterations(n: int, iters: int, seed: int):
    """Training iterations (forward, loss, backward, Adam) at n^3 on a seeded random vorticity and target;
    prints {"ms_per_train_iter": ...}.  Every iteration launches the same kernels in the same order."""
    from . import surrogate as S

    torch.cuda.set_device(0)
    g = torch.Generator(device="cpu").manual_seed(seed)
    net = S.UNet("cuda:0", seed=seed)
    nvox = n ** 3
    om = torch.randn((3, n, n, n), generator=g, dtype=torch.float64).to("cuda:0")
    xb = S.pack_input(om, 1.0, 500.0)
    tg = (torch.randn(nvox * S.USED, generator=g) * 0.01).to("cuda:0", torch.float32)

    def it():
        y = net.forward(xb, n, train=True)
        net.loss_and_grad(y, tg, nvox, fused=True)
        net.backward(None)
        net.adam(lr=1e-4)

    it()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(iters):
        it()
    e1.record()
    torch.cuda.synchronize()
    print(json.dumps({"grid": n, "iters": iters, "ms_per_train_iter": round(e0.elapsed_time(e1) / iters, 3)}), flush=True)


if __name__ == "__main__":
    main()
