"""Generate data with the plain FP64 step, train the surrogate U-Net and run the judged roll-out.

  python -m paper_1601_00035_amd.surrogate_run --n 128 --trajectories 20 --steps 100 --iters 3000 \
      --out report.json

Data: `trajectories` perturbed rings (sigma/R ~ U[0.1, 0.3], Re ~ U[250, 1000], seeded) at n^3 with
dx = R/24 (n = 128) or dx = 2 (R + 5 sigma)/(n - 16) (smaller boxes), `steps` Scheme A steps each,
every step's vorticity kept (trajectories x (steps + 1) snapshots).  Training: Adam on random
(w_k, w_{k+h}) pairs.  Evaluation: judged roll-out on a held-out ring, against the persistence
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
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-blocks", type=int, default=6)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)

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

    net = S.UNet("cuda:0", seed=a.seed)
    t0 = time.perf_counter()
    losses = S.train(net, trajs, res, a.horizon, a.iters, lr=a.lr, seed=a.seed, log_every=max(1, a.iters // 20))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    for it, l in losses:
        print(f"iter {it}: loss {l:.4e}", file=sys.stderr, flush=True)
    del trajs
    torch.cuda.empty_cache()

    sig, re, seed = eval_spec
    ro = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, a.eval_blocks, a.horizon, a.tol)
    gain = [p / e for e, p in zip(ro["err"], ro["persistence_err"])]
    report = {
        "grid": n, "trajectories": len(train_specs), "snapshots": snapshots, "steps_per_trajectory": a.steps,
        "horizon": a.horizon, "train_iters": a.iters, "data_gen_s": round(gen_s, 2), "train_s": round(train_s, 2),
        "ms_per_train_iter": round(1e3 * train_s / max(1, a.iters), 3),
        "loss_first": losses[0][1], "loss_last": losses[-1][1],
        "eval": {"sigma": sig, "Re": re, "tol": a.tol, "rel_err": ro["err"], "persistence_rel_err": ro["persistence_err"],
                 "error_reduction_vs_persistence": gain, "extrapolation_rel_err": ro["extrapolation_err"],
                 "accepted": ro["accepted"],
                 "accept_rate": sum(ro["accepted"]) / len(ro["accepted"]),
                 "ms_surrogate_proposal": ro["ms_surrogate"], "ms_plain_horizon": ro["ms_plain"]},
    }
    line = json.dumps(report)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
