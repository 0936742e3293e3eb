"""Writes tests/golden/elongated_box.npz: the oracle's integrating factor and IF-HERK steps (Schemes A
and C, FP64) on an elongated box, sampled at fixed points.  Calls only oracle/ and workloads/.

The box, (nz, ny, nx) = (200, 136, 16), is chosen for the code paths it reaches on the GPU: a padded
z length of 512 (2 nz - 1 > 384), a y extent above 128 rows (the fused x-y integrating-factor pass
splits a plane into row tiles: by default three of 46 rows, boundaries at y = 46 and 92; two of 68
with 128 rows per workgroup) and z lines long enough for the interior segments of the z
integrating-factor pass.  The initial velocity is three compact random blobs, around y = 40, 92 and 128
(the first two across the default tile boundaries); it is not divergence-free, so the first pressure
solve has a source everywhere the blobs are.

The oracle needs about half an hour on eight cores for the three results; the GPU tests read the
samples and the full-field maxima from the file.  Run from the repository root:
    python tests/golden/make_elongated.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SHAPE = (200, 136, 16)
CENTRES = ((100, 128, 8), (45, 40, 7), (150, 92, 8))
RADIUS = 13.0
SEED = 21
DX, RE, CFL, N_BUF = 0.05, 500.0, 0.5, 2
ALPHA_IF = 0.0213
OUT = os.path.join(ROOT, "tests", "golden", "elongated_box.npz")


def initial_velocity():
    import workloads

    u = workloads.compact_blob(SHAPE, CENTRES, RADIUS, SEED)
    return u * (0.5 / np.abs(u).max())


def sample_index():
    """Flat indices into one scalar component: full rows around the row-tile boundaries (y = 46, 92 by
    default, 68 with 128 rows per workgroup) and the top rows in several z planes, whole z lines at
    several (y, x), and seeded random points."""
    nz, ny, nx = SHAPE
    idx = []
    rows = list(range(38, 54)) + list(range(62, 75)) + list(range(84, 100)) + list(range(118, 136))
    for k in (0, 1, 44, 45, 99, 100, 101, 150, 151, 198, 199):
        for j in rows:
            idx.extend(k * ny * nx + j * nx + np.arange(nx))
    for j in (0, 40, 45, 46, 67, 68, 91, 92, 127, 128, 129, 135):
        for i in (0, 7, 8, 15):
            idx.extend(np.arange(nz) * ny * nx + j * nx + i)
    rng = np.random.default_rng(5)
    idx.extend(rng.choice(nz * ny * nx, size=4000, replace=False))
    return np.unique(np.array(idx, dtype=np.int64))


def main():
    from oracle import ifherk, intfac

    u0 = initial_velocity()
    dt = ifherk.dt_from_cfl(u0, DX, CFL)
    idx = sample_index()
    out = {"shape": np.array(SHAPE), "idx": idx, "dt": np.array(dt), "dx": np.array(DX), "re": np.array(RE),
           "n_buf": np.array(N_BUF), "alpha_if": np.array(ALPHA_IF)}
    t0 = time.time()
    e = intfac.apply_vec(u0, ALPHA_IF)
    out["if_samples"] = e.reshape(3, -1)[:, idx]
    out["if_max"] = np.array(np.abs(e).max())
    print(f"integrating factor done in {time.time() - t0:.0f} s", flush=True)
    for scheme in ("A", "C"):
        t0 = time.time()
        u1, d1 = ifherk.step(u0, dt, DX, RE, scheme, n_buf=N_BUF)
        out[f"u_{scheme}"] = u1.reshape(3, -1)[:, idx]
        out[f"d_{scheme}"] = d1.reshape(-1)[idx]
        out[f"umax_{scheme}"] = np.array(np.abs(u1).max())
        out[f"dmax_{scheme}"] = np.array(np.abs(d1).max())
        print(f"scheme {scheme} step done in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
