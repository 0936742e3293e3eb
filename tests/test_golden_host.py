"""The stored oracle samples of the elongated box match their recipe (CPU only): the box, the step
parameters, the step size the CFL rule gives for the recipe's input, and sample indices inside the
box that include full rows around the row-tile boundaries of the fused x-y integrating-factor pass."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_elongated as mk  # noqa: E402

Z = np.load(os.path.join(HERE, "golden", "elongated_box.npz"))


def test_golden_matches_the_recipe_on_the_host():
    from oracle import ifherk

    assert tuple(Z["shape"]) == mk.SHAPE and float(Z["dx"]) == mk.DX and float(Z["re"]) == mk.RE
    assert int(Z["n_buf"]) == mk.N_BUF and float(Z["alpha_if"]) == mk.ALPHA_IF
    assert float(Z["dt"]) == ifherk.dt_from_cfl(mk.initial_velocity(), mk.DX, mk.CFL)
    idx = Z["idx"]
    assert np.array_equal(idx, mk.sample_index())
    nz, ny, nx = mk.SHAPE
    assert idx.min() >= 0 and idx.max() < nz * ny * nx
    rows = set(((idx // nx) % ny).tolist())
    for j in (45, 46, 67, 68, 91, 92, 127, 128):  # both sides of every tile boundary used on the GPU
        assert j in rows, j
    for key in ("if_samples", "u_A", "u_C"):
        assert Z[key].shape == (3, idx.size)
    for key in ("d_A", "d_C"):
        assert Z[key].shape == (idx.size,)
