"""The launch tuner: every launch-shape choice (fused x-y IF rows per workgroup, z-pass outputs per
thread, point-kernel workgroup shape) gives results bit-identical to the defaults, the tuner picks
valid choices, and recorded choices survive a JSON save / load into another handle."""
import ctypes
import itertools
import json

import numpy as np
import pytest
import torch

import paper_1601_00035_amd as nslgf
import workloads
from oracle import ifherk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# boxes used by no other test, so that the choices recorded on the process's handle stay local
BOX = (20, 132, 44)  # (nx, ny, nz): two or three row tiles per plane, padded lengths 48 / 320 / 96


def _state():
    nx, ny, nz = BOX
    u0 = workloads.compact_blob((nz, ny, nx), [(22, 70, 10), (30, 125, 9)], 9.0, 31)
    u0 *= 0.5 / np.abs(u0).max()
    dx = 0.05
    return u0, dx, ifherk.dt_from_cfl(u0, dx, 0.5), 400.0


def _run(u0, dx, dt, re):
    u = torch.from_numpy(u0).to(DEV)
    st = nslgf.HerkState(u, dx, dt, re, "C", n_buf=2)
    st.step()
    e = nslgf.if_apply(torch.from_numpy(u0).to(DEV), 0.03)
    return u, st.d, e


def _entry(rows, seg, shape, launch=1):
    nx, ny, nz = BOX
    return {"nx": nx, "ny": ny, "nz": nz, "dtype": "f64", "Px": 48, "Py": 320, "Pz": 96, "vy": -1, "vz": -1,
            "launch": launch, "if_rows": rows, "if_seg": seg, "cell_shape": shape}


def test_every_launch_choice_is_bit_identical(tmp_path):
    u0, dx, dt, re = _state()
    ref = _run(u0, dx, dt, re)
    try:
        for rows, seg, shape in itertools.product((32, 64, 128, 256), (16, 32), range(4)):
            path = tmp_path / f"t_{rows}_{seg}_{shape}.json"
            path.write_text(json.dumps({"format": "nslgf-tuning-1", "entries": [_entry(rows, seg, shape)]}))
            nslgf.tuning_load(str(path))
            got = _run(u0, dx, dt, re)
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (rows, seg, shape)
    finally:
        # back to the defaults for this box on the process's handle (an entry without launch choices)
        path = tmp_path / "default.json"
        path.write_text(json.dumps({"format": "nslgf-tuning-1", "entries": [_entry(128, 32, 0, launch=0)]}))
        nslgf.tuning_load(str(path))


def test_auto_tuning_and_save_load(tmp_path):
    u0, dx, dt, re = _state()
    box = (28, 30, 26)
    nslgf.set_tuning(nslgf.TUNE_AUTO)
    try:
        info = nslgf.tuning_info(*box)
    finally:
        nslgf.set_tuning(nslgf.TUNE_DEFAULT)
    assert info["if_rows"] in (32, 64, 128, 256) and info["if_seg"] in (16, 32) and 0 <= info["cell_shape"] < 4
    path = tmp_path / "tuned.json"
    nslgf.tuning_save(str(path))
    doc = json.loads(path.read_text())
    assert doc["format"] == "nslgf-tuning-1"
    mine = [e for e in doc["entries"] if (e["nx"], e["ny"], e["nz"]) == box]
    assert len(mine) == 1 and mine[0]["launch"] == 1 and mine[0]["if_rows"] == info["if_rows"]
    # a second handle reads the file and uses the recorded choices without tuning
    L = nslgf.lib()
    h = ctypes.c_void_p()
    assert L.nslgf_create(ctypes.byref(h), 0) == 0
    try:
        assert L.nslgf_tuning_load(h, str(path).encode()) == 0
        out = (ctypes.c_int * 5)()
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        assert L.nslgf_tuning_info(h, *box, 0, s, out) == 0
        assert list(out)[2:] == [info["if_rows"], info["if_seg"], info["cell_shape"]]
        assert list(out)[:2] == [info["vy"], info["vz"]]
        bad = tmp_path / "bad.json"
        bad.write_text(json.dumps({"format": "nslgf-tuning-1", "entries": [dict(_entry(96, 32, 0))]}))
        assert L.nslgf_tuning_load(h, str(bad).encode()) == -1  # 96 rows is not a choice
        bad.write_text("{}")
        assert L.nslgf_tuning_load(h, str(bad).encode()) == -1
    finally:
        L.nslgf_destroy(h)


def test_default_launch_shapes_follow_the_box():
    """Without recorded choices a box gets the defaults for its size: x-y IF rows per workgroup 32 up to
    128 cells along y, 64 up to 192, else 128; z IF outputs per thread 16 up to 192 cells along z, else 32."""
    for box, rows, seg in (((24, 120, 40), 32, 16), ((24, 150, 200), 64, 32), ((24, 200, 30), 128, 16)):
        info = nslgf.tuning_info(*box)
        assert (info["if_rows"], info["if_seg"], info["cell_shape"]) == (rows, seg, 0), (box, info)
