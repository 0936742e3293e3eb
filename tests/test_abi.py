"""The C ABI library loads and exports every entry point declared in include/nslgf.h and
include/nslgf_surrogate.h, and the host-side
LGF evaluation of the table builder (same method as the GPU builder) agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1601_00035_amd as nslgf
from oracle import lgf as olgf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nslgf.h")).read() + open(os.path.join(ROOT, "include",
                                                                                   "nslgf_surrogate.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|size_t|char|void)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    L = nslgf.lib()
    names = _declared()
    assert "lgf_convolve" in names and "herk_stage" in names and "if_apply" in names and "lgf_table" in names
    assert "sur_conv3d_fwd" in names and "sur_cast_bf16_ex" in names and "sur_bwd_weight_blocked_work_bytes" in names
    for n in names:
        assert hasattr(L, n), n
    assert nslgf.version().startswith("nslgf")


def test_host_lgf_value_matches_oracle():
    cube = olgf.lgf_cube(60)
    rng = np.random.default_rng(0)
    pts = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (39, 0, 0), (40, 0, 0), (23, 23, 23), (60, 60, 60), (0, 0, 60)]
    pts += [tuple(int(v) for v in rng.integers(0, 61, 3)) for _ in range(60)]
    for p in pts:
        v = nslgf.lgf_value(*p)
        ref = cube[p]
        assert abs(v - ref) <= 2e-15 * abs(ref), (p, v, ref)
    # symmetry of the host evaluation and the closed form at the origin
    assert nslgf.lgf_value(-3, 7, -2) == nslgf.lgf_value(7, 2, 3)
    assert abs(nslgf.lgf_value(0, 0, 0) - olgf.g0_closed_form()) < 1e-16


def test_state_bytes():
    L = nslgf.lib()
    # 25 fields of the box (q, w1, w2, r, pressure, two 6-component IF temporaries) plus the
    # one-component convolution workspaces, then 256 bytes of step-guard accumulators at a 256-byte
    # boundary
    b64, b32 = L.nslgf_state_bytes(8, 8, 8, 0), L.nslgf_state_bytes(8, 8, 8, 1)
    assert b64 >= 25 * 512 * 8 + 256 and b32 >= 25 * 512 * 4 + 256
    assert b64 % 256 == 0 and b32 % 256 == 0 and b64 > b32
    assert L.nslgf_state_bytes(0, 8, 8, 0) == 0
    assert L.nslgf_state_bytes(8, 300, 8, 0) == 0


def test_null_handle_is_rejected_without_a_device():
    """Every handle-taking entry point of the refresh, ring-integral and active-domain calls returns
    NSLGF_EINVAL for a null handle before it touches a device (host-only check)."""
    L = nslgf.lib()
    d = ctypes.c_double()
    i = ctypes.c_int()
    buf = (ctypes.c_double * 16)()
    org = (ctypes.c_double * 3)()
    calls = [
        L.max_component_abs(None, None, 8, 8, 8, 1, 0, ctypes.byref(d), None),
        L.velocity_refresh(None, None, 8, 8, 8, 1, 0.1, 0, None),
        L.herk_run(None, None, 1, 1e-6, 10, ctypes.byref(i), None),
        L.herk_run_adaptive(None, None, 1, 4, 1e-4, 1e-2, 1, ctypes.byref(i), ctypes.byref(i), None),
        L.flow_diagnostics(None, None, 8, 8, 8, 1, 0.1, org, 0, buf, None),
        L.block_weights(None, None, 8, 8, 8, 4, 1, 0.1, 0, buf, buf, None),
        L.herk_check(None, None, 1, ctypes.byref(d), None),
    ]
    assert all(c == -1 for c in calls), calls
    assert b"null handle" in L.nslgf_last_error()
