"""Oracle: build and call the plain-C direct lattice sum (direct_sum.c).  Test infrastructure only.

The shared object is built with gcc into oracle/_build/ (no HIP, nothing shared with the GPU
library).  `build()` compiles unconditionally; `load()` compiles only if nothing is built yet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import lgf

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct_sum.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_SO = os.path.join(_OUT_DIR, "liboracle_direct.so")
_lib = None


def build() -> str:
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _SO + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _SO)
    return _SO


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        f = lib.oracle_lgf_direct
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p]
        _lib = lib
    return _lib


def lgf_direct_targets(src: np.ndarray, dx: float, targets: np.ndarray) -> np.ndarray:
    """y(n) = dx^2 sum_m g(n - m) s(m) at the given (k, j, i) targets (int64 [T, 3]; targets may lie
    outside the box).  src: float64 [nz, ny, nx]."""
    src = np.ascontiguousarray(src, dtype=np.float64)
    targets = np.ascontiguousarray(targets, dtype=np.int64).reshape(-1, 3)
    nz, ny, nx = src.shape
    span = max(nz, ny, nx) - 1
    if len(targets):
        lo = targets.min(axis=0)
        hi = targets.max(axis=0)
        span = max(span, int(max(hi[0], nz - 1 - lo[0], hi[1], ny - 1 - lo[1], hi[2], nx - 1 - lo[2])))
    cube = lgf.lgf_cube(span)
    out = np.empty(len(targets))
    rc = load().oracle_lgf_direct(cube.ctypes.data, cube.shape[0], src.ctypes.data, nz, ny, nx,
                                  targets.ctypes.data, len(targets), dx * dx, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_lgf_direct failed ({rc})")
    return out


def lgf_direct(src: np.ndarray, dx: float) -> np.ndarray:
    """Full-box LGF convolution by direct summation: returns float64 of src.shape."""
    nz, ny, nx = src.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tg = np.stack([k.ravel(), j.ravel(), i.ravel()], axis=1)
    return lgf_direct_targets(src, dx, tg).reshape(src.shape)
