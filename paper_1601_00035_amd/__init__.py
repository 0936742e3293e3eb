"""MI355X-native fast lattice Green's function (LGF) hot path of the NS-LGF method.

Thin Python binding of libnslgf.so, whose C ABI is declared in include/nslgf.h.  Every step of the
method runs in the library's HIP kernels; this module only marshals torch tensors (device pointers,
sizes, the current HIP stream) into the C calls.  There is no CPU fallback: if the library is not
built, or a tensor is not on the GPU, the call raises.

Field layout: scalar fields are [nz, ny, nx] tensors, vector fields [3, nz, ny, nx], float64 or
float32, contiguous, on a CUDA (HIP) device.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libnslgf.so")

F64, F32 = 0, 1
SCHEME = {"A": 0, "B": 1, "C": 2}
OP = {"grad": 0, "div": 1, "curl": 2, "curl_bar": 3, "nonlinear": 4, "laplacian": 5}
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSUPPORTED", -5: "ESTATE", -6: "ENONFINITE"}
ENONFINITE = -6


class NslgfError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with {_STATUS.get(code, code)}: {msg}")
        self.code = code


class _State(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dtype", ctypes.c_int),
                ("scheme", ctypes.c_int), ("n_buf", ctypes.c_int), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("re", ctypes.c_double), ("t", ctypes.c_double), ("u", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("work", ctypes.c_void_p), ("stage_done", ctypes.c_int), ("guard", ctypes.c_int),
                ("supp_blocks", ctypes.c_void_p), ("soln_blocks", ctypes.c_void_p), ("block", ctypes.c_int),
                ("guard_margin", ctypes.c_int), ("div_max", ctypes.c_double)]


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is not built; run paper_1601_00035_amd/build.py first")
                L = ctypes.CDLL(LIB_PATH)
                vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
                sig = {
                    "nslgf_create": [ctypes.POINTER(vp), i],
                    "nslgf_destroy": [vp],
                    "lgf_value": [i, i, i, ctypes.POINTER(d)],
                    "lgf_table": [vp, i, i, i, i, vp],
                    "lgf_convolve": [vp, vp, vp, i, i, i, i, d, i, vp],
                    "lgf_convolve_noalloc": [vp, vp, vp, i, i, i, i, d, i, vp],
                    "if_apply": [vp, vp, vp, i, i, i, i, d, i, vp],
                    "herk_stage": [vp, ctypes.POINTER(_State), i, vp],
                    "herk_step": [vp, ctypes.POINTER(_State), vp],
                    "herk_check": [vp, ctypes.POINTER(_State), i, ctypes.POINTER(d), vp],
                    "herk_step_batched": [vp, ctypes.POINTER(ctypes.POINTER(_State)), i, vp],
                    "vor2vel": [vp, vp, vp, i, i, i, d, i, vp],
                    "stencil_apply": [vp, i, vp, vp, i, i, i, i, d, i, vp],
                    "max_cell_speed": [vp, vp, i, i, i, i, ctypes.POINTER(d), vp],
                    "nslgf_profile_enable": [vp, i],
                    "nslgf_set_fft_plan": [vp, i],
                    "nslgf_plan_info": [vp, i, i, i, i, vp, ctypes.POINTER(i), ctypes.POINTER(i)],
                    "nslgf_profile_read": [vp, i, ctypes.c_char_p, i, ctypes.POINTER(ctypes.c_longlong),
                                           ctypes.POINTER(d)],
                    "nslgf_copy": [vp, vp, vp, ctypes.c_size_t, i, vp],
                    "if_trunc_error": [d, i, ctypes.POINTER(d)],
                    "refresh_interval": [d, i, d, d, i, ctypes.POINTER(i)],
                    "max_component_abs": [vp, vp, i, i, i, i, i, ctypes.POINTER(d), vp],
                    "velocity_refresh": [vp, vp, i, i, i, i, d, i, vp],
                    "herk_run": [vp, ctypes.POINTER(_State), i, d, i, ctypes.POINTER(i), vp],
                    "flow_diagnostics": [vp, vp, i, i, i, i, d, ctypes.POINTER(d), i, ctypes.POINTER(d), vp],
                    "block_weights": [vp, vp, i, i, i, i, i, d, i, vp, vp, vp],
                    "herk_run_adaptive": [vp, ctypes.POINTER(_State), i, i, d, d, i, ctypes.POINTER(i),
                                          ctypes.POINTER(i), vp],
                    "classify_blocks": [vp, vp, i, i, i, d, d, i, vp, vp, vp, vp],
                    "herk_run_active": [vp, ctypes.POINTER(_State), i, i, d, d, i, ctypes.POINTER(i),
                                        ctypes.POINTER(i), ctypes.POINTER(i), vp],
                    "nslgf_set_tuning": [vp, i],
                    "nslgf_set_batch_mode": [vp, i],
                    "nslgf_batch_info": [vp, ctypes.POINTER(i), ctypes.POINTER(i)],
                    "nslgf_tuning_info": [vp, i, i, i, i, vp, ctypes.POINTER(i)],
                    "nslgf_tuning_save": [vp, ctypes.c_char_p],
                    "nslgf_tuning_load": [vp, ctypes.c_char_p],
                }
                for name, args in sig.items():
                    f = getattr(L, name)
                    f.argtypes = args
                    f.restype = i
                L.nslgf_state_bytes.argtypes = [i, i, i, i]
                L.nslgf_state_bytes.restype = ctypes.c_size_t
                L.nslgf_last_error.restype = ctypes.c_char_p
                L.nslgf_version.restype = ctypes.c_char_p
                _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != 0:
        raise NslgfError(fn, rc, lib().nslgf_last_error().decode())


_handles: dict[int, ctypes.c_void_p] = {}


def handle(device: int | None = None) -> ctypes.c_void_p:
    """The library handle of a device (created on first use, kept for the process lifetime)."""
    if device is None:
        device = torch.cuda.current_device()
    h = _handles.get(device)
    if h is None:
        h = ctypes.c_void_p()
        _check("nslgf_create", lib().nslgf_create(ctypes.byref(h), device))
        _handles[device] = h
    return h


def _dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype} (float64 or float32)")


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (there is no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _box(t: torch.Tensor, vector: bool | None = None):
    if t.dim() == 3:
        return 1, t.shape[2], t.shape[1], t.shape[0]
    if t.dim() == 4:
        return t.shape[0], t.shape[3], t.shape[2], t.shape[1]
    raise ValueError("fields are [nz, ny, nx] or [ncomp, nz, ny, nx]")


def version() -> str:
    return lib().nslgf_version().decode()


def lgf_value(n1: int, n2: int, n3: int) -> float:
    """g(n) of the 7-point Laplacian (host evaluation, same method as the table builder)."""
    out = ctypes.c_double()
    _check("lgf_value", lib().lgf_value(int(n1), int(n2), int(n3), ctypes.byref(out)))
    return out.value


def lgf_table(nx: int, ny: int, nz: int, dtype: torch.dtype = torch.float64, device: int | None = None):
    """Build the LGF spectrum for a box (otherwise built lazily by the first convolution)."""
    code = F64 if dtype == torch.float64 else F32
    dev = torch.cuda.current_device() if device is None else device
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check("lgf_table", lib().lgf_table(handle(dev), nx, ny, nz, code, s))


def lgf_convolve(src: torch.Tensor, dx: float = 1.0, out: torch.Tensor | None = None) -> torch.Tensor:
    """dst = dx^2 (g * src) per component on the box (L^{-1} src with zero conditions at infinity)."""
    _dev(src, "src")
    ncomp, nx, ny, nz = _box(src)
    if out is None:
        out = torch.empty_like(src)
    _dev(out, "out")
    if out.shape != src.shape or out.dtype != src.dtype:
        raise ValueError("out must match src")
    _check("lgf_convolve", lib().lgf_convolve(handle(src.device.index), src.data_ptr(), out.data_ptr(), ncomp, nx, ny,
                                              nz, float(dx), _dtype(src), _stream(src)))
    return out


def lgf_convolve_noalloc(src: torch.Tensor, dx: float, out: torch.Tensor) -> torch.Tensor:
    """lgf_convolve without any device allocation inside the library (workspaces in its fixed scratch
    array); lgf_table must have been called for the box and dtype, and out is the caller's."""
    _dev(src, "src")
    _dev(out, "out")
    ncomp, nx, ny, nz = _box(src)
    if out.shape != src.shape or out.dtype != src.dtype:
        raise ValueError("out must match src")
    _check("lgf_convolve_noalloc", lib().lgf_convolve_noalloc(handle(src.device.index), src.data_ptr(),
                                                              out.data_ptr(), ncomp, nx, ny, nz, float(dx),
                                                              _dtype(src), _stream(src)))
    return out


def if_apply(src: torch.Tensor, alpha: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """M E(alpha) M src per component (in place if out is src)."""
    _dev(src, "src")
    ncomp, nx, ny, nz = _box(src)
    if out is None:
        out = torch.empty_like(src)
    _dev(out, "out")
    _check("if_apply", lib().if_apply(handle(src.device.index), src.data_ptr(), out.data_ptr(), ncomp, nx, ny, nz,
                                      float(alpha), _dtype(src), _stream(src)))
    return out


def stencil(op: str, src: torch.Tensor, dx: float) -> torch.Tensor:
    """One point operator of the staggered grid: grad, div, curl, curl_bar, nonlinear, laplacian."""
    _dev(src, "src")
    code = OP[op]
    if code == OP["grad"]:
        nz, ny, nx = src.shape
        out = torch.empty((3, nz, ny, nx), dtype=src.dtype, device=src.device)
        ncomp = 1
    elif code == OP["div"]:
        _, nz, ny, nx = src.shape
        out = torch.empty((nz, ny, nx), dtype=src.dtype, device=src.device)
        ncomp = 3
    elif code == OP["laplacian"]:
        ncomp, nx, ny, nz = _box(src)
        out = torch.empty_like(src)
    else:
        _, nz, ny, nx = src.shape
        out = torch.empty_like(src)
        ncomp = 3
    _check("stencil_apply", lib().stencil_apply(handle(src.device.index), code, src.data_ptr(), out.data_ptr(), ncomp,
                                                nx, ny, nz, float(dx), _dtype(src), _stream(src)))
    return out


def vor2vel(w: torch.Tensor, dx: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """u = Cbar a, a = -L^{-1} w (edge vorticity -> face velocity)."""
    _dev(w, "w")
    _, nz, ny, nx = w.shape
    if out is None:
        out = torch.empty_like(w)
    _check("vor2vel", lib().vor2vel(handle(w.device.index), w.data_ptr(), out.data_ptr(), nx, ny, nz, float(dx),
                                    _dtype(w), _stream(w)))
    return out


def max_cell_speed(u: torch.Tensor) -> float:
    _dev(u, "u")
    _, nz, ny, nx = u.shape
    out = ctypes.c_double()
    _check("max_cell_speed", lib().max_cell_speed(handle(u.device.index), u.data_ptr(), nx, ny, nz, _dtype(u),
                                                  ctypes.byref(out), _stream(u)))
    return out.value


def if_trunc_error(alpha: float, k: int) -> float:
    """d_alpha(k) = sum_{n >= k} e^{-2 alpha} I_n(2 alpha): the masked integrating factor's deficit for a
    uniform unit field at the k-th point inside a face (host evaluation)."""
    out = ctypes.c_double()
    _check("if_trunc_error", lib().if_trunc_error(float(alpha), int(k), ctypes.byref(out)))
    return out.value


def refresh_interval(beta: float, n_buf: int, umax: float, eps: float, q_cap: int = 10000) -> int:
    """q_max: the largest number of steps whose estimated truncation error on the solution domain,
    umax d_{q beta}(n_buf + 1), stays within eps (host evaluation)."""
    out = ctypes.c_int()
    _check("refresh_interval", lib().refresh_interval(float(beta), int(n_buf), float(umax), float(eps), int(q_cap),
                                                      ctypes.byref(out)))
    return out.value


def max_component_abs(u: torch.Tensor, n_buf: int) -> float:
    """Largest |u^(q)| on the box shrunk by n_buf points (synchronises the stream)."""
    _dev(u, "u")
    _, nz, ny, nx = u.shape
    out = ctypes.c_double()
    _check("max_component_abs", lib().max_component_abs(handle(u.device.index), u.data_ptr(), nx, ny, nz, int(n_buf),
                                                        _dtype(u), ctypes.byref(out), _stream(u)))
    return out.value


def velocity_refresh(u: torch.Tensor, dx: float, n_buf: int) -> torch.Tensor:
    """In place: u = Cbar a, a = -L^{-1} w, w = M_supp C u (support = box shrunk by n_buf points)."""
    _dev(u, "u")
    _, nz, ny, nx = u.shape
    _check("velocity_refresh", lib().velocity_refresh(handle(u.device.index), u.data_ptr(), nx, ny, nz, int(n_buf),
                                                      float(dx), _dtype(u), _stream(u)))
    return u


def flow_diagnostics(u: torch.Tensor, dx: float, origin, n_buf: int) -> dict:
    """Impulse I, energy K, enstrophy E, helicity J and centroid X of the face velocity u (vorticity
    C u on the box shrunk by n_buf points, zero elsewhere); origin = coordinates of vertex (0, 0, 0).
    Synchronises the stream."""
    _dev(u, "u")
    _, nz, ny, nx = u.shape
    org = (ctypes.c_double * 3)(*[float(v) for v in origin])
    out = (ctypes.c_double * 9)()
    _check("flow_diagnostics", lib().flow_diagnostics(handle(u.device.index), u.data_ptr(), nx, ny, nz, int(n_buf),
                                                      float(dx), org, _dtype(u), out, _stream(u)))
    v = list(out)
    return {"I": v[0:3], "K": v[3], "E": v[4], "J": v[5], "X": v[6:9]}


def block_weights(u: torch.Tensor, dx: float, nb: int, n_buf: int):
    """(mu, nu) per block of nb^3 cells as numpy arrays [bz, by, bx]: the largest |C u| component and
    |G^T Ntilde(u)| over the block, away from the box faces by n_buf points (synchronises the stream)."""
    _dev(u, "u")
    _, nz, ny, nx = u.shape
    # (the library rejects nb < 1 before it writes anything)
    shape = (-(-nz // nb), -(-ny // nb), -(-nx // nb)) if nb >= 1 else (1, 1, 1)
    mu = np.zeros(shape)
    nu = np.zeros(shape)
    _check("block_weights", lib().block_weights(handle(u.device.index), u.data_ptr(), nx, ny, nz, int(nb), int(n_buf),
                                                float(dx), _dtype(u), mu.ctypes.data, nu.ctypes.data, _stream(u)))
    return mu, nu


def classify_blocks(mu, nu, eps_supp: float, eps_soln: float, n_xb: int):
    """(W, supp, soln, xsoln) block arrays from the weights (host evaluation)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    if mu.shape != nu.shape or mu.ndim != 3:
        raise ValueError("mu and nu must be block arrays [bz, by, bx] of one shape")
    bz, by, bx = mu.shape
    W = np.zeros(mu.shape)
    masks = [np.zeros(mu.shape, dtype=np.uint8) for _ in range(3)]
    _check("classify_blocks", lib().classify_blocks(mu.ctypes.data, nu.ctypes.data, bx, by, bz, float(eps_supp),
                                                    float(eps_soln), int(n_xb), W.ctypes.data,
                                                    *[m.ctypes.data for m in masks]))
    return (W, *masks)


FFT_PLAN_AUTOTUNE = -2


def set_fft_plan(choice: int, device: int | None = None):
    """Column-pass FFT plan of convolution plans built from now on (lengths 256 and 512): -1 the
    default, 0 narrow, 1 wide, 2 narrow radices on fewer elements per thread, -2 autotune
    (time every variant when a plan is built and keep the fastest)."""
    _check("nslgf_set_fft_plan", lib().nslgf_set_fft_plan(handle(device), int(choice)))


TUNE_DEFAULT, TUNE_AUTO = 0, 1
CELL_SHAPES = ((64, 4), (128, 2), (32, 8), (256, 1))


def set_tuning(mode: int, device: int | None = None):
    """TUNE_DEFAULT: the measured default launch shapes; TUNE_AUTO: time every choice on the first use of
    a box and dtype and keep the fastest (launch shapes never change results; column plans change the
    order of rounding only)."""
    _check("nslgf_set_tuning", lib().nslgf_set_tuning(handle(device), int(mode)))


def tuning_info(nx: int, ny: int, nz: int, dtype=torch.float64, device: int | None = None) -> dict:
    """The choices used for a box and dtype (tuned first if the handle tunes and none is recorded)."""
    out = (ctypes.c_int * 5)()
    code = F64 if dtype == torch.float64 else F32
    dev = torch.cuda.current_device() if device is None else device
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check("nslgf_tuning_info", lib().nslgf_tuning_info(handle(dev), nx, ny, nz, code, s, out))
    return {"vy": out[0], "vz": out[1], "if_rows": out[2], "if_seg": out[3], "cell_shape": out[4]}


def tuning_save(path: str, device: int | None = None):
    """Write every recorded choice (JSON, format nslgf-tuning-1)."""
    _check("nslgf_tuning_save", lib().nslgf_tuning_save(handle(device), os.fsencode(path)))


def tuning_load(path: str, device: int | None = None):
    """Read recorded choices written by tuning_save (they replace the defaults for their boxes)."""
    _check("nslgf_tuning_load", lib().nslgf_tuning_load(handle(device), os.fsencode(path)))


def plan_info(nx: int, ny: int, nz: int, dtype=torch.float64, device: int | None = None) -> tuple:
    """(y variant, z variant) of the convolution plan for this box and dtype (built if needed)."""
    vy, vz = ctypes.c_int(), ctypes.c_int()
    code = F64 if dtype == torch.float64 else F32
    dev = torch.cuda.current_device() if device is None else device
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check("nslgf_plan_info", lib().nslgf_plan_info(handle(dev), nx, ny, nz, code, s, ctypes.byref(vy),
                                                    ctypes.byref(vz)))
    return vy.value, vz.value


def profile_enable(on: bool = True, device: int | None = None):
    """Start (and clear) or stop per-kernel event timing inside the library."""
    _check("nslgf_profile_enable", lib().nslgf_profile_enable(handle(device), 1 if on else 0))


def profile_read(device: int | None = None) -> dict:
    """{kernel name: (launches, total ms)} collected since profile_enable(True)."""
    out = {}
    h = handle(device)
    i = 0
    buf = ctypes.create_string_buffer(64)
    calls = ctypes.c_longlong()
    ms = ctypes.c_double()
    while lib().nslgf_profile_read(h, i, buf, 64, ctypes.byref(calls), ctypes.byref(ms)) == 0:
        out[buf.value.decode()] = (calls.value, ms.value)
        i += 1
    return out


def copy(src: torch.Tensor, dst: torch.Tensor):
    """Plain device copy through the library's streaming kernel (byte-counter calibration)."""
    _dev(src, "src")
    _dev(dst, "dst")
    if src.numel() != dst.numel() or src.dtype != dst.dtype:
        raise ValueError("copy: size/dtype mismatch")
    _check("nslgf_copy", lib().nslgf_copy(handle(src.device.index), src.data_ptr(), dst.data_ptr(), src.numel(),
                                          _dtype(src), _stream(src)))


class HerkState:
    """IF-HERK state of one box: the caller's velocity u (updated in place), the pressure d and the
    library workspace, plus the step parameters."""

    def __init__(self, u: torch.Tensor, dx: float, dt: float, re: float, scheme: str = "A", n_buf: int = 0,
                 t: float = 0.0, guard: bool = False, guard_margin: int = 0):
        _dev(u, "u")
        _, nz, ny, nx = u.shape
        self.u = u
        self.d = torch.zeros((nz, ny, nx), dtype=u.dtype, device=u.device)
        nbytes = lib().nslgf_state_bytes(nx, ny, nz, _dtype(u))
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=u.device)
        self.c = _State(nx=nx, ny=ny, nz=nz, dtype=_dtype(u), scheme=SCHEME[scheme], n_buf=int(n_buf), dx=float(dx),
                        dt=float(dt), re=float(re), t=float(t), u=u.data_ptr(), d=self.d.data_ptr(),
                        work=self.work.data_ptr(), stage_done=0, guard=1 if guard else 0,
                        guard_margin=int(guard_margin))

    @property
    def t(self) -> float:
        return self.c.t

    @property
    def div_max(self) -> float:
        """Largest FP64 |Dbar u^i| of the last guarded step (over the stages and the checked cells)."""
        return self.c.div_max

    def check(self, margin: int) -> float:
        """FP64 max |Dbar u| over the cells at least margin cells from every face; raises NslgfError
        (code ENONFINITE) if u or d holds a non-finite value.  Synchronises the stream."""
        out = ctypes.c_double()
        _check("herk_check", lib().herk_check(handle(self.u.device.index), ctypes.byref(self.c), int(margin),
                                              ctypes.byref(out), _stream(self.u)))
        return out.value

    def set_dt(self, dt: float):
        self.c.dt = float(dt)

    def set_blocks(self, supp, soln, block: int):
        """Active domain as unions of blocks of block^3 cells (0/1 arrays [bz, by, bx], e.g. from
        classify_blocks): supp restricts the pressure source, soln the nonlinear term; None for both
        returns to the box shrunk by n_buf."""
        if supp is None and soln is None:
            self._blocks = None
            self.c.supp_blocks = self.c.soln_blocks = None
            self.c.block = 0
            return
        nz, ny, nx = self.u.shape[1:]
        shape = (-(-nz // block), -(-ny // block), -(-nx // block))
        t = []
        for m in (supp, soln):
            a = np.ascontiguousarray(np.asarray(m, dtype=np.uint8))
            if a.shape != shape:
                raise ValueError(f"block mask shape {a.shape}, expected {shape}")
            t.append(torch.from_numpy(a).to(self.u.device))
        self._blocks = t  # keeps the device copies alive
        self.c.supp_blocks, self.c.soln_blocks = t[0].data_ptr(), t[1].data_ptr()
        self.c.block = int(block)

    def stage(self, i: int):
        _check("herk_stage", lib().herk_stage(handle(self.u.device.index), ctypes.byref(self.c), int(i),
                                              _stream(self.u)))

    def step(self):
        _check("herk_step", lib().herk_step(handle(self.u.device.index), ctypes.byref(self.c), _stream(self.u)))

    def run_adaptive(self, nsteps: int, block: int, eps_supp: float, eps_soln: float, n_xb: int = 1):
        """nsteps steps on an active domain of blocks re-classified every step; returns (number of
        re-initialisations, steps whose expanded domain reached the box's outer block layer)."""
        nre, nedge = ctypes.c_int(), ctypes.c_int()
        # the run classifies into handle memory and leaves the state's own domain (set_blocks or n_buf)
        # in place when it returns
        _check("herk_run_adaptive", lib().herk_run_adaptive(handle(self.u.device.index), ctypes.byref(self.c),
                                                            int(nsteps), int(block), float(eps_supp), float(eps_soln),
                                                            int(n_xb), ctypes.byref(nre), ctypes.byref(nedge),
                                                            _stream(self.u)))
        return nre.value, nedge.value

    def run_active(self, nsteps: int, block: int, eps_supp: float, eps_soln: float, n_xb: int = 1):
        """nsteps steps on an active box (the bounding box of the expanded solution domain) that follows
        the flow; u and d keep the box's values and zero elsewhere.  Returns (re-initialisations, box
        changes, box first cell (x, y, z) and sizes (x, y, z))."""
        nre, nrg = ctypes.c_int(), ctypes.c_int()
        box = (ctypes.c_int * 6)()
        _check("herk_run_active", lib().herk_run_active(handle(self.u.device.index), ctypes.byref(self.c), int(nsteps),
                                                        int(block), float(eps_supp), float(eps_soln), int(n_xb),
                                                        ctypes.byref(nre), ctypes.byref(nrg), box, _stream(self.u)))
        return nre.value, nrg.value, tuple(box[:3]), tuple(box[3:])

    def run(self, nsteps: int, eps: float, q_cap: int = 10000) -> int:
        """nsteps steps with a velocity refresh after every q_max steps (q_max from eps); returns the
        number of refreshes."""
        n = ctypes.c_int()
        _check("herk_run", lib().herk_run(handle(self.u.device.index), ctypes.byref(self.c), int(nsteps), float(eps),
                                          int(q_cap), ctypes.byref(n), _stream(self.u)))
        return n.value


BATCH_PASSES, BATCH_PER_PROBLEM = 0, 1


def set_batch_mode(mode: int, device: int | None = None):
    """BATCH_PASSES (default): one launch per kernel of the step over every group of like problems;
    BATCH_PER_PROBLEM: each problem's kernels on a branch stream of its own.  Same results."""
    _check("nslgf_set_batch_mode", lib().nslgf_set_batch_mode(handle(device), int(mode)))


def batch_info(device: int | None = None) -> tuple:
    """(groups, kernel launches) of the last captured batch graph (groups 0: the per-problem form)."""
    g, l = ctypes.c_int(), ctypes.c_int()
    _check("nslgf_batch_info", lib().nslgf_batch_info(handle(device), ctypes.byref(g), ctypes.byref(l)))
    return g.value, l.value


def herk_step_batched(states: list) -> None:
    """One step of every state, captured once into a HIP graph and replayed while the batch is
    unchanged (same boxes, pointers and step parameters)."""
    if not states:
        return
    dev = states[0].u.device
    arr = (ctypes.POINTER(_State) * len(states))(*[ctypes.pointer(st.c) for st in states])
    _check("herk_step_batched", lib().herk_step_batched(handle(dev.index), arr, len(states), _stream(states[0].u)))
