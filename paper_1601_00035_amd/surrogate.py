"""Learned surrogate of the IF-HERK step (not part of the paper): a 3D convolutional U-Net.

The network maps the edge vorticity w_k (3 channels, scaled) and a Reynolds-number feature to the
change w_{k+S} - w_k over S steps; a proposal is w_k plus that change.  The plain step of the library
judges every proposal (Vor2Vel + S IF-HERK steps from the same state) and replaces it when its error
exceeds the tolerance.  This module only wires layers together: every layer, forward and backward,
and every optimiser update runs in the library's kernels (include/nslgf_surrogate.h), on BF16 matrix
cores with FP32 accumulation.

Architecture (4 levels, 32-128 channels, 3x3x3 convolutions, ReLU, average pooling, nearest
upsampling, additive skips):
  R:   conv 16->32, conv 32->32 (e1) | R/2: conv 32->64 (e2) | R/4: conv 64->96 (e3)
  R/8: conv 96->128, conv 128->96 | up + e3 -> conv 96->64 | up + e2 -> conv 64->32
  up + e1 -> conv 32->32 -> conv 32->32 (linear; channels 0..2 are the output)
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _check, _stream, handle, lib

IN_CH = 16
OUT_CH = 32
USED = 3
LAYERS = [(16, 32), (32, 32), (32, 64), (64, 96), (96, 128), (128, 96), (96, 64), (64, 32), (32, 32), (32, 32)]
LEVEL = [0, 0, 1, 2, 3, 3, 2, 1, 0, 0]
RELU = [1, 1, 1, 1, 1, 1, 1, 1, 1, 0]

_bound = False


def _bind():
    global _bound
    if _bound:
        return
    L = lib()
    vp, i, d, f, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_float, ctypes.c_longlong
    sig = {
        "sur_conv3d_fwd": [vp, vp, vp, vp, i, i, i, i, i, i, vp],
        "sur_conv3d_bwd_data": [vp, vp, vp, vp, i, i, i, i, i, vp],
        "sur_conv3d_bwd_weight": [vp, vp, vp, vp, vp, i, i, i, i, i, vp],
        "sur_weight_transpose": [vp, vp, vp, i, i, vp],
        "sur_cast_bf16": [vp, vp, vp, ll, vp],
        "sur_cast_bf16_ex": [vp, vp, vp, vp, vp, ll, i, vp],
        "sur_cast_bf16_up": [vp, vp, d, vp, vp, vp, vp, i, i, i, i, vp],
        "sur_to_blocked8": [vp, vp, vp, ll, i, vp],
        "sur_conv3d_bwd_weight_blocked": [vp, vp, vp, vp, vp, i, i, i, i, i, vp],
        "sur_relu_bwd": [vp, vp, vp, ll, vp],
        "sur_add": [vp, vp, vp, vp, ll, vp],
        "sur_pool2_fwd": [vp, vp, vp, i, i, i, i, vp],
        "sur_pool2_bwd": [vp, vp, vp, i, i, i, i, vp],
        "sur_up2_fwd": [vp, vp, vp, i, i, i, i, vp],
        "sur_up2_bwd": [vp, vp, vp, i, i, i, i, vp],
        "sur_mse": [vp, vp, vp, vp, vp, ll, i, i, vp],
        "sur_mse_cast": [vp, vp, vp, vp, vp, vp, ll, i, i, vp],
        "sur_adam": [vp, vp, vp, vp, vp, vp, ll, f, f, f, f, i, vp],
        "sur_pack_input": [vp, vp, vp, i, i, i, d, d, vp],
        "sur_pack_input_pair": [vp, vp, vp, vp, i, i, i, d, d, d, vp],
        "sur_combine3": [vp, vp, vp, vp, vp, ll, d, d, d, vp],
        "sur_pack_target": [vp, vp, vp, i, i, i, d, vp],
        "sur_unpack_update": [vp, vp, vp, vp, i, i, i, i, d, vp],
        "sur_mfma_selftest": [vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = i
    L.sur_bwd_weight_work_bytes.argtypes = [i, i, i, i, i]
    L.sur_bwd_weight_work_bytes.restype = ctypes.c_size_t
    L.sur_bwd_weight_blocked_work_bytes.argtypes = [i, i, i, i, i]
    L.sur_bwd_weight_blocked_work_bytes.restype = ctypes.c_size_t
    _bound = True


def call(name: str, *args):
    """Call one surrogate entry point on the current device and stream (tensors -> pointers)."""
    _bind()
    dev = torch.cuda.current_device()
    conv = []
    for a in args:
        conv.append(a.data_ptr() if isinstance(a, torch.Tensor) else a)
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(name, getattr(lib(), name)(handle(dev), *conv, s))


def bf16_empty(n: int, device) -> torch.Tensor:
    """Raw BF16 storage (16-bit words) for the kernels."""
    return torch.empty(n, dtype=torch.int16, device=device)


def mfma_selftest(a_bf16: torch.Tensor, b_bf16: torch.Tensor) -> torch.Tensor:
    c = torch.empty((32, 32), dtype=torch.float32, device=a_bf16.device)
    call("sur_mfma_selftest", a_bf16, b_bf16, c)
    return c


class UNet:
    """Weights, optimiser state and activation buffers of the surrogate network."""

    def __init__(self, device="cuda:0", seed: int = 0, out_scale: float = 0.1, in_real: int = 4):
        self.device = torch.device(device)
        g = torch.Generator().manual_seed(seed)
        self.w, self.wb, self.wt, self.gw, self.m, self.v = [], [], [], [], [], []
        for li, (ci, co) in enumerate(LAYERS):
            fan_in = 27 * (in_real if li == 0 else ci)
            std = math.sqrt(2.0 / fan_in) * (out_scale if li == len(LAYERS) - 1 else 1.0)
            w = torch.randn((27, co, ci), generator=g) * std
            if li == 0:
                w[:, :, in_real:] = 0.0  # only the real input channels (4, or 7 in the correction form)
            w = w.to(self.device, torch.float32).contiguous()
            self.w.append(w)
            wb = bf16_empty(w.numel(), self.device)
            call("sur_cast_bf16", w, wb, w.numel())
            self.wb.append(wb)
            self.wt.append(bf16_empty(w.numel(), self.device))
            self.gw.append(torch.zeros_like(w))
            self.m.append(torch.zeros_like(w))
            self.v.append(torch.zeros_like(w))
        self.t = 0
        self.bufs = {}

    # ---- buffers ------------------------------------------------------------------------------
    def _buf(self, key, n, bf16=False):
        b = self.bufs.get(key)
        if b is None or b.numel() < n:
            b = bf16_empty(n, self.device) if bf16 else torch.empty(n, dtype=torch.float32, device=self.device)
            self.bufs[key] = b
        return b

    def _cast(self, src, key, n):
        dst = self._buf(key + "_b", n, bf16=True)
        call("sur_cast_bf16", src, dst, n)
        return dst

    def _cast_ex(self, src, key, nvox, c, act=None, blocked=True):
        """BF16 copy of an FP32 tensor [nvox][c] (after the ReLU backward of `act` when given) and, when
        `blocked`, its blocked copy for the weight gradient (key + "_k")."""
        dst = self._buf(key + "_b", nvox * c, bf16=True)
        blk = self._buf(key + "_k", nvox * c, bf16=True) if blocked else None
        call("sur_cast_bf16_ex", src, act, dst, blk, nvox, c)
        return dst

    def _cast_up(self, coarse, scale, skip, key, lv, c, blocked, act=None):
        """BF16 copy of scale * (coarse resampled to level lv) + skip, after the ReLU backward of `act` when
        given, and, when `blocked`, its blocked copy (key + "_k"): the upsampling (scale 1) or pooling
        adjoint (scale 1/8), the skip sum and the cast in one pass."""
        n = self.R >> lv
        dst = self._buf(key + "_b", n ** 3 * c, bf16=True)
        blk = self._buf(key + "_k", n ** 3 * c, bf16=True) if blocked else None
        call("sur_cast_bf16_up", coarse, float(scale), skip, act, dst, blk, n, n, n, c)
        return dst

    # ---- forward ------------------------------------------------------------------------------
    def forward(self, xb: torch.Tensor, R: int, train: bool = False) -> torch.Tensor:
        """xb: BF16 input [R^3][16]; returns the FP32 output [R^3][32] (channels 0..2 meaningful).  With
        `train`, the BF16 layer inputs also get the blocked copies the weight gradients read."""
        assert R % 16 == 0 and R >= 32
        r = [R >> l for l in range(4)]
        nv = [x ** 3 for x in r]
        A = {}
        self.R = R
        A["x_b"] = xb
        if train:
            A["x_k"] = self._buf("x_k", nv[0] * IN_CH, bf16=True)
            call("sur_to_blocked8", xb, A["x_k"], nv[0], IN_CH)

        def cast(src, key, lv, c):
            if train:
                return self._cast_ex(src, key, nv[lv], c)
            return self._cast(src, key, nv[lv] * c)

        def conv(li, src_b, key):
            ci, co = LAYERS[li]
            lv = LEVEL[li]
            out = self._buf(key, nv[lv] * co)
            call("sur_conv3d_fwd", src_b, self.wb[li], out, r[lv], r[lv], r[lv], ci, co, RELU[li])
            return out

        A["a0"] = conv(0, xb, "a0")
        A["a0_b"] = cast(A["a0"], "a0", 0, 32)
        A["e1"] = conv(1, A["a0_b"], "e1")
        A["p1"] = self._buf("p1", nv[1] * 32)
        call("sur_pool2_fwd", A["e1"], A["p1"], r[0], r[0], r[0], 32)
        A["p1_b"] = cast(A["p1"], "p1", 1, 32)
        A["e2"] = conv(2, A["p1_b"], "e2")
        A["p2"] = self._buf("p2", nv[2] * 64)
        call("sur_pool2_fwd", A["e2"], A["p2"], r[1], r[1], r[1], 64)
        A["p2_b"] = cast(A["p2"], "p2", 2, 64)
        A["e3"] = conv(3, A["p2_b"], "e3")
        A["p3"] = self._buf("p3", nv[3] * 96)
        call("sur_pool2_fwd", A["e3"], A["p3"], r[2], r[2], r[2], 96)
        A["p3_b"] = cast(A["p3"], "p3", 3, 96)
        A["b4"] = conv(4, A["p3_b"], "b4")
        A["b4_b"] = cast(A["b4"], "b4", 3, 128)
        A["b5"] = conv(5, A["b4_b"], "b5")
        # decoder inputs u = up2(coarser output) + skip, cast to BF16 in the same pass
        A["u3_b"] = self._cast_up(A["b5"], 1.0, A["e3"], "u3", 2, 96, train)
        A["d3"] = conv(6, A["u3_b"], "d3")
        A["u2_b"] = self._cast_up(A["d3"], 1.0, A["e2"], "u2", 1, 64, train)
        A["d2"] = conv(7, A["u2_b"], "d2")
        A["u1_b"] = self._cast_up(A["d2"], 1.0, A["e1"], "u1", 0, 32, train)
        A["d1"] = conv(8, A["u1_b"], "d1")
        A["d1_b"] = cast(A["d1"], "d1", 0, 32)
        A["y"] = conv(9, A["d1_b"], "y")
        self.A = A
        return A["y"][: nv[0] * OUT_CH]

    # ---- backward -----------------------------------------------------------------------------
    def backward(self, gy: torch.Tensor | None):
        """gy: FP32 gradient of the loss w.r.t. the output [R^3][32], or None for the BF16 copies that
        loss_and_grad(..., fused=True) wrote; fills self.gw.  After a forward with
        `train`, the weight gradients read blocked copies written by the casts (the ReLU backward folded
        into the gradient casts); otherwise they copy their operands themselves.  Same results."""
        A = self.A
        R = self.R
        r = [R >> l for l in range(4)]
        nv = [x ** 3 for x in r]
        blk = "x_k" in A

        def wgrad(li, gkey, g_b, xkey):
            ci, co = LAYERS[li]
            lv = LEVEL[li]
            nbytes = lib().sur_bwd_weight_blocked_work_bytes(r[lv], r[lv], r[lv], ci, co) if blk else 0
            if nbytes:  # (0: a volume the blocked form does not take, W % 8 != 0)
                work = self._buf("wgrad_work", nbytes // 4 + 1)
                call("sur_conv3d_bwd_weight_blocked", self.bufs[gkey + "_k"], self.bufs[xkey + "_k"], self.gw[li], work,
                     r[lv], r[lv], r[lv], ci, co)
            else:
                nbytes = lib().sur_bwd_weight_work_bytes(r[lv], r[lv], r[lv], ci, co)
                work = self._buf("wgrad_work", nbytes // 4 + 1)
                call("sur_conv3d_bwd_weight", g_b, A[xkey + "_b"], self.gw[li], work, r[lv], r[lv], r[lv], ci, co)

        def dgrad(li, g_b, key):
            ci, co = LAYERS[li]
            lv = LEVEL[li]
            call("sur_weight_transpose", self.wb[li], self.wt[li], ci, co)
            out = self._buf(key, nv[lv] * ci)
            call("sur_conv3d_bwd_data", g_b, self.wt[li], out, r[lv], r[lv], r[lv], ci, co)
            return out

        def castg(g, key, lv, c, act=None):
            """BF16 copy of a gradient, after the ReLU backward of the activation `act` when given."""
            if blk:
                return self._cast_ex(g, key, nv[lv], c, act=act)
            if act is not None:
                call("sur_relu_bwd", act, g, nv[lv] * c)
            return self._cast(g, key, nv[lv] * c)

        if gy is None and not getattr(self, "_gy_cast", False):
            raise ValueError("backward(None) needs loss_and_grad(..., fused=True) first")
        gy_b = self.bufs["gy_b"] if gy is None else castg(gy, "gy", 0, 32)  # (None: cast by loss_and_grad)
        self._gy_cast = False
        wgrad(9, "gy", gy_b, "d1")
        gd1 = dgrad(9, gy_b, "gd1")
        gd1_b = castg(gd1, "gd1", 0, 32, A["d1"])
        wgrad(8, "gd1", gd1_b, "u1")
        gu1 = dgrad(8, gd1_b, "gu1")                       # also the gradient of e1 through the skip
        gd2 = self._buf("gd2", nv[1] * 32)
        call("sur_up2_bwd", gu1, gd2, r[0], r[0], r[0], 32)
        gd2_b = castg(gd2, "gd2", 1, 32, A["d2"])
        wgrad(7, "gd2", gd2_b, "u2")
        gu2 = dgrad(7, gd2_b, "gu2")
        gd3 = self._buf("gd3", nv[2] * 64)
        call("sur_up2_bwd", gu2, gd3, r[1], r[1], r[1], 64)
        gd3_b = castg(gd3, "gd3", 2, 64, A["d3"])
        wgrad(6, "gd3", gd3_b, "u3")
        gu3 = dgrad(6, gd3_b, "gu3")
        gb5 = self._buf("gb5", nv[3] * 96)
        call("sur_up2_bwd", gu3, gb5, r[2], r[2], r[2], 96)
        gb5_b = castg(gb5, "gb5", 3, 96, A["b5"])
        wgrad(5, "gb5", gb5_b, "b4")
        gb4 = dgrad(5, gb5_b, "gb4")
        gb4_b = castg(gb4, "gb4", 3, 128, A["b4"])
        wgrad(4, "gb4", gb4_b, "p3")
        gp3 = dgrad(4, gb4_b, "gp3")
        # encoder gradients ge = pool2 adjoint of gp + the skip gradient gu, ReLU backward and cast in one pass
        ge3_b = self._cast_up(gp3, 0.125, gu3, "ge3", 2, 96, blk, act=A["e3"])
        wgrad(3, "ge3", ge3_b, "p2")
        gp2 = dgrad(3, ge3_b, "gp2")
        ge2_b = self._cast_up(gp2, 0.125, gu2, "ge2", 1, 64, blk, act=A["e2"])
        wgrad(2, "ge2", ge2_b, "p1")
        gp1 = dgrad(2, ge2_b, "gp1")
        ge1_b = self._cast_up(gp1, 0.125, gu1, "ge1", 0, 32, blk, act=A["e1"])
        wgrad(1, "ge1", ge1_b, "a0")
        ga0 = dgrad(1, ge1_b, "ga0")
        ga0_b = castg(ga0, "ga0", 0, 32, A["a0"])
        wgrad(0, "ga0", ga0_b, "x")

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for li in range(len(LAYERS)):
            call("sur_adam", self.w[li], self.wb[li], self.gw[li], self.m[li], self.v[li], self.w[li].numel(),
                 lr, b1, b2, eps, self.t)

    def loss_and_grad(self, y: torch.Tensor, target: torch.Tensor, nvox: int, fused: bool = False):
        """Per-block partial sums of the squared error and the FP32 gradient of the loss w.r.t. y; with
        `fused`, the gradient is written only as the BF16 copy (and, after a training forward, the blocked
        copy) that backward(None) reads, and None is returned in its place."""
        part = torch.empty(1024, dtype=torch.float64, device=self.device)
        self._gy_cast = fused
        if fused:
            gb = self._buf("gy_b", nvox * OUT_CH, bf16=True)
            gk = self._buf("gy_k", nvox * OUT_CH, bf16=True) if "x_k" in self.A else None
            call("sur_mse_cast", y, target, part, gb, gk, nvox, OUT_CH, USED)
            return part, None
        grad = self._buf("gy_f", nvox * OUT_CH)
        call("sur_mse", y, target, grad, part, nvox, OUT_CH, USED)
        return part, grad

    def state_dict(self):
        return {"w": [w.cpu() for w in self.w], "t": self.t}


# ---- fields <-> network tensors -------------------------------------------------------------------
def re_feature(re: float) -> float:
    return math.log(re / 500.0)


def pack_input(omega: torch.Tensor, scale: float, re: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """omega: planar FP64 [3][R][R][R] -> BF16 network input [R^3][16]."""
    R = omega.shape[-1]
    if out is None:
        out = bf16_empty(R ** 3 * IN_CH, omega.device)
    call("sur_pack_input", omega, out, R, R, R, float(scale), float(re_feature(re)))
    return out


def pack_input_pair(omega: torch.Tensor, delta: torch.Tensor, scale: float, dscale: float, re: float,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """Input of the correction form: omega * scale, the Re feature, delta * dscale (planar FP64 fields)."""
    R = omega.shape[-1]
    if out is None:
        out = bf16_empty(R ** 3 * IN_CH, omega.device)
    call("sur_pack_input_pair", omega, delta, out, R, R, R, float(scale), float(dscale), float(re_feature(re)))
    return out


def combine3(a: torch.Tensor, b: torch.Tensor, c, ca: float, cb: float, cc: float = 0.0) -> torch.Tensor:
    """ca a + cb b (+ cc c) of FP64 fields, on the GPU."""
    out = torch.empty_like(a)
    call("sur_combine3", a, b, c, out, a.numel(), float(ca), float(cb), float(cc))
    return out


def pack_target(delta: torch.Tensor, scale: float, out: torch.Tensor | None = None) -> torch.Tensor:
    R = delta.shape[-1]
    if out is None:
        out = torch.empty(R ** 3 * USED, dtype=torch.float32, device=delta.device)
    call("sur_pack_target", delta, out, R, R, R, float(scale))
    return out


def unpack_update(base: torch.Tensor, y: torch.Tensor, scale: float) -> torch.Tensor:
    R = base.shape[-1]
    out = torch.empty_like(base)
    call("sur_unpack_update", base, y, out, R, R, R, OUT_CH, float(scale))
    return out


# ---- data, training, judged roll-out ------------------------------------------------------------
def vorticity(u: torch.Tensor, dx: float) -> torch.Tensor:
    from . import stencil

    return stencil("curl", u, dx)


def make_trajectory(n: int, dx: float, sigma: float, re: float, seed: int, steps: int, cfl: float = 0.5,
                    n_buf: int = 8, zc: float = -0.5):
    """Vorticity snapshots w_0..w_steps (FP32, planar [3][n][n][n], on the GPU) of one ring advanced by
    the plain FP64 IF-HERK step, and the step size."""
    import workloads

    from . import HerkState, max_cell_speed, vor2vel

    ring = workloads.Ring(R=1.0, sigma=sigma, gamma=1.0, eps=1e-4, seed=seed, zc=zc)
    w0 = torch.from_numpy(workloads.ring_edge_vorticity(n, dx, ring, quad=2)).to("cuda")
    u = vor2vel(w0, dx)
    dt = cfl * dx / max_cell_speed(u)
    st = HerkState(u, dx, dt, re, "A", n_buf=n_buf)
    snaps = [vorticity(u, dx).float()]
    for _ in range(steps):
        st.step()
        snaps.append(vorticity(u, dx).float())
    return torch.stack(snaps), dt


def train(net: UNet, trajs: list, res: list, horizon: int, iters: int, lr: float = 1e-3, gain: float = 5.0,
          seed: int = 0, log_every: int = 0, mode: str = "persist", dgain: float = 10.0, lr_min: float | None = None):
    """Adam on random (w_k, w_{k+horizon}) pairs, s = 1 / max|w_0| of the trajectory.  With lr_min the
    step size follows a cosine from lr down to lr_min over the iterations (without it, constant lr).
    mode "persist": input w_k s, target (w_{k+h} - w_k) s gain.
    mode "correct": input w_k s and the one-step change (w_{k+1} - w_k) s dgain, target the error of the
    linear extrapolation, (w_{k+h} - w_k - h (w_{k+1} - w_k)) s gain.
    trajs[i]: snapshots [T][3][n][n][n]; res[i]: Re."""
    g = torch.Generator().manual_seed(seed)
    R = trajs[0].shape[-1]
    nvox = R ** 3
    xb = bf16_empty(nvox * IN_CH, net.device)
    tg = torch.empty(nvox * USED, dtype=torch.float32, device=net.device)
    scales = [1.0 / float(t[0].abs().max()) for t in trajs]
    losses = []
    for it in range(iters):
        i = int(torch.randint(len(trajs), (1,), generator=g))
        T = trajs[i].shape[0]
        k = int(torch.randint(T - horizon, (1,), generator=g))
        w_k = trajs[i][k].double()
        w_h = trajs[i][k + horizon].double()
        if mode == "correct":
            w_1 = trajs[i][k + 1].double()
            pack_input_pair(w_k, combine3(w_1, w_k, None, 1.0, -1.0), scales[i], scales[i] * dgain, res[i], out=xb)
            pack_target(combine3(w_h, w_k, w_1, 1.0, horizon - 1.0, -float(horizon)), scales[i] * gain, out=tg)
        else:
            pack_input(w_k, scales[i], res[i], out=xb)
            pack_target(combine3(w_h, w_k, None, 1.0, -1.0), scales[i] * gain, out=tg)
        y = net.forward(xb, R, train=True)
        part, _ = net.loss_and_grad(y, tg, nvox, fused=True)
        net.backward(None)
        lr_it = lr if lr_min is None else lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / max(1, iters - 1)))
        net.adam(lr=lr_it)
        if log_every and (it % log_every == 0 or it == iters - 1):
            losses.append((it, part.sum().item() / (nvox * USED)))
    return losses


def propose(net: UNet, w_k: torch.Tensor, scale: float, re: float, gain: float = 5.0) -> torch.Tensor:
    """The surrogate's proposal w_k + net(w_k) / (scale gain), FP64 planar."""
    R = w_k.shape[-1]
    xb = pack_input(w_k.double(), scale, re)
    y = net.forward(xb, R)
    return unpack_update(w_k.double(), y, scale * gain)


def propose_correct(net: UNet, w_k: torch.Tensor, w_1: torch.Tensor, scale: float, re: float, horizon: int,
                    gain: float, dgain: float) -> torch.Tensor:
    """The correction form's proposal: the extrapolation w_k + h (w_1 - w_k) plus net(w_k, w_1 - w_k) /
    (scale gain), FP64 planar."""
    R = w_k.shape[-1]
    w_k, w_1 = w_k.double(), w_1.double()
    xb = pack_input_pair(w_k, combine3(w_1, w_k, None, 1.0, -1.0), scale, scale * dgain, re)
    y = net.forward(xb, R)
    return unpack_update(combine3(w_k, w_1, None, 1.0 - horizon, float(horizon)), y, scale * gain)


def judged_rollout(net: UNet, n: int, dx: float, sigma: float, re: float, seed: int, blocks: int, horizon: int = 4,
                   tol: float = 1e-3, cfl: float = 0.5, n_buf: int = 8, gain: float = 5.0, mode: str = "persist",
                   dgain: float = 10.0):
    """Every `horizon` steps the surrogate proposes w_{k+h}; the plain FP64 step judges it from the
    same state (rel. max error of the vorticity) and the roll-out continues from the proposal if the
    error is within tol (velocity rebuilt by Vor2Vel), else from the plain result.  In mode "correct"
    the proposal also takes the first plain step (whose cost it then includes).  Returns per-block
    errors, two baselines (persistence w_{k+h} ~ w_k, and linear extrapolation of the first plain step
    w_{k+h} ~ w_k + h (w_{k+1} - w_k)) and timings."""
    import workloads

    from . import HerkState, max_cell_speed, vor2vel

    ring = workloads.Ring(R=1.0, sigma=sigma, gamma=1.0, eps=1e-4, seed=seed, zc=-0.5)
    w0 = torch.from_numpy(workloads.ring_edge_vorticity(n, dx, ring, quad=2)).to("cuda")
    u = vor2vel(w0, dx)
    dt = cfl * dx / max_cell_speed(u)
    scale = 1.0 / float(vorticity(u, dx).abs().max())
    out = {"err": [], "persistence_err": [], "extrapolation_err": [], "accepted": [], "ms_surrogate": [],
           "ms_plain": []}
    for _ in range(blocks):
        w_k = vorticity(u, dx)
        e0, e1, e2, e3, e4 = (torch.cuda.Event(enable_timing=True) for _ in range(5))
        e0.record()
        if mode == "correct":
            st = HerkState(u.clone(), dx, dt, re, "A", n_buf=n_buf)
            st.step()
            e1.record()
            w_1 = vorticity(st.u, dx)
            prop = propose_correct(net, w_k, w_1, scale, re, horizon, gain, dgain)
            u_prop = vor2vel(prop, dx)
            e2.record()
            e3.record()
        else:
            prop = propose(net, w_k, scale, re, gain)
            u_prop = vor2vel(prop, dx)
            e1.record()
            st = HerkState(u.clone(), dx, dt, re, "A", n_buf=n_buf)
            st.step()
            e2.record()
            w_1 = vorticity(st.u, dx)
            e3.record()
        for _ in range(horizon - 1):
            st.step()
        e4.record()
        torch.cuda.synchronize()
        w_ref = vorticity(st.u, dx)
        den = float(w_ref.abs().max())
        err = float((prop - w_ref).abs().max()) / den
        perr = float((w_k - w_ref).abs().max()) / den
        xerr = float((w_k + horizon * (w_1 - w_k) - w_ref).abs().max()) / den
        ok = err <= tol
        out["err"].append(err)
        out["persistence_err"].append(perr)
        out["extrapolation_err"].append(xerr)
        out["accepted"].append(ok)
        if mode == "correct":
            out["ms_surrogate"].append(e0.elapsed_time(e2))
            out["ms_plain"].append(e0.elapsed_time(e1) + e3.elapsed_time(e4))
        else:
            out["ms_surrogate"].append(e0.elapsed_time(e1))
            out["ms_plain"].append(e1.elapsed_time(e2) + e3.elapsed_time(e4))
        u = u_prop if ok else st.u
    return out
