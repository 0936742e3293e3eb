"""Oracle: FP64 reference of the learned surrogate's layers.  Test infrastructure only.

Not part of the paper.  Plain definitions, channels-last arrays [D, H, W, C]:
* conv_fwd:    y[v, o] = sum_{tap, i} x[v + off(tap), i] w[tap, o, i]   (3x3x3, zero padding 1)
* conv_bwd_data:   gx[v, i] = sum_{tap, o} gy[v - off(tap), o] w[tap, o, i]   (adjoint in x)
* conv_bwd_weight: gw[tap, o, i] = sum_v gy[v, o] x[v + off(tap), i]          (adjoint in w)
* pool2 (2x2x2 average), up2 (nearest) and their adjoints.
* unet_forward / unet_backward: the surrogate network wired as in the product, in FP64, with the
  option of rounding each layer input to BF16 the way the matrix-core path does.
tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1).
"""
from __future__ import annotations

import numpy as np

TAPS = [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _shifted(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """out[v] = x[v + (dz, dy, dx)] with zeros outside."""
    D, H, W = x.shape[:3]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]


def conv_fwd(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += _shifted(x, dz, dy, dx) @ w[t].T
    return y


def conv_bwd_data(gy: np.ndarray, w: np.ndarray) -> np.ndarray:
    gx = np.zeros(gy.shape[:3] + (w.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        gx += _shifted(gy, -dz, -dy, -dx) @ w[t]
    return gx


def conv_bwd_weight(gy: np.ndarray, x: np.ndarray) -> np.ndarray:
    C_o, C_i = gy.shape[3], x.shape[3]
    gw = np.zeros((27, C_o, C_i))
    g2 = gy.reshape(-1, C_o)
    for t, (dz, dy, dx) in enumerate(TAPS):
        gw[t] = g2.T @ _shifted(x, dz, dy, dx).reshape(-1, C_i)
    return gw


def pool2(x: np.ndarray) -> np.ndarray:
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool2_adj(g: np.ndarray) -> np.ndarray:
    return up2(g) / 8.0


def up2(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(x, 2, axis=0), 2, axis=1), 2, axis=2)


def up2_adj(g: np.ndarray) -> np.ndarray:
    D, H, W, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def unet_forward(x: np.ndarray, ws: list, bf16: bool = False) -> dict:
    """x [R, R, R, 16]; ws: 10 weights [27, co, ci]; returns every activation (post-ReLU)."""
    q = bf16_round if bf16 else (lambda a: a)
    A = {"x": x}
    A["a0"] = relu(conv_fwd(q(x), ws[0]))
    A["e1"] = relu(conv_fwd(q(A["a0"]), ws[1]))
    A["p1"] = pool2(A["e1"])
    A["e2"] = relu(conv_fwd(q(A["p1"]), ws[2]))
    A["p2"] = pool2(A["e2"])
    A["e3"] = relu(conv_fwd(q(A["p2"]), ws[3]))
    A["p3"] = pool2(A["e3"])
    A["b4"] = relu(conv_fwd(q(A["p3"]), ws[4]))
    A["b5"] = relu(conv_fwd(q(A["b4"]), ws[5]))
    A["u3"] = up2(A["b5"]) + A["e3"]
    A["d3"] = relu(conv_fwd(q(A["u3"]), ws[6]))
    A["u2"] = up2(A["d3"]) + A["e2"]
    A["d2"] = relu(conv_fwd(q(A["u2"]), ws[7]))
    A["u1"] = up2(A["d2"]) + A["e1"]
    A["d1"] = relu(conv_fwd(q(A["u1"]), ws[8]))
    A["y"] = conv_fwd(q(A["d1"]), ws[9])
    return A


def unet_backward(A: dict, ws: list, gy: np.ndarray, bf16: bool = False) -> list:
    """Weight gradients for the output gradient gy (chain rule through unet_forward)."""
    q = bf16_round if bf16 else (lambda a: a)
    gw = [None] * 10
    mask = lambda a: (a > 0).astype(np.float64)

    def layer(li, g, inp):
        gw[li] = conv_bwd_weight(q(g), q(inp))
        return conv_bwd_data(q(g), ws[li])

    gd1 = layer(9, gy, A["d1"]) * mask(A["d1"])
    gu1 = layer(8, gd1, A["u1"])
    gd2 = up2_adj(gu1) * mask(A["d2"])
    gu2 = layer(7, gd2, A["u2"])
    gd3 = up2_adj(gu2) * mask(A["d3"])
    gu3 = layer(6, gd3, A["u3"])
    gb5 = up2_adj(gu3) * mask(A["b5"])
    gb4 = layer(5, gb5, A["b4"]) * mask(A["b4"])
    gp3 = layer(4, gb4, A["p3"])
    ge3 = (pool2_adj(gp3) + gu3) * mask(A["e3"])
    gp2 = layer(3, ge3, A["p2"])
    ge2 = (pool2_adj(gp2) + gu2) * mask(A["e2"])
    gp1 = layer(2, ge2, A["p1"])
    ge1 = (pool2_adj(gp1) + gu1) * mask(A["e1"])
    ga0 = layer(1, ge1, A["a0"]) * mask(A["a0"])
    gw[0] = conv_bwd_weight(q(ga0), q(A["x"]))
    return gw
