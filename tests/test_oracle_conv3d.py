"""Pins of the surrogate-layer oracle: exact adjointness of the backward maps, a delta kernel is a
shift, pooling/upsampling adjoints, BF16 rounding against known values, and finite differences of the
whole network's loss against its backward pass."""
import numpy as np

from oracle import conv3d as C


def test_bf16_rounding_known_values():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, 3.14159265, -2.5e-3, 65504.0])
    got = C.bf16_round(v)
    assert got[0] == 1.0
    assert got[1] == 1.0                       # tie to even
    assert got[2] == 1.0 + 2 ** -6 - 2 ** -7  # 1.0078125 + ... rounds to 8 significant bits
    assert abs(got[3] - 3.140625) < 1e-12
    assert np.all(np.abs(got - v) <= np.abs(v) * 2 ** -8)


def test_conv_adjoints_exact():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, 6, 5, 3))
    w = rng.standard_normal((27, 7, 3))
    g = rng.standard_normal((4, 6, 5, 7))
    y = C.conv_fwd(x, w)
    assert abs(np.sum(y * g) - np.sum(x * C.conv_bwd_data(g, w))) < 1e-10 * np.abs(y * g).sum()
    assert abs(np.sum(y * g) - np.sum(w * C.conv_bwd_weight(g, x))) < 1e-10 * np.abs(y * g).sum()


def test_delta_kernel_is_shift():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 5, 5, 2))
    w = np.zeros((27, 2, 2))
    t = 1 * 9 + 2 * 3 + 0  # dz = 0, dy = +1, dx = -1
    w[t] = np.eye(2)
    y = C.conv_fwd(x, w)
    assert np.array_equal(y[:, :-1, 1:], x[:, 1:, :-1])
    assert not y[:, -1, :].any() and not y[:, :, 0].any()


def test_resampling_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6, 8, 3))
    g = rng.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(C.pool2(x) * g) - np.sum(x * C.pool2_adj(g))) < 1e-12
    assert abs(np.sum(C.up2(g) * x) - np.sum(g * C.up2_adj(x))) < 1e-12
    assert np.allclose(C.pool2(C.up2(g)), g)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(3)
    LAYERS = [(16, 32), (32, 32), (32, 64), (64, 96), (96, 128), (128, 96), (96, 64), (64, 32), (32, 32), (32, 32)]
    R = 16
    x = np.zeros((R, R, R, 16))
    x[..., :4] = rng.standard_normal((R, R, R, 4))
    ws = [rng.standard_normal((27, co, ci)) * np.sqrt(2.0 / (27 * ci)) for ci, co in LAYERS]
    target = rng.standard_normal((R, R, R, 32))

    def loss(ws_):
        y = C.unet_forward(x, ws_)["y"]
        return 0.5 * np.sum((y - target) ** 2)

    A = C.unet_forward(x, ws)
    gw = C.unet_backward(A, ws, A["y"] - target)
    for li, idx in [(0, (13, 5, 2)), (4, (3, 100, 50)), (9, (26, 0, 31)), (6, (7, 10, 20))]:
        eps = 1e-6
        wp = [w.copy() for w in ws]
        wm = [w.copy() for w in ws]
        wp[li][idx] += eps
        wm[li][idx] -= eps
        fd = (loss(wp) - loss(wm)) / (2 * eps)
        assert abs(fd - gw[li][idx]) <= 1e-5 * max(1.0, abs(fd)), (li, fd, gw[li][idx])
