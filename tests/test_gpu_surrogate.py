"""GPU parity of the surrogate's BF16 matrix-core layers against the FP64 oracle (on BF16-exact
inputs the FP32-accumulated results must agree to ~1e-5), the whole U-Net forward and backward
against the oracle network, and training that lowers the loss."""
import numpy as np
import pytest
import torch

import paper_1601_00035_amd.surrogate as S
from oracle import conv3d as C

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_bf16_bits(a: np.ndarray) -> torch.Tensor:
    """float64 values that are exactly BF16 -> int16 storage on the GPU."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    bits = (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.from_numpy(bits.copy()).to(DEV)


def rand_bf16(shape, seed, scale=1.0):
    return C.bf16_round(np.random.default_rng(seed).standard_normal(shape) * scale)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def test_mfma_operand_layout():
    A = rand_bf16((32, 16), 1)
    B = rand_bf16((16, 32), 2)
    got = S.mfma_selftest(to_bf16_bits(A), to_bf16_bits(B)).double().cpu().numpy()
    assert rel(got, A @ B) < 1e-6


# W % 32 == 0, H % 8 == 0 and D % 2 == 0 take the LDS-staged kernels (halo blocks of 2 x 8 rows of 32
# voxels; several blocks per axis, and volume faces on every side); the other shapes the gathering ones
@pytest.mark.parametrize("dims,cin,cout", [((8, 8, 8), 32, 64), ((4, 8, 12), 16, 32), ((8, 4, 4), 96, 128),
                                           ((4, 6, 16), 16, 32), ((2, 4, 24), 96, 128), ((2, 4, 32), 16, 32),
                                           ((4, 16, 64), 32, 64), ((2, 8, 32), 16, 32), ((6, 16, 32), 96, 128),
                                           ((2, 8, 96), 64, 96), ((4, 8, 32), 128, 32)])
def test_conv_layers(dims, cin, cout):
    D, H, W = dims
    x = rand_bf16((D, H, W, cin), 3)
    w = rand_bf16((27, cout, cin), 4, 0.1)
    gy = rand_bf16((D, H, W, cout), 5)
    xb, wb, gyb = to_bf16_bits(x), to_bf16_bits(w), to_bf16_bits(gy)
    nv = D * H * W
    y = torch.empty(nv * cout, dtype=torch.float32, device=DEV)
    S.call("sur_conv3d_fwd", xb, wb, y, D, H, W, cin, cout, 0)
    ref = C.conv_fwd(x, w)
    assert rel(y.double().cpu().numpy().reshape(ref.shape), ref) < 1e-5
    S.call("sur_conv3d_fwd", xb, wb, y, D, H, W, cin, cout, 1)
    assert rel(y.double().cpu().numpy().reshape(ref.shape), np.maximum(ref, 0)) < 1e-5
    # weight gradient
    nbytes = S.lib().sur_bwd_weight_work_bytes(D, H, W, cin, cout)
    work = torch.empty(nbytes // 4 + 1, dtype=torch.float32, device=DEV)
    gw = torch.empty(27 * cout * cin, dtype=torch.float32, device=DEV)
    S.call("sur_conv3d_bwd_weight", gyb, xb, gw, work, D, H, W, cin, cout)
    refw = C.conv_bwd_weight(gy, x)
    assert rel(gw.double().cpu().numpy().reshape(refw.shape), refw) < 1e-5
    if cin % 32 == 0:
        wt = S.bf16_empty(w.size, DEV)
        S.call("sur_weight_transpose", wb, wt, cin, cout)
        gx = torch.empty(nv * cin, dtype=torch.float32, device=DEV)
        S.call("sur_conv3d_bwd_data", gyb, wt, gx, D, H, W, cin, cout)
        refx = C.conv_bwd_data(gy, w)
        assert rel(gx.double().cpu().numpy().reshape(refx.shape), refx) < 1e-5


def test_resampling_and_elementwise():
    rng = np.random.default_rng(6)
    D, H, W, c = 4, 6, 8, 5
    x = rng.standard_normal((D, H, W, c)).astype(np.float32)
    g = rng.standard_normal((D // 2, H // 2, W // 2, c)).astype(np.float32)
    xt, gt = torch.from_numpy(x).to(DEV), torch.from_numpy(g).to(DEV)
    out_c = torch.empty(g.size, dtype=torch.float32, device=DEV)
    out_f = torch.empty(x.size, dtype=torch.float32, device=DEV)
    S.call("sur_pool2_fwd", xt, out_c, D, H, W, c)
    assert rel(out_c.cpu().numpy().reshape(g.shape), C.pool2(x.astype(np.float64))) < 1e-6
    S.call("sur_pool2_bwd", gt, out_f, D, H, W, c)
    assert rel(out_f.cpu().numpy().reshape(x.shape), C.pool2_adj(g.astype(np.float64))) < 1e-6
    S.call("sur_up2_fwd", gt, out_f, D, H, W, c)
    assert rel(out_f.cpu().numpy().reshape(x.shape), C.up2(g.astype(np.float64))) < 1e-7
    S.call("sur_up2_bwd", xt, out_c, D, H, W, c)
    assert rel(out_c.cpu().numpy().reshape(g.shape), C.up2_adj(x.astype(np.float64))) < 1e-6
    y = xt.clone()
    gg = torch.ones_like(xt)
    S.call("sur_relu_bwd", y, gg, y.numel())
    assert torch.equal(gg, (y > 0).float())
    # squared error: gradient 2 (p - t) / (nvox used) on the used channels (16-byte stores for 32
    # channels, one at a time for 6)
    for nvox, cc, used in ((64, 32, 3), (50, 6, 3)):
        p = torch.randn(nvox * cc, device=DEV)
        t = torch.randn(nvox * used, device=DEV)
        grad = torch.full_like(p, float("nan"))
        part = torch.empty(1024, dtype=torch.float64, device=DEV)
        S.call("sur_mse", p, t, grad, part, nvox, cc, used)
        pn, tn = p.double().cpu().numpy().reshape(nvox, cc), t.double().cpu().numpy().reshape(nvox, used)
        assert abs(part.sum().item() - ((pn[:, :used] - tn) ** 2).sum()) < 1e-9
        gref = np.zeros_like(pn)
        gref[:, :used] = 2 * (pn[:, :used] - tn) / (nvox * used)
        assert rel(grad.double().cpu().numpy().reshape(nvox, cc), gref) < 1e-6, cc


def test_unet_forward_backward_vs_oracle():
    R = 32
    net = S.UNet(DEV, seed=1, out_scale=1.0)
    ws = [w.double().cpu().numpy() for w in net.w]
    wsb = [C.bf16_round(w) for w in ws]  # the matrix cores see the BF16 copies
    rng = np.random.default_rng(7)
    x = np.zeros((R, R, R, 16))
    x[..., :4] = C.bf16_round(rng.standard_normal((R, R, R, 4)))
    y = net.forward(to_bf16_bits(x).reshape(-1), R)
    A = C.unet_forward(x, wsb, bf16=True)
    yref = A["y"]
    assert rel(y.double().cpu().numpy().reshape(yref.shape), yref) < 2e-2
    gy = rng.standard_normal(yref.shape)
    net.backward(torch.from_numpy(gy.astype(np.float32).reshape(-1)).to(DEV))
    gref = C.unet_backward(A, wsb, gy, bf16=True)
    # BF16 rounding of the gradient at every layer compounds along the chain: compare in relative L2
    for li in range(10):
        got = net.gw[li].double().cpu().numpy()
        l2 = np.linalg.norm(got - gref[li]) / np.linalg.norm(gref[li])
        assert l2 < 6e-2, (li, l2)
        assert rel(got, gref[li]) < 1.5e-1, li
    # the training path (blocked copies written by the casts, the ReLU backward folded into the gradient
    # casts, the blocked weight gradient) gives the same output and gradients bit for bit
    plain = [g.clone() for g in net.gw]
    y2 = net.forward(to_bf16_bits(x).reshape(-1), R, train=True)
    assert torch.equal(y2, y)
    net.backward(torch.from_numpy(gy.astype(np.float32).reshape(-1)).to(DEV))
    for li in range(10):
        assert torch.equal(net.gw[li], plain[li]), li


def test_fused_cast_and_blocked_weight_gradient():
    """sur_cast_bf16_ex equals sur_relu_bwd, sur_cast_bf16 and sur_to_blocked8 in turn, bit for bit (with
    and without the ReLU mask, zeros and negative values included); the blocked weight gradient equals
    the plain one bit for bit."""
    rng = np.random.default_rng(12)
    D, H, W, c = 4, 8, 16, 32
    nv = D * H * W
    g = rng.standard_normal((nv, c)).astype(np.float32)
    g[::7] = 0.0
    act = rng.standard_normal((nv, c)).astype(np.float32)
    act[::5] = 0.0
    gt, at = torch.from_numpy(g).to(DEV).reshape(-1), torch.from_numpy(act).to(DEV).reshape(-1)
    for use_act in (False, True):
        ref = gt.clone()
        if use_act:
            S.call("sur_relu_bwd", at, ref, nv * c)
        ref_b = S.bf16_empty(nv * c, DEV)
        S.call("sur_cast_bf16", ref, ref_b, nv * c)
        ref_k = S.bf16_empty(nv * c, DEV)
        S.call("sur_to_blocked8", ref_b, ref_k, nv, c)
        y, yk = S.bf16_empty(nv * c, DEV), S.bf16_empty(nv * c, DEV)
        S.call("sur_cast_bf16_ex", gt, at if use_act else None, y, yk, nv, c)
        assert torch.equal(y, ref_b) and torch.equal(yk, ref_k), use_act
    cin, cout = 32, 64
    x = to_bf16_bits(rand_bf16((D, H, W, cin), 13)).reshape(-1)
    dy = to_bf16_bits(rand_bf16((D, H, W, cout), 14)).reshape(-1)
    work = torch.empty(S.lib().sur_bwd_weight_work_bytes(D, H, W, cin, cout) // 4 + 1, dtype=torch.float32, device=DEV)
    gw = torch.empty(27 * cout * cin, dtype=torch.float32, device=DEV)
    S.call("sur_conv3d_bwd_weight", dy, x, gw, work, D, H, W, cin, cout)
    xk, dyk = S.bf16_empty(x.numel(), DEV), S.bf16_empty(dy.numel(), DEV)
    S.call("sur_to_blocked8", x, xk, nv, cin)
    S.call("sur_to_blocked8", dy, dyk, nv, cout)
    work2 = torch.empty(S.lib().sur_bwd_weight_blocked_work_bytes(D, H, W, cin, cout) // 4 + 1, dtype=torch.float32,
                        device=DEV)
    gw2 = torch.full_like(gw, float("nan"))
    S.call("sur_conv3d_bwd_weight_blocked", dyk, xk, gw2, work2, D, H, W, cin, cout)
    assert torch.equal(gw, gw2)


def test_training_lowers_loss():
    """Fit a fixed smooth target from a fixed input with Adam: the loss must fall."""
    R = 32
    net = S.UNet(DEV, seed=2)
    z, y, x = np.meshgrid(*(np.linspace(-1, 1, R),) * 3, indexing="ij")
    om = np.stack([np.exp(-4 * (x * x + y * y + z * z)), np.sin(2 * x) * np.exp(-y * y), z * np.exp(-x * x)])
    omt = torch.from_numpy(om).to(DEV)
    xb = S.pack_input(omt, 1.0, 500.0)
    tgt = S.pack_target(0.3 * omt * omt, 1.0)
    losses = []
    for it in range(60):
        out = net.forward(xb, R)
        part, grad = net.loss_and_grad(out, tgt, R ** 3)
        losses.append(part.sum().item() / (R ** 3 * 3))
        net.backward(grad)
        net.adam(lr=2e-3)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])


def test_judged_rollout_small():
    """Small-scale end to end: data from the plain step at 32^3, a short training run, then the judged
    roll-out on a held-out ring.  The fallback must hand back exactly the plain result when the
    tolerance rejects every proposal, and the trained network must beat the persistence baseline."""
    import workloads
    from paper_1601_00035_amd import HerkState, max_cell_speed, vor2vel

    n = 32
    specs = workloads.surrogate_specs(4, seed=3)
    dx_of = lambda s: 2.0 * (1.0 + 5.0 * s) / (n - 16)
    trajs, res = [], []
    for (sig, re, seed) in specs[:3]:
        snaps, _ = S.make_trajectory(n, dx_of(sig), sig, re, seed, 16, n_buf=2)
        trajs.append(snaps)
        res.append(re)
    net = S.UNet(DEV, seed=0)
    losses = S.train(net, trajs, res, 4, 300, lr=1e-3, log_every=50)
    assert losses[-1][1] < losses[0][1]
    sig, re, seed = specs[3]
    ro = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, blocks=3, horizon=4, tol=0.0, n_buf=2)
    assert not any(ro["accepted"])
    assert np.mean(ro["err"]) < np.mean(ro["persistence_err"]), (ro["err"], ro["persistence_err"])
    ro_all = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, blocks=1, horizon=4, tol=1e9, n_buf=2)
    assert all(ro_all["accepted"])


def test_correction_form_packing():
    """The correction form's input packing and the FP64 combination kernel against their definitions."""
    R = 8
    rng = np.random.default_rng(8)
    om = torch.from_numpy(rng.standard_normal((3, R, R, R))).to(DEV)
    dl = torch.from_numpy(rng.standard_normal((3, R, R, R)) * 0.1).to(DEV)
    x = S.pack_input_pair(om, dl, 0.7, 9.0, 250.0)
    got = x.view(torch.int16).cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    got = got.view(np.float32).reshape(R ** 3, 16).astype(np.float64)
    o, d = om.cpu().numpy().reshape(3, -1).T, dl.cpu().numpy().reshape(3, -1).T
    ref = np.zeros((R ** 3, 16))
    ref[:, 0:3] = C.bf16_round((o * 0.7).astype(np.float32))
    ref[:, 3] = C.bf16_round(np.float32(S.re_feature(250.0)))
    ref[:, 4:7] = C.bf16_round((d * 9.0).astype(np.float32))
    assert np.array_equal(got, ref)
    # (the kernel may fuse a product into the sum: agreement to FP64 rounding, exact for unit weights)
    c = torch.from_numpy(rng.standard_normal((3, R, R, R))).to(DEV)
    out = S.combine3(om, dl, c, 1.0, 3.0, -4.0)
    ref = 1.0 * om + 3.0 * dl + (-4.0) * c
    assert float((out - ref).abs().max()) <= 4e-16 * float(ref.abs().max())
    out = S.combine3(om, dl, None, -3.0, 4.0)
    ref = -3.0 * om + 4.0 * dl
    assert float((out - ref).abs().max()) <= 4e-16 * float(ref.abs().max())
    assert torch.equal(S.combine3(om, dl, None, 1.0, -1.0), om - dl)


def test_correction_form_rollout_small():
    """The correction form end to end at 32^3: it trains, its proposal starts from the extrapolation of
    one plain step (an untrained network's output scale keeps it near that extrapolation), and the
    judge's fallback works as in the persistence form."""
    import workloads

    n = 32
    specs = workloads.surrogate_specs(4, seed=3)
    dx_of = lambda s: 2.0 * (1.0 + 5.0 * s) / (n - 16)
    trajs, res = [], []
    for (sig, re, seed) in specs[:3]:
        snaps, _ = S.make_trajectory(n, dx_of(sig), sig, re, seed, 16, n_buf=2)
        trajs.append(snaps)
        res.append(re)
    net = S.UNet(DEV, seed=0, in_real=7)
    sig, re, seed = specs[3]
    ro0 = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, blocks=2, horizon=4, tol=0.0, n_buf=2, gain=30.0,
                           mode="correct")
    # untrained: the output layer's small initial scale leaves the proposal close to the extrapolation
    assert all(abs(e - x) < 0.5 * x for e, x in zip(ro0["err"], ro0["extrapolation_err"])), ro0
    losses = S.train(net, trajs, res, 4, 300, lr=1e-3, log_every=50, mode="correct", gain=30.0)
    assert losses[-1][1] < losses[0][1]
    ro = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, blocks=3, horizon=4, tol=0.0, n_buf=2, gain=30.0,
                          mode="correct")
    assert not any(ro["accepted"]) and np.isfinite(ro["err"]).all()
    assert np.mean(ro["err"]) < np.mean(ro["persistence_err"]), (ro["err"], ro["persistence_err"])
    ro_all = S.judged_rollout(net, n, dx_of(sig), sig, re, seed, blocks=1, horizon=4, tol=1e9, n_buf=2, gain=30.0,
                              mode="correct")
    assert all(ro_all["accepted"])


def test_misaligned_tensors_are_refused():
    """The 16-byte vector kernels refuse tensors that do not start on 16 bytes (a host-side check)."""
    D, H, W, cin, cout = 2, 8, 32, 16, 32
    x = S.bf16_empty(D * H * W * cin + 8, DEV)
    w = S.bf16_empty(27 * cout * cin, DEV)
    y = torch.empty(D * H * W * cout, dtype=torch.float32, device=DEV)
    with pytest.raises(Exception):
        S.call("sur_conv3d_fwd", x[1:], w, y, D, H, W, cin, cout, 0)
    src = torch.zeros(64 * 8 + 4, dtype=torch.float32, device=DEV)
    out = S.bf16_empty(64 * 8, DEV)
    with pytest.raises(Exception):
        S.call("sur_cast_bf16_ex", src[1:], None, out, None, 64, 8)
    coarse = torch.zeros(8 * 8 + 4, dtype=torch.float32, device=DEV)
    with pytest.raises(Exception):
        S.call("sur_cast_bf16_up", coarse[1:], 1.0, src[:64 * 8], None, out, None, 4, 4, 4, 8)


@pytest.mark.parametrize("c,D,H,W", [(32, 4, 6, 10), (96, 4, 6, 10), (32, 6, 4, 16), (64, 2, 2, 24)])
def test_fused_resample_skip_cast(c, D, H, W):
    """sur_cast_bf16_up equals the separate passes bit for bit: scale 1 = sur_up2_fwd, sur_add and
    sur_cast_bf16_ex; scale 1/8 with the ReLU mask = sur_pool2_bwd, sur_add and sur_cast_bf16_ex (zeros,
    negative activations included), with and without the blocked copy; rows of 8-voxel groups (W % 8 ==
    0) and groups that straddle rows (W = 10)."""
    rng = np.random.default_rng(21 + c + W)
    nv, nc = D * H * W, (D // 2) * (H // 2) * (W // 2)
    coarse = torch.from_numpy(rng.standard_normal(nc * c).astype(np.float32)).to(DEV)
    skip = torch.from_numpy(rng.standard_normal(nv * c).astype(np.float32)).to(DEV)
    act_np = rng.standard_normal(nv * c).astype(np.float32)
    act_np[::6] = 0.0
    act = torch.from_numpy(act_np).to(DEV)
    for scale, up, use_act in ((1.0, "sur_up2_fwd", False), (0.125, "sur_pool2_bwd", True), (1.0, "sur_up2_fwd", True)):
        fine = torch.empty(nv * c, dtype=torch.float32, device=DEV)
        S.call(up, coarse, fine, D, H, W, c)
        S.call("sur_add", fine, skip, fine, nv * c)
        ref_b, ref_k = S.bf16_empty(nv * c, DEV), S.bf16_empty(nv * c, DEV)
        S.call("sur_cast_bf16_ex", fine, act if use_act else None, ref_b, ref_k, nv, c)
        for blocked in (True, False):
            y, yk = S.bf16_empty(nv * c, DEV), S.bf16_empty(nv * c, DEV)
            yk.fill_(7)
            S.call("sur_cast_bf16_up", coarse, scale, skip, act if use_act else None, y, yk if blocked else None,
                   D, H, W, c)
            assert torch.equal(y, ref_b), (scale, use_act, blocked)
            if blocked:
                assert torch.equal(yk, ref_k), (scale, use_act)
            else:
                assert bool((yk == 7).all())


def test_fused_loss_gradient():
    """sur_mse_cast writes the bits of sur_mse followed by sur_cast_bf16_ex of its gradient (BF16 and
    blocked copies) and the same loss up to the order of its FP64 partial sums; training with it
    (loss_and_grad(fused=True), backward(None)) gives the weight gradients of the FP32 path bit for bit."""
    nvox, c, used = 4 * 8 * 16, 32, 3
    g = torch.Generator(device="cpu").manual_seed(5)
    p = torch.randn(nvox * c, generator=g).to(DEV)
    t = torch.randn(nvox * used, generator=g).to(DEV)
    grad = torch.empty_like(p)
    part = torch.empty(1024, dtype=torch.float64, device=DEV)
    S.call("sur_mse", p, t, grad, part, nvox, c, used)
    ref_b, ref_k = S.bf16_empty(nvox * c, DEV), S.bf16_empty(nvox * c, DEV)
    S.call("sur_cast_bf16_ex", grad, None, ref_b, ref_k, nvox, c)
    y, yk = S.bf16_empty(nvox * c, DEV), S.bf16_empty(nvox * c, DEV)
    part2 = torch.empty(1024, dtype=torch.float64, device=DEV)
    S.call("sur_mse_cast", p, t, part2, y, yk, nvox, c, used)
    assert torch.equal(y, ref_b) and torch.equal(yk, ref_k)
    assert abs(part2.sum().item() - part.sum().item()) <= 1e-12 * part.sum().item()
    # the training path
    R = 32
    net = S.UNet(DEV, seed=3)
    x = np.zeros((R, R, R, 16))
    x[..., :4] = C.bf16_round(np.random.default_rng(8).standard_normal((R, R, R, 4)))
    xb = to_bf16_bits(x).reshape(-1)
    tg = torch.randn(R ** 3 * S.USED, generator=g).to(DEV)
    out = net.forward(xb, R, train=True)
    _, gfp = net.loss_and_grad(out, tg, R ** 3)
    net.backward(gfp)
    plain = [w.clone() for w in net.gw]
    out1 = out.clone()
    out2 = net.forward(xb, R, train=True)
    assert torch.equal(out1, out2)
    _, none = net.loss_and_grad(out2, tg, R ** 3, fused=True)
    assert none is None
    net.backward(None)
    for li in range(10):
        assert torch.equal(net.gw[li], plain[li]), li
    with pytest.raises(ValueError):  # the cast gradient is used once
        net.backward(None)
