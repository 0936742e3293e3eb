"""GPU parity of the LGF convolution (Sec. 2.2, Eq. dpoisson_conv) against the oracle's direct
lattice sum, through the C ABI.  FP64 within 1e-12 and FP32 within 1e-6, relative to max|oracle|."""
import numpy as np
import pytest
import torch

import paper_1601_00035_amd as nslgf
import workloads
from oracle import native

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_conv(src_np, dx, dtype=torch.float64):
    t = torch.from_numpy(src_np).to(DEV, dtype)
    return nslgf.lgf_convolve(t, dx).double().cpu().numpy()


def test_compact_sphere_32_fp64_fp32():
    s = workloads.compact_random_source(32, 12.0, seed=0)
    ref = native.lgf_direct(s, 1.0)
    assert rel(gpu_conv(s, 1.0), ref) < 1e-12
    assert rel(gpu_conv(s, 1.0, torch.float32), ref) < 1e-6


@pytest.mark.parametrize("shape", [(9, 13, 20), (33, 24, 40), (8, 12, 70), (5, 6, 150), (6, 150, 5), (150, 5, 6),
                                   (4, 5, 170), (5, 170, 4), (170, 4, 5), (1, 1, 1), (2, 3, 1), (17, 17, 17)])
def test_ragged_boxes_fp64(shape):
    """Non-cubic boxes whose padded sizes exercise radix 2, 3, 4, 5 and 8, several column tiles and a
    ragged last tile; an axis of 150 (170) pads to 320 (384) on the row, y-column and fused z passes,
    whose column passes exchange real and imaginary parts through LDS one after the other."""
    rng = np.random.default_rng(sum(shape))
    s = rng.standard_normal(shape)
    dx = 0.37
    ref = native.lgf_direct(s, dx)
    assert rel(gpu_conv(s, dx), ref) < 1e-12, shape
    assert rel(gpu_conv(s, dx, torch.float32), ref) < 2e-6, shape


def test_three_components_and_delta():
    n = 24
    s = np.zeros((3, n, n, n))
    s[0, 3, 5, 7] = 1.0
    s[1] = workloads.compact_random_source(n, 9.0, seed=4)
    s[2, 20, 1, 2] = -2.0
    dx = 0.5
    ref = np.stack([native.lgf_direct(s[q], dx) for q in range(3)])
    out = gpu_conv(s, dx)
    assert rel(out, ref) < 1e-12
    for q in range(3):
        assert rel(out[q], ref[q]) < 1e-12


def test_zero_source_and_linearity():
    n = 20
    z = np.zeros((n, n, n))
    assert not gpu_conv(z, 1.0).any()
    rng = np.random.default_rng(9)
    a, b = rng.standard_normal((2, n, n, n))
    ya, yb, yab = gpu_conv(a, 1.0), gpu_conv(b, 1.0), gpu_conv(2 * a - 3 * b, 1.0)
    assert rel(yab, 2 * ya - 3 * yb) < 1e-13


def test_laplacian_returns_source_128():
    """At 128^3 (the IF-HERK step size) the 7-point Laplacian of the result equals the source
    away from the box faces (where the stencil would need values outside the box)."""
    n = 128
    s = workloads.compact_random_source(n, 40.0, seed=2)
    y = torch.from_numpy(gpu_conv(s, 1.0)).to(DEV)
    lap = nslgf.stencil("laplacian", y, 1.0).cpu().numpy()
    inner = (slice(1, -1),) * 3
    assert np.abs(lap[inner] - s[inner]).max() < 1e-12 * np.abs(s).max()


@pytest.mark.parametrize("n,dtype,tol", [(128, torch.float64, 1e-12), (256, torch.float64, 1e-12),
                                         (256, torch.float32, 1e-6)])
def test_ring_vorticity_sampled(n, dtype, tol):
    """Full-size boxes in the benchmark's launch configuration (three vorticity components at once),
    checked at seeded sample points against direct sums at those points."""
    if n == 256:
        _, dx, ring, _, _ = workloads.ring_case("conv256")
    else:
        _, dx, ring, _, _ = workloads.ring_case("step128")
    w = workloads.ring_edge_vorticity(n, dx, ring)
    out = nslgf.lgf_convolve(torch.from_numpy(w).to(DEV, dtype), dx).double().cpu().numpy()
    tg = workloads.sample_targets(n, 64, seed=n)
    tg = np.concatenate([tg, np.array([[0, 0, 0], [n - 1, n - 1, n - 1], [n // 2, n // 2, n // 2]])])
    for q in (0, 1):
        ref = native.lgf_direct_targets(w[q], dx, tg)
        got = out[q][tg[:, 0], tg[:, 1], tg[:, 2]]
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() < tol * scale, (q, np.abs(got - ref).max() / scale)
    assert not out[2].any()  # omega_z = 0 convolves to exactly 0


@pytest.mark.parametrize("shape", [(200, 100, 9), (100, 250, 20)])
def test_fft_plans_agree(shape):
    """Every column-pass plan variant (narrow, wide, fewer elements per thread) at
    padded lengths 256 and 512 along y and z, with ragged column tiles, against direct sums at seeded
    sample points, and against each other."""
    rng = np.random.default_rng(shape[0])
    s = rng.standard_normal(shape)
    dx = 0.21
    nz, ny, nx = shape
    flat = rng.choice(nz * ny * nx, size=48, replace=False)
    tg = np.stack([flat // (ny * nx), (flat // nx) % ny, flat % nx], axis=1).astype(np.int64)
    tg = np.concatenate([tg, np.array([[0, 0, 0], [nz - 1, ny - 1, nx - 1]])])
    ref = native.lgf_direct_targets(s, dx, tg)
    scale = np.abs(ref).max()
    outs = {}
    try:
        for choice in (0, 1, 2):
            nslgf.set_fft_plan(choice)
            for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-6)):
                out = gpu_conv(s, dx, dtype)
                got = out[tg[:, 0], tg[:, 1], tg[:, 2]]
                assert np.abs(got - ref).max() < tol * scale, (choice, dtype, np.abs(got - ref).max() / scale)
                outs[(choice, dtype)] = out
    finally:
        nslgf.set_fft_plan(-1)
    for choice in (1, 2):
        assert rel(outs[(choice, torch.float64)], outs[(0, torch.float64)]) < 1e-13, choice
    with pytest.raises(nslgf.NslgfError):
        nslgf.set_fft_plan(3)
    with pytest.raises(nslgf.NslgfError):
        nslgf.set_fft_plan(-3)


@pytest.mark.parametrize("choice", [-1, 0, 1, 2])
def test_repeated_solves_bitwise(choice):
    """Repeated solves of one source give bitwise equal results in every plan variant and dtype (no
    order-dependent reduction and no race between the workgroup's threads), at padded lengths 256 and
    512 along y and z."""
    rng = np.random.default_rng(11)
    s = torch.from_numpy(rng.standard_normal((2, 200, 100, 9))).to(DEV)
    try:
        nslgf.set_fft_plan(choice)
        for dtype in (torch.float64, torch.float32):
            src = s.to(dtype)
            first = nslgf.lgf_convolve(src, 0.5)
            for _ in range(4):
                assert torch.equal(nslgf.lgf_convolve(src, 0.5), first), (choice, dtype)
    finally:
        nslgf.set_fft_plan(-1)


def test_fft_plan_autotune():
    """The autotuner picks existing variants for padded lengths 512 (z) and 256 (y), and its plan
    matches the direct sum; plans of other choices are unaffected."""
    shape = (200, 100, 9)
    rng = np.random.default_rng(7)
    s = rng.standard_normal(shape)
    dx = 0.3
    tg = np.array([[0, 0, 0], [199, 99, 8], [100, 50, 4], [13, 77, 2]], dtype=np.int64)
    ref = native.lgf_direct_targets(s, dx, tg)
    try:
        nslgf.set_fft_plan(nslgf.FFT_PLAN_AUTOTUNE)
        for dtype, tol, valid in ((torch.float64, 1e-12, (0, 1, 2)), (torch.float32, 1e-6, (0, 1, 2))):
            vy, vz = nslgf.plan_info(9, 100, 200, dtype)
            assert vy in valid and vz in valid, (dtype, vy, vz)
            out = gpu_conv(s, dx, dtype)
            got = out[tg[:, 0], tg[:, 1], tg[:, 2]]
            assert np.abs(got - ref).max() < tol * np.abs(ref).max()
    finally:
        nslgf.set_fft_plan(-1)
    assert nslgf.plan_info(9, 100, 200, torch.float64) == (0, 2)  # the default table in FP64
    assert nslgf.plan_info(9, 100, 200, torch.float32) == (0, 1)  # and in FP32 (narrow y, wide z)


def test_invalid_arguments():
    t = torch.zeros((4, 4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(nslgf.NslgfError):
        nslgf.lgf_convolve(t, -1.0)
    with pytest.raises(nslgf.NslgfError):
        nslgf.lgf_convolve(t, 1.0, out=t)
    big = torch.zeros((1, 1, 300), dtype=torch.float64, device=DEV)
    with pytest.raises(nslgf.NslgfError):
        nslgf.lgf_convolve(big, 1.0)
    with pytest.raises(ValueError):
        nslgf.lgf_convolve(torch.zeros((4, 4, 4), dtype=torch.float64), 1.0)
    # empty boxes are refused
    with pytest.raises((nslgf.NslgfError, ValueError)):
        nslgf.lgf_convolve(torch.zeros((0, 4, 4), dtype=torch.float64, device=DEV), 1.0)
