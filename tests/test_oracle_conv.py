"""Pins of the oracle's direct LGF convolution (Sec. 2.2, Eq. dpoisson_conv): applying the 7-point
Laplacian to the result returns the source (inside the box) and zero (outside it); a delta source
returns the shifted table; translation invariance."""
import numpy as np

from oracle import lgf, native, stencils
import workloads


def _ext_targets(n, pad):
    r = np.arange(-pad, n + pad)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([k.ravel(), j.ravel(), i.ravel()], axis=1), len(r)


def test_laplacian_returns_source_compact_sphere():
    n, dx = 32, 1.0
    s = workloads.compact_random_source(n, 12.0, seed=0)
    tg, m = _ext_targets(n, 2)
    y = native.lgf_direct_targets(s, dx, tg).reshape(m, m, m)
    lap = stencils.laplacian(y, dx)[1:-1, 1:-1, 1:-1]  # valid on [-1, n]^3
    expect = np.pad(s, 1)
    scale = np.abs(s).max()
    assert np.abs(lap - expect).max() < 1e-13 * scale


def test_laplacian_returns_source_asymmetric_dx():
    """A source with no symmetry and dx != 1 (a transposed index or a wrong dx power fails here)."""
    rng = np.random.default_rng(3)
    nz, ny, nx = 6, 9, 13
    s = rng.standard_normal((nz, ny, nx))
    dx = 0.37
    r = [np.arange(-1, m + 1) for m in (nz, ny, nx)]
    k, j, i = np.meshgrid(*r, indexing="ij")
    tg = np.stack([k.ravel(), j.ravel(), i.ravel()], axis=1)
    y = native.lgf_direct_targets(s, dx, tg).reshape(nz + 2, ny + 2, nx + 2)
    lap = stencils.laplacian(y, dx)[1:-1, 1:-1, 1:-1]
    assert np.abs(lap - s).max() < 1e-12 * np.abs(s).max()


def test_delta_source_gives_table():
    n, dx = 10, 0.5
    s = np.zeros((n, n, n))
    m0 = (3, 7, 2)
    s[m0] = 1.0
    y = native.lgf_direct(s, dx)
    cube = lgf.lgf_cube(n)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    expect = dx * dx * cube[np.abs(k - m0[0]), np.abs(j - m0[1]), np.abs(i - m0[2])]
    assert np.array_equal(y, expect)


def test_translation_invariance_and_linearity():
    rng = np.random.default_rng(5)
    n = 12
    s = np.zeros((n, n, n))
    s[2:7, 3:8, 1:6] = rng.standard_normal((5, 5, 5))
    y = native.lgf_direct(s, 1.0)
    s2 = np.roll(s, (2, 1, 3), axis=(0, 1, 2))
    y2 = native.lgf_direct(s2, 1.0)
    assert np.allclose(y2[2:, 1:, 3:], y[:-2, :-1, :-3], rtol=0, atol=1e-15 * np.abs(y).max())
    y3 = native.lgf_direct(2.5 * s - s2, 1.0)
    assert np.allclose(y3, 2.5 * y - y2, rtol=0, atol=1e-14 * np.abs(y).max())
