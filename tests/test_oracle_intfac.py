"""Pins of the oracle's integrating factor (Sec. 2.3, Appendix B): the paper's decay example,
mass and variance of the 1D kernel, the semigroup property, the generator dE/dalpha = L E and the
plane-wave eigenvalue exp(alpha sigma(xi))."""
import math

import numpy as np
import pytest

from oracle import intfac, stencils
import workloads


def test_paper_decay_example(paper_values):
    ex = paper_values["if_decay_example"]
    for alpha, n_first in ex["cases"]:
        w = intfac.weights(alpha)
        ratio = w / w[0]
        first = int(np.nonzero(ratio < ex["threshold"])[0][0])
        assert first == n_first, (alpha, first)


@pytest.mark.parametrize("alpha", [0.01, 0.0237, 0.5, 2.0])
def test_kernel_mass_and_variance(alpha):
    w = intfac.weights(alpha)
    k = np.arange(len(w))
    assert abs(w[0] + 2 * w[1:].sum() - 1.0) < 1e-15          # sum_k I_k(z) = e^z
    assert abs(2 * (k * k * w).sum() - 2 * alpha) < 1e-14      # variance of the lattice heat kernel


def _compact(n, inner, seed):
    h = np.zeros((n, n, n))
    h[inner:-inner, inner:-inner, inner:-inner] = workloads.random_field((n - 2 * inner,) * 3, seed)
    return h


def test_semigroup():
    n = 30
    h = _compact(n, 11, 1)
    a, b = 0.03, 0.05
    lhs = intfac.apply(intfac.apply(h, a), b)
    rhs = intfac.apply(h, a + b)
    assert np.abs(lhs - rhs).max() < 1e-15 * np.abs(h).max() * 10


def test_generator():
    n = 24
    h = _compact(n, 9, 2)
    lap = stencils.laplacian(h, 1.0)
    errs = []
    for alpha in (1e-3, 5e-4):
        d = (intfac.apply(h, alpha) - h) / alpha
        errs.append(np.abs(d - lap).max())
    assert errs[1] < 0.6 * errs[0]  # first-order convergence in alpha
    # with the next term of exp(alpha L) the remainder drops to O(alpha^2)
    lap2 = stencils.laplacian(lap, 1.0)
    alpha = 5e-4
    d = (intfac.apply(h, alpha) - h) / alpha
    assert np.abs(d - lap - 0.5 * alpha * lap2).max() < 1e-5 * np.abs(lap).max()


def test_plane_wave_eigenvalue():
    n = 30
    alpha = 0.08
    xi = np.array([0.7, -1.1, 2.3])
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    h = np.cos(xi[0] * i + xi[1] * j + xi[2] * k)
    out = intfac.apply(h, alpha)
    sigma = 2 * np.cos(xi).sum() - 6.0
    R = len(intfac.weights(alpha)) - 1
    inner = slice(R, n - R)
    assert np.abs(out[inner, inner, inner] - math.exp(alpha * sigma) * h[inner, inner, inner]).max() < 1e-14


def test_negative_alpha_rejected():
    with pytest.raises(ValueError):
        intfac.weights(-0.1)
