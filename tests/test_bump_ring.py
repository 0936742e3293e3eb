"""The bump ring of the refinement studies (Sec. 6.1, Eq. initial_omega_bump).  Its printed constant
alpha = 0.54857674 is the integral of the unscaled bump over a meridional half-plane, so omega_theta
integrates to Gamma with alpha as a divisor (the printed equation has it as a factor, which would give
0.30 Gamma); the sampled edge vorticity carries that circulation through the half-plane of dual faces
on y = 0."""
import math

import numpy as np
from scipy.integrate import dblquad, quad

import workloads


def test_alpha_makes_omega_theta_integrate_to_gamma():
    ring = workloads.BumpRing(R=1.3, gamma=2.0)
    # over the disc s <= R of the meridional half-plane, in polar coordinates about the core centre
    f = lambda s: ring.omega_theta(ring.R + s, 0.0) * 2.0 * math.pi * s  # noqa: E731 (radial symmetry in s)
    total, err = quad(f, 0.0, ring.R, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(total / ring.gamma - 1.0) < 1e-8, total  # alpha is printed to 8 digits
    # the same integral over the half-plane in (r, z), with the sampler's own r, z dependence
    total2, _ = dblquad(lambda z, r: ring.omega_theta(np.array(r), np.array(z)), 0.0, 2 * ring.R,
                        -ring.R, ring.R, epsabs=1e-10, epsrel=1e-9)
    assert abs(total2 / ring.gamma - 1.0) < 1e-7
    # the printed constant is the integral of the unscaled bump exp(-4 t^2 / (1 - t^2)) over the unit disc
    bump, _ = quad(lambda t: math.exp(-4 * t * t / (1 - t * t)) * 2 * math.pi * t, 0.0, 1.0, epsabs=1e-15,
                   epsrel=1e-14, limit=200)
    assert abs(bump - 0.54857674) < 5e-9


def test_bump_is_compact_and_flat_at_its_edge():
    ring = workloads.BumpRing()
    assert ring.omega_theta(np.array(2.0), np.array(0.0)) == 0.0  # s = R: at the axis side and the outer rim
    assert ring.omega_theta(np.array(0.0), np.array(0.0)) == 0.0
    assert ring.omega_theta(np.array(1.0), np.array(1.0)) == 0.0
    assert ring.omega_theta(np.array(1.0), np.array(0.0)) == ring.gamma / (ring.alpha * ring.R ** 2)
    # all derivatives vanish at s = R: the value falls faster than any power of the distance
    assert ring.omega_theta(np.array(1.99), np.array(0.0)) < 1e-80
    assert ring.omega_theta(np.array(1.999), np.array(0.0)) == 0.0  # exp(-1996) underflows


def test_sampled_circulation_through_the_half_plane():
    """The edge vorticity is the dual-face flux of omega / dx^2; on a box centred on the ring with an
    even n, the dual faces of edges (2) with j = n/2 tile the plane y = 0, and those with x > 0 the
    half-plane that the ring's core crosses once: their summed flux is Gamma (to the face quadrature)."""
    ring = workloads.BumpRing()
    n, dx = 40, 0.125
    w = workloads.ring_edge_vorticity(n, dx, ring)
    x = (np.arange(n) - (n - 1) / 2.0) * dx  # x of edge (2) (not shifted along x)
    flux = w[1][:, n // 2, :][:, x > 0].sum() * dx * dx
    # (alpha is printed to 8 digits: 0.54857674 against 0.5485767423, a relative 4e-9)
    assert abs(flux - ring.gamma) < 1e-8, flux
    flux_neg = w[1][:, n // 2, :][:, x < 0].sum() * dx * dx  # the other crossing: -Gamma
    assert abs(flux_neg + ring.gamma) < 1e-8
