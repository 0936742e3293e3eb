"""Seeded synthetic inputs shared by the oracle-side tests, the GPU-side tests and the benchmark.

This module holds no arithmetic of the method itself (no lattice Green's function, no stencil,
no integrating factor, no time stepping).  It only draws random numbers and samples analytic
initial fields onto the staggered grid, so that the oracle and the GPU path can be fed the
very same arrays.

Layout of every grid field: a float64 numpy array of shape [nz, ny, nx] per scalar component
(x fastest), vector fields stacked as [3, nz, ny, nx] in component order (1), (2), (3).

Grid geometry (the paper's grid-cell figure is missing; this is the reading under which every
point operator of the operator appendix is a centred second-order difference): vertex (i, j, k)
sits at ((i, j, k) - c) * dx with c = (n - 1) / 2 per axis, so the box is centred on the origin.
Edge (1) of index (i, j, k) sits half a cell below the vertex along x, i.e. at (i - 1/2, j, k),
and cyclically edge (2) at (i, j - 1/2, k) and edge (3) at (i, j, k - 1/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Sizes of the batched workload (one problem = one cubic box).
BATCH_SIZES = (48, 64, 96, 128, 160, 192)


def compact_random_source(n: int = 32, radius: float = 12.0, seed: int = 0) -> np.ndarray:
    """Scalar source for the single Poisson-solve case: i.i.d. N(0,1) values on the cells whose
    index lies within `radius` of the box centre ((n-1)/2 per axis), zero elsewhere, with the
    mean over the sphere cells removed.  Returns float64 [n, n, n]."""
    rng = np.random.default_rng(seed)
    c = (n - 1) / 2.0
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    mask = (i - c) ** 2 + (j - c) ** 2 + (k - c) ** 2 <= radius * radius
    s = np.zeros((n, n, n))
    vals = rng.standard_normal(int(mask.sum()))
    vals -= vals.mean()
    s[mask] = vals
    return s


def random_field(shape, seed: int, integer: bool = False, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Seeded dense field, either N(0,1) or integers in [lo, hi] stored as float64."""
    rng = np.random.default_rng(seed)
    if integer:
        return rng.integers(lo, hi + 1, size=shape).astype(np.float64)
    return rng.standard_normal(shape)


@dataclass
class Ring:
    """Gaussian-core vortex ring, axis z, centred in the box.

    omega_theta(rho, z) = Gamma / (pi sigma^2) exp(-((rho - rho_c(theta))^2 + z^2) / sigma^2),
    rho_c(theta) = R (1 + eps * sum_{m=1..8} A_m cos(m theta + phi_m)), with A_m ~ U[-1, 1] and
    phi_m ~ U[0, 2 pi) drawn from `seed` (eps = 0 gives the unperturbed ring)."""

    R: float = 1.0
    sigma: float = 0.2
    gamma: float = 1.0
    eps: float = 0.0
    seed: int = 0
    zc: float = 0.0  # height of the ring plane above the box centre

    def modes(self):
        rng = np.random.default_rng(self.seed)
        A = rng.uniform(-1.0, 1.0, 8)
        phi = rng.uniform(0.0, 2.0 * math.pi, 8)
        return A, phi

    def omega(self, x, y, z):
        """Vorticity (wx, wy, wz) at points (arrays of equal shape)."""
        A, phi = self.modes()
        z = z - self.zc
        rho = np.sqrt(x * x + y * y)
        th = np.arctan2(y, x)
        rc = np.full_like(rho, self.R)
        if self.eps != 0.0:
            pert = np.zeros_like(rho)
            for m in range(8):
                pert += A[m] * np.cos((m + 1) * th + phi[m])
            rc = self.R * (1.0 + self.eps * pert)
        wt = self.gamma / (math.pi * self.sigma ** 2) * np.exp(-((rho - rc) ** 2 + z * z) / self.sigma ** 2)
        return -wt * np.sin(th), wt * np.cos(th), np.zeros_like(wt)

    def extent(self, cutoff: float = 9.0):
        """(rmax, zmax): beyond rho = rmax or |z - zc| = zmax the Gaussian core is below
        exp(-cutoff^2)."""
        return self.R * (1.0 + 10.0 * abs(self.eps)) + cutoff * self.sigma, cutoff * self.sigma + abs(self.zc)


@dataclass
class BumpRing:
    """The "fat" vortex ring of the refinement studies (Sec. 6.1, Eq. initial_omega_bump), axis z,
    centred at the origin:

        omega_theta(r, z) = Gamma / (alpha R^2) exp(-4 s^2 / (R^2 - s^2))  for s <= R, else 0,
        s^2 = z^2 + (r - R)^2,  omega_z = 0,

    with alpha = 0.54857674, the value printed with the equation.  The equation prints alpha as a
    factor, but the stated purpose (omega_theta integrates to Gamma over a meridional half-plane) needs
    it as a divisor: alpha is the integral of the unscaled bump, 2 pi int_0^1 exp(-4t^2/(1-t^2)) t dt
    = 0.548576742...  Its vorticity is compactly supported (0 <= r <= 2R, |z| <= R) and smooth, also at
    the axis."""

    R: float = 1.0
    gamma: float = 1.0
    alpha: float = 0.54857674

    def omega_theta(self, r, z):
        s2 = z * z + (r - self.R) ** 2
        inside = s2 < self.R * self.R
        d = np.where(inside, self.R * self.R - s2, 1.0)
        return np.where(inside, self.gamma / (self.alpha * self.R ** 2) * np.exp(-4.0 * s2 / d), 0.0)

    def omega(self, x, y, z):
        rho = np.sqrt(x * x + y * y)
        th = np.arctan2(y, x)
        wt = self.omega_theta(rho, z)
        return -wt * np.sin(th), wt * np.cos(th), np.zeros_like(wt)

    def extent(self, cutoff: float = 9.0):
        """(rmax, zmax): the vorticity vanishes beyond rho = rmax or |z| = zmax."""
        return 2.0 * self.R, self.R


def _gauss_legendre(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * x, 0.5 * w  # nodes on [-1/2, 1/2], weights summing to 1


def ring_edge_vorticity(n: int, dx: float, ring, quad: int = 4, cutoff: float = 9.0,
                        origin: float | None = None) -> np.ndarray:
    """Discrete vorticity w on the edges: w(q) = (flux of omega_q through the dual face of the
    edge) / dx^2, each flux by quad x quad Gauss-Legendre.  Returns float64 [3, n, n, n].

    Vertex (0, 0, 0) sits at (origin, origin, origin); the default origin -(n - 1) dx / 2 centres the
    box on the ring.  Cells outside the ring's extent (for the Gaussian core, further than `cutoff`
    core radii from the nominal centreline, where it is below exp(-81)) are skipped."""
    w = np.zeros((3, n, n, n))
    o = -(n - 1) / 2.0 * dx if origin is None else float(origin)
    gx, gw = _gauss_legendre(quad)
    rmax, zmax = ring.extent(cutoff)
    idx = np.arange(n)
    for q in range(3):
        # edge (q) position offsets in index units: -1/2 along axis q
        off = [0.0, 0.0, 0.0]
        off[q] = -0.5
        xs = o + (idx + off[0]) * dx
        ys = o + (idx + off[1]) * dx
        zs = o + (idx + off[2]) * dx
        ix = np.nonzero(np.abs(xs) <= rmax + dx)[0]
        iy = np.nonzero(np.abs(ys) <= rmax + dx)[0]
        iz = np.nonzero(np.abs(zs) <= zmax + dx)[0]
        if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
            continue
        # the dual face of edge (q) spans the two axes other than q
        a1, a2 = [a for a in range(3) if a != q]
        acc = np.zeros((len(iz), len(iy), len(ix)))
        Z, Y, X = np.meshgrid(zs[iz], ys[iy], xs[ix], indexing="ij")
        base = [X, Y, Z]
        for u, wu in zip(gx, gw):
            for v, wv in zip(gx, gw):
                p = [base[0], base[1], base[2]]
                p = [pp.copy() for pp in p]
                p[a1] = p[a1] + u * dx
                p[a2] = p[a2] + v * dx
                comp = ring.omega(p[0], p[1], p[2])[q]
                acc += wu * wv * comp
        w[q][np.ix_(iz, iy, ix)] = acc
    return w


def ring_case(name: str):
    """Named ring workloads: (n, dx, Ring, Re, CFL)."""
    if name == "step128":
        return 128, 1.0 / 24.0, Ring(R=1.0, sigma=0.2, gamma=1.0, eps=1e-4, seed=1), 500.0, 0.5
    if name == "conv256":
        return 256, 1.0 / 48.0, Ring(R=1.0, sigma=0.1, gamma=1.0), 500.0, 0.5
    raise KeyError(name)


def small_ring_case(n: int = 32, seed: int = 1):
    """A coarse ring that fits a small box with an 8-cell margin: same physics as the 128^3 step
    case (sigma = 0.2 R, Re = 500, CFL = 0.5) at dx = 2 (R + 5 sigma) / (n - 16)."""
    R, sig = 1.0, 0.2
    dx = 2.0 * (R + 5.0 * sig) / (n - 16)
    return n, dx, Ring(R=R, sigma=sig, gamma=1.0, eps=1e-4, seed=seed), 500.0, 0.5


def batch_specs(count: int = 32, seed: int = 0, sizes=None):
    """Uneven batch: per problem (n, dx, Ring, Re, CFL) with n ~ U{48..192} (or U(sizes)), R = 1,
    sigma/R ~ U[0.1, 0.3], dx = 2 (R + 5 sigma) / (n - 16)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.choice(BATCH_SIZES if sizes is None else tuple(sizes)))
        sr = float(rng.uniform(0.1, 0.3))
        dx = 2.0 * (1.0 + 5.0 * sr) / (n - 16)
        out.append((n, dx, Ring(R=1.0, sigma=sr, gamma=1.0, eps=1e-4, seed=1000 + b), 500.0, 0.5))
    return out


def sample_targets(n: int, count: int, seed: int = 0) -> np.ndarray:
    """`count` distinct seeded cell indices of an n^3 box as int64 [count, 3] in (k, j, i) order."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n ** 3, size=min(count, n ** 3), replace=False)
    flat.sort()
    k = flat // (n * n)
    j = (flat // n) % n
    i = flat % n
    return np.stack([k, j, i], axis=1).astype(np.int64)


def surrogate_specs(count: int, seed: int = 0):
    """Trajectory parameters of the surrogate's training data: (sigma/R, Re, perturbation seed) with
    sigma/R ~ U[0.1, 0.3] and Re ~ U[250, 1000]; the ring starts half a radius below the centre."""
    rng = np.random.default_rng(seed)
    return [(float(rng.uniform(0.1, 0.3)), float(rng.uniform(250.0, 1000.0)), 2000 + i) for i in range(count)]


def compact_blob(shape, centres, radius: float, seed: int, ncomp: int = 3) -> np.ndarray:
    """Compactly supported random field for parity tests on elongated boxes: i.i.d. N(0,1) values
    times the smooth window (1 - r^2 / radius^2)^3 around each centre (index units, (k, j, i)),
    zero where r >= radius, the windows of several centres added.  Returns float64
    [ncomp, *shape]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    win = np.zeros(shape)
    for (ck, cj, ci) in centres:
        r2 = ((k - ck) ** 2 + (j - cj) ** 2 + (i - ci) ** 2) / (radius * radius)
        win += np.where(r2 < 1.0, (1.0 - r2) ** 3, 0.0)
    return rng.standard_normal((ncomp,) + tuple(shape)) * win
