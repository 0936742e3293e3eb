"""Oracle: the volume integrals of an isolated vortex ring (Sec. 6.2, Eq. int_quantities) on the
staggered box.  Test infrastructure only.

    I = 1/2 int x cross w,   K = int u . (x cross w),   E = 1/2 int |w|^2,   J = int u . w,
    X = 1/2 int ((x cross w) . I / |I|^2) x,            (u_inf = 0)

with the vorticity w = M_supp C u: zero outside the box (the footnote of Sec. 6.2) and on the edges
closer than n_buf points to a face, where the curl of the zero-extended velocity is not the flow's
vorticity (the velocity does not vanish at the faces, so the outermost edges see a spurious jump).

Discretisation (a reading; the paper does not spell it out): every integral is a sum over the box
times dx^3.  I, E and X are linear or quadratic in w alone, so each of their terms is taken at the
position of the edge that carries it: (x cross w)_1 x_p = y w_3 x_p - z w_2 x_p with w_3 at edge (3)
positions and w_2 at edge (2) positions, and so on.  K and J multiply u and w, which sit at different
points: both are averaged to cell centres (u^(1) from its two faces along x, w^(1) from its four edges
around the cell along y and z, and cyclically) and multiplied there.

Positions: the vertex (i, j, k) is at origin + (i, j, k) dx; face (q) sits half a cell back on the two
axes other than q, edge (q) half a cell back along q, the cell centre half a cell back on all three.
"""
from __future__ import annotations

import numpy as np

from . import ifherk, stencils


def _coords(shape, dx, origin, back):
    """x, y, z of the points with index offsets -1/2 on the axes flagged in `back` (x, y, z order)."""
    nz, ny, nx = shape
    x = origin[0] + (np.arange(nx) - 0.5 * back[0]) * dx
    y = origin[1] + (np.arange(ny) - 0.5 * back[1]) * dx
    z = origin[2] + (np.arange(nz) - 0.5 * back[2]) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def integrals(u: np.ndarray, w: np.ndarray, dx: float, origin) -> dict:
    """The quantities of Eq. int_quantities for face velocity u and edge vorticity w [3, nz, ny, nx]."""
    shape = w.shape[1:]
    dv = dx ** 3
    # edge positions: edge (q) is half a cell back along axis q
    pos = [_coords(shape, dx, origin, [1 if a == q else 0 for a in range(3)]) for q in range(3)]
    # x cross w, term by term at the edge of each vorticity component:
    # (x cross w)_q = x_{q+1} w_{q+2} - x_{q+2} w_{q+1}  (indices mod 3)
    S = np.zeros(3)
    M = np.zeros((3, 3))
    for q in range(3):
        a, b = (q + 1) % 3, (q + 2) % 3
        # + x_a w_b at edge (b) positions, - x_b w_a at edge (a) positions
        S[q] = (pos[b][a] * w[b]).sum() - (pos[a][b] * w[a]).sum()
        for p in range(3):
            M[q, p] = (pos[b][a] * pos[b][p] * w[b]).sum() - (pos[a][b] * pos[a][p] * w[a]).sum()
    I = 0.5 * dv * S
    E = 0.5 * dv * float((w * w).sum())
    # cell-centre averages (zero outside the box)
    sh = stencils.sh
    uc = np.stack([0.5 * (u[0] + sh(u[0], di=-1)), 0.5 * (u[1] + sh(u[1], dj=-1)), 0.5 * (u[2] + sh(u[2], dk=-1))])
    wc = np.stack([
        0.25 * (w[0] + sh(w[0], dj=-1) + sh(w[0], dk=-1) + sh(w[0], dj=-1, dk=-1)),
        0.25 * (w[1] + sh(w[1], dk=-1) + sh(w[1], di=-1) + sh(w[1], dk=-1, di=-1)),
        0.25 * (w[2] + sh(w[2], di=-1) + sh(w[2], dj=-1) + sh(w[2], di=-1, dj=-1)),
    ])
    xc = _coords(shape, dx, origin, [1, 1, 1])
    xw = np.stack([xc[1] * wc[2] - xc[2] * wc[1], xc[2] * wc[0] - xc[0] * wc[2], xc[0] * wc[1] - xc[1] * wc[0]])
    K = dv * float((uc * xw).sum())
    J = dv * float((uc * wc).sum())
    X = 0.5 * dv * (I @ M) / float(I @ I)
    return {"I": I, "K": K, "E": E, "J": J, "X": X}


def of_velocity(u: np.ndarray, dx: float, origin, n_buf: int) -> dict:
    """The integrals of a face velocity u with its own vorticity w = M_supp C u (support = box shrunk
    by n_buf points)."""
    return integrals(u, ifherk.inner_mask(u.shape[1:], n_buf) * stencils.curl(u, dx), dx, origin)


def box_origin(shape, dx):
    """Origin that puts the box centre at 0 (the ring workloads' convention: vertex i at (i - (n-1)/2) dx)."""
    nz, ny, nx = shape
    return (-(nx - 1) / 2.0 * dx, -(ny - 1) / 2.0 * dx, -(nz - 1) / 2.0 * dx)


def saffman_speed(gamma: float, R: float, sigma: float) -> float:
    """Propagation speed of a thin Gaussian-core ring (Sec. 6.3, Eq. u_saffman) without its error term:
    Gamma / (4 pi R) (log(8 / eps) - beta_0), eps = sigma / R, beta_0 = (1 - gamma_E + log 2) / 2."""
    euler = 0.5772156649015329
    beta0 = 0.5 * (1.0 - euler + np.log(2.0))
    return gamma / (4.0 * np.pi * R) * (np.log(8.0 * R / sigma) - beta0)
