"""Oracle: point operators of the staggered grid (Appendix A).  Test infrastructure only.

Every field is one float64 array [nz, ny, nx] per component (index [k, j, i]); vector fields are
[3, nz, ny, nx] with components (1), (2), (3).  All values outside the box are zero (the mask
operators of Sec. 4.1): each operator reads its input with zero extension and returns values on
the box only, i.e. it computes M A M x.

Components (2) and (3) follow from the printed component (1) by the cyclic permutation of
(component, axis): 1 -> 2 -> 3 -> 1 together with x -> y -> z -> x.
"""
from __future__ import annotations

import numpy as np


def sh(a: np.ndarray, di: int = 0, dj: int = 0, dk: int = 0) -> np.ndarray:
    """Zero-extended shift: out[k, j, i] = a[k + dk, j + dj, i + di] (0 outside the array)."""
    nz, ny, nx = a.shape
    out = np.zeros_like(a)

    def rng(n, d):
        lo_o, hi_o = max(0, -d), min(n, n - d)
        return slice(lo_o, hi_o), slice(lo_o + d, hi_o + d)

    ok, ik = rng(nz, dk)
    oj, ij = rng(ny, dj)
    oi, ii = rng(nx, di)
    if ok.start < ok.stop and oj.start < oj.stop and oi.start < oi.stop:
        out[ok, oj, oi] = a[ik, ij, ii]
    return out


def grad(c: np.ndarray, dx: float) -> np.ndarray:
    """G: cells -> faces.  dx [Gc]^(1)_{ijk} = c_{i+1,j,k} - c_{ijk}."""
    return np.stack([sh(c, di=1) - c, sh(c, dj=1) - c, sh(c, dk=1) - c]) / dx


def div(f: np.ndarray, dx: float) -> np.ndarray:
    """Dbar = -G^T: faces -> cells.
    dx [Dbar f]_{ijk} = sum_q f^(q)_{ijk} - f^(1)_{i-1,j,k} - f^(2)_{i,j-1,k} - f^(3)_{i,j,k-1}."""
    return (f[0] + f[1] + f[2] - sh(f[0], di=-1) - sh(f[1], dj=-1) - sh(f[2], dk=-1)) / dx


def curl(f: np.ndarray, dx: float) -> np.ndarray:
    """C: faces -> edges.  dx [Cf]^(1)_{ijk} = f^(2)_{ijk} - f^(2)_{i,j,k+1} + f^(3)_{i,j+1,k} - f^(3)_{ijk}."""
    f1, f2, f3 = f
    e1 = f2 - sh(f2, dk=1) + sh(f3, dj=1) - f3
    e2 = f3 - sh(f3, di=1) + sh(f1, dk=1) - f1
    e3 = f1 - sh(f1, dj=1) + sh(f2, di=1) - f2
    return np.stack([e1, e2, e3]) / dx


def curl_bar(e: np.ndarray, dx: float) -> np.ndarray:
    """Cbar = C^T: edges -> faces.  dx [Cbar e]^(1)_{ijk} = e^(2)_{i,j,k-1} - e^(2)_{ijk} + e^(3)_{ijk} - e^(3)_{i,j-1,k}."""
    e1, e2, e3 = e
    f1 = sh(e2, dk=-1) - e2 + e3 - sh(e3, dj=-1)
    f2 = sh(e3, di=-1) - e3 + e1 - sh(e1, dk=-1)
    f3 = sh(e1, dj=-1) - e1 + e2 - sh(e2, di=-1)
    return np.stack([f1, f2, f3]) / dx


def div_edge(e: np.ndarray, dx: float) -> np.ndarray:
    """D: edges -> vertices.  dx [De]_{ijk} = e^(1)_{i+1,j,k} + e^(2)_{i,j+1,k} + e^(3)_{i,j,k+1} - sum_q e^(q)_{ijk}."""
    e1, e2, e3 = e
    return (sh(e1, di=1) + sh(e2, dj=1) + sh(e3, dk=1) - e1 - e2 - e3) / dx


def grad_vertex(v: np.ndarray, dx: float) -> np.ndarray:
    """Gbar = -D^T: vertices -> edges.  dx [Gbar v]^(1)_{ijk} = v_{ijk} - v_{i-1,j,k}."""
    return np.stack([v - sh(v, di=-1), v - sh(v, dj=-1), v - sh(v, dk=-1)]) / dx


def laplacian(a: np.ndarray, dx: float) -> np.ndarray:
    """7-point Laplacian of one scalar component: dx^2 [La] = -6a + sum of the six neighbours."""
    return (-6.0 * a + sh(a, di=1) + sh(a, di=-1) + sh(a, dj=1) + sh(a, dj=-1) + sh(a, dk=1) + sh(a, dk=-1)) / (dx * dx)


def nonlinear(f: np.ndarray, dx: float) -> np.ndarray:
    """Ntilde: faces -> faces (Eq. opr_def_nonlin), rotational form ~ (curl f) x f:
        [N(f)]^(1)_{ijk} = 1/4 sum_{q in {-1,0}} [ e^(2)_{i,j,k+q} (f^(3)_{i,j,k+q} + f^(3)_{i+1,j,k+q})
                                                 - e^(3)_{i,j+q,k} (f^(2)_{i,j+q,k} + f^(2)_{i+1,j+q,k}) ],
    e = C f.  The input is zero-extended, e = C f is the unbounded-grid curl of that extension (so
    e one layer outside the box is kept), and the result is masked to the box."""
    fp = np.pad(f, ((0, 0), (1, 1), (1, 1), (1, 1)))
    e1, e2, e3 = curl(fp, dx)
    f1, f2, f3 = fp
    n1 = np.zeros_like(f1)
    n2 = np.zeros_like(f1)
    n3 = np.zeros_like(f1)
    for q in (-1, 0):
        n1 += sh(e2, dk=q) * (sh(f3, dk=q) + sh(f3, di=1, dk=q)) - sh(e3, dj=q) * (sh(f2, dj=q) + sh(f2, di=1, dj=q))
        n2 += sh(e3, di=q) * (sh(f1, di=q) + sh(f1, di=q, dj=1)) - sh(e1, dk=q) * (sh(f3, dk=q) + sh(f3, dj=1, dk=q))
        n3 += sh(e1, dj=q) * (sh(f2, dj=q) + sh(f2, dj=q, dk=1)) - sh(e2, di=q) * (sh(f1, di=q) + sh(f1, di=q, dk=1))
    out = 0.25 * np.stack([n1, n2, n3])
    return np.ascontiguousarray(out[:, 1:-1, 1:-1, 1:-1])


def cyclic(f: np.ndarray) -> np.ndarray:
    """Lattice rotation x -> y -> z -> x applied to a vector field: the new component (q+1) on the
    new axis order is the old component (q).  Used by covariance tests."""
    # array axes are (z, y, x); the rotation maps old axis x to new axis y, y -> z, z -> x
    rot = lambda a: np.transpose(a, (1, 2, 0))
    return np.stack([rot(f[2]), rot(f[0]), rot(f[1])])
