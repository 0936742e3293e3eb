"""Oracle: block weights and the active-domain classification (Sec. 4.2, 4.3).  Test infrastructure
only.

Followed passages:
* Blocks (Sec. 4.2): the box is tiled by blocks of nb^3 cells (the last block along an axis may be
  shorter), indexed (bz, by, bx).
* Weight function (Sec. 4.3, Eq. weight_fun):
      mu(B) = max over B of |C u|,   nu(B) = max over B of |G^T Ntilde(u)| (= |Dbar Ntilde(u)|),
      W(B) = max(mu(B) / mu_global, nu(B) / nu_global)
  with |C u| read as the largest magnitude of the three edge components at a point.  Values closer
  than n_buf points to a box face are left out (the section zeroes the values in the buffer that the
  finite box has contaminated before it takes the weights).
* Domains (Sec. 4.3, Eqs. d_supp, d_soln; Sec. 4.2, Eq. def_xsoln): D_supp = {W > eps_supp},
  D_soln = {W > eps_soln} (the same weight function, its own threshold), D_xsoln = every block at most
  N_b blocks away from a block of D_soln, the distance read as the largest index difference over the
  three axes (a cube of blocks around each), restricted to the block grid of the box.
"""
from __future__ import annotations

import numpy as np

from . import ifherk, stencils


def block_max(field: np.ndarray, nb: int) -> np.ndarray:
    """Largest value of a nonnegative cell field [nz, ny, nx] over each block of nb^3 cells."""
    nz, ny, nx = field.shape
    bz, by, bx = -(-nz // nb), -(-ny // nb), -(-nx // nb)
    out = np.zeros((bz, by, bx))
    for k in range(bz):
        for j in range(by):
            for i in range(bx):
                blk = field[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb]
                out[k, j, i] = blk.max()
    return out


def weights(u: np.ndarray, dx: float, nb: int, n_buf: int):
    """(mu, nu) per block for the face velocity u."""
    m = ifherk.inner_mask(u.shape[1:], n_buf)
    w = np.abs(stencils.curl(u, dx)).max(axis=0) * m
    q = np.abs(stencils.div(stencils.nonlinear(u, dx), dx)) * m
    return block_max(w, nb), block_max(q, nb)


def classify(mu: np.ndarray, nu: np.ndarray, eps_supp: float, eps_soln: float, n_xb: int):
    """(W, supp, soln, xsoln) block arrays; the masks are 0/1 uint8."""
    mg, ng = mu.max(), nu.max()
    W = np.maximum(mu / mg if mg > 0 else np.zeros_like(mu), nu / ng if ng > 0 else np.zeros_like(nu))
    supp = (W > eps_supp).astype(np.uint8)
    soln = (W > eps_soln).astype(np.uint8)
    xsoln = np.zeros_like(soln)
    bz, by, bx = soln.shape
    for k, j, i in zip(*np.nonzero(soln)):
        xsoln[max(0, k - n_xb):min(bz, k + n_xb + 1), max(0, j - n_xb):min(by, j + n_xb + 1),
              max(0, i - n_xb):min(bx, i + n_xb + 1)] = 1
    return W, supp, soln, xsoln


def cell_mask(block_mask: np.ndarray, nb: int, shape) -> np.ndarray:
    """0/1 cell array of the box from a block mask [bz, by, bx] of nb^3-cell blocks (the union of the
    blocks, Sec. 4.2)."""
    m = np.repeat(np.repeat(np.repeat(block_mask.astype(np.float64), nb, axis=0), nb, axis=1), nb, axis=2)
    nz, ny, nx = shape
    return np.ascontiguousarray(m[:nz, :ny, :nx])

