"""Oracle: velocity refresh and its cadence (Sec. 4.4, Appendix D).  Test infrastructure only.

Followed passages:
* Truncation error of the masked integrating factor (Appendix D, Eq. if_finite_error).  For a uniform
  field on a half-space (the mask keeps the points k >= 1 along one axis), [I - M E(a) M] u at the
  point k equals |u| times the mass of the one-dimensional kernel at distances k and beyond:
      d_a(k) = sum_{n >= k} e^{-2a} I_n(2a),   k >= 1.
  (The printed index of the sum is garbled; this is the sum that the stated mask gives.)  On a box
  the first point inside a face has k = 1, so the point with 0-based index i along that axis has
  d(i + 1) from the near face and d(n - i) from the far one.
* Cadence (Sec. 4.4).  The integrating factors of q steps compose to E(q beta), beta = dt / (dx^2 Re),
  so the estimated error on the solution domain (the box shrunk by n_buf points, whose first point
  has k = n_buf + 1) after q steps is umax d_{q beta}(n_buf + 1), with umax the largest magnitude of
  any velocity component on the solution domain (Appendix D).  q_max is the largest q whose estimate
  stays within eps (capped at q_cap; 0 when one step already exceeds it).
* Refresh (Sec. 4.4): after q_max steps the velocity on the box is recomputed from the vorticity on
  the support domain with Vor2Vel: w = M_supp C u, u = Cbar a, a = -L^{-1} w.
* Active box (Sec. 4.2, 4.3, and the grid update of Sec. 5): steps computed on the bounding box of the
  expanded solution domain, which follows the flow (run_active).
"""
from __future__ import annotations

import numpy as np
from scipy.special import ive

from . import ifherk, stencils


def trunc_error(alpha: float, k: int) -> float:
    """d_alpha(k) = sum_{n >= k} e^{-2 alpha} I_n(2 alpha) for k >= 1 (terms until they no longer
    change the sum)."""
    if k < 1:
        raise ValueError("k >= 1")
    if alpha < 0:
        raise ValueError("alpha >= 0")
    if alpha == 0.0:
        return 0.0
    total = 0.0
    n = k
    while True:
        t = float(ive(n, 2.0 * alpha))
        total += t
        # the terms fall once n passes the peak at 0; stop when they are below rounding of the sum
        if t == 0.0 or t < 1e-18 * total:
            break
        n += 1
    return total


def estimate(beta: float, q: int, n_buf: int, umax: float) -> float:
    """Estimated error on the solution domain after q steps."""
    return umax * trunc_error(q * beta, n_buf + 1)


def refresh_interval(beta: float, n_buf: int, umax: float, eps: float, q_cap: int = 10000) -> int:
    """q_max: the largest q <= q_cap with estimate(q) <= eps, by trying q = 1, 2, ..."""
    if umax == 0.0 or beta == 0.0:
        return q_cap
    q = 0
    while q < q_cap and estimate(beta, q + 1, n_buf, umax) <= eps:
        q += 1
    return q


def component_max(u: np.ndarray, n_buf: int) -> float:
    """Largest magnitude of any velocity component on the solution domain."""
    m = ifherk.inner_mask(u.shape[1:], n_buf)
    return float(np.abs(u * m).max())


def velocity_refresh(u: np.ndarray, dx: float, n_buf: int) -> np.ndarray:
    """u = Cbar a, a = -L^{-1} w, w = M_supp C u."""
    w = ifherk.inner_mask(u.shape[1:], n_buf) * stencils.curl(u, dx)
    return ifherk.vor2vel(w, dx)


def run(u: np.ndarray, nsteps: int, dt: float, dx: float, re: float, scheme: str, n_buf: int, eps: float,
        q_cap: int = 10000):
    """nsteps IF-HERK steps, refreshing the velocity after every q_max steps (q_max from the velocity
    at the start and again after each refresh).  Returns (u, d, number of refreshes, [q_max ...])."""
    beta = dt / (dx * dx * re)
    qs = [refresh_interval(beta, n_buf, component_max(u, n_buf), eps, q_cap)]
    if qs[-1] == 0:
        raise ValueError("the buffer is too thin for eps: one step already exceeds it")
    count = 0
    refreshes = 0
    d = np.zeros(u.shape[1:])
    for _ in range(nsteps):
        u, d = ifherk.step(u, dt, dx, re, scheme, n_buf=n_buf)
        count += 1
        if count == qs[-1]:
            u = velocity_refresh(u, dx, n_buf)
            refreshes += 1
            count = 0
            qs.append(refresh_interval(beta, n_buf, component_max(u, n_buf), eps, q_cap))
            if qs[-1] == 0:
                raise ValueError("the buffer is too thin for eps: one step already exceeds it")
    return u, d, refreshes, qs


def run_adaptive(u: np.ndarray, nsteps: int, dt: float, dx: float, re: float, scheme: str, n_buf: int, nb: int,
                 eps_supp: float, eps_soln: float, n_xb: int):
    """nsteps IF-HERK steps on an active domain of blocks (Sec. 4.3): at the beginning of every step the
    block weights of u (values closer than n_buf to a box face left out) give D_supp and D_soln; the
    step restricts the pressure source to D_supp and the nonlinear term to D_soln; when either differs
    from the previous step's, the velocity is re-initialised from the vorticity on the new support,
    u = Cbar a, a = -L^{-1} M_supp C u (Eq. vel_refresh).  The first classification only sets the
    domain.  Returns (u, d, number of re-initialisations, [W of each step], [xsoln touches the outer
    block layer, per step])."""
    from . import blocks

    shape = u.shape[1:]
    prev = None
    reinit = 0
    Ws, edge = [], []
    d = np.zeros(shape)
    for _ in range(nsteps):
        mu, nu = blocks.weights(u, dx, nb, n_buf)
        W, supp, soln, xsoln = blocks.classify(mu, nu, eps_supp, eps_soln, n_xb)
        Ws.append(W)
        edge.append(bool(xsoln[0].any() or xsoln[-1].any() or xsoln[:, 0].any() or xsoln[:, -1].any()
                         or xsoln[:, :, 0].any() or xsoln[:, :, -1].any()))
        cs = blocks.cell_mask(supp, nb, shape)
        cn = blocks.cell_mask(soln, nb, shape)
        if prev is not None and not (np.array_equal(prev[0], supp) and np.array_equal(prev[1], soln)):
            u = ifherk.vor2vel(cs * stencils.curl(u, dx), dx)
            reinit += 1
        prev = (supp, soln)
        u, d = ifherk.step(u, dt, dx, re, scheme, soln_mask=cn, supp_mask=cs)
    return u, d, reinit, Ws, edge


def run_active(u: np.ndarray, nsteps: int, dt: float, dx: float, re: float, scheme: str, n_buf: int, nb: int,
               eps_supp: float, eps_soln: float, n_xb: int):
    """nsteps IF-HERK steps computed on an active box that follows the flow (Sec. 4.2, 4.3 and the grid
    update of Sec. 5).  The grid G of u is tiled by blocks of nb^3 cells (its sizes must be multiples of
    nb).  At the beginning of every step, on the current box B (a box of whole blocks; at first G):
      * the block weights of u_B (values closer than n_buf to a face of B left out) give D_supp = {W >
        eps_supp} and D_soln = {W > eps_soln} united with D_supp (the domains are nested, D_supp in
        D_soln), in the block coordinates of G;
      * D_xsoln = every block of G at most n_xb blocks from D_soln (along each axis), and the new box B'
        is the bounding box of D_xsoln: the blocks of B' outside D_xsoln are computed too;
      * first step: u is restricted to B' (the classification only sets the domain); later, when D_supp
        or D_soln changed, u is re-initialised on B' from the vorticity on the new support, copied from
        B (Sec. 5, grid update and velocity refresh): u_B' = Vor2Vel(transfer(M_supp C u_B));
      * the step runs on B' with the pressure source on D_supp and the nonlinear term on D_soln.
    Returns (u on G, d on G, both zero outside the final box, number of re-initialisations, number of
    box changes after the first step, [box per step as (lo, hi) block corners, z y x order])."""
    from . import blocks

    G = u.shape[1:]
    if any(s % nb for s in G):
        raise ValueError("the grid sizes must be multiples of the block size")
    gb = tuple(s // nb for s in G)
    lo, hi = (0, 0, 0), gb
    ub = u.copy()
    prev = None
    reinit = regrid = 0
    boxes = []

    def transfer(f, lo0, hi0, lo1, hi1):
        """f on box (lo0, hi0) -> box (lo1, hi1), zero where the new box leaves the old one."""
        out = np.zeros((f.shape[0],) + tuple((h - l) * nb for l, h in zip(lo1, hi1)))
        a = [max(l0, l1) for l0, l1 in zip(lo0, lo1)]
        b = [min(h0, h1) for h0, h1 in zip(hi0, hi1)]
        if all(x < y for x, y in zip(a, b)):
            src = tuple(slice((x - l0) * nb, (y - l0) * nb) for x, y, l0 in zip(a, b, lo0))
            dst = tuple(slice((x - l1) * nb, (y - l1) * nb) for x, y, l1 in zip(a, b, lo1))
            out[(slice(None),) + dst] = f[(slice(None),) + src]
        return out

    def box_of(mask):
        idx = np.argwhere(mask)
        return tuple(int(v) for v in idx.min(axis=0)), tuple(int(v) + 1 for v in idx.max(axis=0))

    d = None
    for _ in range(nsteps):
        mu, nu = blocks.weights(ub, dx, nb, n_buf)
        _, supp, soln, _ = blocks.classify(mu, nu, eps_supp, eps_soln, 0)
        soln = np.maximum(soln, supp)
        gs = np.zeros(gb, dtype=np.uint8)
        gn = np.zeros(gb, dtype=np.uint8)
        box = tuple(slice(l, h) for l, h in zip(lo, hi))
        gs[box] = supp
        gn[box] = soln
        gx = np.zeros_like(gn)
        for k, j, i in zip(*np.nonzero(gn)):
            gx[max(0, k - n_xb):k + n_xb + 1, max(0, j - n_xb):j + n_xb + 1, max(0, i - n_xb):i + n_xb + 1] = 1
        nlo, nhi = box_of(gx)
        if prev is None:
            ub = transfer(ub, lo, hi, nlo, nhi)
        elif not (np.array_equal(prev[0], gs) and np.array_equal(prev[1], gn)):
            w = blocks.cell_mask(gs[box], nb, ub.shape[1:]) * stencils.curl(ub, dx)
            ub = ifherk.vor2vel(transfer(w, lo, hi, nlo, nhi), dx)
            reinit += 1
            regrid += int((nlo, nhi) != (lo, hi))
        lo, hi = nlo, nhi
        prev = (gs, gn)
        boxes.append((lo, hi))
        box = tuple(slice(l, h) for l, h in zip(lo, hi))
        shape = ub.shape[1:]
        ub, db = ifherk.step(ub, dt, dx, re, scheme, soln_mask=blocks.cell_mask(gn[box], nb, shape),
                             supp_mask=blocks.cell_mask(gs[box], nb, shape))
        d = db
    uf = np.zeros_like(u)
    df = np.zeros(G)
    cells = tuple(slice(l * nb, h * nb) for l, h in zip(lo, hi))
    uf[(slice(None),) + cells] = ub
    if d is not None:
        df[cells] = d
    return uf, df, reinit, regrid, boxes
