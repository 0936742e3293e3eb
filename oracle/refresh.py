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
