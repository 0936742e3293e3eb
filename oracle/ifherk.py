"""Oracle: one IF-HERK time step on a fixed box, and Vor2Vel.  Test infrastructure only.

Followed passages:
* HERK tableaus (Sec. 3.2, Eq. ifherk_schemes) and the shifted tableau (Sec. 3.1, Eq. herk_shift):
  a~_{i,j} = a_{i+1,j} (i < s), a~_{s,j} = b_j; c~_i = c_{i+1} (i < s), c~_s = 1; c~_0 = 0.
* IF-HERK step (Sec. 3.2), plain recursion (not the final-stage shortcut of its footnote):
    g^i   = -a~_{ii} dt Ntilde(u^{i-1})                               (Eq. ifherk_g, minus sign as in Sec. 3.2)
    q^1   = u_k,  q^i = H^{i-1} q^{i-1}                                (Eq. ifherk_q)
    w^{i,j} = H^{i-1} w^{i-1,j} for j < i
    r^i   = q^i + dt sum_{j<i} a~_{ij} w^{i,j} + g^i                    (Eq. ifherk_aux_1)
    d^i   = -L^{-1} G^T r^i = L^{-1} Dbar r^i,  u^i = H^i (r^i - G d^i)  (projection, Eq. proj_final)
    w^{i,i} = (g^i - G d^i) / (a~_{ii} dt)
  finalize: u_{k+1} = u^s, d_{k+1} = d^s / (a~_{ss} dt), t_{k+1} = t_k + dt.
  H^i = E((c~_i - c~_{i-1}) dt / (dx^2 Re)).
* Masked form on one box (Sec. 5, xIF-HERK): every operator output is restricted to the box (the
  expanded solution domain) and every input is zero outside it.  The two exceptions of Sec. 5 are
  kept: the nonlinear term is restricted to the solution domain (Eq. rhs_final) and the pressure
  source to the support domain (Eq. dpoisson_final); both are the box shrunk by `n_buf` cells on
  every side (the buffer region).  n_buf = 0 makes the three domains coincide.  u_inf = 0.
* Vor2Vel (Sec. 4.1, Eq. vel_vor / vel_refresh): a = -L^{-1} w (per component), u = Cbar a.
"""
from __future__ import annotations

import math

import numpy as np

from . import intfac, native, stencils

S3 = math.sqrt(3.0)

# Butcher tableaus (A, b, c) of Eq. ifherk_schemes
SCHEMES = {
    "A": (np.array([[0, 0, 0], [0.5, 0, 0], [S3 / 3, (3 - S3) / 3, 0]]),
          np.array([(3 + S3) / 6, -S3 / 3, (3 + S3) / 6]), np.array([0.0, 0.5, 1.0])),
    "B": (np.array([[0, 0, 0], [1 / 3, 0, 0], [-1.0, 2.0, 0]]),
          np.array([0.0, 0.75, 0.25]), np.array([0.0, 1 / 3, 1.0])),
    "C": (np.array([[0, 0, 0], [8 / 15, 0, 0], [0.25, 5 / 12, 0]]),
          np.array([0.25, 0.0, 0.75]), np.array([0.0, 8 / 15, 2 / 3])),
}


def shifted(scheme: str):
    """(at, ct) with at[i][j] = a~_{i,j} and ct[i] = c~_i for 1-based i, j (index 0 unused except ct[0] = 0)."""
    A, b, c = SCHEMES[scheme]
    s = len(b)
    at = np.zeros((s + 1, s + 1))
    ct = np.zeros(s + 1)
    for i in range(1, s + 1):
        for j in range(1, s + 1):
            at[i, j] = A[i, j - 1] if i < s else b[j - 1]
        ct[i] = c[i] if i < s else 1.0
    return at, ct


def lgf_solve(src: np.ndarray, dx: float) -> np.ndarray:
    """L^{-1} src with uniform (zero) conditions at infinity = dx^2 (g * src) by direct summation."""
    return native.lgf_direct(src, dx)


def vor2vel(w: np.ndarray, dx: float) -> np.ndarray:
    """u = Cbar a with a = -L^{-1} w (three scalar LGF solves, then the curl of the potential)."""
    a = np.stack([-lgf_solve(w[q], dx) for q in range(3)])
    return stencils.curl_bar(a, dx)


def inner_mask(shape, n_buf: int) -> np.ndarray:
    """1 on the box shrunk by n_buf cells on every side (support = solution domain), else 0."""
    m = np.zeros(shape)
    nz, ny, nx = shape
    m[n_buf:nz - n_buf, n_buf:ny - n_buf, n_buf:nx - n_buf] = 1.0
    return m


def step(u: np.ndarray, dt: float, dx: float, re: float, scheme: str = "A", nonlinear: bool = True,
         n_buf: int = 0, soln_mask: np.ndarray | None = None, supp_mask: np.ndarray | None = None):
    """One IF-HERK step.  Returns (u_{k+1}, d_{k+1}); both restricted to the box.  soln_mask and
    supp_mask (0/1 cell arrays of the box, e.g. unions of blocks, Sec. 4.2) replace the box shrunk by
    n_buf as the solution domain (nonlinear term) and the support domain (pressure source)."""
    at, ct = shifted(scheme)
    s = len(ct) - 1
    beta = dt / (dx * dx * re)

    def H(i, x):
        return intfac.apply_vec(x, (ct[i] - ct[i - 1]) * beta)

    msk = inner_mask(u.shape[1:], n_buf)
    m_soln = msk if soln_mask is None else soln_mask
    m_supp = msk if supp_mask is None else supp_mask
    q = {1: u}
    w = {}
    u_prev = u
    dhat = None
    for i in range(1, s + 1):
        if i > 1:
            q[i] = H(i - 1, q[i - 1])
            for j in range(1, i):
                w[(i, j)] = H(i - 1, w[(i - 1, j)])
        if nonlinear:
            g = -at[i, i] * dt * m_soln * stencils.nonlinear(u_prev, dx)
        else:
            g = np.zeros_like(u)
        r = q[i] + g
        for j in range(1, i):
            r = r + dt * at[i, j] * w[(i, j)]
        dhat = lgf_solve(m_supp * stencils.div(r, dx), dx)
        gd = stencils.grad(dhat, dx)
        u_prev = H(i, r - gd)
        w[(i, i)] = (g - gd) / (at[i, i] * dt)
    return u_prev, dhat / (at[s, s] * dt)


def cell_speed_max(u: np.ndarray) -> float:
    """max over cells of |u| with each component averaged from its two faces to the cell centre."""
    c1 = 0.5 * (u[0] + stencils.sh(u[0], di=-1))
    c2 = 0.5 * (u[1] + stencils.sh(u[1], dj=-1))
    c3 = 0.5 * (u[2] + stencils.sh(u[2], dk=-1))
    return float(np.sqrt(c1 * c1 + c2 * c2 + c3 * c3).max())


def dt_from_cfl(u: np.ndarray, dx: float, cfl: float) -> float:
    """dt = CFL dx / max|u| (the step size rule of Sec. 6, cell-centred velocity magnitude)."""
    return cfl * dx / cell_speed_max(u)
