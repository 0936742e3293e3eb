"""Oracle: the integrating factor E(alpha) (Sec. 2.3).  Test infrastructure only.

E(alpha) = F^{-1} exp(alpha sigma) F solves the discrete diffusion equation dh/dt = kappa L h with
alpha = kappa (t - tau) / dx^2 (Eq. if_def, ddifussion_soln).  Its kernel is the product of three
one-dimensional factors (Appendix B, Eq. lgf_intfac, read with the sign that makes it the decaying
heat kernel): G_E(alpha)(n) = prod_j e^{-2 alpha} I_{|n_j|}(2 alpha).

The oracle evaluates e^{-2a} I_k(2a) with scipy's exponentially scaled Bessel function and applies
the kernel as one unseparated 3D sum over the box (values outside the box are zero, Sec. 4.1):
    [E(a) h](n) = sum_{m in box, |n - m|_inf <= R} prod_j w[|n_j - m_j|] h(m),
with R the first offset where w[R] / w[0] < 1e-20.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ive



def weights(alpha: float, rel_cut: float = 1e-20) -> np.ndarray:
    """w[k] = e^{-2 alpha} I_k(2 alpha) for k = 0..R (alpha >= 0)."""
    if alpha < 0:
        raise ValueError("E(alpha) is only bounded for alpha >= 0")
    if alpha == 0.0:
        return np.array([1.0])
    k = 0
    w = []
    w0 = ive(0, 2.0 * alpha)
    while True:
        v = ive(k, 2.0 * alpha)
        w.append(v)
        if v / w0 < rel_cut and k > 0:
            break
        k += 1
    return np.array(w)


def apply(h: np.ndarray, alpha: float) -> np.ndarray:
    """E(alpha) applied to one scalar component [nz, ny, nx] as an unseparated 3D sum."""
    w = weights(alpha)
    R = len(w) - 1
    nz, ny, nx = h.shape
    hp = np.pad(h, R)  # zero extension by R on every side
    out = np.zeros_like(h)
    for dk in range(-R, R + 1):
        for dj in range(-R, R + 1):
            for di in range(-R, R + 1):
                c = w[abs(dk)] * w[abs(dj)] * w[abs(di)]
                # h(n + d) for every n of the box
                out += c * hp[R + dk:R + dk + nz, R + dj:R + dj + ny, R + di:R + di + nx]
    return out


def apply_vec(f: np.ndarray, alpha: float) -> np.ndarray:
    """Component-wise E(alpha) of a face or edge field [3, nz, ny, nx]."""
    return np.stack([apply(f[q], alpha) for q in range(f.shape[0])])
