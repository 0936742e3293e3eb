"""Oracle: lattice Green's function g(n) of the 7-point Laplacian.  Test infrastructure only.

Definition followed (Appendix B, Bessel form of G_L): the dimensionless LGF
    g(n) = - int_0^inf e^{-6t} I_{n1}(2t) I_{n2}(2t) I_{n3}(2t) dt
satisfies -6 g(n) + sum of its six neighbours = delta_{n,0}.  With the dimensional Laplacian
(dx^2 L a = -6 a + neighbours, Appendix A) the solution operator is L^{-1} f = dx^2 (g * f).

Method (plain, slow): the integrand is written with scipy's exponentially scaled Bessel function
ive(n, x) = e^{-x} I_n(x), so e^{-6t} prod I_{nj}(2t) = prod ive(nj, 2t).  The interval [0, T] is
split at powers of two and each piece is integrated by scipy's adaptive vector quadrature
(Gauss-Kronrod), every table entry scaled by its expected magnitude so that the error control is
relative per entry.  Beyond T the large-argument (Hankel) series of e^{-z} I_n(z) is multiplied out
for the three factors and integrated term by term in closed form.
"""
from __future__ import annotations

import math
import os
from functools import lru_cache

import numpy as np
from scipy.integrate import quad_vec
from scipy.special import ive

_HANKEL_TERMS = 8


def wedge_entries(nmax: int) -> np.ndarray:
    """All (n1, n2, n3) with nmax >= n1 >= n2 >= n3 >= 0, int64 [M, 3]."""
    out = [(a, b, c) for a in range(nmax + 1) for b in range(a + 1) for c in range(b + 1)]
    return np.array(out, dtype=np.int64)


def _hankel_coefs(nmax: int, terms: int) -> np.ndarray:
    """c[n, k] with e^{-2t} I_n(2t) ~ (4 pi t)^{-1/2} sum_k c[n, k] t^{-k} (large t)."""
    c = np.zeros((nmax + 1, terms))
    for n in range(nmax + 1):
        mu = 4.0 * n * n
        a = 1.0
        for k in range(terms):
            if k > 0:
                a *= (mu - (2 * k - 1) ** 2) / (k * 8.0)
            c[n, k] = (-1) ** k * a / 2.0 ** k
    return c


def _tail(ents: np.ndarray, nmax: int, T: float) -> np.ndarray:
    """int_T^inf prod_j e^{-2t} I_{nj}(2t) dt from the product of the three Hankel series:
    the coefficient of t^{-m} in the product is sum_{i+j+l=m} c[n1,i] c[n2,j] c[n3,l], and
    int_T^inf (4 pi t)^{-3/2} t^{-m} dt = (4 pi)^{-3/2} T^{-1/2-m} / (m + 1/2)."""
    c = _hankel_coefs(nmax, _HANKEL_TERMS)
    ca, cb, cd = c[ents[:, 0]], c[ents[:, 1]], c[ents[:, 2]]
    out = np.zeros(len(ents))
    K = _HANKEL_TERMS
    for i in range(K):
        for j in range(K):
            for l in range(K):
                m = i + j + l
                out += ca[:, i] * cb[:, j] * cd[:, l] * (T ** (-0.5 - m) / (m + 0.5))
    return out * (4.0 * math.pi) ** -1.5


def _integrate(ents: np.ndarray, nmax: int) -> np.ndarray:
    T = max(1.0e5, 400.0 * nmax * nmax)
    ns = np.arange(nmax + 1)
    r = np.sqrt((ents.astype(np.float64) ** 2).sum(axis=1))
    scale = 1.0 / (4.0 * math.pi * np.maximum(r, 1.0))

    def f(t):
        a = ive(ns, 2.0 * t)
        return a[ents[:, 0]] * a[ents[:, 1]] * a[ents[:, 2]] / scale

    pts = [0.0] + [2.0 ** k for k in range(-4, int(math.log2(T)) + 1)] + [T]
    pts = sorted(set(p for p in pts if p <= T))
    tot = np.zeros(len(ents))
    for lo, hi in zip(pts[:-1], pts[1:]):
        v, _ = quad_vec(f, lo, hi, epsabs=1e-21, epsrel=1e-15, norm="max", limit=4000)
        tot += v
    return -(tot * scale + _tail(ents, nmax, T))


def _cache_path(nmax: int):
    d = os.environ.get("NSLGF_ORACLE_CACHE", os.path.join(os.environ.get("TMPDIR", "/tmp"), "nslgf_oracle_cache"))
    return d, os.path.join(d, f"lgf_wedge_{nmax}.npy")


@lru_cache(maxsize=8)
def lgf_wedge(nmax: int) -> tuple[np.ndarray, np.ndarray]:
    """(entries [M,3], g [M]) for the wedge nmax >= n1 >= n2 >= n3 >= 0.  Results are cached on
    disk (computed here, by this module only) because large tables take a minute."""
    ents = wedge_entries(nmax)
    d, path = _cache_path(nmax)
    if os.path.exists(path):
        g = np.load(path)
        if g.shape == (len(ents),):
            return ents, g
    chunk = 40000
    parts = [ents[i:i + chunk] for i in range(0, len(ents), chunk)]
    if len(parts) > 2:
        # worker processes started as fresh interpreters (never forked from a GPU process)
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor

        workers = min(16, len(parts), os.cpu_count() or 1)
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            g = np.concatenate(list(ex.map(_integrate, parts, [nmax] * len(parts))))
    else:
        g = np.concatenate([_integrate(p, nmax) for p in parts])
    try:
        os.makedirs(d, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npy"
        np.save(tmp, g)
        os.replace(tmp, path)
    except OSError:
        pass
    return ents, g


@lru_cache(maxsize=8)
def lgf_cube(nmax: int) -> np.ndarray:
    """g(|n1|, |n2|, |n3|) on the cube [0, nmax]^3 (float64, C-contiguous), filled from the
    wedge by the 48-fold lattice symmetry (g depends only on the sorted absolute offsets)."""
    ents, g = lgf_wedge(nmax)
    cube = np.empty((nmax + 1,) * 3)
    a, b, c = ents[:, 0], ents[:, 1], ents[:, 2]
    for p in ((a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)):
        cube[p] = g
    return np.ascontiguousarray(cube)


def lgf_value(n1: int, n2: int, n3: int) -> float:
    """Single value g(n) (through the cube of size max|n_j|)."""
    m = max(abs(n1), abs(n2), abs(n3))
    return float(lgf_cube(max(m, 1))[abs(n1), abs(n2), abs(n3)])


def g0_closed_form() -> float:
    """g(0) = -W/6 with Watson's integral W = sqrt(6)/(32 pi^3) Gamma(1/24) Gamma(5/24)
    Gamma(7/24) Gamma(11/24) (Glasser & Zucker's closed form of the simple cubic lattice
    integral), evaluated at 40 digits.  Independent of the quadrature above."""
    import mpmath

    with mpmath.workdps(40):
        W = (mpmath.sqrt(6) / (32 * mpmath.pi ** 3) * mpmath.gamma(mpmath.mpf(1) / 24)
             * mpmath.gamma(mpmath.mpf(5) / 24) * mpmath.gamma(mpmath.mpf(7) / 24)
             * mpmath.gamma(mpmath.mpf(11) / 24))
        return float(-W / 6)


def asymptotic_two_term(n) -> float:
    """The far-field expansion printed in Appendix B (two terms, error O(|n|^-5))."""
    n1, n2, n3 = (float(v) for v in n)
    r = math.sqrt(n1 * n1 + n2 * n2 + n3 * n3)
    p4 = n1 ** 4 + n2 ** 4 + n3 ** 4 - 3 * n1 * n1 * n2 * n2 - 3 * n1 * n1 * n3 * n3 - 3 * n2 * n2 * n3 * n3
    return -1.0 / (4.0 * math.pi * r) - p4 / (16.0 * math.pi * r ** 7)
