#!/usr/bin/env python3
"""Generate lgf_asym_coefs.h: far-field expansion of the 7-point-Laplacian LGF to order PMAX.

The paper prints the first two terms of the expansion (Appendix B) and points to the
symbol-expansion procedure behind it.  This script carries that procedure further in exact rational
arithmetic:

  g(n) = (2 pi)^-3 int e^{-i n.xi} / sigma(xi) dxi,   sigma(xi) = sum_j (2 cos xi_j - 2).

  -sigma = |xi|^2 - h(xi), h = sum_{m>=2} sum_j 2 (-1)^m xi_j^{2m} / (2m)!, so
  1/sigma = -(1/|xi|^2) sum_k (h/|xi|^2)^k.  Grouping by homogeneity, order p collects the terms
  monomial(xi) / |xi|^{2K} of degree 2p - 2.  The inverse transform of |xi|^{-2K} in 3D is
  c_K r^{2K-3}, c_K = (-1)^{K-1} / (4 pi (2K-2)!), and a factor xi^a becomes (i d/dn)^a.
  Order p therefore contributes r^{-1-2p} Q_p(u), u = n / r.

Each Q_p is symmetric and even in u, so on the unit sphere it is a polynomial in
e2 = u1^2 u2^2 + u1^2 u3^2 + u2^2 u3^2 and e3 = u1^2 u2^2 u3^2 (e1 = |u|^2 = 1).  The header stores,
per order, the coefficients of Q_p(e2, e3) * pi (so g = sum_p r^{-1-2p} Q_p / pi).

Order 1 reproduces the printed second term.  Run:  python gen_lgf_asym.py > lgf_asym_coefs.h
"""
from __future__ import annotations

import sys
from fractions import Fraction as F
from functools import lru_cache
from math import factorial

PMAX = 6


def padd(p, q, s=1):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, 0) + s * v
        if r[k] == 0:
            del r[k]
    return r


def pmul(p, q):
    r = {}
    for k1, v1 in p.items():
        for k2, v2 in q.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            r[k] = r.get(k, 0) + v1 * v2
    return {k: v for k, v in r.items() if v != 0}


def hm(m):
    p = {}
    for j in range(3):
        e = [0, 0, 0]
        e[j] = 2 * m
        p[tuple(e)] = F(2 * (-1) ** m, factorial(2 * m))
    return p


H = {m: hm(m) for m in range(2, PMAX + 3)}


@lru_cache(None)
def hpow_deg(k, d):
    """Part of h^k of total degree d (as a frozen item tuple)."""
    if k == 0:
        return (((0, 0, 0), F(1)),) if d == 0 else ()
    res = {}
    for m in range(2, d // 2 + 1):
        sub = dict(hpow_deg(k - 1, d - 2 * m))
        if sub:
            res = padd(res, pmul(H[m], sub))
    return tuple(sorted(res.items()))


def dvar(expr, j):
    """d/dn_j of sum_q P_q(n) r^q."""
    out = {}
    for q, p in expr.items():
        dp = {}
        for k, v in p.items():
            if k[j] > 0:
                kk = list(k)
                kk[j] -= 1
                dp[tuple(kk)] = dp.get(tuple(kk), 0) + v * k[j]
        dp = {k: v for k, v in dp.items() if v != 0}
        if dp:
            out[q] = padd(out.get(q, {}), dp)
        if q != 0:
            xp = {}
            for k, v in p.items():
                kk = list(k)
                kk[j] += 1
                xp[tuple(kk)] = v * q
            out[q - 2] = padd(out.get(q - 2, {}), xp)
    return {q: p for q, p in out.items() if p}


@lru_cache(None)
def deriv(a, q):
    if a == (0, 0, 0):
        return {q: {(0, 0, 0): F(1)}}
    j = next(i for i in range(3) if a[i] > 0)
    aa = list(a)
    aa[j] -= 1
    return dvar(deriv(tuple(aa), q), j)


def c_K(K):
    """Inverse transform of |xi|^{-2K} is c_K r^{2K-3}; returned times pi."""
    return F((-1) ** (K - 1), 4 * factorial(2 * K - 2))


def order_terms(p):
    """Q_p as a dict of u-monomials (times pi)."""
    U = {}
    for k in range(0, p + 1):
        num = dict(hpow_deg(k, 2 * p + 2 * k)) if k > 0 else ({(0, 0, 0): F(1)} if p == 0 else {})
        K = k + 1
        for a, coef in num.items():
            s = F((-1) ** (sum(a) // 2)) * c_K(K) * (-coef)
            for q, poly in deriv(a, 2 * K - 3).items():
                for mono, v in poly.items():
                    assert sum(mono) + q == -1 - 2 * p
                    U[mono] = U.get(mono, 0) + s * v
    return {k: v for k, v in U.items() if v != 0}


def to_e2e3(U):
    """Rewrite a symmetric even polynomial in u on |u| = 1 as a polynomial in (e2, e3)."""
    # variables x_i = u_i^2
    P = {}
    for k, v in U.items():
        assert all(e % 2 == 0 for e in k)
        kk = tuple(e // 2 for e in k)
        P[kk] = P.get(kk, 0) + v
    P = {k: v for k, v in P.items() if v != 0}
    # elementary symmetric polynomials in x
    e1 = {(1, 0, 0): F(1), (0, 1, 0): F(1), (0, 0, 1): F(1)}
    e2 = {(1, 1, 0): F(1), (1, 0, 1): F(1), (0, 1, 1): F(1)}
    e3 = {(1, 1, 1): F(1)}

    def ppow(p, n):
        r = {(0, 0, 0): F(1)}
        for _ in range(n):
            r = pmul(r, p)
        return r

    out = {}  # (i, j, l) -> coef of e1^i e2^j e3^l
    while P:
        lead = max(P.keys(), key=lambda k: (sum(k), k))
        a, b, c = lead
        assert a >= b >= c, lead
        coef = P[lead]
        key = (a - b, b - c, c)
        out[key] = out.get(key, 0) + coef
        term = pmul(pmul(ppow(e1, a - b), ppow(e2, b - c)), ppow(e3, c))
        P = padd(P, {k: v * coef for k, v in term.items()}, -1)
    Q = {}
    for (i, j, l), v in out.items():  # e1 = 1
        Q[(j, l)] = Q.get((j, l), 0) + v
    return {k: v for k, v in Q.items() if v != 0}


def main():
    orders = [to_e2e3(order_terms(p)) for p in range(PMAX + 1)]
    # check order 1 against the printed term: -(sum u^4 - 3 sum u_i^2 u_j^2)/(16 pi r^3)
    # sum u^4 = 1 - 2 e2  ->  -(1 - 5 e2)/16
    assert orders[1] == {(0, 0): F(-1, 16), (1, 0): F(5, 16)}, orders[1]
    assert orders[0] == {(0, 0): F(-1, 4)}
    out = sys.stdout
    out.write("// Generated by gen_lgf_asym.py -- far-field expansion of the 7-point LGF.\n")
    out.write("// g(n) = (1/pi) sum_{p=0..%d} r^{-1-2p} Q_p(e2, e3), u = n/r,\n" % PMAX)
    out.write("// e2 = u1^2u2^2 + u1^2u3^2 + u2^2u3^2, e3 = u1^2u2^2u3^2.  Entries: {p, j, l, coef} for coef e2^j e3^l.\n")
    out.write("#pragma once\n\nnamespace nslgf {\n\n")
    out.write("constexpr int kLgfAsymOrders = %d;\n" % (PMAX + 1))
    rows = []
    for p, Q in enumerate(orders):
        for (j, l), v in sorted(Q.items()):
            rows.append((p, j, l, v))
    out.write("struct LgfAsymTerm { int p, j, l; double c; };\n")
    out.write("constexpr int kLgfAsymTerms = %d;\n" % len(rows))
    out.write("constexpr LgfAsymTerm kLgfAsym[kLgfAsymTerms] = {\n")
    for p, j, l, v in rows:
        out.write("    {%d, %d, %d, %s},  // %s\n" % (p, j, l, repr(float(v)), str(v)))
    out.write("};\n\n}  // namespace nslgf\n")


if __name__ == "__main__":
    main()
