"""Pins of the oracle's lattice Green's function against what the paper and the mathematics fix
(Appendix B): the closed form at the origin, the defining difference equation, the printed
far-field expansion and its remainder order."""
import math

import numpy as np
import pytest

from oracle import lgf


def test_origin_closed_form(paper_values):
    g0 = lgf.lgf_value(0, 0, 0)
    assert abs(g0 - lgf.g0_closed_form()) <= 2e-16
    pv = paper_values["lgf_origin"]["value"]
    assert abs(g0 - pv) < 1e-13


def test_difference_equation_whole_table():
    """-6 g(n) + sum of the six neighbours = delta_{n,0} at every n of the table: a relation the
    quadrature does not use, so a dropped factor, a wrong tail or a mis-scaled integrand fails it."""
    nmax = 24
    cube = lgf.lgf_cube(nmax)
    full = np.concatenate([cube[:0:-1], cube], axis=0)
    full = np.concatenate([full[:, :0:-1], full], axis=1)
    full = np.concatenate([full[:, :, :0:-1], full], axis=2)  # g on [-nmax, nmax]^3
    c = full[1:-1, 1:-1, 1:-1]
    lap = (-6 * c + full[2:, 1:-1, 1:-1] + full[:-2, 1:-1, 1:-1] + full[1:-1, 2:, 1:-1]
           + full[1:-1, :-2, 1:-1] + full[1:-1, 1:-1, 2:] + full[1:-1, 1:-1, :-2])
    delta = np.zeros_like(lap)
    delta[nmax - 1, nmax - 1, nmax - 1] = 1.0
    assert np.abs(lap - delta).max() < 1e-15
    # the neighbour of the origin then follows exactly
    assert abs(lgf.lgf_value(1, 0, 0) - (lgf.g0_closed_form() + 1.0 / 6.0)) < 1e-16


def test_far_field_expansion_remainder(paper_values):
    """The printed two-term expansion leaves an O(|n|^-5) remainder: doubling |n| along a fixed
    direction must shrink the error by about 2^5, and the leading term alone by about 2^3."""
    assert paper_values["asymptotic_two_term"]["remainder_order"] == 5
    for d in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0)]:
        errs, errs1 = [], []
        for s in (8, 16):
            n = tuple(s * v for v in d)
            g = lgf.lgf_value(*n)
            errs.append(abs(g - lgf.asymptotic_two_term(n)))
            errs1.append(abs(g + 1.0 / (4 * math.pi * math.sqrt(sum(x * x for x in n)))))
        ratio = errs[0] / errs[1]
        assert 20 < ratio < 50, (d, ratio)
        ratio1 = errs1[0] / errs1[1]
        assert 5 < ratio1 < 11, (d, ratio1)


def test_wedge_symmetry_and_sign():
    ents, g = lgf.lgf_wedge(12)
    assert np.all(g < 0)
    # monotone along an axis (the LGF of the negative-definite Laplacian increases towards 0)
    along = [lgf.lgf_value(k, 0, 0) for k in range(13)]
    assert all(a < b for a, b in zip(along, along[1:]))
    cube = lgf.lgf_cube(12)
    assert np.array_equal(cube, np.transpose(cube, (1, 0, 2)))
    assert np.array_equal(cube, np.transpose(cube, (2, 1, 0)))
