"""Pins of the oracle's vortex-ring integrals (Sec. 6.2, Eq. int_quantities; Sec. 6.3, Eq. u_saffman):
closed forms of a resolved Gaussian ring, the centroid of a lifted ring, translation covariance, and
exact identities that tie the cell-centre sums (K, J) to the edge sums (I) for a uniform velocity."""
import math

import numpy as np
import pytest

import workloads
from oracle import diagnostics as dg
from oracle import ifherk

R, SIG, DX, N = 1.0, 0.3, 0.05, 96


@pytest.fixture(scope="module")
def ring_w():
    return {zc: workloads.ring_edge_vorticity(N, DX, workloads.Ring(R=R, sigma=SIG, zc=zc)) for zc in (0.0, 0.3)}


def test_impulse_and_enstrophy_closed_forms(ring_w):
    """I_z = pi Gamma (R^2 + sigma^2 / 2) and E = Gamma^2 R / (2 sigma^2) for the Gaussian core; the
    edge values are dual-face averages of the vorticity, which lowers E by sigma-relative
    (dx / sigma)^2 / 6 (two averaged directions)."""
    w = ring_w[0.0]
    r = dg.integrals(np.zeros_like(w), w, DX, dg.box_origin(w.shape[1:], DX))
    assert abs(r["I"][2] / (math.pi * (R * R + SIG * SIG / 2)) - 1) < 1e-7
    assert abs(r["I"][0]) < 1e-12 and abs(r["I"][1]) < 1e-12
    e_ref = R / (2 * SIG * SIG) * (1 - DX * DX / (6 * SIG * SIG))
    assert abs(r["E"] / e_ref - 1) < 1e-3
    # the flux-averaged E is below the continuum value by about that amount, not by more
    assert 0.002 < 1 - r["E"] / (R / (2 * SIG * SIG)) < 0.006


def test_centroid_of_a_lifted_ring_and_translation(ring_w):
    o = dg.box_origin(ring_w[0.3].shape[1:], DX)
    r = dg.integrals(np.zeros_like(ring_w[0.3]), ring_w[0.3], DX, o)
    assert abs(r["X"][2] - 0.3) < 1e-9
    assert abs(r["X"][0]) < 1e-9 and abs(r["X"][1]) < 1e-9
    # moving the origin by a leaves I alone (the vorticity sums to zero) and moves X by a along the
    # impulse; across it the printed definition moves X by 3/2 a, since int x w_y = -int y w_x = I_z
    # for a divergence-free w, so X is a centroid along I only (Sec. 6.3 uses its I-component)
    a = np.array([0.7, -1.3, 0.4])
    r2 = dg.integrals(np.zeros_like(ring_w[0.3]), ring_w[0.3], DX, tuple(np.array(o) + a))
    assert np.abs(np.array(r2["I"]) - np.array(r["I"])).max() < 1e-9
    assert np.abs(np.array(r2["X"]) - np.array(r["X"]) - a * np.array([1.5, 1.5, 1.0])).max() < 1e-6


def test_uniform_velocity_ties_cell_centre_sums_to_edge_sums(ring_w):
    """For u = U uniform and w vanishing near the faces, K = U . (2 I) and J = dx^3 U . sum w exactly
    (the cell-centre averages are linear, and the centre positions average to the edge positions)."""
    w = ring_w[0.3]
    U = np.array([0.3, -0.7, 1.1])
    u = np.stack([np.full(w.shape[1:], U[q]) for q in range(3)])
    r = dg.integrals(u, w, DX, dg.box_origin(w.shape[1:], DX))
    assert abs(r["K"] - 2 * U @ np.array(r["I"])) < 1e-9 * abs(r["K"])
    assert abs(r["J"] - DX ** 3 * U @ w.sum(axis=(1, 2, 3))) < 1e-9
    # rigid rotation u = Omega cross x (sampled on the faces, so exact at the cell centres):
    # J = sum (Omega cross x) . w dx^3 = 2 Omega . I
    om = np.array([0.2, -0.5, 0.9])
    o = dg.box_origin(w.shape[1:], DX)
    pos = [dg._coords(w.shape[1:], DX, o, [0 if a == q else 1 for a in range(3)]) for q in range(3)]
    rot = np.stack([np.cross(om, np.stack(pos[q]), axis=0)[q] for q in range(3)])
    r3 = dg.integrals(rot, w, DX, o)
    assert abs(r3["J"] - 2 * om @ np.array(r3["I"])) < 1e-9 * abs(r3["J"])


def test_integrals_of_the_vor2vel_velocity():
    """Vor2Vel then the masked curl gives back the sampled vorticity inside the box (C Cbar (-L^{-1})
    is the identity on a divergence-free w), so the integrals of u = Vor2Vel(w) with one masked layer
    equal those of w; without the mask the curl of the truncated velocity at the outermost edges
    dominates them."""
    n, dx = 24, 4.4 / 24
    w = workloads.ring_edge_vorticity(n, dx, workloads.Ring(R=1.0, sigma=0.3))
    o = dg.box_origin(w.shape[1:], dx)
    u = ifherk.vor2vel(w, dx)
    ref = dg.integrals(u, w, dx, o)
    got = dg.of_velocity(u, dx, o, 1)
    for key in ("K", "E"):
        assert abs(got[key] / ref[key] - 1) < 1e-5, key
    assert abs(got["I"][2] / ref["I"][2] - 1) < 1e-5
    assert abs(dg.of_velocity(u, dx, o, 0)["I"][2] / ref["I"][2] - 1) > 0.5
    # K > 0 is the kinetic energy of the ring (Sec. 6.2), J = 0 without swirl
    assert got["K"] > 0 and abs(got["J"]) < 1e-9 * got["K"]


def test_saffman_speed_constants():
    """beta_0 = (1 - gamma_E + log 2) / 2 = 0.557966 (Sec. 6.3) and U = Gamma/(4 pi R)(log(8/eps) - beta_0)."""
    euler = 0.5772156649015329
    assert abs(0.5 * (1 - euler + math.log(2)) - 0.557966) < 1e-6
    assert abs(dg.saffman_speed(1.0, 1.0, 0.2) - (math.log(40) - 0.557966) / (4 * math.pi)) < 1e-7
