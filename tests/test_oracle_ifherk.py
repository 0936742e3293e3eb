"""Pins of the oracle's IF-HERK step and Vor2Vel (Sec. 3, 4.1, 5; Appendix C): tableau
invariants and the stability limit, the projection's divergence-free result, the Stokes special
case H^1 H^2 H^3 = E(beta), and the temporal orders of Table 1."""
import math

import numpy as np
import pytest

from oracle import ifherk, intfac, native, stencils
import workloads


@pytest.mark.parametrize("scheme", ["A", "B", "C"])
def test_tableau_and_stability(scheme, paper_values):
    A, b, c = ifherk.SCHEMES[scheme]
    assert np.allclose(A.sum(axis=1), c)            # row sums are the nodes
    assert abs(b.sum() - 1.0) < 1e-15
    at, ct = ifherk.shifted(scheme)
    assert ct[3] == 1.0 and ct[0] == 0.0
    # stability function R(z) = 1 + z b^T (I - zA)^{-1} e (Appendix C, Eq. stability_region)
    def R(z):
        return 1 + z * b @ np.linalg.solve(np.eye(3) - z * A, np.ones(3))
    for z in (0.3, -1.1, 0.5j, 1.2 - 0.4j):
        assert abs(R(z) - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-13
    # largest mu with |R(i mu)| <= 1, divided by gamma/CFL = sqrt(3)
    mus = np.linspace(0.0, 3.0, 300001)
    ok = np.abs(1 + 1j * mus - mus ** 2 / 2 - 1j * mus ** 3 / 6) <= 1 + 1e-12
    mu_star = mus[ok].max()
    assert abs(mu_star / math.sqrt(3.0) - paper_values["cfl_max"]["value"]) < 1e-4


def test_scheme_a_shifted_constants():
    at, ct = ifherk.shifted("A")
    s3 = math.sqrt(3.0)
    assert at[1, 1] == 0.5
    assert abs(at[2, 1] - s3 / 3) < 1e-16 and abs(at[2, 2] - (3 - s3) / 3) < 1e-16
    assert abs(at[3, 1] - (3 + s3) / 6) < 1e-16 and abs(at[3, 2] + s3 / 3) < 1e-16 and abs(at[3, 3] - (3 + s3) / 6) < 1e-16
    assert list(ct) == [0.0, 0.5, 1.0, 1.0]


def test_projection_removes_divergence():
    """d = L^{-1} Dbar r makes Dbar (r - G d) vanish everywhere but the outermost layer (where the
    gradient of the masked pressure is cut); the opposite sign would double the divergence."""
    n, dx = 14, 0.3
    r = workloads.random_field((3, n, n, n), 21)
    d = native.lgf_direct(stencils.div(r, dx), dx)
    y = r - stencils.grad(d, dx)
    dv = stencils.div(y, dx)
    assert np.abs(dv[1:-1, 1:-1, 1:-1]).max() < 1e-11 * np.abs(stencils.div(r, dx)).max()


def _compact_velocity(n, inner, dx, seed):
    a = np.zeros((3, n, n, n))
    a[:, inner:-inner, inner:-inner, inner:-inner] = workloads.random_field((3,) + (n - 2 * inner,) * 3, seed)
    return stencils.curl_bar(a, dx)


def test_stokes_special_case():
    """Without the nonlinear term a divergence-free compact u_k needs no pressure and the stage
    factors compose to E(beta): u_{k+1} = E(beta) u_k, d_{k+1} = 0."""
    n, dx, re, dt = 30, 0.5, 50.0, 0.3
    beta = dt / (dx * dx * re)
    R = len(intfac.weights(beta)) - 1
    u = _compact_velocity(n, R + 2, dx, 3)
    u1, d1 = ifherk.step(u, dt, dx, re, "A", nonlinear=False)
    expect = intfac.apply_vec(u, beta)
    assert np.abs(u1 - expect).max() < 1e-13 * np.abs(u).max()
    assert np.abs(d1).max() < 1e-12 * np.abs(u).max() / dt


def test_zero_stays_zero():
    u = np.zeros((3, 8, 8, 8))
    u1, d1 = ifherk.step(u, 0.1, 0.5, 100.0)
    assert not u1.any() and not d1.any()


def _ring_u0(n, dx, ring):
    w = workloads.ring_edge_vorticity(n, dx, ring)
    return w, ifherk.vor2vel(w, dx)


def test_vor2vel_properties():
    n, dx = 24, 0.15
    ring = workloads.Ring(R=1.0, sigma=0.3)
    w, u = _ring_u0(n, dx, ring)
    # exactly divergence free (Dbar Cbar = 0)
    assert np.abs(stencils.div(u, dx)).max() < 1e-12 * np.abs(u).max() / dx
    # the ring moves in +z: u^(3) at the centre (the face nearest the axis) is positive
    c = n // 2
    assert u[2, c, c, c] > 0
    # curl returns the vorticity where D w ~ 0 (away from the box edge)
    cw = stencils.curl(u, dx)
    inner = slice(4, n - 4)
    err = np.abs(cw[:, inner, inner, inner] - w[:, inner, inner, inner]).max()
    assert err < 1e-3 * np.abs(w).max()


def _apparent_orders(p):
    """log2 error ratios of runs with 1, 2, 4 steps measured against an 8-step reference when the
    true error is C dt^p (the finite reference biases them upward)."""
    e = [2.0 ** (-p * k) - 8.0 ** (-p) for k in range(3)]
    return math.log2(e[0] / e[1]), math.log2(e[1] / e[2])


@pytest.mark.parametrize("scheme", ["A", "B", "C"])
def test_temporal_order(scheme, paper_values):
    """Velocity and pressure errors at a fixed time against a dt/8 reference fall with the orders of
    Table 1 (A: 2, 2; B: 3, 2; C: 3, 1).  The initial velocity is compactly supported inside the box:
    a field that is not small on the box faces (a vortex ring on a box a few radii wide) adds an
    error of first order in dt that comes from the box, not from the scheme, because integrating
    factors truncated at the box faces only compose approximately, E(a1) E(a2) != E(a1 + a2) there."""
    n, dx, re, n_buf = 16, 0.3, 100.0, 2
    u0 = _compact_velocity(n, 5, dx, 7)
    u0 = u0 * (0.5 / np.abs(u0).max())
    T = ifherk.dt_from_cfl(u0, dx, 0.5)

    def run(m):
        u = u0
        for _ in range(m):
            u, d = ifherk.step(u, T / m, dx, re, scheme, n_buf=n_buf)
        return u, d

    ref, dref = run(8)
    eu, ed = [], []
    for m in (1, 2, 4):
        u, d = run(m)
        eu.append(np.abs(u - ref).max())
        ed.append(np.abs(d - dref).max())
    want = paper_values["scheme_orders"][scheme]
    for var, e in (("y", eu), ("z", ed)):
        got = (math.log2(e[0] / e[1]), math.log2(e[1] / e[2]))
        expect = _apparent_orders(want[var])
        assert all(abs(g - x) < 0.3 for g, x in zip(got, expect)), (var, got, expect)
