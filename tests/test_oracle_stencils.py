"""Pins of the oracle's point operators (Appendix A) against the mimetic identities of Sec. 2.1,
adjointness, the Laplacian identity L_F = -G G^T - C^T C, exactness of the nonlinear operator on
linear fields, and covariance under the lattice rotation."""
import numpy as np
import pytest

from oracle import stencils as st
import workloads


N = 10


def _int_vec(seed):
    return workloads.random_field((3, N, N, N), seed, integer=True)


def _int_scal(seed):
    return workloads.random_field((N, N, N), seed, integer=True)


def test_mimetic_null_identities_exact():
    dx = 1.0
    c, f, e, v = _int_scal(1), _int_vec(2), _int_vec(3), _int_scal(4)
    assert np.array_equal(st.curl(st.grad(c, dx), dx), np.zeros((3, N, N, N)))
    assert np.array_equal(st.div_edge(st.curl(f, dx), dx), np.zeros((N, N, N)))
    assert np.array_equal(st.curl_bar(st.grad_vertex(v, dx), dx), np.zeros((3, N, N, N)))
    assert np.array_equal(st.div(st.curl_bar(e, dx), dx), np.zeros((N, N, N)))


def test_adjointness():
    dx = 0.7
    c, f, e, v = (workloads.random_field(s, k) for s, k in [((N, N, N), 5), ((3, N, N, N), 6), ((3, N, N, N), 7), ((N, N, N), 8)])
    assert abs(np.sum(st.grad(c, dx) * f) + np.sum(c * st.div(f, dx))) < 1e-12 * np.abs(f).sum()
    assert abs(np.sum(st.curl(f, dx) * e) - np.sum(f * st.curl_bar(e, dx))) < 1e-12 * np.abs(f).sum()
    assert abs(np.sum(st.grad_vertex(v, dx) * e) + np.sum(v * st.div_edge(e, dx))) < 1e-12 * np.abs(e).sum()


def test_face_laplacian_identity():
    """L_F = G Dbar - Cbar C equals the 7-point stencil per component (compact support)."""
    dx = 0.5
    f = np.zeros((3, N, N, N))
    f[:, 3:-3, 3:-3, 3:-3] = workloads.random_field((3, N - 6, N - 6, N - 6), 9, integer=True)
    lhs = st.grad(st.div(f, dx), dx) - st.curl_bar(st.curl(f, dx), dx)
    rhs = np.stack([st.laplacian(f[q], dx) for q in range(3)])
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12)
    c = np.zeros((N, N, N))
    c[3:-3, 3:-3, 3:-3] = workloads.random_field((N - 6,) * 3, 10, integer=True)
    assert np.allclose(st.div(st.grad(c, dx), dx), st.laplacian(c, dx), rtol=0, atol=1e-12)


def _face_positions(n, dx):
    c = (n - 1) / 2.0
    idx = np.arange(n)
    K, J, I = np.meshgrid(idx, idx, idx, indexing="ij")
    # face (q) sits half a cell below the vertex along the two axes other than q
    pos = []
    for q in range(3):
        off = [-0.5, -0.5, -0.5]
        off[q] = 0.0
        pos.append(((I + off[0] - c) * dx, (J + off[1] - c) * dx, (K + off[2] - c) * dx))
    return pos


def test_nonlinear_uniform_and_linear_fields():
    n, dx = 12, 0.3
    # uniform flow: no vorticity, no nonlinear term away from the box edge
    u = np.ones((3, n, n, n)) * np.array([0.3, -1.2, 0.7])[:, None, None, None]
    nl = st.nonlinear(u, dx)
    assert np.abs(nl[:, 2:-2, 2:-2, 2:-2]).max() < 1e-14
    # solid-body rotation plus a uniform flow: omega = 2 Omega, Ntilde = omega x u exactly
    Om = np.array([0.4, -0.9, 1.3])
    U0 = np.array([0.2, 0.1, -0.5])
    pos = _face_positions(n, dx)
    u = np.zeros((3, n, n, n))
    for q in range(3):
        x = np.stack(pos[q])
        vel = np.cross(Om[:, None, None, None], x, axis=0) + U0[:, None, None, None]
        u[q] = vel[q]
    nl = st.nonlinear(u, dx)
    om = 2 * Om
    for q in range(3):
        x = np.stack(pos[q])
        vel = np.cross(Om[:, None, None, None], x, axis=0) + U0[:, None, None, None]
        expect = np.cross(om[:, None, None, None], vel, axis=0)[q]
        assert np.abs(nl[q, 2:-2, 2:-2, 2:-2] - expect[2:-2, 2:-2, 2:-2]).max() < 1e-12, q


@pytest.mark.parametrize("op", ["grad", "div", "curl", "curl_bar", "nonlinear"])
def test_cyclic_covariance(op):
    """The three components come from one printed component by the cyclic rule; rotating the
    lattice (x -> y -> z -> x) must commute with every operator."""
    dx = 1.0
    rng = np.random.default_rng(11)
    f = rng.standard_normal((3, N, N, N))
    c = rng.standard_normal((N, N, N))
    rot = lambda a: np.transpose(a, (1, 2, 0))
    if op == "grad":
        assert np.allclose(st.grad(rot(c), dx), st.cyclic(st.grad(c, dx)), atol=1e-14)
    elif op == "div":
        assert np.allclose(st.div(st.cyclic(f), dx), rot(st.div(f, dx)), atol=1e-14)
    elif op == "curl":
        assert np.allclose(st.curl(st.cyclic(f), dx), st.cyclic(st.curl(f, dx)), atol=1e-14)
    elif op == "curl_bar":
        assert np.allclose(st.curl_bar(st.cyclic(f), dx), st.cyclic(st.curl_bar(f, dx)), atol=1e-14)
    else:
        assert np.allclose(st.nonlinear(st.cyclic(f), dx), st.cyclic(st.nonlinear(f, dx)), atol=1e-13)
