"""Pins of the oracle's block weights and active-domain classification (Sec. 4.2, 4.3): closed forms
for a rigid rotation, the footprint of a point vortex, and the block counts of the expanded domain."""
import numpy as np

from oracle import blocks, ifherk, stencils
from oracle import diagnostics as dg


def _faces(shape, dx, fn):
    """Face field whose component q is fn(x, y, z)[q] at face (q) positions."""
    o = dg.box_origin(shape, dx)
    out = []
    for q in range(3):
        X, Y, Z = dg._coords(shape, dx, o, [0 if a == q else 1 for a in range(3)])
        out.append(fn(X, Y, Z)[q])
    return np.stack(out)


def test_rigid_rotation_weights():
    """u = Omega x x: C u = 2 Omega on every edge and Ntilde(u) = (2 Omega) x u exactly (Ntilde is exact on
    linear fields), whose divergence is -4 |Omega|^2; away from the faces every block sees them."""
    shape, dx, nb, n_buf = (20, 16, 24), 0.25, 4, 3
    om = np.array([0.3, -0.8, 0.5])
    u = _faces(shape, dx, lambda X, Y, Z: (om[1] * Z - om[2] * Y, om[2] * X - om[0] * Z, om[0] * Y - om[1] * X))
    mu, nu = blocks.weights(u, dx, nb, n_buf)
    assert mu.shape == (5, 4, 6)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.abs(mu[inner] - 2 * np.abs(om).max()).max() < 1e-12
    assert np.abs(nu[inner] - 4 * om @ om).max() < 1e-11


def test_point_vortex_footprint():
    """u = Cbar of one potential value: C u is nonzero only near that edge, so with a tiny threshold D_supp is
    the block holding it and D_xsoln the cube of (2 N_b + 1)^3 blocks around it."""
    n, dx, nb = 24, 0.5, 4
    a = np.zeros((3, n, n, n))
    a[2, 10, 9, 13] = 1.0  # inside block (2, 2, 3), one point away from its faces
    u = stencils.curl_bar(a, dx)
    mu, nu = blocks.weights(u, dx, nb, 1)
    W, supp, soln, xsoln = blocks.classify(mu, nu, 1e-3, 1e-3, 1)
    # the curl of Cbar a reaches one point around the edge, which stays inside the block
    assert supp.sum() == 1 and supp[2, 2, 3] == 1
    assert W.max() == 1.0
    assert xsoln.sum() == 27 and xsoln[1:4, 1:4, 2:5].all()


def test_expanded_domain_clipped_at_the_box():
    mu = np.zeros((4, 5, 6))
    nu = np.zeros((4, 5, 6))
    mu[0, 0, 0] = 2.0   # corner block
    nu[3, 2, 5] = 7.0   # on a face of the block grid
    W, supp, soln, xsoln = blocks.classify(mu, nu, 0.5, 0.5, 2)
    assert W[0, 0, 0] == 1.0 and W[3, 2, 5] == 1.0 and W.sum() == 2.0
    corner = np.zeros_like(xsoln)
    corner[0:3, 0:3, 0:3] = 1
    face = np.zeros_like(xsoln)
    face[1:4, 0:5, 3:6] = 1
    assert (xsoln == np.maximum(corner, face)).all()
    # a higher solution threshold keeps the support but drops the block from D_soln
    W, supp, soln, xsoln = blocks.classify(mu, nu, 0.5, 1.0, 2)
    assert supp.sum() == 2 and soln.sum() == 0 and xsoln.sum() == 0


def test_block_domains_in_the_step():
    """The solution and support domains as unions of blocks (Sec. 4.2, 4.3) inside the IF-HERK step:
    blocks equal to the box shrunk by n_buf reproduce the n_buf step exactly; a solution domain that
    misses every block where the flow is leaves no nonlinear term, so the step is the Stokes step; a
    support domain that misses the source gives no pressure."""
    n, dx, nb = 16, 0.3, 4
    f = np.zeros((3, n, n, n))
    f[:, 6:10, 6:10, 6:10] = np.random.default_rng(3).standard_normal((3, 4, 4, 4))
    u = stencils.curl_bar(f, dx)
    dt, re = 0.05, 50.0
    inner = np.zeros((4, 4, 4), dtype=np.uint8)
    inner[1:3, 1:3, 1:3] = 1
    m = blocks.cell_mask(inner, nb, (n, n, n))
    ref = ifherk.step(u, dt, dx, re, "A", n_buf=4)
    got = ifherk.step(u, dt, dx, re, "A", soln_mask=m, supp_mask=m)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    corner = np.zeros((4, 4, 4), dtype=np.uint8)
    corner[0, 0, 0] = 1
    mc = blocks.cell_mask(corner, nb, (n, n, n))
    stokes = ifherk.step(u, dt, dx, re, "A", nonlinear=False)
    got = ifherk.step(u, dt, dx, re, "A", soln_mask=mc, supp_mask=m)
    assert np.abs(got[0] - stokes[0]).max() < 1e-13 * np.abs(u).max()
    got = ifherk.step(u, dt, dx, re, "A", soln_mask=m, supp_mask=mc)
    assert np.abs(got[1]).max() < 1e-12 * np.abs(ref[1]).max()

