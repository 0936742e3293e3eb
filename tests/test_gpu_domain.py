"""GPU parity of the active-domain block weights (Sec. 4.3, Eq. weight_fun) against the oracle through
the C ABI, their closed form for a rigid rotation, and the classification of a ring's blocks."""
import numpy as np
import pytest
import torch

import paper_1601_00035_amd as nslgf
import workloads
from oracle import blocks, ifherk
from oracle import diagnostics as dg

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("shape,nb,n_buf", [((24, 24, 24), 4, 2), ((20, 26, 22), 5, 1), ((16, 16, 16), 16, 0)])
def test_block_weights_parity(shape, nb, n_buf):
    nz, ny, nx = shape
    dx = 4.4 / min(shape)
    m = max(shape)
    w = workloads.ring_edge_vorticity(m, dx, workloads.Ring(R=1.0, sigma=0.3, eps=0.05, seed=4))
    o = (m - nx) // 2, (m - ny) // 2, (m - nz) // 2
    w = np.ascontiguousarray(w[:, o[2]:o[2] + nz, o[1]:o[1] + ny, o[0]:o[0] + nx])
    u = ifherk.vor2vel(w, dx)
    mu_r, nu_r = blocks.weights(u, dx, nb, n_buf)
    mu, nu = nslgf.block_weights(torch.from_numpy(u).to(DEV), dx, nb, n_buf)
    assert mu.shape == mu_r.shape
    assert np.abs(mu - mu_r).max() <= 1e-12 * mu_r.max()
    assert np.abs(nu - nu_r).max() <= 1e-12 * nu_r.max()
    mu32, nu32 = nslgf.block_weights(torch.from_numpy(u).to(DEV, torch.float32), dx, nb, n_buf)
    assert np.abs(mu32 - mu_r).max() <= 1e-5 * mu_r.max()
    assert np.abs(nu32 - nu_r).max() <= 1e-5 * nu_r.max()
    # the classification of the GPU weights equals the oracle's wherever W is not within rounding of eps
    eps = 1e-3
    W_r, s_r, _, x_r = blocks.classify(mu_r, nu_r, eps, eps, 1)
    W, s, _, x = nslgf.classify_blocks(mu, nu, eps, eps, 1)
    clear = np.abs(W_r - eps) > 1e-9
    assert np.array_equal(s[clear], s_r[clear])
    assert np.abs(W - W_r).max() < 1e-11


def test_block_weights_rigid_rotation():
    shape, dx, nb, n_buf = (20, 16, 24), 0.25, 4, 3
    om = np.array([0.3, -0.8, 0.5])
    o = dg.box_origin(shape, dx)
    u = []
    for q in range(3):
        X, Y, Z = dg._coords(shape, dx, o, [0 if a == q else 1 for a in range(3)])
        u.append((om[1] * Z - om[2] * Y, om[2] * X - om[0] * Z, om[0] * Y - om[1] * X)[q])
    u = torch.from_numpy(np.stack(u)).to(DEV)
    mu, nu = nslgf.block_weights(u, dx, nb, n_buf)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.abs(mu[inner] - 2 * np.abs(om).max()).max() < 1e-12
    assert np.abs(nu[inner] - 4 * om @ om).max() < 1e-11


def test_block_weights_errors():
    u = torch.zeros((3, 8, 8, 8), dtype=torch.float64, device=DEV)
    for nb, n_buf, dx in ((0, 1, 0.1), (4, -1, 0.1), (4, 1, 0.0)):
        with pytest.raises(nslgf.NslgfError):
            nslgf.block_weights(u, dx, nb, n_buf)


@pytest.mark.parametrize("scheme", ["A", "C"])
def test_step_with_block_domains(scheme):
    """IF-HERK steps whose support and solution domains are unions of blocks (Sec. 4.2, 4.3) taken from
    the classification of the flow's own weights, against the oracle's step with the same cell masks."""
    n, dx, ring, re, cfl = workloads.small_ring_case(24, seed=6)
    w = workloads.ring_edge_vorticity(n, dx, ring)
    u0 = ifherk.vor2vel(w, dx)
    dt = ifherk.dt_from_cfl(u0, dx, cfl)
    nb = 4
    mu, nu = blocks.weights(u0, dx, nb, 1)
    _, supp, soln, _ = blocks.classify(mu, nu, 1e-4, 1e-1, 1)
    assert 0 < soln.sum() < supp.sum() < supp.size
    cs, cn = blocks.cell_mask(supp, nb, u0.shape[1:]), blocks.cell_mask(soln, nb, u0.shape[1:])
    u_ref, d_ref = ifherk.step(u0, dt, dx, re, scheme, soln_mask=cn, supp_mask=cs)
    u = torch.from_numpy(u0).to(DEV)
    st = nslgf.HerkState(u, dx, dt, re, scheme, n_buf=0)
    st.set_blocks(supp, soln, nb)
    st.step()
    assert np.abs(u.cpu().numpy() - u_ref).max() <= 1e-12 * np.abs(u_ref).max()
    assert np.abs(st.d.cpu().numpy() - d_ref).max() <= 1e-12 * np.abs(d_ref).max()


def test_blocks_equal_to_the_buffer_form():
    """Blocks covering exactly the box shrunk by n_buf give the n_buf step bit for bit (same kernels,
    same arithmetic), one by one and in the batched graph."""
    n, dx, ring, re, cfl = workloads.small_ring_case(24, seed=7)
    u0 = torch.from_numpy(ifherk.vor2vel(workloads.ring_edge_vorticity(n, dx, ring), dx)).to(DEV)
    dt = cfl * dx / nslgf.max_cell_speed(u0)
    inner = np.zeros((6, 6, 6), dtype=np.uint8)
    inner[1:5, 1:5, 1:5] = 1
    a, b, c = u0.clone(), u0.clone(), u0.clone()
    sa = nslgf.HerkState(a, dx, dt, re, "B", n_buf=4)
    sb = nslgf.HerkState(b, dx, dt, re, "B", n_buf=0)
    sb.set_blocks(inner, inner, 4)
    sc = nslgf.HerkState(c, dx, dt, re, "B", n_buf=0)
    sc.set_blocks(inner, inner, 4)
    sa.step()
    sb.step()
    nslgf.herk_step_batched([sc])
    assert torch.equal(a, b) and torch.equal(sa.d, sb.d)
    assert torch.equal(a, c) and torch.equal(sa.d, sc.d)
    with pytest.raises(ValueError):
        sb.set_blocks(inner[:5], inner, 4)
    sb.c.block = 0
    with pytest.raises(nslgf.NslgfError):
        sb.step()


def test_run_adaptive():
    """Four steps on an active domain re-classified every step (Sec. 4.3) against the oracle: the same
    domains (the thresholds sit clear of every block weight), the same re-initialisations, and the
    same velocity and pressure."""
    from oracle import refresh

    n, dx, ring, re, cfl = workloads.small_ring_case(24, seed=6)
    u0 = ifherk.vor2vel(workloads.ring_edge_vorticity(n, dx, ring), dx)
    dt = ifherk.dt_from_cfl(u0, dx, cfl)
    args = dict(nb=4, eps_supp=1e-4, eps_soln=1e-1, n_xb=1)
    u_ref, d_ref, nre, Ws, edge = refresh.run_adaptive(u0, 4, dt, dx, 100.0, "A", 1, **args)
    for W in Ws:
        assert np.abs(W - args["eps_supp"]).min() > 1e-9 and np.abs(W - args["eps_soln"]).min() > 1e-9
    assert nre >= 1
    u = torch.from_numpy(u0).to(DEV)
    st = nslgf.HerkState(u, dx, dt, 100.0, "A", n_buf=1)
    got = st.run_adaptive(4, args["nb"], args["eps_supp"], args["eps_soln"], args["n_xb"])
    assert got == (nre, sum(edge))
    assert np.abs(u.cpu().numpy() - u_ref).max() <= 1e-12 * np.abs(u_ref).max()
    assert np.abs(st.d.cpu().numpy() - d_ref).max() <= 1e-12 * np.abs(d_ref).max()
    with pytest.raises(nslgf.NslgfError):
        st.run_adaptive(1, 0, 1e-4, 1e-1)


def test_run_adaptive_fp32():
    """The FP32 form of the adaptive run takes the same domain decisions as FP64 (the block weights sit
    far from the thresholds at FP32 resolution) and stays within FP32 rounding of it."""
    n, dx, ring, re, cfl = workloads.small_ring_case(24, seed=6)
    u0 = ifherk.vor2vel(workloads.ring_edge_vorticity(n, dx, ring), dx)
    dt = ifherk.dt_from_cfl(u0, dx, cfl)
    out = {}
    for dtype in (torch.float64, torch.float32):
        u = torch.from_numpy(u0).to(DEV, dtype)
        st = nslgf.HerkState(u, dx, dt, 100.0, "A", n_buf=1)
        counts = st.run_adaptive(4, 4, 1e-4, 1e-1, 1)
        out[dtype] = (counts, u.double().cpu().numpy())
    assert out[torch.float32][0] == out[torch.float64][0]
    ref = out[torch.float64][1]
    assert np.abs(out[torch.float32][1] - ref).max() <= 1e-5 * np.abs(ref).max()


def test_full_size_refresh_weights_and_integrals():
    """At the benchmark's 256^3 FP64 ring (the launch shapes the bench times), properties that hold at
    any size: the refresh returns a Vor2Vel velocity whose vorticity lies inside the support; the
    largest block weight mu equals the largest |C u| over the trusted points (same curl arithmetic);
    the impulse of the velocity matches the sampled ring's closed form."""
    import math

    n, dx, ring, re, cfl = workloads.ring_case("conv256")
    w = torch.from_numpy(workloads.ring_edge_vorticity(n, dx, ring)).to(DEV)
    u = nslgf.vor2vel(w, dx)
    v = nslgf.velocity_refresh(u.clone(), dx, 16)
    assert ((v - u).abs().max() / u.abs().max()).item() < 1e-10
    mu, nu = nslgf.block_weights(u, dx, 16, 16)
    cu = nslgf.stencil("curl", u, dx)[:, 16:-16, 16:-16, 16:-16]
    assert mu.max() == cu.abs().max().item()
    assert nu.max() > 0 and mu.shape == (16, 16, 16)
    r = nslgf.flow_diagnostics(u, dx, dg.box_origin((n, n, n), dx), 16)
    assert abs(r["I"][2] / (math.pi * (ring.R ** 2 + ring.sigma ** 2 / 2)) - 1) < 1e-4


def test_run_adaptive_leaves_the_state_domain_in_place():
    """An adaptive run classifies into handle memory and restores the state's own masks when it
    returns: a state given masks by set_blocks keeps them after its adaptive run, even after another
    state's adaptive run on a larger box has reused (and grown) the handle's mask memory."""
    n, dx, ring, re, cfl = workloads.small_ring_case(24, seed=6)
    u0 = ifherk.vor2vel(workloads.ring_edge_vorticity(n, dx, ring), dx)
    dt = ifherk.dt_from_cfl(u0, dx, cfl)
    inner = np.zeros((6, 6, 6), dtype=np.uint8)
    inner[1:-1, 1:-1, 1:-1] = 1
    b = torch.from_numpy(u0).to(DEV)
    sb = nslgf.HerkState(b, dx, dt, 100.0, "A", n_buf=0)
    sb.set_blocks(inner, inner, 4)
    sb.run_adaptive(2, 4, 1e-4, 1e-1, 1)
    assert sb.c.supp_blocks == sb._blocks[0].data_ptr() and sb.c.soln_blocks == sb._blocks[1].data_ptr()
    assert sb.c.block == 4
    m, dxm, rm, rem, cflm = workloads.small_ring_case(40, seed=7)
    um = ifherk.vor2vel(workloads.ring_edge_vorticity(m, dxm, rm), dxm)
    sc = nslgf.HerkState(torch.from_numpy(um).to(DEV), dxm, ifherk.dt_from_cfl(um, dxm, cflm), 100.0, "A", n_buf=1)
    sc.run_adaptive(1, 2, 1e-4, 1e-1, 1)
    assert sc.c.supp_blocks is None and sc.c.soln_blocks is None
    ref = nslgf.HerkState(b.clone(), dx, dt, 100.0, "A", n_buf=0)
    ref.set_blocks(inner, inner, 4)
    ref.step()
    sb.step()
    assert torch.equal(ref.u, sb.u) and torch.equal(ref.d, sb.d)
