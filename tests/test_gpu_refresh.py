"""GPU parity of the velocity refresh and the multi-step driver with its refresh cadence (Sec. 4.4,
Appendix D) against the oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import paper_1601_00035_amd as nslgf
import workloads
from oracle import ifherk, refresh

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_max_component_abs():
    u = workloads.random_field((3, 13, 17, 21), 41)
    for n_buf in (0, 1, 4):
        ref = refresh.component_max(u, n_buf)
        assert nslgf.max_component_abs(torch.from_numpy(u).to(DEV), n_buf) == ref
    u32 = torch.from_numpy(u).to(DEV, torch.float32)
    ref32 = refresh.component_max(u32.double().cpu().numpy(), 2)
    assert nslgf.max_component_abs(u32, 2) == ref32


@pytest.mark.parametrize("shape,n_buf", [((20, 22, 26), 3), ((16, 16, 16), 0), ((24, 18, 20), 5)])
def test_velocity_refresh(shape, n_buf):
    dx = 0.37
    u = workloads.random_field((3,) + shape, 43)
    ref = refresh.velocity_refresh(u, dx, n_buf)
    got = nslgf.velocity_refresh(torch.from_numpy(u).to(DEV), dx, n_buf).cpu().numpy()
    assert rel(got, ref) < 1e-12
    got32 = nslgf.velocity_refresh(torch.from_numpy(u).to(DEV, torch.float32), dx, n_buf).double().cpu().numpy()
    assert rel(got32, ref) < 1e-6


def _ring(n=20, seed=3):
    n, dx, ring, _, cfl = workloads.small_ring_case(n, seed)
    u0 = ifherk.vor2vel(workloads.ring_edge_vorticity(n, dx, ring), dx)
    return n, dx, u0, 100.0, ifherk.dt_from_cfl(u0, dx, cfl)


@pytest.mark.parametrize("scheme", ["A", "C"])
def test_run_with_refresh(scheme):
    """Five steps with eps set between the estimates after two and three steps: the velocity is
    refreshed after steps 2 and 4 on both sides."""
    n, dx, u0, re, dt = _ring()
    n_buf = 3
    beta = dt / (dx * dx * re)
    umax = refresh.component_max(u0, n_buf)
    eps = math.sqrt(refresh.estimate(beta, 2, n_buf, umax) * refresh.estimate(beta, 3, n_buf, umax))
    u_ref, d_ref, nref, qs = refresh.run(u0, 5, dt, dx, re, scheme, n_buf, eps)
    assert nref == 2 and qs == [2, 2, 2]
    u = torch.from_numpy(u0).to(DEV)
    st = nslgf.HerkState(u, dx, dt, re, scheme, n_buf=n_buf)
    assert st.run(5, eps) == 2
    assert rel(u.cpu().numpy(), u_ref) < 1e-12
    assert rel(st.d.cpu().numpy(), d_ref) < 1e-12
    assert abs(st.t - 5 * dt) < 1e-14


def test_run_without_refresh_equals_steps():
    """A cadence longer than the run: herk_run is plain herk_step calls (bitwise)."""
    n, dx, u0, re, dt = _ring(18)
    a = torch.from_numpy(u0).to(DEV)
    b = a.clone()
    sa = nslgf.HerkState(a, dx, dt, re, "A", n_buf=3)
    sb = nslgf.HerkState(b, dx, dt, re, "A", n_buf=3)
    assert sa.run(3, 1.0) == 0
    for _ in range(3):
        sb.step()
    assert torch.equal(a, b) and torch.equal(sa.d, sb.d)
    # zero steps leave the state alone
    c = a.clone()
    assert sa.run(0, 1.0) == 0 and torch.equal(a, c)


def test_run_errors():
    n, dx, u0, re, dt = _ring(18)
    u = torch.from_numpy(u0).to(DEV)
    st = nslgf.HerkState(u, dx, dt, re, "A", n_buf=0)
    with pytest.raises(nslgf.NslgfError):
        st.run(2, 1e-30)  # no buffer: one step already exceeds eps
    st = nslgf.HerkState(u, dx, dt, re, "A", n_buf=2)
    for nsteps, eps, cap in ((-1, 1e-6, 10), (2, 0.0, 10), (2, 1e-6, 0)):
        with pytest.raises(nslgf.NslgfError):
            st.run(nsteps, eps, cap)
    with pytest.raises(nslgf.NslgfError):
        nslgf.velocity_refresh(u, -1.0, 2)
    with pytest.raises(nslgf.NslgfError):
        nslgf.velocity_refresh(u, dx, -1)


def test_run_with_refresh_fp32():
    """The FP32 run refreshes after the same steps as FP64 (eps sits between the estimates after two
    and three steps, a factor of five apart) and stays within FP32 rounding of it."""
    n, dx, u0, re, dt = _ring()
    n_buf = 3
    beta = dt / (dx * dx * re)
    umax = refresh.component_max(u0, n_buf)
    eps = math.sqrt(refresh.estimate(beta, 2, n_buf, umax) * refresh.estimate(beta, 3, n_buf, umax))
    out = {}
    for dtype in (torch.float64, torch.float32):
        u = torch.from_numpy(u0).to(DEV, dtype)
        st = nslgf.HerkState(u, dx, dt, re, "A", n_buf=n_buf)
        out[dtype] = (st.run(5, eps), u.double().cpu().numpy())
    assert out[torch.float32][0] == out[torch.float64][0] == 2
    ref = out[torch.float64][1]
    assert rel(out[torch.float32][1], ref) < 1e-5
