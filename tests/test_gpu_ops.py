"""GPU parity of the integrating factor (Sec. 2.3) and the staggered point operators (Appendix A)
against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_1601_00035_amd as nslgf
import workloads
from oracle import intfac, stencils

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("alpha", [0.0, 0.012, 0.0237, 0.3, 2.5])
def test_if_apply_fp64_fp32(alpha):
    shape = (2, 13, 17, 22)
    h = workloads.random_field(shape, 7)
    ref = np.stack([intfac.apply(h[q], alpha) for q in range(2)])
    out = nslgf.if_apply(torch.from_numpy(h).to(DEV), alpha).cpu().numpy()
    assert rel(out, ref) < 1e-13
    out32 = nslgf.if_apply(torch.from_numpy(h).to(DEV, torch.float32), alpha).double().cpu().numpy()
    assert rel(out32, ref) < 1e-6


def test_if_apply_in_place_six_components():
    shape = (6, 16, 9, 11)
    h = workloads.random_field(shape, 3)
    alpha = 0.04
    ref = np.stack([intfac.apply(h[q], alpha) for q in range(6)])
    t = torch.from_numpy(h).to(DEV)
    nslgf.if_apply(t, alpha, out=t)
    assert rel(t.cpu().numpy(), ref) < 1e-13


def test_if_apply_rejects_negative_alpha():
    t = torch.zeros((3, 4, 4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(nslgf.NslgfError):
        nslgf.if_apply(t, -0.1)
    # a diffusion so wide that the kernel radius exceeds the supported one is refused, not truncated
    with pytest.raises(nslgf.NslgfError):
        nslgf.if_apply(t, 1.0e4)
    with pytest.raises(nslgf.NslgfError):
        nslgf.if_apply(t, float("nan"))
    with pytest.raises(nslgf.NslgfError):
        nslgf.if_apply(torch.zeros((7, 4, 4, 4), dtype=torch.float64, device=DEV), 0.1)  # ncomp > 6


OPS = {
    "grad": (lambda f, dx: stencils.grad(f, dx), "scalar"),
    "div": (lambda f, dx: stencils.div(f, dx), "vector"),
    "curl": (lambda f, dx: stencils.curl(f, dx), "vector"),
    "curl_bar": (lambda f, dx: stencils.curl_bar(f, dx), "vector"),
    "nonlinear": (lambda f, dx: stencils.nonlinear(f, dx), "vector"),
}


@pytest.mark.parametrize("op", list(OPS))
@pytest.mark.parametrize("shape", [(7, 11, 16), (20, 20, 20), (1, 3, 2)])
def test_stencils(op, shape):
    fn, kind = OPS[op]
    dx = 0.41
    src = workloads.random_field(shape if kind == "scalar" else (3,) + shape, 17)
    ref = fn(src, dx)
    out = nslgf.stencil(op, torch.from_numpy(src).to(DEV), dx).cpu().numpy()
    assert rel(out, ref) < 1e-14
    out32 = nslgf.stencil(op, torch.from_numpy(src).to(DEV, torch.float32), dx).double().cpu().numpy()
    assert rel(out32, ref) < 2e-6


def test_laplacian_components():
    src = workloads.random_field((3, 9, 10, 11), 5)
    ref = np.stack([stencils.laplacian(src[q], 0.3) for q in range(3)])
    out = nslgf.stencil("laplacian", torch.from_numpy(src).to(DEV), 0.3).cpu().numpy()
    assert rel(out, ref) < 1e-14


def test_mimetic_identities_exact_on_gpu():
    n = 24
    c = torch.from_numpy(workloads.random_field((n, n, n), 1, integer=True)).to(DEV)
    f = torch.from_numpy(workloads.random_field((3, n, n, n), 2, integer=True)).to(DEV)
    assert not nslgf.stencil("curl", nslgf.stencil("grad", c, 1.0), 1.0).any()
    assert not nslgf.stencil("div", nslgf.stencil("curl_bar", f, 1.0), 1.0).any()


def test_max_cell_speed():
    u = workloads.random_field((3, 10, 12, 14), 4)
    from oracle import ifherk
    ref = ifherk.cell_speed_max(u)
    got = nslgf.max_cell_speed(torch.from_numpy(u).to(DEV))
    assert abs(got - ref) < 1e-14 * ref
