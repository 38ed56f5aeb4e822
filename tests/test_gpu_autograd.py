"""Adjoints and autograd on the GPU (T399 on O400, 137 fields, FP32, and a
tiny FP64 plan for torch.autograd.gradcheck)."""
import numpy as np
import pytest

import synth_inputs as si
from error_metrics import spec_errors

pytestmark = pytest.mark.gpu


def _setup(key="t399_o400", prec="fp32"):
    import torch
    import paper_1908_06097_amd as shtx
    if not torch.cuda.is_available():
        pytest.fail("GPU test without a GPU")
    wl = si.WORKLOADS[key]
    plan = shtx.Plan(wl.trunc, wl.grid, wl.nlat, wl.nfld, prec)
    return torch, shtx, wl, plan


def _rdot(x, y):
    """Euclidean inner product over all real components, in float64."""
    import torch
    if x.is_complex():
        x, y = torch.view_as_real(x), torch.view_as_real(y)
    return float((x.double() * y.double()).sum())


@pytest.fixture(scope="module")
def c4():
    torch, shtx, wl, plan = _setup()
    print(f"{wl.name}: plan ready", flush=True)
    a = torch.from_numpy(si.spectral_fields(wl.trunc, wl.key, range(wl.nfld))).to(torch.complex64).cuda()
    yield torch, shtx, wl, plan, a
    plan.close()


def test_dot_product_inverse(c4):
    torch, shtx, wl, plan, a = c4
    y = torch.from_numpy(np.stack([si.white_noise_grid(plan.npts, 700 + f) for f in range(wl.nfld)])).float().cuda()
    lhs = _rdot(plan.inv(a), y)
    rhs = _rdot(a, plan.inv_adj(y))
    print(f"  <inv a, y> = {lhs:.9e}  <a, inv_adj y> = {rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_dot_product_direct(c4):
    torch, shtx, wl, plan, a = c4
    y = torch.from_numpy(np.stack([si.white_noise_grid(plan.npts, 800 + f) for f in range(wl.nfld)])).float().cuda()
    b = a.clone()
    lhs = _rdot(plan.dir(y), b)
    rhs = _rdot(y, plan.dir_adj(b))
    print(f"  <dir y, b> = {lhs:.9e}  <y, dir_adj b> = {rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_finite_differences_ten_directions(c4):
    """L(a) = sum g^2, g = inv(a).  L is quadratic, so the central difference
    is exact up to rounding for any step; compare with <grad, d>."""
    torch, shtx, wl, plan, a = c4
    x = a.clone().requires_grad_(True)
    g = shtx.InvTrans.apply(x, plan)
    loss = (g.double() ** 2).sum()
    loss.backward()
    grad = x.grad.detach()
    gnorm = float(torch.linalg.vector_norm(g.detach().double()))
    grad_norm = float(torch.linalg.vector_norm(torch.view_as_real(grad).double()))
    for k in range(10):
        d = torch.from_numpy(si.random_unit((wl.nfld, plan.nspec), 9000 + k, complex_=True)).to(torch.complex64).cuda()
        # step sized so that the perturbation of the grid is as large as the grid
        eps = gnorm / float(torch.linalg.vector_norm(plan.inv(d).double()))
        lp = float((plan.inv(a + eps * d).double() ** 2).sum())
        lm = float((plan.inv(a - eps * d).double() ** 2).sum())
        fd = (lp - lm) / (2 * eps)
        an = _rdot(grad, d)
        # |d| = 1, so |<grad, d>| <= |grad|: measure the defect against that bound
        print(f"  dir {k}: fd {fd:.8e} autograd {an:.8e} bound {grad_norm:.3e}", flush=True)
        assert abs(fd - an) <= 1e-5 * grad_norm


def test_gradient_vs_oracle(c4):
    import oracle
    torch, shtx, wl, plan, a = c4
    x = a.clone().requires_grad_(True)
    g = shtx.InvTrans.apply(x, plan)
    (g.double() ** 2).sum().backward()
    grad = x.grad.detach().cpu().numpy()
    fields = [0, 68, 136]
    a_np = si.spectral_fields(wl.trunc, wl.key, fields)
    nlon = plan.ring_lengths()
    ref = 2 * oracle.inv_adj(wl.trunc, nlon, oracle.inv(wl.trunc, nlon, a_np))
    em, er = spec_errors(grad[fields], ref, wl.trunc)
    print(f"  grad e_max {em.max():.2e} e_rms {er.max():.2e}", flush=True)
    assert er.max() < 1e-5


def test_dir_autograd_matches_adjoint(c4):
    torch, shtx, wl, plan, a = c4
    y = plan.inv(a).detach().clone().requires_grad_(True)
    s = shtx.DirTrans.apply(y, plan)
    w = torch.from_numpy(si.spectral_fields(wl.trunc, 55, range(wl.nfld))).to(torch.complex64).cuda()
    (torch.view_as_real(s) * torch.view_as_real(w)).sum().backward()
    ref = plan.dir_adj(w)
    assert torch.equal(y.grad, ref)


def test_gradcheck_fp64_tiny():
    import torch
    import paper_1908_06097_amd as shtx
    plan = shtx.Plan(15, "octahedral", 32, 2, "fp64")
    a = torch.from_numpy(si.spectral_fields(15, 3, [0, 1])).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: shtx.InvTrans.apply(x, plan), (a,), eps=1e-6, atol=1e-8)
    g = torch.from_numpy(np.stack([si.white_noise_grid(plan.npts, 40 + f) for f in range(2)])).cuda()
    g.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: shtx.DirTrans.apply(x, plan), (g,), eps=1e-6, atol=1e-8)
    plan.close()
