"""The projector pair as torch.autograd functions (HIP kernels through the C ABI).

Checks: torch.autograd.gradcheck of both directions on 8^3 and 16^3 volumes in true FP64
(the library's FP64 instantiation of the pair; finite differences with eps 1e-3 are
exact up to FP64 rounding for a linear map, so the tolerance is atol 1e-9); the same
gradcheck through the FP32 kernels, whose finite-difference Jacobian carries the FP32
rounding of the outputs divided by 2*eps (about 1e-6 / 2e-3), hence atol 2e-3, rtol
1e-3 there; second derivatives (A^T A v); a directional finite difference of the
mini-batch objective at 128^3 with 180 views (the objective is quadratic, so the central
difference is exact up to rounding); the adjoint dot-product identity through
vector-Jacobian products; the gradient against the FP64 oracle; and the FP64 pair itself
against the oracle to 1e-12.
"""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fbl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2605_12085_amd as fbl
    return fbl


@pytest.mark.parametrize("n,det", [(8, 12), (16, 20)])
def test_gradcheck_fp64_project_and_backproject(fbl, n, det):
    # true FP64: FP64 tensors run the FP64 instantiation of the pair in both directions
    import torch
    g = syn.tiny_geometry(n=n, det=det, views=16)
    views = [0, 3, 6, 13]   # both axis classes
    rng = np.random.default_rng(7)
    with fbl.Plan(g) as plan:
        x = torch.tensor(rng.uniform(0, 1, g.vol_shape), dtype=torch.float64, device="cuda", requires_grad=True)
        r = torch.tensor(rng.standard_normal((len(views), g.nv, g.nu)), dtype=torch.float64, device="cuda",
                         requires_grad=True)
        fp = lambda t: fbl.project(t, plan, views)
        bp = lambda t: fbl.backproject(t, plan, views)
        assert fp(x).dtype == torch.float64
        # the FP64 transpose adds with atomics, so repeated backward calls may differ by
        # FP64 rounding: nondet_tol admits that and nothing larger
        assert torch.autograd.gradcheck(fp, (x,), eps=1e-3, atol=1e-9, rtol=1e-7, nondet_tol=1e-12,
                                        fast_mode=n > 8)
        assert torch.autograd.gradcheck(bp, (r,), eps=1e-3, atol=1e-9, rtol=1e-7, nondet_tol=1e-12,
                                        fast_mode=n > 8)


def test_gradcheck_fp32_project_and_backproject(fbl):
    # the fast FP32 kernels, checked at the FP32 resolution of the finite differences
    import torch
    g = syn.tiny_geometry(n=8, det=12, views=16)
    views = [0, 3, 6, 13]
    rng = np.random.default_rng(7)
    with fbl.Plan(g) as plan:
        x = torch.tensor(rng.uniform(0, 1, g.vol_shape), dtype=torch.float64, device="cuda", requires_grad=True)
        r = torch.tensor(rng.standard_normal((len(views), g.nv, g.nu)), dtype=torch.float64, device="cuda",
                         requires_grad=True)
        fp = lambda t: fbl.project(t.float(), plan, views).double()
        bp = lambda t: fbl.backproject(t.float(), plan, views).double()
        assert torch.autograd.gradcheck(fp, (x,), eps=1e-3, atol=2e-3, rtol=1e-3, fast_mode=False)
        assert torch.autograd.gradcheck(bp, (r,), eps=1e-3, atol=2e-3, rtol=1e-3, fast_mode=False)


def test_fp64_pair_matches_oracle(fbl, orc):
    # the FP64 instantiation against the FP64 oracle: equal up to FP64 rounding (1e-12),
    # on odd sizes with axis-aligned and oblique views, both directions
    import torch
    g = syn.Geometry(29, 41, 37, 0.9, 1.1, 1.0, 50, 33, 1.7, 1.9, 400.0, 900.0, 12,
                     angles=[0.0, np.pi / 4, np.pi / 2, np.pi, 3 * np.pi / 2, 0.3, 1.7, 2.9, 4.0, 5.5, 0.05, 6.2])
    views = np.arange(g.n_views, dtype=np.int32)
    rng = np.random.default_rng(31)
    x = rng.uniform(-1, 1, g.vol_shape)
    r = rng.standard_normal((g.n_views, g.nv, g.nu))
    y_ref = orc.forward(g, x, views)
    g_ref = orc.backproject(g, r, views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward_f64(plan, torch.from_numpy(x).cuda(), views).cpu().numpy()
        gg = fbl.fb_lisa_backproject_f64(plan, torch.from_numpy(r).cuda(), views, grad_scale=1.0).cpu().numpy()
        # the gradient scale, and repeated views in one batch
        vv = np.array([0, 0, 3, 7, 7, 11], dtype=np.int32)
        rr = rng.standard_normal((len(vv), g.nv, g.nu))
        g2 = fbl.fb_lisa_backproject_f64(plan, torch.from_numpy(rr).cuda(), vv, grad_scale=0.5).cpu().numpy()
    for b in range(g.n_views):
        assert np.abs(y[b] - y_ref[b]).max() <= 1e-12 * np.abs(y_ref[b]).max(), b
    assert np.abs(gg - g_ref).max() <= 1e-12 * np.abs(g_ref).max()
    g2_ref = 0.5 * orc.backproject(g, rr, vv)
    assert np.abs(g2 - g2_ref).max() <= 1e-12 * np.abs(g2_ref).max()
    # adjoint identity in FP64
    lhs, rhs = float(np.sum(y * r)), float(np.sum(x * gg))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_second_derivative_is_normal_operator(fbl):
    import torch
    g = syn.tiny_geometry(n=8, det=12, views=16)
    views = [1, 5, 9, 12]
    rng = np.random.default_rng(8)
    with fbl.Plan(g) as plan:
        x = torch.tensor(rng.uniform(0, 1, g.vol_shape), dtype=torch.float32, device="cuda", requires_grad=True)
        v = torch.tensor(rng.uniform(-1, 1, g.vol_shape), dtype=torch.float32, device="cuda")
        loss = 0.5 * (fbl.project(x, plan, views) ** 2).sum()
        (grad,) = torch.autograd.grad(loss, x, create_graph=True)
        (hv,) = torch.autograd.grad(grad, x, grad_outputs=v)
        ref = fbl.fb_lisa_backproject(plan, fbl.fb_lisa_forward(plan, v, views), views, grad_scale=1.0)
        # grad = A^T A x
        gref = fbl.fb_lisa_backproject(plan, fbl.fb_lisa_forward(plan, x.detach(), views), views, grad_scale=1.0)
        torch.testing.assert_close(grad.detach(), gref, rtol=1e-5, atol=1e-5 * float(gref.abs().max()))
        torch.testing.assert_close(hv, ref, rtol=1e-5, atol=1e-5 * float(ref.abs().max()))


def test_directional_difference_of_objective_128(fbl):
    import torch
    g = syn.config_geometry("c4")
    B = syn.CONFIGS["c4"]["batch"]
    rng = np.random.default_rng(9)
    views = np.sort(rng.choice(g.n_views, B, replace=False))
    b = torch.tensor(syn.random_projections(g, g.n_views, seed=10, scale=0.5), dtype=torch.float32, device="cuda")
    x = torch.tensor(syn.random_volume(g, seed=11), device="cuda", requires_grad=True)
    d = torch.tensor(syn.random_volume(g, seed=12, lo=-0.02, hi=0.02), device="cuda")
    with fbl.Plan(g, max_batch=B) as plan:
        f = fbl.data_fidelity(x, plan, views, b)
        (grad,) = torch.autograd.grad(f, x)
        slope = float((grad.double() * d.double()).sum())
        eps = 1e-3
        fp = float(fbl.data_fidelity((x + eps * d).detach(), plan, views, b))
        fm = float(fbl.data_fidelity((x - eps * d).detach(), plan, views, b))
    fd = (fp - fm) / (2 * eps)
    assert fd == pytest.approx(slope, rel=1e-3), (fd, slope)


def test_adjoint_identity_through_vjp(fbl):
    import torch
    g = syn.config_geometry("c4")
    rng = np.random.default_rng(13)
    views = np.sort(rng.choice(g.n_views, 10, replace=False))
    x = torch.tensor(syn.random_volume(g, seed=14), device="cuda", requires_grad=True)
    y = torch.tensor(rng.standard_normal((len(views), g.nv, g.nu)), dtype=torch.float32, device="cuda")
    with fbl.Plan(g, max_batch=10) as plan:
        ax = fbl.project(x, plan, views)
        (aty,) = torch.autograd.grad(ax, x, grad_outputs=y)
    lhs = float((ax.detach().double() * y.double()).sum())
    rhs = float((x.detach().double() * aty.double()).sum())
    assert lhs == pytest.approx(rhs, rel=1e-5)


def test_gradient_matches_oracle(fbl, orc):
    import torch
    g = syn.Geometry(29, 41, 37, 0.9, 1.1, 1.0, 50, 33, 1.7, 1.9, 400.0, 900.0, 12)
    views = np.array([0, 2, 5, 7, 11], dtype=np.int32)
    x32 = syn.random_volume(g, seed=15)
    b32 = syn.random_projections(g, g.n_views, seed=16, scale=0.3).astype(np.float32)
    f_ref, g_ref, _ = orc.objective_and_gradient(g, x32.astype(np.float64), b32.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        x = torch.tensor(x32, device="cuda", requires_grad=True)
        f = fbl.data_fidelity(x, plan, views, torch.from_numpy(b32).cuda())
        (grad,) = torch.autograd.grad(3.0 * f, x)   # an upstream scale reaches the gradient
    assert float(f) == pytest.approx(f_ref, rel=1e-5)
    got = grad.cpu().numpy().astype(np.float64) / 3.0
    assert np.linalg.norm(got - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    assert np.abs(got - g_ref).max() <= 1e-5 * np.abs(g_ref).max()
