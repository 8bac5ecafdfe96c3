"""The projector pair as differentiable torch operations.

The forward projector A_N (Joseph, eq. 2.4/2.5 mini-batch of views) is linear, so its
vector-Jacobian product is the matched backprojection A_N^T, and that of A_N^T is
A_N.  Both directions run in the library's kernels:

  project(x, plan, views)         y = A_N x           backward: A_N^T grad_y
  backproject(r, plan, views)     g = A_N^T r         backward: A_N grad_g
  data_fidelity(x, plan, views, b)
      f_N(x) = n_theta/(2|N|) ||A_N x - b_N||^2 (eq. 2.5), an FP64 scalar;
      backward: grad_f * n_theta/|N| * A_N^T (A_N x - b_N), the gradient the method uses.

Because each backward is itself one of these differentiable operations, higher-order
derivatives (for instance Hessian-vector products A_N^T A_N v) are available too.
Volumes are [nz][ny][nx] CUDA tensors in the plan's layout, projections [B][nv][nu]:
FP32 tensors run the library's fast kernels, FP64 tensors its FP64 check instantiation
(project and backproject), so that torch.autograd.gradcheck can work in true FP64.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch
from torch.autograd.function import once_differentiable

from ._lib import Plan, fb_lisa_backproject, fb_lisa_backproject_f64, fb_lisa_forward, fb_lisa_forward_f64


def _fp(plan, x, views):
    # FP64 tensors take the FP64 check instantiation of the pair, FP32 ones the fast path
    if x.dtype == torch.float64:
        return fb_lisa_forward_f64(plan, x.contiguous(), views)
    return fb_lisa_forward(plan, x.contiguous(), views)


def _bp(plan, r, views):
    if r.dtype == torch.float64:
        return fb_lisa_backproject_f64(plan, r.contiguous(), views, grad_scale=1.0)
    return fb_lisa_backproject(plan, r.contiguous(), views, grad_scale=1.0)


def _as_views(views) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(views, dtype=np.int32).ravel())


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan, views: np.ndarray) -> torch.Tensor:
        ctx.plan, ctx.views = plan, views
        return _fp(plan, x, views)

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        return _Backproject.apply(grad_y, ctx.plan, ctx.views), None, None


class _Backproject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r: torch.Tensor, plan: Plan, views: np.ndarray) -> torch.Tensor:
        ctx.plan, ctx.views = plan, views
        return _bp(plan, r, views)

    @staticmethod
    def backward(ctx, grad_g: torch.Tensor):
        return _Project.apply(grad_g, ctx.plan, ctx.views), None, None


class _DataFidelity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan, views: np.ndarray, b: torch.Tensor) -> torch.Tensor:
        B = len(views)
        loss = torch.zeros(1, dtype=torch.float64, device=x.device)
        r = fb_lisa_forward(plan, x.contiguous(), views, b, loss=loss, loss_scale=plan.n_views / (2.0 * B))
        ctx.plan, ctx.views = plan, views
        ctx.save_for_backward(r)
        return loss[0]

    @staticmethod
    @once_differentiable
    def backward(ctx, grad_f: torch.Tensor):
        (r,) = ctx.saved_tensors
        B = len(ctx.views)
        # n_theta/|N| A^T r, then the upstream scalar (kept on the device: no host sync)
        g = fb_lisa_backproject(ctx.plan, r, ctx.views, grad_scale=ctx.plan.n_views / float(B))
        return g * grad_f.to(g.dtype), None, None, None


def project(x: torch.Tensor, plan: Plan, views: Sequence[int]) -> torch.Tensor:
    """y = A_views x, differentiable in x (vector-Jacobian product: the backprojection)."""
    return _Project.apply(x, plan, _as_views(views))


def backproject(r: torch.Tensor, plan: Plan, views: Sequence[int]) -> torch.Tensor:
    """g = A_views^T r, differentiable in r (vector-Jacobian product: the forward projection)."""
    return _Backproject.apply(r, plan, _as_views(views))


def data_fidelity(x: torch.Tensor, plan: Plan, views: Sequence[int], b: torch.Tensor) -> torch.Tensor:
    """f_N(x) of eq. 2.5 as a 0-dim FP64 tensor, differentiable in x; its gradient is
    n_theta/|N| A_N^T (A_N x - b_N) from one backprojection of the stored residual (first
    order only: the residual is not tracked as a function of x)."""
    return _DataFidelity.apply(x, plan, _as_views(views), b)
