"""Learned initial step for the FB-LISA line search.

Algorithm 1 restarts every line search from the same alpha_0 (Step 2d) and backtracks
(Step 2c, alpha <- beta alpha) until the sufficient-decrease test (2.3) holds, paying one
forward projection per rejected trial.  Here a small perceptron proposes the first trial
step of each iteration from statistics the method already has on the host; the
backtracking is unchanged and still accepts or rejects every proposal, so the accepted
step satisfies (2.3) exactly as before and the appendix's convergence argument (any
initial guess no larger than alpha_max) still applies: proposals are clipped to
[alpha_min, alpha_0].

Features of iteration k >= 1 (all scale-free, known on the host without a device
read-back), computed from iteration k-1:
  1. (t - 1) / T                         epoch progress
  2. log10(2 fbar / (n_theta n_p))       mean squared residual per ray at x^k (the
                                         accepted trial's objective, on batch k-1)
  3. log10(||grad f_{N_{k-1}}|| / sqrt(d))  gradient norm per voxel
  4. log10(alpha_{k-1} / alpha_0)        last accepted step
  5. m_{k-1}                             backtracks of the last line search
Target: log10(alpha_k / alpha_0) of the accepted step.

The perceptron (5-64-64-1, ReLU, FP32) is trained on the GPU by the library's own
kernels (fbl_mlp_loss_grad, fbl_mlp_adam) and evaluated by fbl_mlp_forward.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from ._lib import MLP_IN, MLP_NPARAMS, mlp_adam, mlp_forward, mlp_loss_grad, mlp_workspace


def iteration_features(run, prev) -> List[float]:
    """Features of the next iteration of ``run`` (an FBLisa) from its last Iteration."""
    g = run.geom
    n_p = int(g.nu) * int(g.nv)
    d = int(g.nx) * int(g.ny) * int(g.nz)
    fbar = max(prev.trials[-1].f_bar, 1e-300)
    gn = max(prev.grad_norm, 1e-300)
    return [(max(run.epoch, 1) - 1) / float(run.epochs),
            math.log10(2.0 * fbar / (run.n * n_p)),
            math.log10(gn / math.sqrt(d)),
            math.log10(prev.alpha / run.alpha0),
            float(prev.backtracks)]


class TraceRecorder:
    """FBLisa.run callback collecting (features, target) pairs of a run."""

    def __init__(self):
        self.X: List[List[float]] = []
        self.t: List[float] = []
        self._prev = None

    def __call__(self, run, it):
        if it.k == 0:
            self._prev = None   # a new run starts
        if self._prev is not None:
            self.X.append(iteration_features(run, self._prev))   # run.epoch is it's epoch here
            self.t.append(math.log10(it.alpha / run.alpha0))
        self._prev = it

    def arrays(self):
        return np.asarray(self.X, dtype=np.float32).reshape(-1, MLP_IN), np.asarray(self.t, dtype=np.float32)


@dataclass
class Normalizer:
    """Per-feature affine standardisation fitted on the training set (part of the model)."""
    mean: np.ndarray
    scale: np.ndarray

    @classmethod
    def fit(cls, X: np.ndarray) -> "Normalizer":
        m = X.mean(axis=0)
        s = X.std(axis=0)
        s[s < 1e-6] = 1.0
        return cls(m.astype(np.float32), s.astype(np.float32))

    def __call__(self, X: np.ndarray) -> np.ndarray:
        return ((np.asarray(X, dtype=np.float32) - self.mean) / self.scale).astype(np.float32)


class StepModel:
    """The perceptron's parameters on the device, with its Adam state."""

    def __init__(self, params0: np.ndarray, device="cuda"):
        p = np.asarray(params0, dtype=np.float32).ravel()
        if p.size != MLP_NPARAMS:
            raise ValueError("need %d parameters" % MLP_NPARAMS)
        self.params = torch.from_numpy(p.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.steps = 0
        self.norm: Optional[Normalizer] = None

    def fit(self, X: np.ndarray, t: np.ndarray, iters: int = 2000, lr: float = 3e-3, beta1: float = 0.9,
            beta2: float = 0.999, eps: float = 1e-8) -> List[float]:
        """Full-batch Adam on the mean-squared error; returns the loss (1/(2n) sum e^2) every
        100 steps.  Features are standardised with statistics of X."""
        self.norm = Normalizer.fit(np.asarray(X, dtype=np.float32))
        Xd = torch.from_numpy(self.norm(X)).to(self.params.device).contiguous()
        td = torch.from_numpy(np.asarray(t, dtype=np.float32)).to(self.params.device).contiguous()
        n = Xd.shape[0]
        work = mlp_workspace(n, self.params.device)
        grad = torch.empty_like(self.params)
        loss = torch.zeros(1, dtype=torch.float64, device=self.params.device)
        curve = []
        for k in range(iters):
            mlp_loss_grad(self.params, Xd, td, work, grad, loss if k % 100 == 0 else None)
            self.steps += 1
            mlp_adam(self.params, grad, self.m, self.v, self.steps, lr, beta1, beta2, eps)
            if k % 100 == 0:
                curve.append(float(loss) / (2 * n))
        return curve

    def predict(self, X: np.ndarray) -> np.ndarray:
        Xd = torch.from_numpy(self.norm(np.asarray(X, dtype=np.float32).reshape(-1, MLP_IN))).to(self.params.device)
        return mlp_forward(self.params, Xd.contiguous()).cpu().numpy()


class LearnedStep:
    """Proposer for FBLisa.run(alpha_init=...): alpha_0 at the first iteration, then
    alpha_0 * beta^j with j the predicted number of halvings rounded down, less `margin`,
    clipped to [0, j_max] -- a proposal on the method's own step grid, never above alpha_0.

    The proposal errs towards the larger step: one above the step the plain search would
    accept costs one more trial (one forward projection) and then lands on that same step,
    while one below it is accepted as is and shortens the step, which costs iterations.
    margin = 1 proposes one notch larger still: the run then follows the plain search's
    steps more closely, at the price of more trials."""

    def __init__(self, model: StepModel, j_max: int = 20, margin: int = 0):
        self.model = model
        self.j_max = j_max
        self.margin = int(margin)
        dev = model.params.device
        self._x = torch.empty((1, MLP_IN), dtype=torch.float32).pin_memory()
        self._xd = torch.empty((1, MLP_IN), dtype=torch.float32, device=dev)
        self._yd = torch.empty(1, dtype=torch.float32, device=dev)
        self._y = torch.empty(1, dtype=torch.float32).pin_memory()

    def __call__(self, run) -> Optional[float]:
        if not run.history:
            return None
        f = self.model.norm(np.asarray([iteration_features(run, run.history[-1])], dtype=np.float32))
        self._x.numpy()[:] = f
        self._xd.copy_(self._x, non_blocking=True)
        mlp_forward(self.model.params, self._xd, self._yd)
        self._y.copy_(self._yd, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        log_ratio = float(self._y[0])
        j = int(math.floor(log_ratio / math.log10(run.beta))) - self.margin if math.isfinite(log_ratio) else 0
        j = min(max(j, 0), self.j_max)
        return run.alpha0 * run.beta ** j
