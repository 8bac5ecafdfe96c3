"""FB-LISA (Algorithm 1 of arXiv 2605.12085) on one GPU through libfblisa.

The loop's host logic is the method's control flow only: the mini-batch size rule
(Step 1), the choice of the mini-batch (Step 2a, from caller-supplied permutations),
the accept/reject decision of the sufficient-decrease test (2.3) on three FP64 scalars
read back once per trial (Step 2c), and the step reset (Step 2d).  Every array
operation runs in the library's kernels: the forward projection with the residual and
the FP64 mini-batch objective, the backprojection (gradient), and the prox trial with
its FP64 inner products.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import Plan, fb_lisa_backproject, fb_lisa_forward, fb_lisa_step, fb_lisa_step_mixed


class LineSearchFailed(RuntimeError):
    pass


def eps_power(k: int, base: float = 0.99) -> float:
    """The summable sequence eps_k = base^k (the paper uses base 0.99)."""
    return math.pow(base, k)


def sr_key(seed: int, k: int, j: int) -> int:
    """Stochastic-rounding key of line-search trial j of iteration k: (seed << 32) +
    (k << 6) + j modulo 2^64 (j < 64: at most j_max + 1 <= 64 trials)."""
    return ((int(seed) << 32) + (int(k) << 6) + int(j)) & 0xFFFFFFFFFFFFFFFF


def _ceil(z: float) -> int:
    # an FP-exact integer is not rounded up by representation noise
    return int(math.ceil(z - 1e-9))


def next_batch_size(n_prev: int, k_hat: int, n: int, n0: int, n_max: int, C: float,
                    eps: Callable[[int], float]) -> int:
    """Step 1: N_t = min{n_max, max{ceil(C / eps_{k_hat + ceil(n / N_{t-1})}), N_0}}."""
    return min(n_max, max(_ceil(C / eps(k_hat + int(math.ceil(n / n_prev)))), n0))


def constant_batch_C(n: int, n0: int, epochs: int, eps: Callable[[int], float] = eps_power) -> float:
    """C for which Step 1 keeps N_t = N_0 for `epochs` epochs."""
    return n0 * eps(epochs * int(math.ceil(n / n0)))


def growing_batch_C(n: int, n0: int, eps: Callable[[int], float] = eps_power) -> float:
    """C for which Step 1 starts at N_0 and grows the batch as eps_k decays."""
    return n0 * eps(int(math.ceil(n / n0)))


@dataclass
class Trial:
    alpha: float
    f_bar: float
    inner: float
    sq: float
    accepted: bool


@dataclass
class Iteration:
    epoch: int
    k: int
    batch: np.ndarray
    f0: float
    alpha: float
    backtracks: int
    grad_norm: float = float("nan")
    trials: List[Trial] = field(default_factory=list)
    seconds: float = 0.0


class FBLisa:
    """GPU FB-LISA on a fixed data set b [n_views][nv][nu] (device tensor).

    x starts at x0 (default 0).  ``alpha_init(state)`` may propose the first trial step
    of an iteration (default: alpha_0, the paper's reset); the sufficient-decrease test
    and the backtracking still decide on every proposal.

    ``mixed=True`` with a 16-bit ``vol_dtype`` keeps the iterate in FP32 (x, xbar) and
    gives the projector a 16-bit copy of it (x16, xbar16, written by the prox trial):
    f and its gradient are evaluated at the copy, the prox step and the inner products
    of (2.3) on the FP32 values.
    """

    def __init__(self, geom, b: torch.Tensor, *, n0: int, epochs: int, alpha0: float = 1e-3, beta: float = 0.5,
                 mu: float = 0.0, lo: float = 0.0, hi: float = math.inf, C: Optional[float] = None,
                 n_max: Optional[int] = None, eps: Callable[[int], float] = eps_power, j_max: int = 50,
                 x0: Optional[torch.Tensor] = None, vol_dtype: str = "f32", proj_dtype: Optional[str] = None,
                 plan: Optional[Plan] = None, sr_seed: Optional[int] = None, mixed: bool = False):
        self.geom = geom
        self.n = int(geom.n_views)
        self.n0, self.epochs = int(n0), int(epochs)
        self.alpha0, self.beta, self.mu, self.lo, self.hi = float(alpha0), float(beta), float(mu), float(lo), float(hi)
        self.n_max = self.n if n_max is None else int(n_max)
        self.eps = eps
        self.C = constant_batch_C(self.n, self.n0, self.epochs, eps) if C is None else float(C)
        self.j_max = int(j_max)
        if proj_dtype is None:
            proj_dtype = {torch.float16: "f16", torch.bfloat16: "bf16"}.get(b.dtype, "f32")
        self.plan = plan if plan is not None else Plan(geom, vol_dtype, proj_dtype, max_batch=self.n_max)
        dev = b.device
        self.b = b
        vt = self.plan.vol_torch
        shape = self.plan.vol_shape
        self.mixed = bool(mixed)
        if self.mixed:
            if vt == torch.float32:
                raise ValueError("mixed storage needs a 16-bit volume type (vol_dtype 'bf16' or 'f16')")
            if sr_seed is not None:
                raise ValueError("mixed storage keeps an FP32 iterate: stochastic rounding does not apply")
            self.x = (torch.zeros(shape, dtype=torch.float32, device=dev) if x0 is None
                      else x0.to(torch.float32).contiguous().clone())
            self.x16 = self.x.to(vt)
            self.xbar16 = torch.empty_like(self.x16)
        else:
            self.x = torch.zeros(shape, dtype=vt, device=dev) if x0 is None else x0.to(vt).contiguous().clone()
            self.x16 = self.x     # the projector reads the iterate itself
        self.xbar = torch.empty_like(self.x)
        self.g = torch.empty(shape, dtype=torch.float32, device=dev)
        self.r = torch.empty((self.n_max, geom.nv, geom.nu), dtype=torch.float32, device=dev)
        self.rbar = torch.empty_like(self.r)
        # device scalars: [0] f(x), [2] f(xbar), [4] <g, d>, [5] ||d||^2, [6] ||g||^2
        self.scal = torch.zeros(8, dtype=torch.float64, device=dev)
        self.host = torch.zeros(8, dtype=torch.float64).pin_memory()
        # stochastic rounding of the stored iterates: trial j of iteration k uses the key
        # (sr_seed << 32) + (k << 6) + j (j < 64 since at most 51 trials run)
        if sr_seed is not None and self.j_max > 63:
            raise ValueError("stochastic rounding keys allow at most 64 trials per iteration (j_max <= 63)")
        self.sr_seed = sr_seed
        self.k = 0
        self.epoch = 0
        self.history: List[Iteration] = []

    # -- one iteration (Steps 2b-2d) ---------------------------------------------------
    def iterate(self, views: Sequence[int], alpha_init=None, epoch: int = 0,
                decisions: Optional[Sequence[bool]] = None) -> Iteration:
        """One iteration (Steps 2b-2d) on the given views.  ``alpha_init`` is the first
        trial step: None (alpha_0), a number, or a callable proposer(self) evaluated once
        the forward projection and the backprojection are enqueued (so a proposer that
        runs device work overlaps them)."""
        t0 = time.perf_counter()
        self.epoch = epoch
        v = np.asarray(views, dtype=np.int32)
        B = len(v)
        f_scale = self.n / (2.0 * B)
        r, rbar = self.r[:B], self.rbar[:B]
        plan = self.plan
        fb_lisa_forward(plan, self.x16, v, self.b, r, self.scal[0:1], f_scale)
        fb_lisa_backproject(plan, r, v, self.n / float(B), self.g)
        if callable(alpha_init):
            alpha_init = alpha_init(self)
        alpha = self.alpha0 if alpha_init is None else float(alpha_init)
        if not alpha > 0.0:
            raise ValueError("initial step must be > 0, got %r" % alpha)
        trials: List[Trial] = []
        stream = torch.cuda.current_stream()
        for j in range(self.j_max + 1):
            key = None if self.sr_seed is None else sr_key(self.sr_seed, self.k, j)
            if self.mixed:
                fb_lisa_step_mixed(plan, self.x, self.g, alpha, self.mu, self.lo, self.hi, self.xbar, self.xbar16,
                                   self.scal[4:7])
                fb_lisa_forward(plan, self.xbar16, v, self.b, rbar, self.scal[2:3], f_scale)
            else:
                fb_lisa_step(plan, self.x, self.g, alpha, self.mu, self.lo, self.hi, self.xbar, self.scal[4:7],
                             key=key)
                fb_lisa_forward(plan, self.xbar, v, self.b, rbar, self.scal[2:3], f_scale)
            self.host.copy_(self.scal, non_blocking=True)
            stream.synchronize()
            h = self.host.tolist()
            f0, f_bar, inner, sq = h[0], h[2], h[4], h[5]
            gnorm = math.sqrt(h[6])
            if not math.isfinite(f0) or not math.isfinite(f_bar):
                raise FloatingPointError("non-finite objective at iteration %d (f=%r, f_bar=%r)" % (self.k, f0, f_bar))
            ok = f_bar <= f0 + inner + sq / (2.0 * alpha)
            if decisions is not None:
                ok = bool(decisions[j])
            trials.append(Trial(alpha, f_bar, inner, sq, ok))
            if ok:
                break
            alpha *= self.beta
        else:
            raise LineSearchFailed("no step satisfied the sufficient-decrease test in %d trials at iteration %d"
                                   % (self.j_max + 1, self.k))
        # Step 2d: accept (swap buffers; x keeps the accepted trial point)
        self.x, self.xbar = self.xbar, self.x
        if self.mixed:
            self.x16, self.xbar16 = self.xbar16, self.x16
        else:
            self.x16 = self.x
        it = Iteration(epoch, self.k, v.copy(), f0, alpha, len(trials) - 1, gnorm, trials,
                       time.perf_counter() - t0)
        self.history.append(it)
        self.k += 1
        return it

    # -- Algorithm 1 --------------------------------------------------------------------
    def run(self, perms: np.ndarray, max_iters: Optional[int] = None,
            alpha_init: Optional[Callable[["FBLisa"], Optional[float]]] = None,
            callback: Optional[Callable[["FBLisa", Iteration], None]] = None,
            decisions: Optional[Sequence[Sequence[bool]]] = None) -> torch.Tensor:
        """Epochs t = 1..T; epoch t runs ceil(n/N_t) iterations on the first N_t views of
        perms[k].  Returns the final iterate."""
        k_hat, n_prev = 0, self.n0
        for t in range(1, self.epochs + 1):
            nt = next_batch_size(n_prev, k_hat, self.n, self.n0, self.n_max, self.C, self.eps)
            iters = int(math.ceil(self.n / nt))
            for k in range(k_hat, k_hat + iters):
                if max_iters is not None and k >= max_iters:
                    return self.x
                it = self.iterate(perms[k][:nt], alpha_init, epoch=t,
                                  decisions=None if decisions is None else decisions[k])
                if callback is not None:
                    callback(self, it)
            k_hat += iters
            n_prev = nt
        return self.x
