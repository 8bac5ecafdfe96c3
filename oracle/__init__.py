"""FP64 CPU oracle of the FB-LISA hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library (``paper_2605_12085_amd``) never imports it, and
it imports nothing from the product; the two share only the seeded input
generators of ``synthetic``.

Contents, each following the paper (arXiv 2605.12085):
  * the cone-beam projector pair (C, FP64; ``fbl_oracle.c``): per-view blocks A_i
    of (2.4), the mini-batch operator A_N of (2.5) and its exact transpose;
  * the mini-batch objective f_N and gradient (2.5), read as
    f_N(x) = n_theta/(2|N|) ||A_N x - b_N||^2, grad = n_theta/|N| A_N^T (A_N x - b_N);
  * the prox of R(x) = mu ||x||_1 + indicator of [lo, hi] (problem (2.1) uses
    mu > 0 and the nonnegative orthant);
  * the sufficient-decrease line search (2.3) with backtracking (Algorithm 1,
    Step 2c) and the step reset of Step 2d;
  * the mini-batch size rule of Algorithm 1, Step 1, and the epoch loop (Steps 2, 3).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fbl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("nu", ctypes.c_int64), ("nv", ctypes.c_int64),
                ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("sod", ctypes.c_double), ("sdd", ctypes.c_double),
                ("n_views", ctypes.c_int64), ("angles", ctypes.POINTER(ctypes.c_double))]


_P = ctypes.c_void_p


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_LIB)
            G = ctypes.POINTER(_Geom)
            lib.orc_forward.argtypes = [G, _P, _P, ctypes.c_int64, _P]
            lib.orc_forward.restype = None
            lib.orc_forward_rays.argtypes = [G, _P, _P, ctypes.c_int64, _P]
            lib.orc_forward_rays.restype = None
            lib.orc_backproject.argtypes = [G, _P, _P, ctypes.c_int64, _P]
            lib.orc_backproject.restype = ctypes.c_int
            lib.orc_backproject_voxels.argtypes = [G, _P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P]
            lib.orc_backproject_voxels.restype = None
            lib.orc_matrix_entry.argtypes = [G, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
            lib.orc_matrix_entry.restype = ctypes.c_double
            lib.orc_ray_value.argtypes = [G, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
            lib.orc_ray_value.restype = ctypes.c_double
            lib.orc_dominant_axes.argtypes = [G, ctypes.c_int64, _P]
            lib.orc_dominant_axes.restype = None
            lib.orc_num_threads.argtypes = []
            lib.orc_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


class _GeomHolder:
    """Keeps the ctypes struct and the angle array it points to alive together."""

    def __init__(self, g):
        self.angles = np.ascontiguousarray(np.asarray(g.angles, dtype=np.float64))
        self.s = _Geom(g.nx, g.ny, g.nz, g.hx, g.hy, g.hz, g.nu, g.nv, g.du, g.dv, g.sod, g.sdd,
                       g.n_views, self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def ref(self):
        return ctypes.byref(self.s)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _views(views):
    v = np.ascontiguousarray(np.asarray(views, dtype=np.int32).ravel())
    return v


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ----------------------------------------------------------------------------------
# projector pair
# ----------------------------------------------------------------------------------

def forward(g, x, views) -> np.ndarray:
    """A_N x for the listed views, FP64 [B][nv][nu] ((2.4), (2.5))."""
    lib = _load()
    x = _f64(x)
    assert x.shape == g.vol_shape
    v = _views(views)
    y = np.zeros((len(v), g.nv, g.nu), dtype=np.float64)
    gh = _GeomHolder(g)
    lib.orc_forward(gh.ref(), x.ctypes.data, v.ctypes.data, len(v), y.ctypes.data)
    return y


def forward_rays(g, x, rays) -> np.ndarray:
    """Values of individual rays; rays is int64 [n][3] of (view, iv, iu)."""
    lib = _load()
    x = _f64(x)
    rr = np.ascontiguousarray(np.asarray(rays, dtype=np.int64).reshape(-1, 3))
    out = np.zeros(len(rr), dtype=np.float64)
    gh = _GeomHolder(g)
    lib.orc_forward_rays(gh.ref(), x.ctypes.data, rr.ctypes.data, len(rr), out.ctypes.data)
    return out


def backproject(g, r, views) -> np.ndarray:
    """A_N^T r (exact transpose of ``forward``), FP64 [nz][ny][nx]."""
    lib = _load()
    v = _views(views)
    r = _f64(r)
    assert r.shape == (len(v), g.nv, g.nu)
    out = np.zeros(g.vol_shape, dtype=np.float64)
    gh = _GeomHolder(g)
    if lib.orc_backproject(gh.ref(), r.ctypes.data, v.ctypes.data, len(v), out.ctypes.data) != 0:
        raise MemoryError("oracle backprojection could not allocate its per-thread volumes")
    return out


def backproject_voxels(g, r, views, voxels) -> np.ndarray:
    """(A_N^T r) at the listed linear voxel indices, by summing matrix entries over all rays."""
    lib = _load()
    v = _views(views)
    r = _f64(r)
    assert r.shape == (len(v), g.nv, g.nu)
    vox = np.ascontiguousarray(np.asarray(voxels, dtype=np.int64).ravel())
    out = np.zeros(len(vox), dtype=np.float64)
    gh = _GeomHolder(g)
    lib.orc_backproject_voxels(gh.ref(), r.ctypes.data, v.ctypes.data, len(v), vox.ctypes.data, len(vox),
                               out.ctypes.data)
    return out


def matrix_entry(g, view, iu, iv, voxel) -> float:
    gh = _GeomHolder(g)
    return float(_load().orc_matrix_entry(gh.ref(), view, iu, iv, voxel))


def ray_value(g, x, view, iu, iv) -> float:
    x = _f64(x)
    gh = _GeomHolder(g)
    return float(_load().orc_ray_value(gh.ref(), x.ctypes.data, view, iu, iv))


def dominant_axes(g, view) -> np.ndarray:
    out = np.zeros((g.nv, g.nu), dtype=np.int32)
    gh = _GeomHolder(g)
    _load().orc_dominant_axes(gh.ref(), view, out.ctypes.data)
    return out


def assemble_matrix(g, views) -> np.ndarray:
    """Explicit A_N (rows = rays [b][iv][iu], cols = voxels) by forward-projecting unit vectors."""
    d = g.d
    cols = []
    e = np.zeros(d, dtype=np.float64)
    for i in range(d):
        e[:] = 0.0
        e[i] = 1.0
        cols.append(forward(g, e.reshape(g.vol_shape), views).ravel())
    return np.stack(cols, axis=1)


def assemble_matrix_transpose(g, views) -> np.ndarray:
    """Explicit A_N^T (rows = voxels) by backprojecting unit vectors of the data space."""
    nb = len(_views(views))
    n = nb * g.n_p
    rows = []
    e = np.zeros(n, dtype=np.float64)
    for i in range(n):
        e[:] = 0.0
        e[i] = 1.0
        rows.append(backproject(g, e.reshape(nb, g.nv, g.nu), views).ravel())
    return np.stack(rows, axis=1)


# ----------------------------------------------------------------------------------
# objective, gradient, prox  ((2.1), (2.5), Algorithm 1 Step 2c)
# ----------------------------------------------------------------------------------

def residual(g, x, b_full, views) -> np.ndarray:
    """A_N x - b_N, FP64 [B][nv][nu]; b_full holds every view [n_theta][nv][nu]."""
    v = _views(views)
    return forward(g, x, v) - _f64(b_full)[v]


def objective(g, x, b_full, views, n_theta: Optional[int] = None) -> float:
    """f_N(x) = n_theta / (2|N|) * ||A_N x - b_N||^2, the mini-batch objective (2.5)."""
    v = _views(views)
    nt = g.n_views if n_theta is None else n_theta
    r = residual(g, x, b_full, v)
    return nt / (2.0 * len(v)) * float(np.dot(r.ravel(), r.ravel()))


def objective_and_gradient(g, x, b_full, views, n_theta: Optional[int] = None):
    """(f_N(x), grad f_N(x), residual) with grad = n_theta/|N| * A_N^T (A_N x - b_N)."""
    v = _views(views)
    nt = g.n_views if n_theta is None else n_theta
    r = residual(g, x, b_full, v)
    f = nt / (2.0 * len(v)) * float(np.dot(r.ravel(), r.ravel()))
    grad = (nt / float(len(v))) * backproject(g, r, v)
    return f, grad, r


def prox(v, alpha: float, mu: float, lo: float = 0.0, hi: float = math.inf) -> np.ndarray:
    """prox of alpha * (mu ||.||_1 + indicator[lo, hi]) for 0 <= lo <= hi.

    The function is separable; on [lo, hi] with lo >= 0 the l1 term is the linear
    term mu * z, so each coordinate minimises (z - v)^2/(2 alpha) + mu * z over an
    interval: the unconstrained minimiser v - alpha*mu clipped to [lo, hi].
    """
    return np.minimum(np.maximum(_f64(v) - alpha * mu, lo), hi)


# ----------------------------------------------------------------------------------
# storage rounding (the precision form stores x in 16-bit types, computes in FP32/FP64)
# ----------------------------------------------------------------------------------

def round_bf16(v) -> np.ndarray:
    """Round FP64 values once to bfloat16 (8 significant bits, FP32 exponent range),
    to nearest with ties to even, returned as FP64.

    From the definition: a finite v with |v| in [2^(e-1), 2^e) has the quantum
    2^(e-8); below the smallest normal 2^-126 the quantum stays 2^-133 (gradual
    underflow).  v / quantum is exact (a power-of-two scaling), np.rint rounds it half
    to even.  Results beyond the largest finite bfloat16 become infinities."""
    v = _f64(v)
    out = v.copy()
    fin = np.isfinite(v) & (v != 0)
    _, e = np.frexp(v[fin])
    q = np.ldexp(1.0, np.maximum(e, -125) - 8)
    r = np.rint(v[fin] / q) * q
    big = np.ldexp(1.0, 128)
    r = np.where(np.abs(r) >= big, np.copysign(np.inf, r), r)
    out[fin] = r
    return out


def round_storage(v, storage) -> np.ndarray:
    """Round FP64 values once to a storage type: "f32", "f16" (numpy's IEEE conversions,
    nearest-even from FP64), "bf16" (round_bf16), or None/"f64" (unchanged)."""
    if storage is None or storage == "f64":
        return _f64(v)
    if storage in ("f32", np.float32):
        return _f64(v).astype(np.float32).astype(np.float64)
    if storage in ("f16", np.float16):
        with np.errstate(over="ignore"):
            return _f64(v).astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return round_bf16(v)
    raise ValueError("unknown storage %r" % (storage,))


_SPLITMIX_GAMMA = 0x9E3779B97F4A7C15
_PRECISION = {"f32": (24, -126), "bf16": (8, -126), "f16": (11, -14)}   # significant bits, min normal exponent


def splitmix64(key: int, counters) -> np.ndarray:
    """Outputs number counters+1 of SplitMix64 (Steele, Lea and Flood, 2014) seeded with
    ``key``: the state after c+1 steps is key + (c+1) * gamma (mod 2^64), mixed by the
    generator's finaliser.  Used as a counter-based generator: voxel i draws output i+1."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * np.uint64(_SPLITMIX_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def trial_key(seed: int, k: int, j: int) -> int:
    """Rounding key of line-search trial j of iteration k: (seed << 32) + (k << 6) + j
    (mod 2^64); j stays below 64 (at most 51 trials)."""
    return ((int(seed) << 32) + (int(k) << 6) + int(j)) & 0xFFFFFFFFFFFFFFFF


def round_stochastic(v, storage: str, key: int) -> np.ndarray:
    """Stochastic rounding of FP64 values to a storage type: a value between the adjacent
    representable numbers a < v < a + q goes up with probability (v - a) / q, decided by
    r < (v - a) / q with r = (splitmix64(key, i) >> 11) * 2^-53 for the value's flat index
    i; representable values are unchanged.  All steps are exact in FP64 (q is a power of
    two, a a multiple of q within one q of v)."""
    v = _f64(v)
    P, emin = _PRECISION[storage]
    flat = v.ravel()
    out = flat.copy()
    fin = np.isfinite(flat) & (flat != 0)
    _, e = np.frexp(flat[fin])                       # |v| in [2^(e-1), 2^e)
    q = np.ldexp(1.0, np.maximum(e - 1, emin) - (P - 1))
    a = np.floor(flat[fin] / q) * q
    p = (flat[fin] - a) / q
    r = (splitmix64(key, np.nonzero(fin)[0]) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    out[fin] = np.where(r < p, a + q, a)
    return out.reshape(v.shape)


def prox_step(x, grad, alpha: float, mu: float, lo: float = 0.0, hi: float = math.inf, storage=None,
              key: Optional[int] = None):
    """Trial point of Algorithm 1 Step 2c and the inner products of (2.3).

    xbar = prox(x - alpha grad); with ``storage`` ("f32", "bf16", "f16" or a numpy
    dtype) the trial point is rounded to that storage type, as a stored iterate would
    be, before d = xbar - x is formed: to nearest, or stochastically with ``key`` (see
    round_stochastic).  Returns (xbar, <grad, d>, ||d||^2, ||grad||^2).
    """
    x64, g64 = _f64(x), _f64(grad)
    xbar = prox(x64 - alpha * g64, alpha, mu, lo, hi)
    if storage is not None:
        xbar = round_storage(xbar, storage) if key is None else round_stochastic(xbar, storage, key)
    d = xbar - x64
    return xbar, float(np.dot(g64.ravel(), d.ravel())), float(np.dot(d.ravel(), d.ravel())), \
        float(np.dot(g64.ravel(), g64.ravel()))


# ----------------------------------------------------------------------------------
# line search and Algorithm 1
# ----------------------------------------------------------------------------------

class LineSearchError(RuntimeError):
    pass


@dataclass
class TrialRecord:
    alpha: float
    f_bar: float
    inner: float
    sq: float
    accepted: bool


def sufficient_decrease(f_bar: float, f0: float, inner: float, sq: float, alpha: float) -> bool:
    """Inequality (2.3): f(xbar) <= f(x) + grad^T (xbar - x) + ||xbar - x||^2 / (2 alpha)."""
    return f_bar <= f0 + inner + sq / (2.0 * alpha)


def line_search(fun: Callable[[np.ndarray], float], x: np.ndarray, f0: float, grad: np.ndarray,
                alpha_init: float, beta: float, mu: float, lo: float, hi: float, j_max: int = 50,
                decide: Optional[Callable[[int], bool]] = None, storage=None,
                key: Optional[Callable[[int], int]] = None):
    """Backtracking of Algorithm 1, Step 2c.

    Starting from alpha_init, forms xbar = prox(x - alpha grad) and accepts the first
    alpha for which (2.3) holds; otherwise alpha <- beta * alpha.  ``decide`` (replay
    mode) overrides the accept/reject decision of trial j.  ``storage`` rounds each
    trial point to a storage type before it is used: to nearest (round_storage), or
    stochastically with the key ``key(j)`` of trial j (round_stochastic).
    Returns (alpha, xbar, f_bar, trials).
    """
    alpha = alpha_init
    trials: List[TrialRecord] = []
    for j in range(j_max + 1):
        xbar = prox(x - alpha * grad, alpha, mu, lo, hi)
        if storage is not None:
            xbar = round_storage(xbar, storage) if key is None else round_stochastic(xbar, storage, key(j))
        dlt = xbar - x
        inner = float(np.dot(grad.ravel(), dlt.ravel()))
        sq = float(np.dot(dlt.ravel(), dlt.ravel()))
        f_bar = fun(xbar)
        ok = sufficient_decrease(f_bar, f0, inner, sq, alpha)
        if decide is not None:
            ok = bool(decide(j))
        trials.append(TrialRecord(alpha, f_bar, inner, sq, ok))
        if ok:
            return alpha, xbar, f_bar, trials
        alpha = beta * alpha
    raise LineSearchError("sufficient decrease not reached in %d trials" % (j_max + 1))


def ceil_tol(z: float) -> int:
    """Ceiling that does not round an FP-exact integer up (tolerance 1e-9)."""
    return int(math.ceil(z - 1e-9))


def batch_size(t: int, n_prev: int, k_hat: int, n: int, n0: int, n_max: int, C: float,
               eps: Callable[[int], float]) -> int:
    """Algorithm 1, Step 1: N_t = min{n_max, max{ceil(C / eps_{k_hat + ceil(n/N_{t-1})}), N_0}}."""
    idx = k_hat + int(math.ceil(n / n_prev))
    return min(n_max, max(ceil_tol(C / eps(idx)), n0))


def eps_default(k: int) -> float:
    """eps_k = 0.99^k, the summable sequence used in the paper's experiments."""
    return math.pow(0.99, k)


def schedule(n: int, n0: int, epochs: int, C: float, n_max: Optional[int] = None,
             eps: Callable[[int], float] = eps_default) -> List[int]:
    """Mini-batch sizes N_1..N_T of Algorithm 1 (epoch t runs ceil(n/N_t) iterations)."""
    n_max = n if n_max is None else n_max
    sizes = []
    n_prev, k_hat = n0, 0
    for t in range(1, epochs + 1):
        nt = batch_size(t, n_prev, k_hat, n, n0, n_max, C, eps)
        sizes.append(nt)
        k_hat += int(math.ceil(n / nt))
        n_prev = nt
    return sizes


def fixed_batch_C(n: int, n0: int, epochs: int, eps: Callable[[int], float] = eps_default) -> float:
    """C that keeps N_t = N_0 for the whole run: N_0 * eps_{K_tot}, K_tot = epochs * ceil(n/N_0)."""
    return n0 * eps(epochs * int(math.ceil(n / n0)))


def growth_C(n: int, n0: int, eps: Callable[[int], float] = eps_default) -> float:
    """C for which Step 1 gives N_1 = N_0 and then grows: N_0 * eps_{ceil(n/N_0)}."""
    return n0 * eps(int(math.ceil(n / n0)))


@dataclass
class IterRecord:
    epoch: int
    k: int
    batch: np.ndarray
    f0: float
    alpha: float
    backtracks: int
    trials: List[TrialRecord] = field(default_factory=list)


def fblisa(g, b_full, *, epochs: int, n0: int, alpha0: float = 1e-3, beta: float = 0.5,
           mu: float = 0.0, lo: float = 0.0, hi: float = math.inf, C: Optional[float] = None,
           n_max: Optional[int] = None, eps: Callable[[int], float] = eps_default,
           x0: Optional[np.ndarray] = None, perms: Optional[np.ndarray] = None,
           j_max: int = 50, decisions: Optional[Sequence[Sequence[bool]]] = None,
           alpha_init: Optional[Callable[[int], float]] = None,
           max_iters: Optional[int] = None, callback=None, storage=None, sr_seed: Optional[int] = None,
           copy_storage=None):
    """Algorithm 1 (FB-LISA) in FP64 with n = n_theta (one f_i per projection angle).

    perms[k] is a permutation of the views for iteration k; the mini-batch is its
    first N_t entries.  ``decisions`` (replay) forces the accept/reject outcome of
    each trial.  ``alpha_init(k)`` replaces alpha_0 as the first trial step.
    ``storage`` keeps the iterates rounded to a storage type (the arithmetic stays FP64),
    to nearest or, with ``sr_seed``, stochastically with trial_key(sr_seed, k, j).
    ``copy_storage`` ("bf16" or "f16") is the mixed form: the iterates are kept in FP32 and
    the objective and its gradient are evaluated at their copies rounded to nearest in
    copy_storage (what a projector reading 16-bit values sees); the prox step and the inner
    products of (2.3) use the FP32 iterates.
    Returns (x, records).
    """
    if copy_storage is not None:
        if sr_seed is not None:
            raise ValueError("the mixed form keeps FP32 iterates: no stochastic rounding")
        storage = "f32"
    seen = (lambda z: z) if copy_storage is None else (lambda z: round_storage(z, copy_storage))
    n = g.n_views
    n_max = n if n_max is None else n_max
    if C is None:
        C = fixed_batch_C(n, n0, epochs, eps)
    x = np.zeros(g.vol_shape, dtype=np.float64) if x0 is None else _f64(x0).copy()
    records: List[IterRecord] = []
    k_hat, n_prev, k = 0, n0, 0
    for t in range(1, epochs + 1):
        nt = batch_size(t, n_prev, k_hat, n, n0, n_max, C, eps)
        iters = int(math.ceil(n / nt))
        for k in range(k_hat, k_hat + iters):
            if max_iters is not None and k >= max_iters:
                return x, records
            views = perms[k][:nt] if perms is not None else np.arange(nt)
            f0, grad, _ = objective_and_gradient(g, seen(x), b_full, views)
            a0 = alpha0 if alpha_init is None else alpha_init(k)
            dec = None
            if decisions is not None:
                dk = decisions[k]
                dec = lambda j, dk=dk: dk[j]
            alpha, xbar, f_bar, trials = line_search(
                lambda z: objective(g, seen(z), b_full, views), x, f0, grad, a0, beta, mu, lo, hi, j_max, dec,
                storage, None if sr_seed is None else (lambda j, k=k: trial_key(sr_seed, k, j)))
            records.append(IterRecord(t, k, np.asarray(views).copy(), f0, alpha, len(trials) - 1, trials))
            x = xbar
            if callback is not None:
                callback(k, x, records[-1])
        k_hat = k + 1
        n_prev = nt
    return x, records


def power_iteration_L(g, views, n_theta: Optional[int] = None, iters: int = 200, seed: int = 0) -> float:
    """Largest eigenvalue of n_theta/|N| A_N^T A_N (Lipschitz constant of grad f_N)."""
    v = _views(views)
    nt = g.n_views if n_theta is None else n_theta
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(g.vol_shape)
    z /= np.linalg.norm(z)
    lam = 0.0
    for _ in range(iters):
        w = (nt / float(len(v))) * backproject(g, forward(g, z, v), v)
        lam = float(np.linalg.norm(w))
        z = w / lam
    return lam


# ----------------------------------------------------------------------------------
# reconstruction quality
# ----------------------------------------------------------------------------------

def rmse(x, x_true) -> float:
    """Root-mean-square error over every voxel (the time-to-quality target of the
    benchmark; Section 3 reports errors of the reconstruction against the reference)."""
    d = _f64(x) - _f64(x_true)
    return math.sqrt(float(np.dot(d.ravel(), d.ravel())) / d.size)


def relative_error(x, x_true) -> float:
    """RE = ||x - x_true||_2 / ||x_true||_2 (Section 3 leaves RE undefined; this is the
    usual reading)."""
    d = _f64(x) - _f64(x_true)
    return float(np.linalg.norm(d.ravel()) / np.linalg.norm(_f64(x_true).ravel()))


def psnr(x, x_true) -> float:
    """PSNR in dB with the peak taken as the largest value of x_true (Section 3 leaves the
    peak unstated): 20 log10(max x_true / RMSE)."""
    peak = float(_f64(x_true).max())
    return 20.0 * math.log10(peak / rmse(x, x_true))
