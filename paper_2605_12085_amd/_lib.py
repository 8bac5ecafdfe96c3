"""ctypes binding of libfblisa.so (include/fblisa.h): argument marshalling only.

Every function here forwards torch tensors' device addresses and the current HIP
stream to the C ABI and raises ``FblError`` on a non-zero status.  All arithmetic of
the hot path runs in the library's HIP kernels; if the library is missing, importing
this module fails.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfblisa.so")

FBL_OK, FBL_E_INVALID, FBL_E_GEOMETRY, FBL_E_RANGE, FBL_E_DTYPE, FBL_E_HIP, FBL_E_NOMEM = range(7)
FBL_F32, FBL_BF16, FBL_F16 = 0, 1, 2
_VOL_DTYPES = {"f32": (FBL_F32, torch.float32), "bf16": (FBL_BF16, torch.bfloat16), "f16": (FBL_F16, torch.float16)}
_PROJ_DTYPES = {"f32": (FBL_F32, torch.float32), "bf16": (FBL_BF16, torch.bfloat16), "f16": (FBL_F16, torch.float16)}

EXPORTED = ("fbl_geometry_check", "fbl_plan_create", "fbl_plan_destroy", "fb_lisa_forward",
            "fb_lisa_backproject", "fb_lisa_step", "fb_lisa_step_sr", "fbl_mlp_workspace_bytes", "fbl_mlp_forward",
            "fbl_mlp_loss_grad", "fbl_mlp_adam", "fbl_timing_enable", "fbl_timing_select", "fbl_timing_read",
            "fbl_last_error", "fb_lisa_step_mixed", "fb_lisa_forward_f64", "fb_lisa_backproject_f64",
            "fb_lisa_step_noalloc")
MLP_IN, MLP_HIDDEN = 5, 64
MLP_NPARAMS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
KERNELS = ("forward", "transpose", "finalize", "prescale", "backproject", "step")  # FBL_K_* order


class FblError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libfblisa error %d: %s" % (code, msg))
        self.code = code


class _Geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("nu", ctypes.c_int64), ("nv", ctypes.c_int64),
                ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("sod", ctypes.c_double), ("sdd", ctypes.c_double),
                ("n_views", ctypes.c_int64), ("angles", ctypes.POINTER(ctypes.c_double))]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfblisa.so is not built (expected at %s); run __graft_entry__.build() "
                          "or python paper_2605_12085_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, G = ctypes.c_void_p, ctypes.POINTER(_Geometry)
    lib.fbl_geometry_check.argtypes = [G]
    lib.fbl_plan_create.argtypes = [G, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P)]
    lib.fbl_plan_destroy.argtypes = [P]
    lib.fbl_plan_destroy.restype = None
    lib.fb_lisa_forward.argtypes = [P, P, P, ctypes.c_int32, P, P, P, ctypes.c_double, P]
    lib.fb_lisa_backproject.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_double, P, P]
    lib.fb_lisa_step.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 P, P, P]
    lib.fb_lisa_step_sr.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_uint64, P, P, P]
    lib.fb_lisa_step_mixed.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       P, P, P, P]
    lib.fb_lisa_step_noalloc.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, P, P, P]
    lib.fb_lisa_forward_f64.argtypes = [P, P, P, ctypes.c_int32, P, P]
    lib.fb_lisa_backproject_f64.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_double, P, P]
    lib.fbl_mlp_workspace_bytes.argtypes = [ctypes.c_int64]
    lib.fbl_mlp_workspace_bytes.restype = ctypes.c_size_t
    lib.fbl_mlp_forward.argtypes = [P, P, ctypes.c_int64, P, P]
    lib.fbl_mlp_loss_grad.argtypes = [P, P, P, ctypes.c_int64, P, P, P, P]
    lib.fbl_mlp_adam.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, P]
    lib.fbl_timing_enable.argtypes = [P, ctypes.c_int]
    lib.fbl_timing_select.argtypes = [P, ctypes.c_uint32]
    lib.fbl_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.fbl_last_error.argtypes = []
    lib.fbl_last_error.restype = ctypes.c_char_p
    for name in ("fbl_geometry_check", "fbl_plan_create", "fb_lisa_forward", "fb_lisa_backproject",
                 "fb_lisa_step", "fb_lisa_step_sr", "fb_lisa_step_mixed", "fb_lisa_forward_f64",
                 "fb_lisa_backproject_f64", "fb_lisa_step_noalloc", "fbl_mlp_forward", "fbl_mlp_loss_grad",
                 "fbl_mlp_adam",
                 "fbl_timing_enable", "fbl_timing_select", "fbl_timing_read"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def _check(rc: int):
    if rc != FBL_OK:
        raise FblError(rc, lib.fbl_last_error().decode())


class _GeomHolder:
    def __init__(self, geom):
        n = int(geom.n_views)
        ang = getattr(geom, "angles", None)
        self.angles = None if ang is None else np.ascontiguousarray(np.asarray(ang, dtype=np.float64))
        if self.angles is not None and self.angles.shape != (n,):
            raise ValueError("angles must have n_views entries")
        ap = None if self.angles is None else self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s = _Geometry(int(geom.nx), int(geom.ny), int(geom.nz), float(geom.hx), float(geom.hy),
                           float(geom.hz), int(geom.nu), int(geom.nv), float(geom.du), float(geom.dv),
                           float(geom.sod), float(geom.sdd), n, ap)


def fbl_geometry_check(geom) -> None:
    """Host-only validation; raises FblError with the library's message."""
    gh = _GeomHolder(geom)
    _check(lib.fbl_geometry_check(ctypes.byref(gh.s)))


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _views(views) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(views, dtype=np.int32).ravel())
    return v


def _need(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


class Plan:
    """A libfblisa plan (fbl_plan_create): geometry tables and workspace on one device."""

    def __init__(self, geom, vol_dtype: str = "f32", proj_dtype: str = "f32", max_batch: Optional[int] = None):
        self.geom = geom
        self.vol_code, self.vol_torch = _VOL_DTYPES[vol_dtype]
        self.proj_code, self.proj_torch = _PROJ_DTYPES[proj_dtype]
        self.vol_dtype, self.proj_dtype = vol_dtype, proj_dtype
        self.max_batch = int(geom.n_views if max_batch is None else max_batch)
        self.vol_shape = (int(geom.nz), int(geom.ny), int(geom.nx))
        self.nv, self.nu, self.n_views = int(geom.nv), int(geom.nu), int(geom.n_views)
        self.device = torch.cuda.current_device()
        self._gh = _GeomHolder(geom)
        h = ctypes.c_void_p()
        _check(lib.fbl_plan_create(ctypes.byref(self._gh.s), self.vol_code, self.proj_code, self.max_batch,
                                   ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.fbl_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self, on: bool = True, kernels: Optional[Sequence[str]] = None) -> None:
        """Start (and clear) or stop per-launch event timing inside the library; ``kernels``
        (names from KERNELS) limits the bracketed launches, default all."""
        mask = (1 << len(KERNELS)) - 1 if kernels is None else sum(1 << KERNELS.index(k) for k in set(kernels))
        _check(lib.fbl_timing_select(self.handle, mask))
        _check(lib.fbl_timing_enable(self.handle, 1 if on else 0))

    def timing_read(self) -> dict:
        """{kernel: (summed ms, launches)} since timing was enabled or last read; clears the record."""
        ms = (ctypes.c_double * len(KERNELS))()
        n = (ctypes.c_int64 * len(KERNELS))()
        _check(lib.fbl_timing_read(self.handle, ms, n))
        return {k: (ms[i], int(n[i])) for i, k in enumerate(KERNELS)}

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def fb_lisa_forward(plan: Plan, x: torch.Tensor, views: Sequence[int], b: Optional[torch.Tensor] = None,
                    y: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None,
                    loss_scale: Optional[float] = None, stream=None) -> torch.Tensor:
    """y = A_views x (or the residual A_views x - b[views]); optionally loss[0] = scale * ||y||^2."""
    v = _views(views)
    _need(x, "x", plan.vol_torch, plan.vol_shape)
    if b is not None:
        _need(b, "b", plan.proj_torch, (plan.n_views, plan.nv, plan.nu))
    if y is None:
        y = torch.empty((len(v), plan.nv, plan.nu), dtype=torch.float32, device=x.device)
    _need(y, "y", torch.float32, (len(v), plan.nv, plan.nu))
    if loss is not None:
        _need(loss, "loss", torch.float64)
        if loss.numel() < 1:
            raise ValueError("loss needs one element")
    if loss_scale is None:
        loss_scale = plan.n_views / (2.0 * len(v))
    _check(lib.fb_lisa_forward(plan.handle, x.data_ptr(), v.ctypes.data, len(v), _ptr(b), y.data_ptr(),
                               _ptr(loss), float(loss_scale), _stream(stream)))
    return y


def fb_lisa_backproject(plan: Plan, r: torch.Tensor, views: Sequence[int], grad_scale: Optional[float] = None,
                        g: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """g = grad_scale * A_views^T r (default scale n_theta/B, the gradient of (2.5))."""
    v = _views(views)
    _need(r, "r", torch.float32, (len(v), plan.nv, plan.nu))
    if g is None:
        g = torch.empty(plan.vol_shape, dtype=torch.float32, device=r.device)
    _need(g, "g", torch.float32, plan.vol_shape)
    if grad_scale is None:
        grad_scale = plan.n_views / float(len(v))
    _check(lib.fb_lisa_backproject(plan.handle, r.data_ptr(), v.ctypes.data, len(v), float(grad_scale),
                                   g.data_ptr(), _stream(stream)))
    return g


def fb_lisa_step(plan: Plan, x: torch.Tensor, g: torch.Tensor, alpha: float, mu: float = 0.0, lo: float = 0.0,
                 hi: float = math.inf, xbar: Optional[torch.Tensor] = None, red: Optional[torch.Tensor] = None,
                 stream=None, key: Optional[int] = None):
    """xbar = prox(x - alpha g); red = [<g, xbar - x>, ||xbar - x||^2, ||g||^2] (FP64).  With a
    ``key`` (an unsigned 64-bit integer) xbar is rounded to the storage type stochastically
    (fb_lisa_step_sr), else to nearest."""
    _need(x, "x", plan.vol_torch, plan.vol_shape)
    _need(g, "g", torch.float32, plan.vol_shape)
    if xbar is None:
        xbar = torch.empty_like(x)
    _need(xbar, "xbar", plan.vol_torch, plan.vol_shape)
    if red is None:
        red = torch.empty(3, dtype=torch.float64, device=x.device)
    _need(red, "red", torch.float64)
    if red.numel() < 3:
        raise ValueError("red needs three elements")
    if key is None:
        _check(lib.fb_lisa_step(plan.handle, x.data_ptr(), g.data_ptr(), float(alpha), float(mu), float(lo),
                                float(hi), xbar.data_ptr(), red.data_ptr(), _stream(stream)))
    else:
        _check(lib.fb_lisa_step_sr(plan.handle, x.data_ptr(), g.data_ptr(), float(alpha), float(mu), float(lo),
                                   float(hi), int(key) & 0xFFFFFFFFFFFFFFFF, xbar.data_ptr(), red.data_ptr(),
                                   _stream(stream)))
    return xbar, red


def fb_lisa_step_mixed(plan: Plan, x: torch.Tensor, g: torch.Tensor, alpha: float, mu: float = 0.0,
                       lo: float = 0.0, hi: float = math.inf, xbar: Optional[torch.Tensor] = None,
                       xbar16: Optional[torch.Tensor] = None, red: Optional[torch.Tensor] = None, stream=None):
    """Prox trial on an FP32 master iterate: xbar (FP32) = prox(x - alpha g) and its 16-bit copy
    xbar16 (the plan's volume storage type, the projector's input); red as fb_lisa_step, on
    the FP32 values."""
    _need(x, "x", torch.float32, plan.vol_shape)
    _need(g, "g", torch.float32, plan.vol_shape)
    if xbar is None:
        xbar = torch.empty_like(x)
    _need(xbar, "xbar", torch.float32, plan.vol_shape)
    if xbar16 is None:
        xbar16 = torch.empty(plan.vol_shape, dtype=plan.vol_torch, device=x.device)
    _need(xbar16, "xbar16", plan.vol_torch, plan.vol_shape)
    if red is None:
        red = torch.empty(3, dtype=torch.float64, device=x.device)
    _need(red, "red", torch.float64)
    if red.numel() < 3:
        raise ValueError("red needs three elements")
    _check(lib.fb_lisa_step_mixed(plan.handle, x.data_ptr(), g.data_ptr(), float(alpha), float(mu), float(lo),
                                  float(hi), xbar.data_ptr(), xbar16.data_ptr(), red.data_ptr(), _stream(stream)))
    return xbar, xbar16, red


def fb_lisa_step_noalloc(x: torch.Tensor, g: torch.Tensor, alpha: float, mu: float, lo: float, hi: float,
                         xbar: torch.Tensor, red: torch.Tensor, stream=None):
    """fb_lisa_step without a plan or allocation: x, xbar in one storage type (FP32, BF16 or
    FP16), g FP32, all of the same number of voxels; red: three FP64 values."""
    codes = {torch.float32: FBL_F32, torch.bfloat16: FBL_BF16, torch.float16: FBL_F16}
    if x.dtype not in codes:
        raise TypeError("x must be float32, bfloat16 or float16")
    _need(x, "x", x.dtype)
    _need(xbar, "xbar", x.dtype, tuple(x.shape))
    _need(g, "g", torch.float32, tuple(x.shape))
    _need(red, "red", torch.float64)
    if red.numel() < 3:
        raise ValueError("red needs three elements")
    _check(lib.fb_lisa_step_noalloc(x.numel(), codes[x.dtype], x.data_ptr(), g.data_ptr(), float(alpha), float(mu),
                                    float(lo), float(hi), xbar.data_ptr(), red.data_ptr(), _stream(stream)))
    return xbar, red


def fb_lisa_forward_f64(plan: Plan, x: torch.Tensor, views: Sequence[int], y: Optional[torch.Tensor] = None,
                        stream=None) -> torch.Tensor:
    """y = A_views x with the FP64 check kernels (x FP64 [nz][ny][nx], y FP64 [B][nv][nu])."""
    v = _views(views)
    _need(x, "x", torch.float64, plan.vol_shape)
    if y is None:
        y = torch.empty((len(v), plan.nv, plan.nu), dtype=torch.float64, device=x.device)
    _need(y, "y", torch.float64, (len(v), plan.nv, plan.nu))
    _check(lib.fb_lisa_forward_f64(plan.handle, x.data_ptr(), v.ctypes.data, len(v), y.data_ptr(), _stream(stream)))
    return y


def fb_lisa_backproject_f64(plan: Plan, r: torch.Tensor, views: Sequence[int], grad_scale: Optional[float] = None,
                            g: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """g = grad_scale * A_views^T r with the FP64 check kernels (default scale n_theta/B)."""
    v = _views(views)
    _need(r, "r", torch.float64, (len(v), plan.nv, plan.nu))
    if g is None:
        g = torch.empty(plan.vol_shape, dtype=torch.float64, device=r.device)
    _need(g, "g", torch.float64, plan.vol_shape)
    if grad_scale is None:
        grad_scale = plan.n_views / float(len(v))
    _check(lib.fb_lisa_backproject_f64(plan.handle, r.data_ptr(), v.ctypes.data, len(v), float(grad_scale),
                                       g.data_ptr(), _stream(stream)))
    return g


# -- learned initial step: perceptron kernels --------------------------------------------

def _need_vec(t: torch.Tensor, name: str, n: int):
    _need(t, name, torch.float32)
    if t.numel() != n:
        raise ValueError("%s must have %d elements, got %d" % (name, n, t.numel()))


def mlp_workspace(n: int, device=None) -> torch.Tensor:
    """A device workspace for mlp_loss_grad on n samples (256-byte aligned)."""
    nbytes = int(lib.fbl_mlp_workspace_bytes(int(n)))
    w = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-w.data_ptr()) % 256
    return w[off:off + nbytes]


def mlp_forward(params: torch.Tensor, X: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
    """out[i] = MLP(X[i]) (X FP32 [n][5])."""
    _need_vec(params, "params", MLP_NPARAMS)
    _need(X, "X", torch.float32)
    if X.dim() != 2 or X.shape[1] != MLP_IN:
        raise ValueError("X must be [n][%d]" % MLP_IN)
    n = X.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=X.device)
    _need_vec(out, "out", n)
    _check(lib.fbl_mlp_forward(params.data_ptr(), X.data_ptr(), n, out.data_ptr(), _stream(stream)))
    return out


def mlp_loss_grad(params: torch.Tensor, X: torch.Tensor, t: torch.Tensor, work: torch.Tensor,
                  grad: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None, stream=None):
    """grad = d/dparams of 1/(2n) sum (MLP(X) - t)^2; loss[0] = sum (MLP(X) - t)^2 (FP64)."""
    _need_vec(params, "params", MLP_NPARAMS)
    _need(X, "X", torch.float32)
    n = X.shape[0]
    _need_vec(t, "t", n)
    if work.numel() < int(lib.fbl_mlp_workspace_bytes(n)):
        raise ValueError("workspace too small for %d samples" % n)
    if grad is None:
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
    _need_vec(grad, "grad", MLP_NPARAMS)
    if loss is not None:
        _need(loss, "loss", torch.float64)
    _check(lib.fbl_mlp_loss_grad(params.data_ptr(), X.data_ptr(), t.data_ptr(), n, grad.data_ptr(), _ptr(loss),
                                 work.data_ptr(), _stream(stream)))
    return grad


def mlp_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
             beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    """One in-place Adam update of params (state m, v)."""
    for t, name in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _need_vec(t, name, MLP_NPARAMS)
    _check(lib.fbl_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr),
                            float(beta1), float(beta2), float(eps), _stream(stream)))
