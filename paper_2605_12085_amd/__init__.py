"""MI355X-native hot path of FB-LISA (arXiv 2605.12085): cone-beam Joseph projector
pair, matched backprojection and prox/line-search step as HIP kernels for gfx950
behind a C ABI (include/fblisa.h), with a thin ctypes binding and the method's host
loop."""
from ._lib import (FBL_BF16, FBL_F16, FBL_F32, FblError, Plan, fb_lisa_backproject, fb_lisa_backproject_f64,
                   fb_lisa_forward, fb_lisa_forward_f64, fb_lisa_step, fb_lisa_step_mixed, fbl_geometry_check)
from .autograd import backproject, data_fidelity, project
from .learned_step import LearnedStep, StepModel, TraceRecorder
from .driver import FBLisa, Iteration, LineSearchFailed, constant_batch_C, growing_batch_C, next_batch_size

__all__ = ["Plan", "FblError", "fb_lisa_forward", "fb_lisa_backproject", "fb_lisa_step", "fb_lisa_step_mixed",
           "fb_lisa_forward_f64", "fb_lisa_backproject_f64", "fbl_geometry_check",
           "FBLisa", "Iteration", "LineSearchFailed", "constant_batch_C", "growing_batch_C", "next_batch_size",
           "FBL_F32", "FBL_BF16", "FBL_F16", "project", "backproject", "data_fidelity",
           "LearnedStep", "StepModel", "TraceRecorder"]
