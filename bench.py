#!/usr/bin/env python
"""Benchmark of the FB-LISA hot path on one MI355X.

The default workload is the 1024^3 one: a 1024^3 FP32 ellipsoid phantom (30 ellipsoids),
1440 views of a 1536x1536 detector, 40-view mini-batches, 10 epochs, nonnegativity prox,
1% Gaussian noise on exact line integrals.  A step is one FB-LISA iteration (Algorithm 1,
Steps 2a-2d) of the plain FP32 method: the forward projection of the mini-batch with
residual and FP64 objective, the backprojection (gradient), and the line search's prox
trials, each followed by a forward projection of the trial point and one read-back of
three FP64 scalars.  Inputs (phantom, noisy data, view draws) are synthetic, seeded and
already resident in device memory when the timed region starts.

value = projector updates per second over the timed steps (GUPS): every forward or
backprojection call over B views counts d*B voxel-view updates (d voxels); the time
includes the step kernels, the reductions and the per-trial host synchronisation.

After the timed steps the same workload runs the time-to-RMSE comparison: the plain FP32
method against the learned initial step with the projector reading a BF16 copy of the
volume and FP16 data, each given the plain run's wall time.  A secondary block repeats
throughput and the comparison at 256^3 (three view orders).

Printed: one JSON line on stdout (diagnostics go to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP+BP GUPS & %HBM roofline; FB-LISA time-to-RMSE, learned+BF16 vs plain"
HBM_PEAK_GBS = 8000.0
# VALU issue peak of the chip without packed FP32: each of 256 CUs issues one wave64 VALU
# instruction per clock (4 SIMDs of 16 lanes, 4 clocks per instruction) at 2.4 GHz, i.e.
# 256 * 64 * 2.4e9 lane operations per second (78.6 TFLOP/s counting an FMA as two).
VALU_PEAK_TLOPS = 256 * 64 * 2.4e9 / 1e12
DEVICE_DATA = ("c3", "c5")   # workloads whose exact line integrals are computed on the GPU


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"fp_kernel": "forward.hip", "bp_kernel": "backproject.hip", "step_kernel": "step.hip"}


def kernel_source_hash(kernel: str) -> str:
    """Hash of a kernel's source, its device helpers, the shared declarations and the host
    code that chooses its launch shapes (plan.hip), comments and spacing removed, so that a
    counter summary stays valid across edits that change no code."""
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES[kernel], "device_util.h", "common.h", "plan.hip"):
        with open(os.path.join(ROOT, "paper_2605_12085_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def profile_value(kernel: str, cfg: str, field: str = "hbm_bytes_per_launch"):
    """A figure of a kernel from the committed rocprofv3 counter summary
    profiles/<kernel>_<cfg>_pmc.json, if it was taken on the current kernel source (else
    None): HBM bytes per launch, VALU issue fraction or L2 hit rate."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.json" % (kernel, cfg))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get(field)


def measured_traffic(kernel: str, cfg: str):
    """HBM bytes per launch of a kernel from its committed counter summary (or None)."""
    return profile_value(kernel, cfg, "hbm_bytes_per_launch")


def host_info():
    """CPU model name (as lscpu reports it, from /proc/cpuinfo) and the logical CPUs."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def make_workload(syn, name):
    """The seeded synthetic workload of a configuration: (geometry, config, seed, FP64
    phantom on the host, FP32 data [n_views][nv][nu] on the GPU).  The data are the exact
    line integrals through the phantom's ellipsoids plus 1% Gaussian noise; for the 512^3
    and 1024^3 workloads they are computed on the GPU and the phantom is voxelised at one
    sample per voxel (the host loops would take a quarter of an hour)."""
    import torch
    cfg = syn.CONFIGS[name]
    g = syn.config_geometry(name)
    seed = 1000 * int(name[1:])
    if name in DEVICE_DATA:
        ells, xt = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"], sub=1)
        b = torch.empty((g.n_views, g.nv, g.nu), dtype=torch.float32, device="cuda")
        chunk = 60
        for v0 in range(0, g.n_views, chunk):   # FP64 line integrals a few views at a time
            vv = np.arange(v0, min(g.n_views, v0 + chunk))
            b[v0:v0 + len(vv)] = syn.ellipsoid_line_integrals_torch(g, ells, vv, device="cuda").float()
        syn.add_noise_torch(b, 0.01, seed=seed + 1)
    else:
        ells, xt = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"])
        clean = syn.ellipsoid_line_integrals(g, ells, np.arange(g.n_views))
        b = torch.from_numpy(syn.add_noise(clean, 0.01, seed=seed + 1).astype(np.float32)).cuda()
        del clean
    torch.cuda.synchronize()
    return g, cfg, seed, xt, b


def cpu_baseline_rays(g, xt, views, min_seconds=10.0, max_rays=1 << 24, seed=77):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: its ray-subset
    forward projector (every slice of each ray, the same per-ray work as a full view)
    on seeded random rays of the mini-batch, in rounds of doubling size until about
    min_seconds of host time.  A full view of n_p rays counts d voxel-view updates, so a
    ray counts d / n_p."""
    import oracle
    x64 = np.ascontiguousarray(np.asarray(xt, dtype=np.float64))
    rng = np.random.default_rng(seed)
    n, done, dt = 256, 0, 0.0
    while dt < min_seconds and done < max_rays:
        rays = np.stack([np.asarray(views)[rng.integers(0, len(views), n)], rng.integers(0, g.nv, n),
                         rng.integers(0, g.nu, n)], 1)
        t0 = time.perf_counter()
        oracle.forward_rays(g, x64, rays)
        dt += time.perf_counter() - t0
        done += n
        n *= 2
    per_ray = dt / done
    hi = host_info()
    return {
        "value": (g.d / g.n_p) / per_ray / 1e9,
        "unit": "GUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "%d seeded random rays of the %d-view mini-batch through the oracle's FP64 ray-subset forward "
                  "projector (%d slices per ray) in %.1f s: %.3g ms per ray; a view's %d rays count %d voxel-view "
                  "updates" % (done, len(views), g.nx, dt, per_ray * 1e3, g.n_p, g.d),
        "seconds_per_ray": per_ray,
        "cpu_model": hi["cpu_model"],
        "logical_cpus": hi["logical_cpus"],
    }


def cpu_baseline_iterations(g, b32, perms, B, alpha0, beta, lo, hi, min_seconds=12.0, max_iters=4):
    """The FP64 oracle, as it stands, on a bounded sample of a small workload: FB-LISA
    iterations from x = 0 on the run's first mini-batches, until about min_seconds of host
    time have passed (at most max_iters iterations)."""
    import oracle
    b64 = b32.astype(np.float64)
    x = np.zeros(g.vol_shape)
    calls = {"fp": 0, "bp": 0}
    n_iter = n_trials = 0
    t0 = time.perf_counter()
    while n_iter < max_iters and (n_iter == 0 or time.perf_counter() - t0 < min_seconds):
        views = perms[n_iter][:B]
        f0, grad, _ = oracle.objective_and_gradient(g, x, b64, views)
        calls["fp"] += 1
        calls["bp"] += 1

        def fun(z, views=views):
            calls["fp"] += 1
            return oracle.objective(g, z, b64, views)

        alpha, x, fbar, trials = oracle.line_search(fun, x, f0, grad, alpha0, beta, 0.0, lo, hi)
        n_iter += 1
        n_trials += len(trials)
    dt = time.perf_counter() - t0
    updates = (calls["fp"] + calls["bp"]) * g.d * B
    return {
        "value": updates / dt / 1e9,
        "unit": "GUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "%d FB-LISA iterations (objective, gradient, %d line-search trials) of the same workload from "
                  "x = 0 on its first %d-view mini-batches: %d forward + %d backprojection calls in %.1f s"
                  % (n_iter, n_trials, B, calls["fp"], calls["bp"], dt),
    }


def train_step_proposer(fbl, syn, n_runs=200, iters=2000, lr=3e-3):
    """The learned-step perceptron, trained on the GPU from the traces of n_runs seeded plain
    FB-LISA runs of the 64^3 / 60-view / 6-view-batch workload."""
    import torch
    rec = fbl.TraceRecorder()
    g = syn.config_geometry("c1")
    cfg = syn.CONFIGS["c1"]
    for rep in range(n_runs):
        seed = 1000 + rep
        ells, _ = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"])
        b = syn.add_noise(syn.ellipsoid_line_integrals(g, ells, np.arange(g.n_views)), 0.01, seed=seed + 1)
        perms = syn.view_permutations(g.n_views, 200, seed=seed + 2)
        run = fbl.FBLisa(g, torch.from_numpy(b.astype(np.float32)).cuda(), n0=cfg["batch"], epochs=cfg["epochs"],
                         lo=cfg["lo"], hi=cfg["hi"])
        run.run(perms, callback=rec)
    X, t = rec.arrays()
    model = fbl.StepModel(syn.mlp_params(7))
    curve = model.fit(X, t, iters=iters, lr=lr)
    return model, len(t), curve


CLOCK_WARMUP_S = 1.0


def warm_clock(fbl, plan, x, views, r, g, seconds=None):
    """Forward and backprojection of x, repeated for `seconds` (no state of a run changes:
    r and g are scratch).  After a pause the GPU's clock needs tens of milliseconds of
    sustained load to reach its working frequency: a projector launch's cycle count stays
    the same while its duration falls by about 10%, so a short timed region that starts
    cold measures the ramp."""
    import torch
    seconds = CLOCK_WARMUP_S if seconds is None else seconds
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            fbl.fb_lisa_forward(plan, x, views, y=r)
            fbl.fb_lisa_backproject(plan, r, views, g=g)
        torch.cuda.synchronize()



def summarize(values):
    v = np.asarray(values, dtype=np.float64)
    return {"median": round(float(np.median(v)), 2), "min": round(float(v.min()), 2),
            "max": round(float(v.max()), 2), "p10": round(float(np.percentile(v, 10)), 2),
            "p90": round(float(np.percentile(v, 90)), 2), "n": int(v.size)}


def rmse_race(fbl, g, cfg, b_f32, xt_dev, perms, runs, warm_s=None):
    """Time to the reconstruction error of the plain FP32 run, at equal wall-clock budgets.

    The plain FP32 method runs its configured epochs; its elapsed time T is every run's
    budget, its final RMSE is the target RMSE*, its smallest RMSE the second target.  Each
    other run (learned initial step, with the projector reading a 16-bit copy of the
    volume and 16-bit data, or FP32) runs for the same wall time T: its configured epochs,
    then, if time remains, more iterations in the last epoch's setting.  Reported per run:
    the time and iterations to RMSE* and to the plain run's minimum, RMSE and RE at T/2
    and T, forward calls per iteration and the backtrack histogram.  Device-synchronised
    host clock; the RMSE evaluations are excluded by timestamps.

    runs: list of (name, dict(vol_dtype, mixed, sr_seed, proj16, learned proposer or None)).
    """
    import torch
    nrm_t = float(torch.linalg.vector_norm(xt_dev.double()))
    sqd = math.sqrt(g.d)

    class Budget(Exception):
        pass

    def go(name, b_dev, vol_dtype, alpha_init, budget, mixed=False, sr_seed=None, stop_below=None):
        B = cfg["batch"]
        run = fbl.FBLisa(g, b_dev, n0=B, epochs=cfg["epochs"], lo=cfg["lo"], hi=cfg["hi"], vol_dtype=vol_dtype,
                         sr_seed=sr_seed, n_max=B, mixed=mixed)
        st = {"excluded": 0.0, "t": [], "rmse": []}

        def cb(r, it):
            t_in = time.perf_counter()
            el = t_in - st["t0"] - st["excluded"]            # the iterate is complete (read back)
            st["t"].append(el)
            e = float(torch.sqrt(torch.mean((r.x.float() - xt_dev) ** 2)))
            st["rmse"].append(e)
            if len(st["rmse"]) % 60 == 0:                    # progress of long runs
                log("  %s: iteration %d, %.1f s, rmse %.4e" % (name, len(st["rmse"]), el, e))
            st["excluded"] += time.perf_counter() - t_in
            if budget is not None and el >= budget:
                raise Budget()
            if stop_below is not None and e <= stop_below:
                raise Budget()

        warm_clock(fbl, run.plan, run.x16, perms[0][:B], run.r[:B], run.g, warm_s)
        torch.cuda.synchronize()
        st["t0"] = time.perf_counter()
        try:
            run.run(perms, alpha_init=alpha_init, callback=cb)
            if budget is not None:
                for k in range(len(run.history), len(perms)):
                    cb(run, run.iterate(perms[k][:B], alpha_init, epoch=run.epochs))
        except Budget:
            pass
        hist = run.history
        run = None
        torch.cuda.empty_cache()
        return hist, st

    hist_p, st_p = go("plain f32", b_f32, "f32", None, None)
    T = st_p["t"][-1]
    target = st_p["rmse"][-1]
    best = min(st_p["rmse"])

    def first(st, thr):
        i = next((i for i, e in enumerate(st["rmse"]) if e <= thr), None)
        return None if i is None else (round(st["t"][i], 4), i + 1)

    def at_time(st, t):
        i = max([j for j, tt in enumerate(st["t"]) if tt <= t], default=None)
        if i is None:
            return None
        return {"rmse": st["rmse"][i], "re": st["rmse"][i] * sqd / nrm_t, "iterations": i + 1}

    def summary(hist, st):
        bt = [it.backtracks for it in hist]
        hist_bt = {}
        for b_ in bt:
            hist_bt[str(b_)] = hist_bt.get(str(b_), 0) + 1
        tt = first(st, target)
        tm = first(st, best)
        return {"to_rmse_target": None if tt is None else {"seconds": tt[0], "iterations": tt[1]},
                "to_plain_min_rmse": None if tm is None else {"seconds": tm[0], "iterations": tm[1]},
                "at_half_budget": at_time(st, 0.5 * T), "at_budget": at_time(st, T),
                "iterations": len(hist), "seconds": round(st["t"][-1], 4),
                "fp_calls_per_iter": round(float(np.mean([2 + b_ for b_ in bt])), 3),
                "backtracks_per_iter": round(float(np.mean(bt)), 3),
                "backtrack_histogram": dict(sorted(hist_bt.items(), key=lambda kv: int(kv[0])))}

    rec = {"rmse_target": target, "plain_min_rmse": best, "budget_s": round(T, 4),
           "rule": "RMSE* is the plain FP32 run's RMSE after its configured epochs; every run gets that run's "
                   "wall time T as its budget (configured epochs, then further iterations in the last epoch's "
                   "setting while time remains); speedup = plain time to RMSE* / run's time to RMSE*",
           "plain_f32": summary(hist_p, st_p)}
    b16 = None
    for name, spec in runs:
        if spec.get("proj16") and b16 is None:
            b16 = b_f32.half()
        b_dev = b16 if spec.get("proj16") else b_f32
        # a run marked "until_targets" stops once it has reached both targets (the budget still caps it)
        hist, st = go(name, b_dev, spec["vol_dtype"], spec.get("proposer"), T, mixed=spec.get("mixed", False),
                      sr_seed=spec.get("sr_seed"), stop_below=min(target, best) if spec.get("until_targets") else None)
        sm = summary(hist, st)
        if spec.get("until_targets") and st["t"][-1] < T:
            sm["at_budget"] = None
            sm["stopped"] = "after reaching both targets"
        sm["storage"] = spec["label"]
        tp = rec["plain_f32"]["to_rmse_target"]["seconds"]
        sm["speedup"] = (round(tp / sm["to_rmse_target"]["seconds"], 3)
                         if sm["to_rmse_target"] is not None else None)
        rec[name] = sm
        log("  %s: speedup %s" % (name, sm["speedup"]))
    del b16
    torch.cuda.empty_cache()
    return rec


LEARNED_RUNS = {
    "learned_bf16": dict(vol_dtype="bf16", mixed=True, proj16=True,
                         label="projector reads a BF16 copy of the FP32 iterate; FP16 data"),
    "learned_bf16_sr": dict(vol_dtype="bf16", sr_seed=2024, proj16=True,
                            label="BF16 iterate with stochastic rounding; FP16 data"),
    "learned_f16": dict(vol_dtype="f16", mixed=True, proj16=True,
                        label="projector reads an FP16 copy of the FP32 iterate; FP16 data"),
    "learned_f16_until": dict(vol_dtype="f16", mixed=True, proj16=True, until_targets=True,
                              label="projector reads an FP16 copy of the FP32 iterate; FP16 data; stopped once "
                                    "both targets are reached"),
    "learned_f32": dict(vol_dtype="f32", label="FP32 iterate and data"),
}


def timed_steps(fbl, g, cfg, b_dev, perms, steps, warmup, clock_warmup, per_iteration_timing):
    """W warmup iterations, then exactly K timed iterations of the plain FP32 method, with
    the projector (and prox-trial) launches bracketed by HIP events on the launch stream."""
    import torch
    B = cfg["batch"]
    run = fbl.FBLisa(g, b_dev, n0=B, epochs=cfg["epochs"], alpha0=1e-3, beta=0.5, lo=cfg["lo"], hi=cfg["hi"],
                     n_max=B)
    warm_clock(fbl, run.plan, run.x, perms[0][:B], run.r[:B], run.g, clock_warmup)
    for k in range(warmup):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    kernels = ("forward", "backproject", "step") if per_iteration_timing else ("forward", "backproject")
    run.plan.timing(True, kernels=kernels)
    n_hist = len(run.history)
    per_it = {k: [] for k in kernels}
    tot = {k: [0.0, 0] for k in kernels}
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        run.iterate(perms[k][:B])
        if per_iteration_timing:   # the iteration has synchronised: its events are complete
            kt = run.plan.timing_read()
            for name in kernels:
                ms, n = kt[name]
                tot[name][0] += ms
                tot[name][1] += n
                if n:
                    per_it[name].append(ms / n * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if not per_iteration_timing:
        kt = run.plan.timing_read()
        for name in kernels:
            tot[name] = [kt[name][0], kt[name][1]]
    run.plan.timing(False)
    timed = run.history[n_hist:]
    # a short supplementary pass with every launch bracketed gives the other kernels' means
    k0 = warmup + steps
    run.plan.timing(True)
    for k in range(k0, k0 + 3):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    ks = run.plan.timing_read()
    run.plan.timing(False)
    return run, timed, t1 - t0, tot, per_it, ks


def phi_cone_fraction(fbl, g, views, B):
    """Fraction of the voxels each view's rays touch (the cone of the view inside the
    volume), from the backprojection of an all-ones residual: every tap weight is
    nonnegative, so a voxel's value is nonzero exactly where some ray of the view reaches it
    with nonzero weight.  Mean over the views."""
    import torch
    fr = []
    with fbl.Plan(g, max_batch=1) as plan:
        ones = torch.ones((1, g.nv, g.nu), dtype=torch.float32, device="cuda")
        gg = torch.empty(g.vol_shape, dtype=torch.float32, device="cuda")
        for v in views[:B]:
            fbl.fb_lisa_backproject(plan, ones, [int(v)], grad_scale=1.0, g=gg)
            fr.append(float((gg != 0).sum()) / g.d)
        del gg, ones
    torch.cuda.empty_cache()
    return float(np.mean(fr))


def projector_block(fbl, syn, name, g, cfg, b_dev, perms, steps, warmup, clock_warmup, per_iteration_timing):
    """Throughput of the timed steps and the projector kernels against their rooflines."""
    B = cfg["batch"]
    run, timed, wall, tot, per_it, ks = timed_steps(fbl, g, cfg, b_dev, perms, steps, warmup, clock_warmup,
                                                    per_iteration_timing)
    n_fp, n_bp = tot["forward"][1], tot["backproject"][1]
    gups = (n_fp + n_bp) * g.d * B / wall / 1e9
    t_fp = tot["forward"][0] / n_fp * 1e-3
    t_bp = tot["backproject"][0] / n_bp * 1e-3
    kernel_us = {k: round(ms / n * 1e3, 2) for k, (ms, n) in ks.items() if n}
    kernel_us.update({k: round(tot[k][0] / tot[k][1] * 1e3, 2) for k in tot if tot[k][1]})
    t_st = (tot["step"][0] / tot["step"][1] * 1e-3) if "step" in tot and tot["step"][1] else \
        ks["step"][0] / ks["step"][1] * 1e-3
    bytes_view = B * (g.d * 4 + 4 * g.n_p)
    bytes_min = g.d * 4 + B * g.n_p * (4 + 4)
    share = {"fp_kernel": tot["forward"][0], "bp_kernel": tot["backproject"][0]}
    dominant = max(share, key=share.get)
    t_dom = t_fp if dominant == "fp_kernel" else t_bp
    other = "bp_kernel" if dominant == "fp_kernel" else "fp_kernel"
    t_other = t_bp if dominant == "fp_kernel" else t_fp
    achieved = bytes_view / t_dom / 1e9
    out = {
        "gups": gups, "wall": wall, "B": B,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dominant, name),
            "kernel": dominant,
            "bytes_per_launch": bytes_view,
            "compulsory_bytes_per_launch": bytes_min,
            "compulsory_frac": round(bytes_min / t_dom / 1e9 / HBM_PEAK_GBS, 4),
            "valu_busy": profile_value(dominant, name, "valu_busy"),
            "l2_hit_rate": profile_value(dominant, name, "l2_hit_rate"),
            "share_of_timed_region": round(share[dominant] / (wall * 1e3), 4),
        },
        "roofline_other": {
            "kernel": other,
            "achieved": round(bytes_view / t_other / 1e9, 1),
            "frac": round(bytes_view / t_other / 1e9 / HBM_PEAK_GBS, 4),
            "compulsory_frac": round(bytes_min / t_other / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(other, name),
            "valu_busy": profile_value(other, name, "valu_busy"),
            "l2_hit_rate": profile_value(other, name, "l2_hit_rate"),
            "share_of_timed_region": round(share[other] / (wall * 1e3), 4),
        },
        "pair_frac": round(2 * bytes_view / (t_fp + t_bp) / 1e9 / HBM_PEAK_GBS, 4),
        "kernel_us": kernel_us,
        "step_hbm": {"bytes_per_launch": 12 * g.d, "achieved": round(12 * g.d / t_st / 1e9, 1),
                     "frac": round(12 * g.d / t_st / 1e9 / HBM_PEAK_GBS, 4)},
        "gups_per_op": {"forward": round(g.d * B / t_fp / 1e9, 2), "backproject": round(g.d * B / t_bp / 1e9, 2)},
        "gsamples_per_s": {"forward": round(B * g.n_p * g.nx / t_fp / 1e9, 2),
                           "backproject": round(B * g.n_p * g.nx / t_bp / 1e9, 2)},
        "calls": {"forward": n_fp, "backproject": n_bp, "step": sum(len(it.trials) for it in timed)},
        "mean_backtracks": float(np.mean([it.backtracks for it in timed])),
    }
    # What binds the projector kernels is VALU issue, not HBM: both against the VALU issue
    # peak, from the committed counter summaries (SQ_INSTS_VALU over the profiled duration).
    alu = {}
    for kern in (dominant, other):
        vb = profile_value(kern, name, "valu_busy")
        if vb is not None:
            alu[kern] = {"bound": "alu", "achieved": round(vb * VALU_PEAK_TLOPS, 2), "peak": round(VALU_PEAK_TLOPS, 2),
                         "unit": "T VALU lane-ops/s", "frac": vb}
    if alu:
        out["roofline_alu"] = alu
    if per_iteration_timing:
        out["per_launch_us"] = {k: summarize(v) for k, v in per_it.items() if v}
    return out, run


def paper_shaped_run(fbl, syn, seconds: float, views: int = 72, n: int = 560, n0: int = 8, seed: int = 5600):
    """The paper's own variant on a synthetic stand-in for its walnut scan: an n^3 volume,
    `views` projections over [0, 2 pi), 2% noise, R = mu ||x||_1 + nonnegativity, the
    growing mini-batch of Step 1 (C = N_0 eps_{ceil(n_theta/N_0)}), run for a wall-clock
    budget.  Reports the batch sizes per epoch and the relative error against time."""
    import torch
    h = 64.0 / n
    det = (3 * n) // 2
    g = syn.Geometry(n, n, n, h, h, h, det, det, 96.0 / det, 96.0 / det, 500.0, 1000.0, views)
    t0 = time.perf_counter()
    ells, xt = syn.phantom(g, 30, seed=seed, sub=2)
    b = syn.add_noise(syn.ellipsoid_line_integrals(g, ells, np.arange(views)), 0.02, seed=seed + 1)
    log("paper-shaped data (%d^3, %d views, %dx%d detector): %.1f s" % (n, views, det, det, time.perf_counter() - t0))
    bd = torch.from_numpy(b.astype(np.float32)).cuda()
    del b
    xt_dev = torch.from_numpy(xt.astype(np.float32)).cuda()
    nrm = float(torch.linalg.vector_norm(xt_dev.double()))
    # mu: 2% of the largest entry of the full-batch gradient at x = 0
    with fbl.Plan(g, max_batch=views) as plan:
        r0 = fbl.fb_lisa_forward(plan, torch.zeros_like(xt_dev), np.arange(views), bd)
        g0 = fbl.fb_lisa_backproject(plan, r0, np.arange(views))
        mu = 0.02 * float(g0.abs().max())
        del r0, g0
    C = fbl.growing_batch_C(views, n0)
    perms = syn.view_permutations(views, 200000, seed=seed + 2)
    run = fbl.FBLisa(g, bd, n0=n0, epochs=100000, mu=mu, C=C)
    st = {"excluded": 0.0, "series": [], "next": 0.0}

    class Budget(Exception):
        pass

    def cb(r, it):
        t_in = time.perf_counter()
        el = t_in - st["t0"] - st["excluded"]
        if el >= st["next"] or el >= seconds:
            re = float(torch.linalg.vector_norm((r.x - xt_dev).double())) / nrm
            st["series"].append({"t": round(el, 3), "k": it.k + 1, "epoch": it.epoch, "batch": len(it.batch),
                                 "re": re})
            st["next"] = el + max(0.5, seconds / 60.0)
            if len(st["series"]) % 10 == 1:
                log("paper-shaped run: %.1f s, iteration %d, epoch %d, batch %d, RE %.4f"
                    % (el, it.k + 1, it.epoch, len(it.batch), re))
        st["excluded"] += time.perf_counter() - t_in
        if el >= seconds:
            raise Budget()

    torch.cuda.synchronize()
    st["t0"] = time.perf_counter()
    try:
        run.run(perms, callback=cb)
    except Budget:
        pass
    per_epoch = {}
    for it in run.history:
        per_epoch.setdefault(it.epoch, len(it.batch))
    return {
        "mode": "paper-shaped growth run",
        "workload": "%d^3 ellipsoid phantom (30), %d views over [0, 2pi), %dx%d detector, 2%% noise, "
                    "mu = %.4g (2%% of max |grad f(0)|), nonnegativity, N_0 = %d, growth C = %.4g"
                    % (n, views, det, det, mu, n0, C),
        "seconds": seconds,
        "iterations": len(run.history),
        "epochs": max(per_epoch) if per_epoch else 0,
        "batch_per_epoch": [per_epoch[e] for e in sorted(per_epoch)],
        "mean_backtracks": float(np.mean([it.backtracks for it in run.history])),
        "series": st["series"],
        "final_re": st["series"][-1]["re"] if st["series"] else None,
    }


def kernel_scaling(fbl, syn, names, reps=5, storage="f32"):
    """Projector and step kernel times alone at several workload sizes, on a voxelised phantom
    and a seeded residual (no measured data needed): forward, backprojection and prox trial
    of one mini-batch of the workload's size, mean over `reps` launches after a clock warm-up.
    `storage` is the volume's storage type (f32, bf16 or f16); the view model then counts
    its bytes per voxel, and the prox trial moves 4 + 2 x (bytes per voxel) bytes per voxel."""
    import torch
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[storage]
    vb = 4 if storage == "f32" else 2
    out = []
    for name in names:
        cfg = syn.CONFIGS[name]
        g = syn.config_geometry(name)
        B = cfg["batch"]
        t0 = time.perf_counter()
        _, xt = syn.phantom(g, cfg["k"], seed=1000 * int(name[1:]), hi=cfg["hi"], sub=1)
        x = torch.from_numpy(xt.astype(np.float32)).cuda().to(tdt).contiguous()
        del xt
        views = syn.view_permutations(g.n_views, 1, seed=7)[0][:B]
        r = torch.from_numpy(syn.random_projections(g, B, seed=8, scale=0.1)).cuda()
        with fbl.Plan(g, storage, "f32", max_batch=B) as plan:
            plan_s = time.perf_counter() - t0
            y = fbl.fb_lisa_forward(plan, x, views)
            gr = fbl.fb_lisa_backproject(plan, r, views)
            xb, red = fbl.fb_lisa_step(plan, x, gr, 1e-3, 0.0, 0.0, math.inf)
            warm_clock(fbl, plan, x, views, y, gr)
            plan.timing(True)
            for _ in range(reps):
                fbl.fb_lisa_forward(plan, x, views, y=y)
                fbl.fb_lisa_backproject(plan, r, views, g=gr)
                fbl.fb_lisa_step(plan, x, gr, 1e-3, 0.0, 0.0, math.inf, xbar=xb, red=red)
            torch.cuda.synchronize()
            kt = plan.timing_read()
            t_mixed = None
            if storage != "f32":
                # the prox trial of the mixed form: FP32 iterate, 16-bit copy (14 bytes per voxel)
                x32 = x.float()
                xb32 = torch.empty_like(x32)
                fbl.fb_lisa_step_mixed(plan, x32, gr, 1e-3, xbar=xb32, xbar16=xb, red=red)
                plan.timing(True, kernels=("step",))
                for _ in range(reps):
                    fbl.fb_lisa_step_mixed(plan, x32, gr, 1e-3, xbar=xb32, xbar16=xb, red=red)
                torch.cuda.synchronize()
                ms, n = plan.timing_read()["step"]
                t_mixed = ms / n * 1e-3
                del x32, xb32
        t = {k: ms / n * 1e-3 for k, (ms, n) in kt.items() if n}
        byts = B * (g.d * vb + 4 * g.n_p)
        rec = {"workload": "%s: %d^3, %d views, %dx%d detector, batch %d" % (name, g.nx, g.n_views, g.nu, g.nv, B),
               "storage": storage,
               "setup_s": round(plan_s, 1),
               "forward_us": round(t["forward"] * 1e6, 1), "backproject_us": round(t["backproject"] * 1e6, 1),
               "step_us": round(t["step"] * 1e6, 1),
               "forward_gups": round(g.d * B / t["forward"] / 1e9, 1),
               "backproject_gups": round(g.d * B / t["backproject"] / 1e9, 1),
               "forward_hbm_frac": round(byts / t["forward"] / 8e12, 4),
               "backproject_hbm_frac": round(byts / t["backproject"] / 8e12, 4),
               "step_hbm_frac": round((4 + 2 * vb) * g.d / t["step"] / 8e12, 4)}
        if t_mixed is not None:
            rec["step_mixed_us"] = round(t_mixed * 1e6, 1)
            rec["step_mixed_hbm_frac"] = round(14 * g.d / t_mixed / 8e12, 4)
        log(json.dumps(rec))
        out.append(rec)
        del x, r, y, gr, xb
        torch.cuda.empty_cache()
    return {"mode": "kernel scaling", storage: out}



def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--clock-warmup", type=float, default=CLOCK_WARMUP_S, metavar="SECONDS",
                    help="projector launches on the initial iterate before the warmup steps, so the timed "
                         "region runs at the GPU's working clock (no state of the run changes)")
    ap.add_argument("--config", default="c5",
                    help="workload (c1..c5); the default, c5 (1024^3, 1440 views, 1536^2, batch 40), is the one "
                         "the metric's time-to-RMSE comparison is defined on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-rmse", action="store_true",
                    help="skip the time-to-RMSE comparison (learned step + BF16 storage against plain FP32)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary 256^3 block (throughput and a three-order time-to-RMSE comparison)")
    ap.add_argument("--no-cone-fraction", action="store_true",
                    help="skip the cone fraction (one single-view backprojection per view of the batch)")
    ap.add_argument("--orders", type=int, default=1,
                    help="view orders of the main time-to-RMSE comparison (seeds base+2, base+3, ...); the median "
                         "speedup over them is reported (one order by default, to stay within minutes at 1024^3)")
    ap.add_argument("--variants", default="learned_bf16,learned_f16_until",
                    help="learned runs of the main comparison, comma-separated from %s" % ",".join(LEARNED_RUNS))
    ap.add_argument("--probe", action="store_true",
                    help="counter-collection run: 3 forward, 1 backprojection, 1 step call of the workload, then "
                         "a plain 512 MiB device copy whose FETCH_SIZE/WRITE_SIZE calibrate the counters")
    ap.add_argument("--paper-run", type=float, default=0.0, metavar="SECONDS",
                    help="instead of the benchmark: the paper's growing-batch variant with mu > 0 on a 560^3 / "
                         "72-view synthetic stand-in, for this many seconds")
    ap.add_argument("--kernel-storage", default="f32", choices=("f32", "bf16", "f16"),
                    help="volume storage type for --kernels")
    ap.add_argument("--kernels", default="", metavar="CONFIGS",
                    help="instead of the benchmark: time the projector and step kernels alone at these workloads "
                         "(comma-separated, e.g. c3,c5)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(--gpus %d / WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        return 2

    import torch
    import synthetic as syn
    import paper_2605_12085_amd as fbl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.kernels:
        print(json.dumps(kernel_scaling(fbl, syn, [c for c in args.kernels.split(",") if c],
                                        storage=args.kernel_storage)), flush=True)
        return 0
    if args.paper_run > 0:
        print(json.dumps(paper_shaped_run(fbl, syn, args.paper_run)), flush=True)
        return 0
    name = args.config
    if args.probe:
        # values do not change the kernels' work: a seeded random volume and zero data
        cfg = syn.CONFIGS[name]
        g = syn.config_geometry(name)
        B = cfg["batch"]
        plan = fbl.Plan(g, max_batch=B)
        x = torch.from_numpy(syn.random_volume(g, seed=5)).cuda()
        b_dev = torch.zeros((g.n_views, g.nv, g.nu), dtype=torch.float32, device="cuda")
        views = syn.view_permutations(g.n_views, 1, seed=1000 * int(name[1:]) + 2)[0][:B]
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        for _ in range(3):
            r = fbl.fb_lisa_forward(plan, x, views, b_dev, loss=loss)
        gr = fbl.fb_lisa_backproject(plan, r, views)
        fbl.fb_lisa_step(plan, x, gr, 1e-3, 0.0, cfg["lo"], cfg["hi"])
        torch.cuda.synchronize()
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": name, "copy_bytes": src.numel() * 4,
                          "forward_bytes_model": B * (g.d * 4 + 4 * g.n_p)}), flush=True)
        return 0

    t_setup = time.perf_counter()
    g, cfg, seed, xt, b_dev = make_workload(syn, name)
    B = cfg["batch"]
    n_it = cfg["epochs"] * math.ceil(g.n_views / B)
    perms = syn.view_permutations(g.n_views, max(args.warmup + args.steps + 3, 3 * n_it), seed=seed + 2)
    log("setup of %s (phantom, exact line integrals, noise): %.1f s" % (name, time.perf_counter() - t_setup))

    blk, run = projector_block(fbl, syn, name, g, cfg, b_dev, perms, args.steps, args.warmup, args.clock_warmup,
                               per_iteration_timing=True)
    del run
    torch.cuda.empty_cache()
    log("%s: %.1f GUPS, %.3f ms per step" % (name, blk["gups"], blk["wall"] / args.steps * 1e3))
    rec = {
        "metric": METRIC,
        "value": round(blk["gups"], 3),
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(blk["wall"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %d^3 fp32 ellipsoid phantom (%d ellipsoids), %d views, %dx%d detector, "
                        "mini-batch %d, %d epochs, prox [%g, %g], 1%% Gaussian noise on exact line integrals"
                        % (name, g.nx, cfg["k"], g.n_views, g.nu, g.nv, B, cfg["epochs"], cfg["lo"], cfg["hi"]),
            "global_batch": B,
            "parallelism": "single GPU",
        },
    }
    for k in ("roofline", "roofline_other", "roofline_alu", "pair_frac", "kernel_us", "per_launch_us", "step_hbm",
              "gups_per_op", "gsamples_per_s", "calls", "mean_backtracks"):
        if k in blk:
            rec[k] = blk[k]
    if not args.no_cone_fraction:
        rec["roofline"]["cone_fraction"] = round(phi_cone_fraction(fbl, g, perms[0], B), 4)
    xt_dev = torch.from_numpy(xt.astype(np.float32)).cuda()
    model = None
    if not args.no_time_to_rmse:
        log("training the step proposer (200 plain runs of the 64^3 workload) ...")
        t_tr = time.perf_counter()
        model, n_samples, curve = train_step_proposer(fbl, syn)
        log("trained on %d samples in %.1f s (loss %.3e -> %.3e)" % (n_samples, time.perf_counter() - t_tr,
                                                                    curve[0], curve[-1]))
        prop = fbl.LearnedStep(model)
        runs = [(v, dict(LEARNED_RUNS[v], proposer=prop)) for v in args.variants.split(",") if v]
        log("time to RMSE at %s ..." % name)
        tt = rmse_race(fbl, g, cfg, b_dev, xt_dev, perms, runs)
        tt["proposer"] = "5-64-64-1 perceptron trained on %d iterations of 200 seeded 64^3 runs" % n_samples
        tt["view_order_seed"] = seed + 2
        if args.orders > 1:
            names = [v for v, _ in runs]
            more = []
            for s_off in range(3, 2 + args.orders):
                log("time to RMSE at %s, view order %d ..." % (name, s_off))
                p_o = syn.view_permutations(g.n_views, 3 * n_it, seed=seed + s_off)
                more.append(rmse_race(fbl, g, cfg, b_dev, xt_dev, p_o, runs))
            orders = [tt] + more
            sp = {v: [o[v]["speedup"] for o in orders] for v in names}
            tt["view_orders"] = {
                "seeds": [seed + s for s in range(2, 2 + args.orders)], "speedup": sp,
                "median_speedup": {v: (float(np.median(x)) if all(y is not None for y in x) else None)
                                   for v, x in sp.items()},
                "plain_seconds_to_target": [o["plain_f32"]["to_rmse_target"]["seconds"] for o in orders],
                "rmse_target": [o["rmse_target"] for o in orders],
                "speedup_to_plain_min": {v: [round(o["plain_f32"]["to_plain_min_rmse"]["seconds"]
                                                   / o[v]["to_plain_min_rmse"]["seconds"], 3)
                                             if o[v]["to_plain_min_rmse"] else None for o in orders] for v in names}}
        rec["time_to_rmse"] = tt
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        if name in DEVICE_DATA:
            rec["cpu_baseline"] = cpu_baseline_rays(g, xt, perms[0][:B])
        else:
            rec["cpu_baseline"] = cpu_baseline_iterations(g, b_dev.cpu().numpy(), perms, B, 1e-3, 0.5, cfg["lo"],
                                                          cfg["hi"])
            rec["cpu_baseline"].update(host_info())
    del xt, xt_dev, b_dev
    torch.cuda.empty_cache()
    if not args.no_secondary and name != "c2":
        log("secondary block: c2 ...")
        g2, cfg2, seed2, xt2, b2 = make_workload(syn, "c2")
        n_it2 = cfg2["epochs"] * math.ceil(g2.n_views / cfg2["batch"])
        perms2 = syn.view_permutations(g2.n_views, max(args.warmup + args.steps + 3, 3 * n_it2), seed=seed2 + 2)
        blk2, run2 = projector_block(fbl, syn, "c2", g2, cfg2, b2, perms2, args.steps, args.warmup,
                                     args.clock_warmup, per_iteration_timing=False)
        del run2
        sec = {"workload": "c2: 256^3, 360 views, 384x384 detector, mini-batch 20, prox [0, 0.03]",
               "value": round(blk2["gups"], 3), "ms_per_step": round(blk2["wall"] / args.steps * 1e3, 3)}
        for k in ("roofline", "roofline_other", "roofline_alu", "pair_frac", "kernel_us", "step_hbm", "calls",
                  "mean_backtracks"):
            sec[k] = blk2[k]
        if model is not None:
            prop = fbl.LearnedStep(model)
            xt2_dev = torch.from_numpy(xt2.astype(np.float32)).cuda()
            names = ("learned_bf16", "learned_bf16_sr", "learned_f16", "learned_f32")
            orders = []
            for s_off in (2, 3, 4):
                p2 = syn.view_permutations(g2.n_views, 3 * n_it2, seed=seed2 + s_off)
                orders.append(rmse_race(fbl, g2, cfg2, b2, xt2_dev, p2,
                                        [(v, dict(LEARNED_RUNS[v], proposer=prop)) for v in names], warm_s=0.5))
            sec["time_to_rmse"] = orders[0]
            sp = {v: [o[v]["speedup"] for o in orders] for v in names}
            sec["view_orders"] = {"seeds": [seed2 + s for s in (2, 3, 4)], "speedup": sp,
                                  "median_speedup": {v: (float(np.median(x)) if all(y is not None for y in x)
                                                         else None) for v, x in sp.items()}}
            del xt2_dev
        rec["secondary"] = sec
        del b2
        torch.cuda.empty_cache()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
