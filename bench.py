#!/usr/bin/env python
"""Benchmark of the FB-LISA hot path on one MI355X.

A step is one FB-LISA iteration (Algorithm 1, Steps 2a-2d) of the 256^3 workload:
the forward projection of a 20-view mini-batch with residual and FP64 objective, the
backprojection (gradient), and the line search's prox trials, each followed by a
forward projection of the trial point and one read-back of three FP64 scalars.
Inputs (phantom, noisy data, view draws) are synthetic, seeded and already resident
in device memory when the timed region starts.

value = projector updates per second over the timed steps (GUPS): every forward or
backprojection call over B views counts d*B voxel-view updates (d voxels); the time
includes the step kernels, the reductions and the per-trial host synchronisation.

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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"fp_kernel": "forward.hip", "bp_kernel": "backproject.hip"}


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


def measured_traffic(kernel: str, cfg: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.json" % (kernel, cfg))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(g, b32, perms, B, alpha0, beta, lo, hi, min_seconds=12.0, max_iters=4):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: FB-LISA
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


def time_to_rmse(fbl, g, cfg, b32, xt, perms, proposer, variants=("bf16", "bf16_nearest", "f16", "f32")):
    """Wall time to the reconstruction error of the plain FP32 run: the plain FP32 run sets
    RMSE* (its error after the configured epochs) and is timed to its first iterate at or
    below RMSE*; the learned-step runs are timed to the same target.  A learned run that has
    not reached it after the configured epochs goes on, in the last epoch's setting, up to
    len(perms) iterations (perms rows beyond the configured ones).  Device-synchronised
    host clock; RMSE evaluations excluded."""
    import torch
    xt_dev = torch.from_numpy(xt.astype(np.float32)).cuda()

    class Reached(Exception):
        pass

    def go(b_dev, vol_dtype, alpha_init, target, sr_seed=None):
        # the constant-batch C keeps N_t = N_0 for the configured epochs, so buffers for
        # one batch suffice (n_max)
        run = fbl.FBLisa(g, b_dev, n0=cfg["batch"], epochs=cfg["epochs"], lo=cfg["lo"], hi=cfg["hi"],
                         vol_dtype=vol_dtype, sr_seed=sr_seed, n_max=cfg["batch"])
        st = {"excluded": 0.0, "t": [], "rmse": []}

        def cb(r, it):
            t_in = time.perf_counter()
            st["t"].append(t_in - st["t0"] - st["excluded"])   # the iterate is complete (read back)
            e = float(torch.sqrt(torch.mean((r.x.float() - xt_dev) ** 2)))
            st["rmse"].append(e)
            if len(st["rmse"]) % 50 == 0:   # progress of long runs (outside the timed intervals)
                log("  %s: iteration %d, rmse %.4e" % (vol_dtype, len(st["rmse"]), e))
            st["excluded"] += time.perf_counter() - t_in
            if target is not None and e <= target:
                raise Reached()

        B0 = cfg["batch"]
        warm_clock(fbl, run.plan, run.x, perms[0][:B0], run.r[:B0], run.g)
        torch.cuda.synchronize()
        st["t0"] = time.perf_counter()
        try:
            run.run(perms, alpha_init=alpha_init, callback=cb)
            if target is not None:
                n_cfg = len(run.history)
                for k in range(n_cfg, len(perms)):
                    cb(run, run.iterate(perms[k][:cfg["batch"]], alpha_init, epoch=run.epochs))
        except Reached:
            pass
        return run.history, st

    b_f32 = b32 if torch.is_tensor(b32) else torch.from_numpy(b32).cuda()
    hist_p, st_p = go(b_f32, "f32", None, None)
    target = st_p["rmse"][-1]
    k_p = next(i for i, e in enumerate(st_p["rmse"]) if e <= target) + 1
    b16 = b_f32.half()
    hist_l, st_l = go(b16, "bf16", proposer, target, sr_seed=2024)
    k_l = len(hist_l)
    reached = st_l["rmse"][-1] <= target
    if "bf16_nearest" in variants:
        hist_n, st_n = go(b16, "bf16", proposer, target)
    if "f16" in variants:
        hist_h, st_h = go(b16, "f16", proposer, target, sr_seed=2024)
    if "f32" in variants:
        hist_f, st_f = go(b_f32, "f32", proposer, target)

    def summary(hist, st, k):
        h = hist[:k]
        return {"seconds": round(st["t"][k - 1], 4), "iterations": k, "rmse": st["rmse"][k - 1],
                "fp_calls_per_iter": round(float(np.mean([2 + it.backtracks for it in h])), 3),
                "backtracks_per_iter": round(float(np.mean([it.backtracks for it in h])), 3)}

    rec = {
        "rmse_target": target,
        "plain_f32": summary(hist_p, st_p, k_p),
        "learned_bf16": dict(summary(hist_l, st_l, k_l), reached=reached,
                             storage="BF16 volume (stochastic rounding), FP16 data"),
    }
    if "bf16_nearest" in variants:
        rec["learned_bf16_nearest"] = dict(summary(hist_n, st_n, len(hist_n)), reached=st_n["rmse"][-1] <= target)
    if "f16" in variants:
        rec["learned_f16"] = dict(summary(hist_h, st_h, len(hist_h)), reached=st_h["rmse"][-1] <= target,
                                  storage="FP16 volume (stochastic rounding), FP16 data")
    if "f32" in variants:
        rec["learned_f32"] = dict(summary(hist_f, st_f, len(hist_f)), reached=st_f["rmse"][-1] <= target)
    rec["speedup"] = round(st_p["t"][k_p - 1] / st_l["t"][k_l - 1], 3) if reached else None
    return rec


def combined_run(fbl, syn, name: str = "c5"):
    """The full combined run on one GPU: plain FP32 FB-LISA against the learned initial step
    with BF16 volume storage (stochastic rounding) and FP16 data, timed to the plain run's
    final RMSE; the same with FP16 volume storage for comparison.  The data are exact line integrals of the workload's ellipsoid phantom plus
    1% Gaussian noise, computed on the GPU (the host loop would take a quarter of an hour at
    1024^3); the phantom is voxelised at one sample per voxel."""
    import torch
    cfg = syn.CONFIGS[name]
    g = syn.config_geometry(name)
    B = cfg["batch"]
    seed = 1000 * int(name[1:])
    t0 = time.perf_counter()
    ells, xt = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"], sub=1)
    t_ph = time.perf_counter() - t0
    y = syn.ellipsoid_line_integrals_torch(g, ells, np.arange(g.n_views), device="cuda")
    syn.add_noise_torch(y, 0.01, seed=seed + 1)
    b32 = y.float()
    del y
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    t_data = time.perf_counter() - t0
    log("combined run %s: phantom %.1f s, data %.1f s" % (name, t_ph, t_data))
    model, n_samples, curve = train_step_proposer(fbl, syn)
    n_it = cfg["epochs"] * math.ceil(g.n_views / B)
    perms = syn.view_permutations(g.n_views, 2 * n_it, seed=seed + 2)
    # BF16 (the run's storage) and, for comparison, FP16 storage with the same proposer
    tt = time_to_rmse(fbl, g, cfg, b32, xt, perms, fbl.LearnedStep(model), variants=("bf16", "f16"))
    return {"mode": "combined run",
            "workload": "%s: %d^3 ellipsoid phantom (%d ellipsoids, voxelised at 1 sample per voxel), %d views, "
                        "%dx%d detector, mini-batch %d, %d epochs, prox [%g, %g], 1%% Gaussian noise on exact line "
                        "integrals" % (name, g.nx, cfg["k"], g.n_views, g.nu, g.nv, B, cfg["epochs"], cfg["lo"],
                                       cfg["hi"]),
            "setup_s": round(t_data, 1),
            "proposer": "5-64-64-1 perceptron trained on %d iterations of 200 seeded 64^3 runs" % n_samples,
            "time_to_rmse": tt}


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
    ap.add_argument("--config", default="c2", help="workload (c1..c4); the default is the metric's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-rmse", action="store_true",
                    help="skip the time-to-RMSE comparison (learned step + BF16 storage against plain FP32)")
    ap.add_argument("--probe", action="store_true",
                    help="counter-collection run: 3 forward, 1 backprojection, 1 step call of the workload, then "
                         "a plain 512 MiB device copy whose FETCH_SIZE/WRITE_SIZE calibrate the counters")
    ap.add_argument("--paper-run", type=float, default=0.0, metavar="SECONDS",
                    help="instead of the benchmark: the paper's growing-batch variant with mu > 0 on a 560^3 / "
                         "72-view synthetic stand-in, for this many seconds")
    ap.add_argument("--kernel-storage", default="f32", choices=("f32", "bf16", "f16"),
                    help="volume storage type for --kernels")
    ap.add_argument("--combined-run", default="", metavar="CONFIG",
                    help="instead of the benchmark: the full combined run (plain FP32 against learned step + BF16 "
                         "storage, time to the plain run's RMSE) at this workload, e.g. c5")
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
    if args.combined_run:
        print(json.dumps(combined_run(fbl, syn, args.combined_run)), flush=True)
        return 0
    if args.paper_run > 0:
        print(json.dumps(paper_shaped_run(fbl, syn, args.paper_run)), flush=True)
        return 0
    cfg = syn.CONFIGS[args.config]
    g = syn.config_geometry(args.config)
    B = cfg["batch"]
    seed = 1000 * int(args.config[1:])
    t_setup = time.perf_counter()
    ells, xt = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"])
    clean = syn.ellipsoid_line_integrals(g, ells, np.arange(g.n_views))
    b32 = syn.add_noise(clean, 0.01, seed=seed + 1).astype(np.float32)
    del clean
    perms = syn.view_permutations(g.n_views, args.warmup + args.steps + 3, seed=seed + 2)
    log("setup (phantom, exact line integrals, noise): %.1f s" % (time.perf_counter() - t_setup))

    b_dev = torch.from_numpy(b32).cuda()
    alpha0, beta = 1e-3, 0.5
    if args.probe:
        plan = fbl.Plan(g, max_batch=B)
        x = torch.from_numpy(xt.astype(np.float32)).cuda()
        views = perms[0][:B]
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        for _ in range(3):
            r = fbl.fb_lisa_forward(plan, x, views, b_dev, loss=loss)
        gr = fbl.fb_lisa_backproject(plan, r, views)
        fbl.fb_lisa_step(plan, x, gr, alpha0, 0.0, cfg["lo"], cfg["hi"])
        torch.cuda.synchronize()
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": args.config, "copy_bytes": src.numel() * 4,
                          "forward_bytes_model": B * (g.d * 4 + 4 * g.n_p)}), flush=True)
        return 0
    run = fbl.FBLisa(g, b_dev, n0=B, epochs=cfg["epochs"], alpha0=alpha0, beta=beta, lo=cfg["lo"], hi=cfg["hi"])
    warm_clock(fbl, run.plan, run.x, perms[0][:B], run.r[:B], run.g, args.clock_warmup)
    for k in range(args.warmup):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    # HIP events (on the launch stream) around the projector kernels' launches only: each
    # bracketed launch adds two event records to the stream, so timing every launch of an
    # iteration would slow the timed region itself
    run.plan.timing(True, kernels=("forward", "backproject"))
    n_hist = len(run.history)
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = run.plan.timing_read()
    run.plan.timing(False)
    timed = run.history[n_hist:]
    # a short supplementary pass with every launch bracketed gives the other kernels' means
    k0 = args.warmup + args.steps
    run.plan.timing(True)
    for k in range(k0, k0 + 3):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    ks = run.plan.timing_read()
    run.plan.timing(False)
    n_fp = kt["forward"][1]
    n_bp = kt["backproject"][1]
    updates = (n_fp + n_bp) * g.d * B
    wall = t1 - t0
    gups = updates / wall / 1e9
    kernel_us = {k: round(ms / n * 1e3, 2) for k, (ms, n) in ks.items() if n}
    kernel_us.update({k: round(kt[k][0] / kt[k][1] * 1e3, 2) for k in ("forward", "backproject")})
    t_fp = kt["forward"][0] / n_fp * 1e-3            # fp_kernel alone (timed region)
    t_bp = kt["backproject"][0] / n_bp * 1e-3        # bp_kernel alone (timed region)
    t_fin = ks["finalize"][0] / max(1, ks["finalize"][1]) * 1e-3
    n_fp_s = max(1, ks["forward"][1])
    t_fp_call = t_fp + ks["transpose"][0] / n_fp_s * 1e-3 + t_fin   # whole forward call
    t_bp_call = t_bp + ks["prescale"][0] / max(1, ks["backproject"][1]) * 1e-3
    t_st = ks["step"][0] / ks["step"][1] * 1e-3                # step_kernel alone

    # roofline of the dominant kernel (the projector kernel with the larger share of the
    # timed region): the per-view block model, each view reads the volume once and writes
    # (forward) or reads (backprojection) its n_p FP32 values
    bytes_view = B * (g.d * 4 + 4 * g.n_p)
    share = {"fp_kernel": kt["forward"][0], "bp_kernel": kt["backproject"][0]}
    dominant = max(share, key=share.get)
    t_dom = t_fp if dominant == "fp_kernel" else t_bp
    achieved = bytes_view / t_dom / 1e9
    other = "bp_kernel" if dominant == "fp_kernel" else "fp_kernel"
    t_other = t_bp if dominant == "fp_kernel" else t_fp

    rec = {
        "metric": METRIC,
        "value": round(gups, 3),
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %d^3 fp32 ellipsoid phantom (%d ellipsoids), %d views, %dx%d detector, "
                        "mini-batch %d, prox [%g, %g], 1%% Gaussian noise on exact line integrals"
                        % (args.config, g.nx, cfg["k"], g.n_views, g.nu, g.nv, B, cfg["lo"], cfg["hi"]),
            "global_batch": B,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dominant, args.config),
            "kernel": dominant,
            "bytes_per_launch": bytes_view,
            "share_of_timed_region": round(share[dominant] / (wall * 1e3), 4),
        },
        "roofline_other": {
            "kernel": other,
            "achieved": round(bytes_view / t_other / 1e9, 1),
            "frac": round(bytes_view / t_other / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(other, args.config),
            "share_of_timed_region": round(share[other] / (wall * 1e3), 4),
        },
        "kernel_us": kernel_us,
        "step_hbm": {"bytes_per_launch": 12 * g.d, "achieved": round(12 * g.d / t_st / 1e9, 1),
                     "frac": round(12 * g.d / t_st / 1e9 / HBM_PEAK_GBS, 4)},
        "per_call_ms": {"forward": round(t_fp_call * 1e3, 4), "backproject": round(t_bp_call * 1e3, 4),
                        "step": round(t_st * 1e3, 4)},
        "gups_per_op": {"forward": round(g.d * B / t_fp / 1e9, 2), "backproject": round(g.d * B / t_bp / 1e9, 2)},
        "calls": {"forward": n_fp, "backproject": n_bp, "step": sum(len(it.trials) for it in timed)},
        "mean_backtracks": float(np.mean([it.backtracks for it in timed])),
    }
    if not args.no_time_to_rmse:
        log("training the step proposer (200 plain runs of the 64^3 workload) ...")
        t_tr = time.perf_counter()
        model, n_samples, curve = train_step_proposer(fbl, syn)
        log("trained on %d samples in %.1f s (loss %.3e -> %.3e)" % (n_samples, time.perf_counter() - t_tr,
                                                                    curve[0], curve[-1]))
        n_it = cfg["epochs"] * math.ceil(g.n_views / B)
        # The iteration at which a run first reaches RMSE* moves by several iterations with
        # small changes of the trajectory (the error curve is flat there), so the comparison
        # is repeated over three view orders; each order's plain run sets its own RMSE*.
        runs = []
        for s_off in (2, 3, 4):
            perms_run = syn.view_permutations(g.n_views, 2 * n_it, seed=seed + s_off)
            runs.append(time_to_rmse(fbl, g, cfg, b32, xt, perms_run, fbl.LearnedStep(model)))
            log("time to RMSE, view order %d: speedup %s" % (s_off, runs[-1]["speedup"]))
        tt = runs[0]
        tt["proposer"] = "5-64-64-1 perceptron trained on %d iterations of 200 seeded 64^3 runs" % n_samples
        variants = ("learned_bf16", "learned_bf16_nearest", "learned_f16", "learned_f32")
        per_order = {v: [round(r["plain_f32"]["seconds"] / r[v]["seconds"], 3) if r[v].get("reached", True) else None
                         for r in runs] for v in variants}
        tt["view_orders"] = {"seeds": [seed + s for s in (2, 3, 4)], "speedup": per_order,
                             "median_speedup": {v: (float(np.median(x)) if all(y is not None for y in x) else None)
                                                for v, x in per_order.items()}}
        rec["time_to_rmse"] = tt
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(g, b32, perms, B, alpha0, beta, cfg["lo"], cfg["hi"])
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
