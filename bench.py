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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("forward.hip", "common.h", "device_util.h"):
        with open(os.path.join(ROOT, "paper_2605_12085_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(cfg: str, bytes_per_launch: float):
    """HBM bytes per forward launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "fp_kernel_%s_pmc.json" % cfg)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", help="workload (c1..c4); the default is the metric's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", action="store_true",
                    help="counter-collection run: 3 forward, 1 backprojection, 1 step call of the workload, then "
                         "a plain 512 MiB device copy whose FETCH_SIZE/WRITE_SIZE calibrate the counters")
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
    cfg = syn.CONFIGS[args.config]
    g = syn.config_geometry(args.config)
    B = cfg["batch"]
    seed = 1000 * int(args.config[1:])
    t_setup = time.perf_counter()
    ells, xt = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"])
    clean = syn.ellipsoid_line_integrals(g, ells, np.arange(g.n_views))
    b32 = syn.add_noise(clean, 0.01, seed=seed + 1).astype(np.float32)
    del clean
    perms = syn.view_permutations(g.n_views, args.warmup + args.steps, seed=seed + 2)
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
    for k in range(args.warmup):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    run.plan.timing(True)  # HIP events around every kernel launch, on the launch stream
    n_hist = len(run.history)
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        run.iterate(perms[k][:B])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = run.plan.timing_read()
    run.plan.timing(False)
    timed = run.history[n_hist:]
    n_fp = kt["forward"][1]
    n_bp = kt["backproject"][1]
    updates = (n_fp + n_bp) * g.d * B
    wall = t1 - t0
    gups = updates / wall / 1e9
    kernel_us = {k: round(ms / n * 1e3, 2) for k, (ms, n) in kt.items() if n}
    t_fp = kt["forward"][0] / n_fp * 1e-3            # fp_kernel alone
    t_bp = kt["backproject"][0] / n_bp * 1e-3        # bp_kernel alone
    t_fin = kt["finalize"][0] / max(1, kt["finalize"][1]) * 1e-3
    t_fp_call = (kt["forward"][0] + kt["transpose"][0]) / n_fp * 1e-3 + t_fin   # whole forward call
    t_bp_call = (kt["backproject"][0] + kt["prescale"][0]) / n_bp * 1e-3
    t_st = kt["step"][0] / kt["step"][1] * 1e-3                # step_kernel alone

    # roofline of the dominant kernel (forward projection): the per-view block model,
    # each view reads the volume once and writes its n_p FP32 values
    bytes_fp = B * (g.d * 4 + 4 * g.n_p)
    achieved = bytes_fp / t_fp / 1e9
    traffic = measured_traffic(args.config, bytes_fp)

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
            "traffic": traffic,
            "kernel": "fp_kernel (forward projection with residual and loss partials)",
            "bytes_per_launch": bytes_fp,
        },
        "kernel_us": kernel_us,
        "backproject_roofline": {"achieved": round(bytes_fp / t_bp / 1e9, 1), "frac": round(bytes_fp / t_bp / 1e9 /
                                                                                          HBM_PEAK_GBS, 4)},
        "step_hbm": {"bytes_per_launch": 12 * g.d, "achieved": round(12 * g.d / t_st / 1e9, 1),
                     "frac": round(12 * g.d / t_st / 1e9 / HBM_PEAK_GBS, 4)},
        "per_call_ms": {"forward": round(t_fp_call * 1e3, 4), "backproject": round(t_bp_call * 1e3, 4),
                        "step": round(t_st * 1e3, 4)},
        "gups_per_op": {"forward": round(g.d * B / t_fp / 1e9, 2), "backproject": round(g.d * B / t_bp / 1e9, 2)},
        "calls": {"forward": n_fp, "backproject": n_bp, "step": kt["step"][1]},
        "mean_backtracks": float(np.mean([it.backtracks for it in timed])),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(g, b32, perms, B, alpha0, beta, cfg["lo"], cfg["hi"])
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
