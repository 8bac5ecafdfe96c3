"""Learned initial step: the perceptron kernels against the FP64 oracle, and what the
trained proposer gains over the plain method.

Kernel parity (FP32 kernels, FP64 oracle): outputs and loss to 1e-5 relative, gradients
to 1e-5 of their largest entry (sums over samples are FP64 on both sides; the FP32
activations carry ~1e-7 relative error each), Adam updates to 1e-6 given the same
gradient.  Gain: the proposer is trained on traces of 200 seeded plain runs of the
64^3 / 60-view / 6-view-batch workload and evaluated on 20 held-out seeds and on the
128^3 / 180-view / 10-view-batch shape: fewer backtracks and forward projections per
iteration at an unchanged reconstruction error.
"""
import math
import time

import numpy as np
import pytest

import synthetic as syn
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fbl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2605_12085_amd as fbl
    return fbl


def _params(seed):
    p = syn.mlp_params(seed)
    p = p + np.random.default_rng(seed + 1).uniform(-0.05, 0.05, p.size).astype(np.float32)
    return p.astype(np.float32)


@pytest.mark.parametrize("n", [1, 37, 1000, 20000])
def test_mlp_kernels_match_oracle(fbl, n):
    import torch
    from paper_2605_12085_amd import _lib
    rng = np.random.default_rng(n)
    p = _params(3)
    X = rng.standard_normal((n, 5)).astype(np.float32)
    t = rng.normal(-0.5, 0.3, n).astype(np.float32)
    pd = torch.from_numpy(p).cuda()
    Xd = torch.from_numpy(X).cuda()
    td = torch.from_numpy(t).cuda()
    y = _lib.mlp_forward(pd, Xd).cpu().numpy().astype(np.float64)
    y_ref, _ = omlp.forward(p, X)
    assert np.abs(y - y_ref).max() <= 1e-5 * max(1.0, np.abs(y_ref).max())
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = _lib.mlp_workspace(n)
    g = _lib.mlp_loss_grad(pd, Xd, td, work, loss=loss).cpu().numpy().astype(np.float64)
    L_ref, g_ref = omlp.loss_and_grad(p, X, t)
    assert float(loss) == pytest.approx(2 * n * L_ref, rel=1e-5)
    assert np.abs(g - g_ref).max() <= 1e-5 * np.abs(g_ref).max()
    assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    # repeatable bit for bit
    g2 = _lib.mlp_loss_grad(pd, Xd, td, work).cpu().numpy().astype(np.float64)
    assert np.array_equal(g, g2)


def test_adam_matches_oracle(fbl):
    import torch
    from paper_2605_12085_amd import _lib
    rng = np.random.default_rng(5)
    p = _params(4)
    pd = torch.from_numpy(p).cuda()
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    pr, mr, vr = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for step in range(1, 4):
        gr = rng.standard_normal(p.size).astype(np.float32) * 10.0 ** rng.uniform(-4, 0, p.size).astype(np.float32)
        _lib.mlp_adam(pd, torch.from_numpy(gr).cuda(), m, v, step, 1e-3)
        pr, mr, vr = omlp.adam_step(pr, gr, mr, vr, step, 1e-3)
    got = pd.cpu().numpy().astype(np.float64)
    assert np.abs(got - pr).max() <= 1e-6 * max(1.0, np.abs(pr).max())
    # the moments mix gradients of either sign, so their error is relative to the largest
    # moment, not to each (possibly cancelled) entry
    assert np.abs(m.cpu().numpy() - mr).max() <= 1e-6 * np.abs(mr).max()
    assert np.abs(v.cpu().numpy() - vr).max() <= 1e-6 * np.abs(vr).max()


def test_mlp_host_checks(fbl):
    import torch
    from paper_2605_12085_amd import _lib
    pd = torch.zeros(_lib.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    ptr = pd.data_ptr()
    assert _lib.lib.fbl_mlp_forward(ptr, ptr, 0, ptr, None) == _lib.FBL_E_RANGE
    assert _lib.lib.fbl_mlp_forward(ptr, None, 4, ptr, None) == _lib.FBL_E_INVALID
    assert _lib.lib.fbl_mlp_loss_grad(ptr, ptr, ptr, 4, ptr, None, ptr + 16, None) == _lib.FBL_E_INVALID
    with pytest.raises(_lib.FblError) as e:
        _lib.mlp_adam(pd, pd, pd.clone(), pd.clone(), 0, 1e-3)
    assert e.value.code == _lib.FBL_E_RANGE


def _workload(name, rep):
    g = syn.config_geometry(name)
    cfg = syn.CONFIGS[name]
    seed = 1000 * int(name[1:]) + rep
    ells, xt = syn.phantom(g, cfg["k"], seed=seed, hi=cfg["hi"])
    b = syn.add_noise(syn.ellipsoid_line_integrals(g, ells, np.arange(g.n_views)), 0.01, seed=seed + 1)
    perms = syn.view_permutations(g.n_views, 1000, seed=seed + 2)
    return g, cfg, xt, b.astype(np.float32), perms


def _run(fbl, name, rep, proposer=None, recorder=None):
    import torch
    g, cfg, xt, b, perms = _workload(name, rep)
    run = fbl.FBLisa(g, torch.from_numpy(b).cuda(), n0=cfg["batch"], epochs=cfg["epochs"], lo=cfg["lo"],
                     hi=cfg["hi"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = run.run(perms, alpha_init=proposer, callback=recorder)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    x = x.cpu().numpy().astype(np.float64)
    bt = np.array([it.backtracks for it in run.history])
    rmse = math.sqrt(float(np.mean((x - xt) ** 2)))
    return dict(backtracks=bt.mean(), fp_per_iter=float(np.mean(2 + bt)), seconds=dt, rmse=rmse,
                iters=len(run.history))


def test_learned_step_gain(fbl, capsys):
    # training traces: 200 seeded plain runs of the 64^3 workload
    rec = fbl.TraceRecorder()
    for rep in range(200):
        _run(fbl, "c1", rep, recorder=rec)
    X, t = rec.arrays()
    assert X.shape == (200 * 99, 5)
    model = fbl.StepModel(syn.mlp_params(7))
    curve = model.fit(X, t, iters=2000, lr=3e-3)
    assert curve[-1] < 0.5 * curve[0]
    prop = fbl.LearnedStep(model)
    rows = {}
    for name, reps in (("c1", range(200, 220)), ("c4", range(2))):
        plain = [_run(fbl, name, r) for r in reps]
        learned = [_run(fbl, name, r, proposer=prop) for r in reps]
        rows[name] = (plain, learned)
    with capsys.disabled():
        print("\nlearned initial step (trained on %d samples; training loss %.3e -> %.3e):"
              % (len(t), curve[0], curve[-1]))
        for name, (plain, learned) in rows.items():
            for label, runs in (("plain", plain), ("learned", learned)):
                print("  %s %-7s: backtracks/iter %.2f  FP calls/iter %.2f  time %.3f s  RMSE %.4e  (%d runs)"
                      % (name, label, np.mean([r["backtracks"] for r in runs]),
                         np.mean([r["fp_per_iter"] for r in runs]), np.median([r["seconds"] for r in runs]),
                         np.median([r["rmse"] for r in runs]), len(runs)), flush=True)
    for name, (plain, learned) in rows.items():
        bp = np.mean([r["backtracks"] for r in plain])
        bl = np.mean([r["backtracks"] for r in learned])
        fp = np.mean([r["fp_per_iter"] for r in plain])
        fl = np.mean([r["fp_per_iter"] for r in learned])
        # The proposal is the predicted halving count rounded down, so even an exact
        # predictor may leave one rejected trial per iteration: the floor of the method is
        # up to one backtrack, i.e. 3 forward calls per iteration against the plain run's
        # 2 + bp.  The bars: at most one backtrack per iteration, at most half the plain
        # run's backtracks, and (what the first implies at these plain counts) at most
        # four fifths of its forward projections, with no loss of accuracy.
        assert bl <= 1.0, (name, bl)
        assert bl <= 0.5 * bp, (name, bl, bp)
        assert fl <= 0.8 * fp, (name, fl, fp)
        for p_, l_ in zip(plain, learned):
            assert l_["rmse"] <= 1.02 * p_["rmse"], (name, l_["rmse"], p_["rmse"])
