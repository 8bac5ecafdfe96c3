"""FB-LISA loop on the GPU against the FP64 oracle's run of Algorithm 1.

Replay: the GPU driver is forced to follow the oracle's accept/reject decisions, so the
two trajectories differ only by arithmetic; every iterate must stay within 1e-4
(relative l2) of the oracle's, and the GPU's own decision must equal the oracle's
wherever the oracle's sufficient-decrease margin exceeds 1e-4 relative (near-ties may
go either way: both outcomes are correct).  Free run: the GPU takes its own decisions.
"""
import math

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu


def _problem(n=32, det=48, views=24, seed=300, k=6):
    h = 64.0 / n
    du = 96.0 / det
    g = syn.Geometry(n, n, n, h, h, h, det, det, du, du, 500.0, 1000.0, views)
    ells, xt = syn.phantom(g, k, seed=seed)
    clean = syn.ellipsoid_line_integrals(g, ells, np.arange(views))
    b = syn.add_noise(clean, 0.01, seed=seed + 1).astype(np.float32)
    perms = syn.view_permutations(views, 200, seed=seed + 2)
    return g, xt, b, perms


def test_replay_and_free_run(orc):
    import torch
    import paper_2605_12085_amd as fbl
    g, xt, b32, perms = _problem()
    epochs, n0 = 2, 4
    xs_orc = []
    x_orc, rec = orc.fblisa(g, b32.astype(np.float64), epochs=epochs, n0=n0, perms=perms, alpha0=1e-3,
                            callback=lambda k, x, r: xs_orc.append(x.copy()))
    decisions = [[t.accepted for t in r.trials] for r in rec]
    assert sum(r.backtracks for r in rec) > 0          # the search is exercised
    bd = torch.from_numpy(b32).cuda()

    xs_gpu = []
    run = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, alpha0=1e-3)
    run.run(perms, decisions=decisions, callback=lambda s, it: xs_gpu.append(s.x.cpu().numpy().astype(np.float64)))
    assert len(xs_gpu) == len(xs_orc) == len(rec)
    for k, (xg, xo, ro, rg) in enumerate(zip(xs_gpu, xs_orc, rec, run.history)):
        assert np.linalg.norm(xg - xo) <= 1e-4 * np.linalg.norm(xo), k
        assert rg.f0 == pytest.approx(ro.f0, rel=1e-4), k
        assert rg.alpha == ro.alpha and rg.backtracks == ro.backtracks
        for tg, to in zip(rg.trials, ro.trials):
            rhs = ro.f0 + to.inner + to.sq / (2 * to.alpha)
            margin = abs(to.f_bar - rhs) / abs(rhs)
            own = tg.f_bar <= rg.f0 + tg.inner + tg.sq / (2 * tg.alpha)
            if margin > 1e-4:
                assert own == to.accepted, (k, margin)

    # free run: the GPU decides on its own values
    free = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, alpha0=1e-3)
    xf = free.run(perms).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(xf - x_orc) <= 1e-3 * np.linalg.norm(x_orc)
    hist_o = np.bincount([r.backtracks for r in rec], minlength=20)
    hist_g = np.bincount([r.backtracks for r in free.history], minlength=20)
    assert np.abs(hist_o - hist_g).sum() <= 2
    # the run reduces the error against the phantom
    assert orc.rmse(xf, xt) < orc.rmse(np.zeros_like(xt), xt)


def test_growth_schedule_with_l1_term_replay(orc):
    # the paper's own variant: the mini-batch grows by Step 1 (C = N_0 eps_{ceil(n/N_0)})
    # and R = mu ||x||_1 + nonnegativity with mu > 0; the GPU follows the oracle's
    # decisions and must keep its iterates within 1e-4 and use the same batch sizes
    import torch
    import paper_2605_12085_amd as fbl
    g, xt, b32, perms = _problem(seed=310)
    epochs, n0 = 4, 4
    C = orc.growth_C(g.n_views, n0)
    b64 = b32.astype(np.float64)
    # mu: a small fraction of the largest gradient entry at x = 0 (full batch)
    _, g0, _ = orc.objective_and_gradient(g, np.zeros(g.vol_shape), b64, np.arange(g.n_views))
    mu = 0.02 * float(np.abs(g0).max())
    xs_orc = []
    x_orc, rec = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms, mu=mu, C=C,
                            callback=lambda k, x, r: xs_orc.append(x.copy()))
    sizes = [len(r.batch) for r in rec]
    assert sizes[0] == n0 and max(sizes) > n0            # the batch grows
    assert all(a <= b for a, b in zip(sizes, sizes[1:]))  # and never shrinks
    assert np.mean(x_orc == 0.0) > 0.05                   # the l1 term zeroes voxels
    decisions = [[t.accepted for t in r.trials] for r in rec]
    bd = torch.from_numpy(b32).cuda()
    xs_gpu = []
    run = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, mu=mu, C=C)
    run.run(perms, decisions=decisions, callback=lambda s, it: xs_gpu.append(s.x.cpu().numpy().astype(np.float64)))
    assert [len(it.batch) for it in run.history] == sizes
    for k, (xg, xo) in enumerate(zip(xs_gpu, xs_orc)):
        assert np.linalg.norm(xg - xo) <= 1e-4 * np.linalg.norm(xo), k


def test_fixed_point_on_gpu(orc):
    # noise-free data of a nonnegative x_true with mu = 0: starting at x_true the
    # gradient is (numerically) zero and every iterate stays at x_true (appendix: a
    # stationary point is a fixed point of the prox-gradient map)
    import torch
    import paper_2605_12085_amd as fbl
    g = syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 30, 1.5, 1.5, 300.0, 600.0, 12)
    _, xt = syn.phantom(g, 4, seed=5)
    x32 = xt.astype(np.float32)
    b = orc.forward(g, x32.astype(np.float64), np.arange(g.n_views)).astype(np.float32)
    perms = syn.view_permutations(g.n_views, 20, seed=6)
    run = fbl.FBLisa(g, torch.from_numpy(b).cuda(), n0=3, epochs=1, x0=torch.from_numpy(x32).cuda())
    x = run.run(perms).cpu().numpy()
    # the FP32 data carries rounding noise, so the residual is tiny, not zero
    assert np.abs(x - x32).max() <= 1e-6 * x32.max()
