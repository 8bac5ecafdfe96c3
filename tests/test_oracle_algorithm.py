"""Pins of the oracle's FB-LISA pieces: objective reading, gradient, prox, line
search, Step 1 schedule and the whole loop, against closed forms, brute force,
library solvers and the paper's Lemma (appendix)."""
import math
import os

import numpy as np
import pytest
import scipy.optimize as so

import synthetic as syn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_problem(seed=0, noise=0.01, zero_frac=0.3):
    """4^3 volume, 16 views of 12x12: every voxel seen, A well conditioned (cond ~ 6)."""
    import oracle as orc
    g = syn.tiny_geometry(n=4, det=12, views=16, du=0.8)
    views = np.arange(g.n_views)
    A = orc.assemble_matrix(g, views)
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0.0, 0.02, g.d)
    xt[rng.random(g.d) < zero_frac] = 0.0
    y = A @ xt
    b = y + noise * np.linalg.norm(y) / math.sqrt(y.size) * rng.standard_normal(y.size)
    return g, A, xt, b


def test_full_batch_objective_is_half_least_squares(orc):
    # Reading of (2.4)/(2.5): with the batch equal to all n_theta views, f_N equals the
    # data term 1/2 ||Ax - b||^2 of (2.1).
    g, A, xt, b = _small_problem()
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 0.02, g.d)
    bf = b.reshape(g.n_views, g.nv, g.nu)
    f = orc.objective(g, x.reshape(g.vol_shape), bf, np.arange(g.n_views))
    ref = 0.5 * float(np.sum((A @ x - b) ** 2))
    assert f == pytest.approx(ref, rel=1e-13)
    # a permuted full batch gives the same value
    f2 = orc.objective(g, x.reshape(g.vol_shape), bf, rng.permutation(g.n_views))
    assert f2 == pytest.approx(ref, rel=1e-13)


def test_minibatch_objective_is_unbiased_average(orc):
    # f_N averages the per-angle terms f_i = n_theta/2 ||A_i x - b_i||^2: the mean of
    # f_N over all batches of size 1 is the full objective.
    g, A, xt, b = _small_problem()
    x = np.full(g.d, 0.01)
    bf = b.reshape(g.n_views, g.nv, g.nu)
    vals = [orc.objective(g, x.reshape(g.vol_shape), bf, [i]) for i in range(g.n_views)]
    ref = 0.5 * float(np.sum((A @ x - b) ** 2))
    assert np.mean(vals) == pytest.approx(ref, rel=1e-13)
    # explicit row block of one view
    i = 5
    Ai = A[i * g.n_p:(i + 1) * g.n_p]
    bi = b[i * g.n_p:(i + 1) * g.n_p]
    assert vals[i] == pytest.approx(g.n_views / 2.0 * float(np.sum((Ai @ x - bi) ** 2)), rel=1e-13)


def test_gradient_central_differences(orc):
    # f_N is quadratic, so the central difference is exact up to rounding for any eps.
    g = syn.Geometry(9, 8, 7, 1.0, 1.0, 1.0, 14, 12, 1.5, 1.5, 300.0, 600.0, 12)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 0.02, g.vol_shape)
    bf = rng.standard_normal((g.n_views, g.nv, g.nu)) * 0.1
    views = np.array([3, 7, 11])
    f0, grad, _ = orc.objective_and_gradient(g, x, bf, views)
    for k in range(4):
        v = rng.standard_normal(g.vol_shape)
        eps = 1e-3
        fp = orc.objective(g, x + eps * v, bf, views)
        fm = orc.objective(g, x - eps * v, bf, views)
        fd = (fp - fm) / (2 * eps)
        assert fd == pytest.approx(float(np.sum(grad * v)), rel=1e-9, abs=1e-12)


def test_gradient_matches_explicit_matrix(orc):
    g, A, xt, b = _small_problem()
    x = np.full(g.d, 0.005)
    views = np.array([2, 9, 13])
    rows = np.concatenate([np.arange(v * g.n_p, (v + 1) * g.n_p) for v in views])
    AN, bN = A[rows], b[rows]
    ref = g.n_views / len(views) * AN.T @ (AN @ x - bN)
    _, grad, _ = orc.objective_and_gradient(g, x.reshape(g.vol_shape), b.reshape(g.n_views, g.nv, g.nu), views)
    assert np.allclose(grad.ravel(), ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def _golden_min(fun, a, b, iters=200):
    gr = (math.sqrt(5) - 1) / 2
    c, d = b - gr * (b - a), a + gr * (b - a)
    for _ in range(iters):
        if fun(c) < fun(d):
            b = d
        else:
            a = c
        c, d = b - gr * (b - a), a + gr * (b - a)
    return 0.5 * (a + b)


def test_prox_brute_force(orc):
    # prox_{alpha R}(v) minimises (z - v)^2/(2 alpha) + mu |z| over [lo, hi].
    rng = np.random.default_rng(4)
    for _ in range(200):
        v = float(rng.uniform(-0.05, 0.08))
        alpha = float(10 ** rng.uniform(-4, 0))
        mu = float(rng.choice([0.0, 0.01, 0.5, 2.0]))
        lo = float(rng.choice([0.0, 0.0, 0.004]))
        hi = float(rng.choice([math.inf, 0.03]))
        top = hi if math.isfinite(hi) else 1.0
        obj = lambda z: (z - v) ** 2 / (2 * alpha) + mu * abs(z)
        z = _golden_min(obj, lo, top)
        got = float(orc.prox(np.array([v]), alpha, mu, lo, hi)[0])
        # golden section locates a quadratic's minimiser only to ~sqrt(eps): compare
        # objective values (the prox may not be worse) and the location loosely
        assert lo <= got <= hi
        assert obj(got) <= obj(z) + 1e-15 * max(1.0, abs(obj(z)))
        assert got == pytest.approx(z, abs=1e-7)


def test_line_search_lemma(orc):
    # Appendix Lemma: any alpha <= 1/L satisfies (2.3), so alpha_0 <= 1/L_N gives no
    # backtracking; starting above, the accepted step satisfies alpha > beta/L_N.
    g = syn.tiny_geometry(n=6, det=10, views=12)
    rng = np.random.default_rng(3)
    bf = rng.uniform(0, 0.5, (g.n_views, g.nv, g.nu))
    views = np.array([1, 4, 8])
    x = rng.uniform(0, 0.02, g.vol_shape)
    L = orc.power_iteration_L(g, views, iters=300)
    f0, grad, _ = orc.objective_and_gradient(g, x, bf, views)
    fun = lambda z: orc.objective(g, z, bf, views)
    for mu, hi in ((0.0, math.inf), (0.05, 0.03)):
        alpha, _, _, trials = orc.line_search(fun, x, f0, grad, 0.999 / L, 0.5, mu, 0.0, hi)
        assert len(trials) == 1 and alpha == 0.999 / L
        backtracked = 0
        for a0 in (1e-3, 1.0, 37.0):
            alpha, xbar, f_bar, trials = orc.line_search(fun, x, f0, grad, a0, 0.5, mu, 0.0, hi)
            # a step reached by backtracking exceeds beta/L; a first guess is kept as is
            assert alpha > 0.5 / L if len(trials) > 1 else alpha == a0
            t = trials[-1]
            assert t.accepted and orc.sufficient_decrease(t.f_bar, f0, t.inner, t.sq, alpha)
            for rej in trials[:-1]:
                assert not rej.accepted and rej.alpha > 1.0 / L
            backtracked += len(trials) > 1
        assert backtracked >= 2


def test_step1_schedules_golden(orc):
    path = os.path.join(GOLDEN, "step1_schedules.txt")
    n_cases = 0
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, seq = line.split(":")
        kind, n, n0, T = head.split()
        n, n0, T = int(n), int(n0), int(T)
        expect = [int(s) for s in seq.split()]
        C = orc.growth_C(n, n0) if kind == "growth" else orc.fixed_batch_C(n, n0, T)
        assert orc.schedule(n, n0, T, C) == expect, line
        n_cases += 1
    assert n_cases == 4


def _full_batch_run(orc, g, b, iters, **kw):
    perms = np.tile(np.arange(g.n_views, dtype=np.int32), (iters + 5, 1))
    x, rec = orc.fblisa(g, b.reshape(g.n_views, g.nv, g.nu), epochs=iters, n0=g.n_views, perms=perms, **kw)
    return x.ravel(), rec


def test_full_batch_converges_to_nnls(orc):
    # With the whole data set as the batch, mu = 0 and the nonnegative orthant the
    # problem is nonnegative least squares; FB-LISA must converge to its solution.
    g, A, xt, b = _small_problem(seed=0)
    xs, _ = so.nnls(A, b, maxiter=10000)
    assert (xs == 0).sum() > 3  # some constraints active
    x, rec = _full_batch_run(orc, g, b, 400, alpha0=1.0)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6


def test_full_batch_converges_to_box_lsq(orc):
    g, A, xt, b = _small_problem(seed=1, noise=0.05)
    b = b * 1.6  # push some voxels above the box
    res = so.lsq_linear(A, b, bounds=(0.0, 0.03), tol=1e-14, method="bvls")
    xs = res.x
    assert (xs >= 0.03 - 1e-12).sum() > 0
    x, rec = _full_batch_run(orc, g, b, 400, alpha0=1.0, hi=0.03)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6


def test_full_batch_converges_to_l1_problem(orc):
    # mu > 0 with the nonnegative orthant (problem (2.1)); on x >= 0 the l1 term is
    # mu * 1^T x, so L-BFGS-B with bounds solves the same problem.
    g, A, xt, b = _small_problem(seed=2)
    mu = 0.05
    fun = lambda x: (0.5 * np.sum((A @ x - b) ** 2) + mu * np.sum(x), A.T @ (A @ x - b) + mu)
    res = so.minimize(fun, np.zeros(g.d), jac=True, method="L-BFGS-B", bounds=[(0, None)] * g.d,
                      options=dict(ftol=1e-16, gtol=1e-13, maxiter=20000, maxcor=50))
    xs = res.x
    x, rec = _full_batch_run(orc, g, b, 400, alpha0=1.0, mu=mu)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6


def test_fixed_point_of_noise_free_data(orc):
    # Noise-free b = A x_true with x_true >= 0 and mu = 0: x_true is a fixed point of
    # the prox-gradient map, so every iterate stays x_true and each trial is accepted
    # at alpha_0 (equality in (2.3)).
    g = syn.tiny_geometry(n=6, det=10, views=12)
    rng = np.random.default_rng(8)
    xt = rng.uniform(0, 0.02, g.vol_shape)
    b = orc.forward(g, xt, np.arange(g.n_views))
    perms = syn.view_permutations(g.n_views, 20, seed=3)
    x, rec = orc.fblisa(g, b, epochs=2, n0=3, x0=xt, perms=perms)
    assert np.array_equal(x, xt)
    assert all(r.backtracks == 0 and r.alpha == 1e-3 for r in rec)


def test_forward_backward_special_case_monotone(orc):
    # Full batch with alpha_0 <= 1/L never backtracks: the method is the plain
    # forward-backward iteration with fixed step, and F is non-increasing.
    g, A, xt, b = _small_problem(seed=4)
    L = float(np.linalg.eigvalsh(A.T @ A).max())
    mu = 0.01
    F = []
    perms = np.tile(np.arange(g.n_views, dtype=np.int32), (60, 1))
    bf = b.reshape(g.n_views, g.nv, g.nu)

    def cb(k, x, r):
        F.append(0.5 * float(np.sum((A @ x.ravel() - b) ** 2)) + mu * float(np.abs(x).sum()))

    x, rec = orc.fblisa(g, bf, epochs=50, n0=g.n_views, perms=perms, alpha0=0.99 / L, mu=mu, callback=cb)
    assert all(r.backtracks == 0 for r in rec)
    assert all(F[i + 1] <= F[i] * (1 + 1e-15) for i in range(len(F) - 1))


def test_minibatch_run_counts_and_replay(orc):
    # Epoch bookkeeping: fixed-batch C gives T * ceil(n/N_0) iterations; replaying the
    # recorded accept/reject decisions reproduces the run exactly.
    g = syn.tiny_geometry(n=6, det=10, views=12)
    rng = np.random.default_rng(9)
    xt = rng.uniform(0, 0.02, g.vol_shape)
    b = syn.add_noise(orc.forward(g, xt, np.arange(g.n_views)), 0.01, seed=1)
    perms = syn.view_permutations(g.n_views, 40, seed=2)
    x1, rec1 = orc.fblisa(g, b, epochs=3, n0=5, perms=perms, alpha0=1.0)
    assert len(rec1) == 3 * math.ceil(12 / 5)
    assert all(len(r.batch) == 5 and len(set(r.batch.tolist())) == 5 for r in rec1)
    decisions = [[t.accepted for t in r.trials] for r in rec1]
    x2, rec2 = orc.fblisa(g, b, epochs=3, n0=5, perms=perms, alpha0=1.0, decisions=decisions)
    assert np.array_equal(x1, x2)


def test_sufficient_decrease_threshold_is_exact(orc):
    # Away from the constraints, xbar - x = -alpha g and f_N is quadratic with
    # Hessian H = n_theta/|N| A_N^T A_N, so (2.3) holds iff
    # alpha <= g^T g / (g^T H g).  Just below that step the first trial is accepted,
    # just above it is rejected.
    g = syn.tiny_geometry(n=6, det=10, views=12)
    rng = np.random.default_rng(12)
    views = np.array([0, 5, 7])
    x = np.ones(g.vol_shape)                      # interior: no clipping at small steps
    bf = rng.uniform(0, 20.0, (g.n_views, g.nv, g.nu))
    f0, grad, _ = orc.objective_and_gradient(g, x, bf, views)
    Hg = orc.forward(g, grad, views)
    a_star = float(np.sum(grad * grad)) / (g.n_views / len(views) * float(np.sum(Hg * Hg)))
    assert np.all(x - 1.01 * a_star * grad > 0)
    fun = lambda z: orc.objective(g, z, bf, views)
    a_ok, _, _, t_ok = orc.line_search(fun, x, f0, grad, 0.99 * a_star, 0.5, 0.0, 0.0, math.inf)
    assert len(t_ok) == 1
    a_bad, _, _, t_bad = orc.line_search(fun, x, f0, grad, 1.01 * a_star, 0.5, 0.0, 0.0, math.inf)
    assert len(t_bad) == 2 and not t_bad[0].accepted and a_bad == 0.5 * 1.01 * a_star
