"""Pins of the oracle's storage rounding (precision form: x stored in BF16/FP16).

round_bf16 is written from the definition of the format (8 significant bits, FP32
exponent range, nearest-even); it is pinned by hand-computed ties, by torch's own
bfloat16 conversion on inputs that are exact in FP32 (where that conversion is a single
rounding), by the half-ulp error bound and by idempotence.  FP16 uses numpy's IEEE
conversion; hand cases pin the storage dispatch.
"""
import math

import numpy as np
import pytest


def test_bf16_hand_ties(orc):
    one = 1.0
    cases = [
        (one + 2.0 ** -8, one),                          # tie between 1 and 1+2^-7: even (1)
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),          # tie between 1+2^-7 and 1+2^-6: even
        (-(one + 2.0 ** -8), -one),
        (one + 2.0 ** -8 + 2.0 ** -40, one + 2.0 ** -7),  # just above a tie (lost if FP32 came first)
        (one + 2.0 ** -8 - 2.0 ** -40, one),
        (255.0 + 0.5, 256.0),                            # 255.5: quantum 1 at [128, 256) -> tie -> 256
        (3.0 * 2.0 ** -130, 3.0 * 2.0 ** -130),          # below 2^-126: quantum 2^-133, exact
        (2.0 ** -134, 0.0),                              # half the smallest subnormal: tie to even 0
        (3.0 * 2.0 ** -134, 2.0 ** -132),                # 1.5 quanta: tie to even (2 quanta)
        (3.39e38, float(np.ldexp(1.0, 128) - np.ldexp(1.0, 120))),   # largest finite bfloat16
        (3.4e38, math.inf),                              # beyond max + half a quantum
        (0.0, 0.0),
    ]
    got = orc.round_bf16(np.array([c[0] for c in cases]))
    for (v, want), r in zip(cases, got):
        assert r == want, (v, r, want)
    assert np.isinf(orc.round_bf16(np.array([2.0 ** 128 * (1 - 2.0 ** -9)]))[0])  # rounds past the max
    assert math.copysign(1.0, orc.round_bf16(np.array([-0.0]))[0]) == -1.0


def test_bf16_matches_torch_on_fp32_inputs(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * 10.0 ** rng.integers(-30, 30, 200000)).astype(np.float32)
    x = np.concatenate([x, rng.uniform(0, 0.03, 100000).astype(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(orc.round_bf16(x.astype(np.float64)), ref)


def test_bf16_error_bound_and_idempotence(orc):
    rng = np.random.default_rng(1)
    v = rng.uniform(-1, 1, 100000) * 10.0 ** rng.uniform(-20, 20, 100000)
    r = orc.round_bf16(v)
    assert np.all(np.abs(r - v) <= 2.0 ** -8 * np.abs(v) * (1 + 1e-15))   # unit roundoff 2^-p, p = 8
    assert np.array_equal(orc.round_bf16(r), r)
    # monotone
    s = np.sort(v)
    assert np.all(np.diff(orc.round_bf16(s)) >= 0)


def test_storage_dispatch(orc):
    v = np.array([2049.0, 2051.0, 1.0 + 2.0 ** -11, 65520.0, 0.1])
    f16 = orc.round_storage(v, "f16")
    assert list(f16[:3]) == [2048.0, 2052.0, 1.0]
    assert np.isinf(f16[3])
    assert orc.round_storage(v, "f32")[4] == float(np.float32(0.1))
    assert orc.round_storage(v, "bf16")[4] == 0.10009765625
    assert np.array_equal(orc.round_storage(v, None), v)


def test_prox_step_with_storage(orc):
    rng = np.random.default_rng(2)
    x = orc.round_bf16(rng.uniform(0, 0.03, 5000))
    grad = rng.standard_normal(5000)
    for st in ("bf16", "f16"):
        xb, inner, sq, gg = orc.prox_step(x, grad, 1e-3, 0.5, 0.0, 0.03, storage=st)
        assert np.array_equal(orc.round_storage(xb, st), xb)
        d = xb - x
        assert inner == pytest.approx(float(grad @ d), rel=1e-13)
        assert sq == pytest.approx(float(d @ d), rel=1e-13)
        exact = np.clip(x - 1e-3 * grad - 1e-3 * 0.5, 0.0, 0.03)
        ulp = 2.0 ** -8 if st == "bf16" else 2.0 ** -11   # unit roundoff
        assert np.all(np.abs(xb - exact) <= ulp * np.abs(exact) + 2.0 ** -24)


def test_splitmix64_published_outputs(orc):
    # the first outputs of SplitMix64 seeded with 0, as published with the generator
    z = orc.splitmix64(0, [0, 1, 2])
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # a stream continues across counters: output c+1 of seed k equals output c of seed k + gamma
    assert int(orc.splitmix64(5, [7])[0]) == int(orc.splitmix64(5 + 0x9E3779B97F4A7C15, [6])[0])


def test_stochastic_rounding_probability_and_bias(orc):
    n = 200000
    for st, q in (("bf16", 2.0 ** -7), ("f16", 2.0 ** -10), ("f32", 2.0 ** -23)):
        for frac in (0.25, 0.5, 0.9):
            v = np.full(n, 1.0 + frac * q)
            r = orc.round_stochastic(v, st, key=77)
            assert set(np.unique(r)) <= {1.0, 1.0 + q}
            up = np.mean(r > 1.0)
            assert abs(up - frac) < 5 * math.sqrt(frac * (1 - frac) / n), (st, frac, up)
    # unbiased on average over keys, and exact where representable
    rng = np.random.default_rng(3)
    v = rng.uniform(0.001, 0.03, 1000)
    mean = np.mean([orc.round_stochastic(v, "bf16", key=k) for k in range(400)], axis=0)
    q = np.ldexp(1.0, np.frexp(v)[1] - 8)
    assert np.all(np.abs(mean - v) < 5 * 0.5 * q / math.sqrt(400))
    rep = orc.round_bf16(v)
    assert np.array_equal(orc.round_stochastic(rep, "bf16", key=9), rep)
    # the result is one of the two neighbours and depends only on (value, key, index)
    r1 = orc.round_stochastic(v, "bf16", key=11)
    assert np.array_equal(r1, orc.round_stochastic(v, "bf16", key=11))
    assert not np.array_equal(r1, orc.round_stochastic(v, "bf16", key=12))
    lo = np.floor(v / q) * q
    assert np.all((r1 == lo) | (r1 == lo + q))


def test_stochastic_rounding_subnormal_quantum(orc):
    # below the smallest normal FP16 number 2^-14 the quantum stays 2^-24
    v = np.full(100000, 3.25 * 2.0 ** -24)
    r = orc.round_stochastic(v, "f16", key=5)
    assert set(np.unique(r)) == {3.0 * 2.0 ** -24, 4.0 * 2.0 ** -24}
    assert abs(np.mean(r == 4.0 * 2.0 ** -24) - 0.25) < 0.01


def test_mixed_form_by_explicit_matrix(orc):
    """The mixed form of the loop (FP32 iterates, objective and gradient at their 16-bit
    copies), checked step by step against the explicit 4^3 matrix: every recorded f(x_k)
    equals n/(2B) ||A_S bf16(x_k) - b_S||^2 and every accepted iterate equals the FP32
    rounding of clip(x_k - alpha_k n/B A_S^T (A_S bf16(x_k) - b_S))."""
    import synthetic as syn
    g = syn.tiny_geometry(n=4, det=12, views=16, du=0.8)
    A = orc.assemble_matrix(g, np.arange(g.n_views))
    rng = np.random.default_rng(5)
    xt = rng.uniform(0.0, 0.02, g.d)
    b = (A @ xt + 1e-4 * rng.standard_normal(A.shape[0])).reshape(g.n_views, g.nv, g.nu)
    perms = np.array([rng.permutation(g.n_views) for _ in range(40)])
    xs = [np.zeros(g.d)]
    _, rec = orc.fblisa(g, b, epochs=3, n0=4, perms=perms, copy_storage="bf16",
                        callback=lambda k, x, r: xs.append(x.ravel().copy()))
    rows = lambda v: np.concatenate([np.arange(i * g.n_p, (i + 1) * g.n_p) for i in v])
    rounded_somewhere = False
    for k, r in enumerate(rec):
        x = xs[k]
        xc = orc.round_bf16(x)
        rounded_somewhere |= not np.array_equal(xc, x)
        R = rows(r.batch)
        res = A[R] @ xc - b.ravel()[R]
        nb = len(r.batch)
        assert r.f0 == pytest.approx(g.n_views / (2.0 * nb) * float(res @ res), rel=1e-12)
        grad = g.n_views / nb * (A[R].T @ res)
        want = np.clip(x - r.alpha * grad, 0.0, np.inf).astype(np.float32).astype(np.float64)
        ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(xs[k + 1] - want) <= ulp)
        assert np.array_equal(xs[k + 1].astype(np.float32).astype(np.float64), xs[k + 1])
    assert rounded_somewhere
