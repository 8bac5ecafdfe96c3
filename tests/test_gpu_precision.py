"""Precision form: volume and data stored in BF16 or FP16, ray sums in FP32, the loss and
the line-search inner products in FP64 (HIP kernels through the C ABI).

Parity with the oracle is taken on the stored values: the oracle receives exactly the
16-bit numbers the GPU reads (rounded by its own round_storage), so the 1e-5 bar of the
FP32 path applies unchanged.  The error of storage itself is stated against FP64:
for a nonnegative volume every ray weight is nonnegative, so rounding each voxel with
relative error <= u gives a ray-sum error <= u * (ray sum); the bound per view is the
unit roundoff u (2^-8 BF16, 2^-11 FP16) plus the FP32 arithmetic.
"""
import math

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

TOL = 1e-5
U = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def fbl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2605_12085_amd as fbl
    return fbl


def _torch_dtype(st):
    import torch
    return {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[st]


def _dev(a64, st):
    """Device tensor holding exactly the FP64 values a64 (already representable in st)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a64.astype(np.float32))).to(_torch_dtype(st))
    assert np.array_equal(t.to(torch.float64).numpy(), a64)
    return t.cuda()


# 33,752,070 voxels: above 2^25, so the prox trial takes its one-pass kernels and a
# second reduction level; two voxels after the last group of four
LARGE = syn.Geometry(331, 330, 309, 0.1, 0.1, 0.1, 64, 64, 0.15, 0.15, 500.0, 1000.0, 4)

ODD = syn.Geometry(29, 41, 37, 0.9, 1.1, 1.0, 50, 33, 1.7, 1.9, 400.0, 900.0, 12,
                   angles=[0.0, np.pi / 4, np.pi / 2, np.pi, 3 * np.pi / 2, 0.3, 1.7, 2.9, 4.0, 5.5, 0.05, 6.2])


def _rel_views(got, ref):
    out = []
    for b in range(ref.shape[0]):
        out.append(np.linalg.norm(got[b] - ref[b]) / np.linalg.norm(ref[b]))
    return np.array(out)


@pytest.mark.parametrize("vol,proj", [("bf16", "f32"), ("f16", "f32"), ("f32", "f16"), ("f32", "bf16"),
                                      ("bf16", "bf16"), ("f16", "f16")])
def test_forward_parity_on_stored_values(fbl, orc, vol, proj):
    import torch
    g = ODD
    rng = np.random.default_rng(21)
    xs = orc.round_storage(rng.uniform(0, 0.03, g.vol_shape), vol)
    views = np.arange(g.n_views, dtype=np.int32)
    y64 = orc.forward(g, xs, views)
    bs = orc.round_storage(0.5 * y64 * rng.uniform(0.5, 1.5, y64.shape), proj)
    r_ref = y64 - bs
    f_ref = g.n_views / (2.0 * len(views)) * float(np.sum(r_ref ** 2))
    with fbl.Plan(g, vol_dtype=vol, proj_dtype=proj) as plan:
        x = _dev(xs, vol)
        b = _dev(bs, proj)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        y = fbl.fb_lisa_forward(plan, x, views).cpu().numpy().astype(np.float64)
        r = fbl.fb_lisa_forward(plan, x, views, b, loss=loss).cpu().numpy().astype(np.float64)
        f = float(loss)
    for got, ref, what in ((y, y64, "forward"), (r, r_ref, "residual")):
        rel = _rel_views(got, ref)
        mx = np.array([np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(len(views))])
        assert rel.max() <= TOL and mx.max() <= TOL, (what, vol, proj, rel.max(), mx.max())
    assert f == pytest.approx(f_ref, rel=TOL)


def _storage_ulp(v, st):
    m, e = np.frexp(np.abs(v))
    p = {"f32": 24, "bf16": 8, "f16": 11}[st]
    emin = {"f32": -125, "bf16": -125, "f16": -13}[st]
    return np.ldexp(1.0, np.maximum(e, emin) - p)


@pytest.mark.parametrize("st", ["bf16", "f16"])
@pytest.mark.parametrize("shape", ["odd", "128", "large"])
def test_step_16bit_rounds_once_like_the_oracle(fbl, orc, st, shape):
    # "odd": 43,993 voxels (a tail of one after the four-voxel passes), three settings;
    # "128": 128^3, where each thread makes several grid-stride passes of four voxels;
    # "large": above 2^25 voxels, the one-pass kernel
    import torch
    g = {"odd": ODD, "128": syn.config_geometry("c4"), "large": LARGE}[shape]
    print("case step 16-bit %s %s (%d voxels)" % (st, shape, g.d), flush=True)
    settings = ((1e-3, 0.0, 0.0, math.inf), (2.5e-3, 0.7, 0.0, 0.03), (1e-4, 2.0, 0.001, 0.025))
    if shape != "odd":
        settings = settings[1:2]
    rng = np.random.default_rng(22)
    xs = orc.round_storage(rng.uniform(0, 0.03, g.vol_shape), st)
    xs[rng.random(g.vol_shape) < 0.2] = 0.0
    grad = (rng.standard_normal(g.vol_shape) * 3.0).astype(np.float32)
    with fbl.Plan(g, vol_dtype=st) as plan:
        for alpha, mu, lo, hi in settings:
            red = torch.zeros(3, dtype=torch.float64, device="cuda")
            xb, red = fbl.fb_lisa_step(plan, _dev(xs, st), torch.from_numpy(grad).cuda(), alpha, mu, lo, hi,
                                       red=red)
            xb = xb.to(torch.float64).cpu().numpy()
            red = red.cpu().numpy()
            xr, inner, sq, gg = orc.prox_step(xs, grad, alpha, mu, lo, hi, storage=st)
            assert np.all(np.abs(xb - xr) <= _storage_ulp(xr, st))
            assert np.mean(xb == xr) > 0.999
            assert red[0] == pytest.approx(inner, rel=1e-9)
            assert red[1] == pytest.approx(sq, rel=1e-9)
            assert red[2] == pytest.approx(gg, rel=1e-12)


def test_precision_report_512_sampled_rays(fbl, orc, capsys):
    """Per-view relative error against the FP64 oracle on the FP64 phantom, on 1% of the
    rays of every view, for FP32, BF16 and FP16 volume storage: 512^3 volume, 720 views,
    768x768 detector, batches of 40 views.  Storage rounding is counted."""
    import torch
    name = "c3"
    g = syn.config_geometry(name)
    cfg = syn.CONFIGS[name]
    _, x64 = syn.phantom(g, cfg["k"], seed=3000, hi=cfg["hi"], sub=2)
    rng = np.random.default_rng(3002)
    n_s = g.n_p // 100
    pix = np.stack([np.sort(rng.choice(g.n_p, n_s, replace=False)) for _ in range(g.n_views)])
    rays = np.stack([np.repeat(np.arange(g.n_views), n_s), (pix // g.nu).ravel(), (pix % g.nu).ravel()], axis=1)
    ref = orc.forward_rays(g, x64, rays).reshape(g.n_views, n_s)
    B = cfg["batch"]
    report = {}
    for st in ("f32", "bf16", "f16"):
        xs = torch.from_numpy(x64.astype(np.float32)).to(_torch_dtype(st)).cuda()
        got = np.empty((g.n_views, n_s))
        with fbl.Plan(g, vol_dtype=st, max_batch=B) as plan:
            for v0 in range(0, g.n_views, B):
                vs = np.arange(v0, v0 + B, dtype=np.int32)
                y = fbl.fb_lisa_forward(plan, xs, vs).view(B, -1)
                idx = torch.from_numpy(pix[v0:v0 + B]).cuda()
                got[v0:v0 + B] = torch.gather(y, 1, idx).cpu().numpy()
        del xs
        torch.cuda.empty_cache()
        rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
        report[st] = rel
    with capsys.disabled():
        print("\nper-view relative error vs FP64 (512^3, 720 views, 1%% of rays = %d per view):" % n_s)
        for st, rel in report.items():
            print("  %-4s storage: median %.3e  p99 %.3e  max %.3e  (unit roundoff %.3e)"
                  % (st, np.median(rel), np.percentile(rel, 99), rel.max(), U[st]), flush=True)
    assert report["f32"].max() <= TOL
    assert report["f16"].max() <= U["f16"] + TOL
    assert report["bf16"].max() <= U["bf16"] + TOL
    assert np.median(report["bf16"]) > np.median(report["f16"]) > np.median(report["f32"])


def _loop_problem(n=32, det=48, views=24, seed=300, k=6):
    h = 64.0 / n
    du = 96.0 / det
    g = syn.Geometry(n, n, n, h, h, h, det, det, du, du, 500.0, 1000.0, views)
    ells, xt = syn.phantom(g, k, seed=seed)
    clean = syn.ellipsoid_line_integrals(g, ells, np.arange(views))
    b = syn.add_noise(clean, 0.01, seed=seed + 1).astype(np.float32)
    perms = syn.view_permutations(views, 200, seed=seed + 2)
    return g, xt, b, perms


@pytest.mark.parametrize("st", ["bf16", "f16"])
def test_16bit_iterates_replay_and_error_against_fp64(fbl, orc, st, capsys):
    """FB-LISA with the iterates stored in 16 bits.  Replay: the GPU follows the decisions
    of the oracle's run with the same storage; its iterates stay within one unit roundoff
    (relative l2) of the oracle's (they differ only where the FP32 gradient moves a value
    across a rounding boundary).  The storage error of the reconstruction is stated
    against the FP64 run and bounded by a few unit roundoffs."""
    import torch
    g, xt, b32, perms = _loop_problem()
    epochs, n0 = 2, 4
    b64 = b32.astype(np.float64)
    x64, _ = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms)
    xs_o = []
    xo, rec = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms, storage=st,
                         callback=lambda k, x, r: xs_o.append(x.copy()))
    assert all(np.array_equal(orc.round_storage(x, st), x) for x in xs_o)
    decisions = [[t.accepted for t in r.trials] for r in rec]
    bd = torch.from_numpy(b32).cuda()
    xs_g = []
    run = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, vol_dtype=st)
    run.run(perms, decisions=decisions,
            callback=lambda s, it: xs_g.append(s.x.to(torch.float64).cpu().numpy()))
    assert len(xs_g) == len(xs_o)
    for k, (a, b) in enumerate(zip(xs_g, xs_o)):
        assert np.linalg.norm(a - b) <= U[st] * np.linalg.norm(b), k
    free = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, vol_dtype=st)
    xf = free.run(perms).to(torch.float64).cpu().numpy()
    f32 = fbl.FBLisa(g, bd, n0=n0, epochs=epochs)
    x32 = f32.run(perms).cpu().numpy().astype(np.float64)
    re_st, re_32 = orc.relative_error(xf, x64), orc.relative_error(x32, x64)
    with capsys.disabled():
        print("\n%s iterates: RE vs FP64 run %.3e (FP32 run %.3e); RMSE vs phantom %.4e (FP32 %.4e, FP64 %.4e)"
              % (st, re_st, re_32, orc.rmse(xf, xt), orc.rmse(x32, xt), orc.rmse(x64, xt)), flush=True)
    assert re_32 <= 1e-3
    assert re_st <= 4 * U[st]


@pytest.mark.parametrize("st,shape", [("bf16", "odd"), ("f16", "odd"), ("f32", "odd"), ("bf16", "large")])
def test_step_stochastic_rounding_matches_oracle(fbl, orc, st, shape):
    # the rounding decision depends only on the FP64 trial value, the key and the voxel
    # index, so the GPU's stored trial point equals the oracle's replay of the same draw
    # ("large": above 2^25 voxels, the one-pass kernel)
    import torch
    g = ODD if shape == "odd" else LARGE
    print("case step stochastic %s %s (%d voxels)" % (st, shape, g.d), flush=True)
    rng = np.random.default_rng(23)
    xs = orc.round_storage(rng.uniform(0, 0.03, g.vol_shape), st)
    xs[rng.random(g.vol_shape) < 0.2] = 0.0
    grad = (rng.standard_normal(g.vol_shape) * 3.0).astype(np.float32)
    with fbl.Plan(g, vol_dtype=st) as plan:
        outs = []
        for key, (alpha, mu, lo, hi) in ((0x1234, (1e-3, 0.0, 0.0, math.inf)), (2 ** 63 + 5, (2.5e-3, 0.7, 0.0, 0.03))):
            red = torch.zeros(3, dtype=torch.float64, device="cuda")
            xb, red = fbl.fb_lisa_step(plan, _dev(xs, st), torch.from_numpy(grad).cuda(), alpha, mu, lo, hi,
                                       red=red, key=key)
            xb = xb.to(torch.float64).cpu().numpy()
            red = red.cpu().numpy()
            xr, inner, sq, gg = orc.prox_step(xs, grad, alpha, mu, lo, hi, storage=st, key=key)
            assert np.mean(xb == xr) > 0.999
            assert np.all(np.abs(xb - xr) <= _storage_ulp(xr, st))
            assert red[0] == pytest.approx(inner, rel=1e-9)
            assert red[1] == pytest.approx(sq, rel=1e-9)
            outs.append(xb)
        # stochastic, not nearest: some values differ from the nearest rounding
        xn, _ = fbl.fb_lisa_step(plan, _dev(xs, st), torch.from_numpy(grad).cuda(), 1e-3, 0.0, 0.0, math.inf)
        assert not np.array_equal(outs[0], xn.to(torch.float64).cpu().numpy())


def test_bf16_stochastic_iterates_replay(fbl, orc, capsys):
    """BF16 iterates with stochastic rounding: the GPU replays the oracle's BF16 run with
    the same keys (trial j of iteration k uses (seed << 32) + (k << 6) + j)."""
    import torch
    g, xt, b32, perms = _loop_problem()
    epochs, n0, seed = 2, 4, 99
    b64 = b32.astype(np.float64)
    x64, _ = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms)
    xs_o = []
    xo, rec = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms, storage="bf16", sr_seed=seed,
                         callback=lambda k, x, r: xs_o.append(x.copy()))
    decisions = [[t.accepted for t in r.trials] for r in rec]
    bd = torch.from_numpy(b32).cuda()
    xs_g = []
    run = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, vol_dtype="bf16", sr_seed=seed)
    run.run(perms, decisions=decisions, callback=lambda s, it: xs_g.append(s.x.to(torch.float64).cpu().numpy()))
    for k, (a, b) in enumerate(zip(xs_g, xs_o)):
        assert np.linalg.norm(a - b) <= U["bf16"] * np.linalg.norm(b), k
    with capsys.disabled():
        print("\nbf16 iterates, stochastic rounding: RE vs FP64 run %.3e; RMSE vs phantom %.4e (FP64 %.4e)"
              % (orc.relative_error(xs_g[-1], x64), orc.rmse(xs_g[-1], xt), orc.rmse(x64, xt)), flush=True)
    assert orc.relative_error(xs_g[-1], x64) <= 4 * U["bf16"]


@pytest.mark.parametrize("st", ["bf16", "f16"])
@pytest.mark.parametrize("shape", ["odd", "128", "large"])
def test_step_mixed_master_and_copy(fbl, orc, st, shape):
    """Mixed storage: the FP32 trial point is the oracle's FP64 prox rounded once to FP32
    (within one FP32 ulp, > 99.9% identical), its 16-bit copy is exactly the nearest
    rounding of the returned FP32 value, and the inner products are those of the FP32
    values ("odd": a tail of one after the four-voxel passes; "128": several grid-stride
    passes per thread; "large": above 2^25 voxels, the one-pass kernel)."""
    import torch
    g = {"odd": ODD, "128": syn.config_geometry("c4"), "large": LARGE}[shape]
    print("case step mixed %s %s (%d voxels)" % (st, shape, g.d), flush=True)
    settings = ((1e-3, 0.0, 0.0, math.inf), (2.5e-3, 0.7, 0.0, 0.03), (1e-4, 2.0, 0.001, 0.025))
    if shape != "odd":
        settings = settings[1:2]
    rng = np.random.default_rng(24)
    x32 = rng.uniform(0, 0.03, g.vol_shape).astype(np.float32)
    x32[rng.random(g.vol_shape) < 0.2] = 0.0
    grad = (rng.standard_normal(g.vol_shape) * 3.0).astype(np.float32)
    with fbl.Plan(g, vol_dtype=st) as plan:
        for alpha, mu, lo, hi in settings:
            red = torch.zeros(3, dtype=torch.float64, device="cuda")
            xb, xb16, red = fbl.fb_lisa_step_mixed(plan, torch.from_numpy(x32).cuda(), torch.from_numpy(grad).cuda(),
                                                   alpha, mu, lo, hi, red=red)
            xb = xb.cpu().numpy().astype(np.float64)
            xb16 = xb16.to(torch.float64).cpu().numpy()
            red = red.cpu().numpy()
            xr, inner, sq, gg = orc.prox_step(x32, grad, alpha, mu, lo, hi, storage="f32")
            assert np.all(np.abs(xb - xr) <= _storage_ulp(xr, "f32"))
            assert np.mean(xb == xr) > 0.999
            assert np.array_equal(xb16, orc.round_storage(xb, st))
            assert np.mean(xb16 == orc.round_storage(xr, st)) > 0.999
            assert red[0] == pytest.approx(inner, rel=1e-9)
            assert red[1] == pytest.approx(sq, rel=1e-9)
            assert red[2] == pytest.approx(gg, rel=1e-12)


def test_step_mixed_rejects_fp32_plan(fbl):
    import torch
    g = ODD
    with fbl.Plan(g) as plan:
        x = torch.zeros(g.vol_shape, dtype=torch.float32, device="cuda")
        with pytest.raises(fbl.FblError) as ei:
            fbl.fb_lisa_step_mixed(plan, x, x.clone(), 1e-3, xbar16=torch.zeros(g.vol_shape, dtype=torch.float32,
                                                                                 device="cuda"))
        assert ei.value.code == 4   # FBL_E_DTYPE


@pytest.mark.parametrize("st", ["bf16", "f16"])
def test_mixed_iterates_replay_and_error_against_fp64(fbl, orc, st, capsys):
    """FB-LISA with an FP32 iterate and a 16-bit copy for the projector.  Replay: the GPU
    follows the decisions of the oracle's mixed run; its FP32 iterates stay within the
    16-bit unit roundoff (relative l2) of the oracle's (the FP32 gradient can move a value
    across a 16-bit rounding boundary, which changes the copy the next gradient sees).
    Against the FP64 run the error stays at a few unit roundoffs of the copy's type."""
    import torch
    g, xt, b32, perms = _loop_problem()
    epochs, n0 = 2, 4
    b64 = b32.astype(np.float64)
    x64, _ = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms)
    xs_o = []
    xo, rec = orc.fblisa(g, b64, epochs=epochs, n0=n0, perms=perms, copy_storage=st,
                         callback=lambda k, x, r: xs_o.append(x.copy()))
    assert all(np.array_equal(orc.round_storage(x, "f32"), x) for x in xs_o)
    decisions = [[t.accepted for t in r.trials] for r in rec]
    bd = torch.from_numpy(b32).cuda()
    xs_g = []
    run = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, vol_dtype=st, mixed=True)
    run.run(perms, decisions=decisions, callback=lambda s, it: xs_g.append(s.x.double().cpu().numpy()))
    assert len(xs_g) == len(xs_o)
    worst = 0.0
    for k, (a, b) in enumerate(zip(xs_g, xs_o)):
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        worst = max(worst, e)
        assert e <= U[st], (k, e)
    # the copy the projector reads is the nearest rounding of the iterate
    assert torch.equal(run.x16, run.x.to(run.x16.dtype))
    free = fbl.FBLisa(g, bd, n0=n0, epochs=epochs, vol_dtype=st, mixed=True)
    xf = free.run(perms).double().cpu().numpy()
    re_m = orc.relative_error(xf, x64)
    with capsys.disabled():
        print("\n%s copy of an FP32 iterate: replay worst RE vs oracle %.3e; free run RE vs FP64 run %.3e; "
              "RMSE vs phantom %.4e (FP64 run %.4e)" % (st, worst, re_m, orc.rmse(xf, xt), orc.rmse(x64, xt)),
              flush=True)
    assert re_m <= 4 * U[st]
