"""GPU (HIP) path against the FP64 oracle, element by element, through the C ABI.

Tolerance (float path, FP32 arithmetic against FP64): per view, relative l2 error
<= 1e-5 and max abs error <= 1e-5 * max|oracle|; the prox trial is within one FP32 ulp
of the oracle's stored trial point and its FP64 reductions agree to 1e-12 relative
(1e-9 where single-ulp differences of the trial point enter); the loss to 1e-5.
"""
import math

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def fbl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2605_12085_amd as fbl
    return fbl


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _cmp_views(gpu, ref, tol=TOL, what=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    for b in range(ref.shape[0]):
        nr = np.linalg.norm(ref[b])
        if nr == 0:
            assert np.abs(gpu[b]).max() == 0, what
            continue
        rel = np.linalg.norm(gpu[b] - ref[b]) / nr
        mx = np.abs(gpu[b] - ref[b]).max() / np.abs(ref[b]).max()
        assert rel <= tol and mx <= tol, "%s view %d: rel l2 %.3g, rel max %.3g" % (what, b, rel, mx)


def _cmp_vol(gpu, ref, tol=TOL, what=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    rel = np.linalg.norm(gpu - ref) / np.linalg.norm(ref)
    mx = np.abs(gpu - ref).max() / np.abs(ref).max()
    assert rel <= tol and mx <= tol, "%s: rel l2 %.3g, rel max %.3g" % (what, rel, mx)


ODD = syn.Geometry(29, 41, 37, 0.9, 1.1, 1.0, 50, 33, 1.7, 1.9, 400.0, 900.0, 12,
                   angles=[0.0, np.pi / 4, np.pi / 2, np.pi, 3 * np.pi / 2, 0.3, 1.7, 2.9, 4.0, 5.5, 0.05, 6.2])


def test_forward_odd_sizes_axis_aligned_views(fbl, orc):
    g = ODD
    print("case forward ODD", flush=True)
    x = syn.random_volume(g, 3)
    views = np.array([0, 1, 2, 3, 4, 7, 10, 11], dtype=np.int32)
    ref = orc.forward(g, x.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x), views).cpu().numpy()
    _cmp_views(y, ref, what="forward")


def test_forward_residual_and_loss(fbl, orc):
    import torch
    g = ODD
    x = syn.random_volume(g, 4)
    b = syn.random_projections(g, g.n_views, 5, scale=2.0)
    views = np.array([5, 2, 9], dtype=np.int32)
    r_ref = orc.forward(g, x.astype(np.float64), views) - b.astype(np.float64)[views]
    f_ref = g.n_views / (2.0 * len(views)) * float(np.sum(r_ref ** 2))
    with fbl.Plan(g, max_batch=5) as plan:
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        r = fbl.fb_lisa_forward(plan, _t(x), views, _t(b), loss=loss).cpu().numpy()
        f_gpu = float(loss.item())
        # repeat: the FP64 reduction order is fixed
        loss2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        fbl.fb_lisa_forward(plan, _t(x), views, _t(b), loss=loss2)
        assert loss2.item() == f_gpu
    _cmp_views(r, r_ref, what="residual")
    assert f_gpu == pytest.approx(f_ref, rel=TOL)


def test_forward_c1_phantom_all_rays(fbl, orc):
    g = syn.config_geometry("c1")
    _, xt = syn.phantom(g, 10, seed=1000)
    x32 = xt.astype(np.float32)
    views = syn.view_permutations(g.n_views, 1, seed=1002)[0][:6]
    ref = orc.forward(g, x32.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x32), views).cpu().numpy()
    _cmp_views(y, ref, what="forward c1")


def test_backproject_odd_sizes(fbl, orc):
    g = ODD
    rng = np.random.default_rng(6)
    views = np.array([0, 1, 2, 3, 4, 7, 10], dtype=np.int32)
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    ref = g.n_views / len(views) * orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        gg = fbl.fb_lisa_backproject(plan, _t(r), views).cpu().numpy()
        gg2 = fbl.fb_lisa_backproject(plan, _t(r), views).cpu().numpy()
    assert np.array_equal(gg, gg2)  # no atomics: bitwise repeatable
    _cmp_vol(gg, ref, what="backprojection")


def test_backproject_c1_all_voxels(fbl, orc):
    g = syn.config_geometry("c1")
    rng = np.random.default_rng(7)
    views = syn.view_permutations(g.n_views, 1, seed=7)[0][:6]
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    ref = 1.7 * orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g, max_batch=6) as plan:
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.7).cpu().numpy()
    _cmp_vol(gg, ref, what="backprojection c1")


def test_backproject_non_finite_residual(fbl, orc):
    # an inf and a NaN residual: every voxel the oracle's gradient makes non-finite is
    # non-finite on the GPU too (the GPU marks the whole z-profile of the bad detector
    # column, a superset), and every voxel the GPU leaves finite agrees with the oracle
    g = ODD
    print("case backprojection non-finite residual", flush=True)
    rng = np.random.default_rng(61)
    views = np.array([0, 5, 9], dtype=np.int32)
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    r[0, g.nv // 2, g.nu // 2] = np.inf
    r[2, g.nv // 3, g.nu // 4] = np.nan
    ref = g.n_views / len(views) * orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        gg = fbl.fb_lisa_backproject(plan, _t(r), views).cpu().numpy().astype(np.float64)
    bad_ref, bad_gpu = ~np.isfinite(ref), ~np.isfinite(gg)
    assert bad_ref.any()
    assert np.all(bad_gpu[bad_ref])
    ok = ~bad_gpu
    assert ok.any()
    err = np.abs(gg[ok] - ref[ok]).max() / np.abs(ref[ok]).max()
    assert err <= TOL, "finite voxels: rel max %.3g" % err


def test_fine_detector_rows_forward_and_backprojection(fbl, orc):
    # detector rows 0.6 voxel apart at the detector (about 0.3 voxel at the volume): the
    # backprojection's residual window for half a tile's z-range exceeds its LDS window on
    # some passes, which then read the residual from device memory
    g = syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 60, 1.5, 0.6, 300.0, 600.0, 12)
    rng = np.random.default_rng(16)
    views = np.arange(g.n_views, dtype=np.int32)
    x = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    y_ref = orc.forward(g, x.astype(np.float64), views)
    g_ref = orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x), views).cpu().numpy()
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
    _cmp_views(y, y_ref, what="forward fine rows")
    _cmp_vol(gg, g_ref, what="backprojection fine rows")


def test_backproject_power_of_two_scaling_is_exact(fbl):
    # The staged z-profiles round each column's residual window to integers relative to
    # its largest entry; the rounding follows a power-of-two scale of the residual, so
    # the result scales by exactly that power (no overflow or underflow here).
    g = syn.config_geometry("c1")
    rng = np.random.default_rng(21)
    views = syn.view_permutations(g.n_views, 1, seed=21)[0][:6]
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    with fbl.Plan(g, max_batch=6) as plan:
        g0 = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
        for e in (60, -60):
            ge = fbl.fb_lisa_backproject(plan, _t(np.ldexp(r, e)), views, grad_scale=1.0).cpu().numpy()
            assert np.array_equal(ge, np.ldexp(g0, e)), e


def test_backproject_wide_dynamic_range(fbl, orc):
    # Residual rows spanning eight decades within each detector column (a few rows 1e4
    # times the rest, the rest down to 1e-4): the rounding is relative to each column's
    # largest entry, so the result keeps the 1e-5 bar on the volume.
    g = syn.config_geometry("c1")
    rng = np.random.default_rng(22)
    views = syn.view_permutations(g.n_views, 1, seed=22)[0][:6]
    r = rng.standard_normal((len(views), g.nv, g.nu)) * 10.0 ** rng.uniform(-4, 0, (len(views), g.nv, 1))
    r[:, rng.integers(0, g.nv, 5), :] *= 1e4
    r = r.astype(np.float32)
    ref = orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g, max_batch=6) as plan:
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
    _cmp_vol(gg, ref, what="backprojection, wide dynamic range")


def test_fine_detector_columns_wide_pair_tables(fbl, orc):
    # detector columns 0.7 voxel apart at the detector (about 0.35 voxel at the volume):
    # up to 55 columns cross one 16-voxel tile slice, so the backprojection takes its
    # 64-column pair tables (two blocks per compute unit)
    g = syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 77, 30, 0.7, 1.5, 300.0, 600.0, 8)
    rng = np.random.default_rng(17)
    views = np.arange(g.n_views, dtype=np.int32)
    x = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    y_ref = orc.forward(g, x.astype(np.float64), views)
    g_ref = orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x), views).cpu().numpy()
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
    _cmp_views(y, y_ref, what="forward fine columns")
    _cmp_vol(gg, g_ref, what="backprojection fine columns")


def test_forward_split_march_two_parts(fbl, orc):
    # 40 views of the 128^3 / 192^2 workload: one march part per ray would give 1440
    # waves, under two per SIMD, so the forward splits each ray's march over two waves
    g = syn.config_geometry("c4")
    cfg = syn.CONFIGS["c4"]
    ells, xt = syn.phantom(g, cfg["k"], seed=41, hi=cfg["hi"])
    views = syn.view_permutations(g.n_views, 1, seed=42)[0][:40]
    b = syn.add_noise(syn.ellipsoid_line_integrals(g, ells, np.arange(g.n_views)), 0.01, seed=43).astype(np.float32)
    x = (0.8 * xt).astype(np.float32)
    y_ref = orc.forward(g, x.astype(np.float64), views) - b[views].astype(np.float64)
    f_ref = g.n_views / (2.0 * len(views)) * float(np.sum(y_ref ** 2))
    import torch
    with fbl.Plan(g, max_batch=40) as plan:
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        y = fbl.fb_lisa_forward(plan, _t(x), views, _t(b), loss=loss).cpu().numpy()
    _cmp_views(y, y_ref, what="forward, split march")
    assert float(loss) == pytest.approx(f_ref, rel=TOL)


def test_adjoint_identity_on_gpu(fbl):
    import torch
    g = syn.Geometry(40, 36, 30, 1.0, 1.0, 1.0, 60, 44, 1.4, 1.4, 400.0, 800.0, 16)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(g.vol_shape).astype(np.float32)
    views = np.arange(0, 16, 3, dtype=np.int32)
    y = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    with fbl.Plan(g) as plan:
        ax = fbl.fb_lisa_forward(plan, _t(x), views).double()
        aty = fbl.fb_lisa_backproject(plan, _t(y), views, grad_scale=1.0).double()
        lhs = float(torch.sum(ax * _t(y).double()))
        rhs = float(torch.sum(_t(x).double() * aty))
    assert lhs == pytest.approx(rhs, rel=1e-5)


def test_explicit_matrix_8cubed(fbl, orc):
    # Columns of A by GPU forward projection of unit voxels, rows by GPU backprojection
    # of unit rays: both equal the oracle's explicit A to FP32 accuracy.
    import torch
    g = syn.tiny_geometry(n=8, det=12, views=16)
    views = np.arange(16, dtype=np.int32)
    A = orc.assemble_matrix(g, views)
    with fbl.Plan(g) as plan:
        e = torch.zeros(g.vol_shape, dtype=torch.float32, device="cuda")
        cols = []
        for i in range(g.d):
            e.view(-1).zero_()
            e.view(-1)[i] = 1.0
            cols.append(fbl.fb_lisa_forward(plan, e, views).reshape(-1).cpu().numpy())
        A_fp = np.stack(cols, axis=1)
        rows = []
        er = torch.zeros((16, g.nv, g.nu), dtype=torch.float32, device="cuda")
        for i in range(0, 16 * g.n_p, 7):     # every 7th ray (a third of the rows)
            er.view(-1).zero_()
            er.view(-1)[i] = 1.0
            rows.append((i, fbl.fb_lisa_backproject(plan, er, views, grad_scale=1.0).reshape(-1).cpu().numpy()))
    # entries are weights w*(1-a)(1-b); the kernels step positions in FP32 relative to an
    # integer base up to ~20 voxels away (resolution ~2e-6 voxel), so an entry is exact to
    # a few 1e-6 of the largest one
    scale = np.abs(A).max()
    assert np.abs(A_fp - A).max() <= 4e-6 * scale
    for i, row in rows:
        assert np.abs(row - A[i]).max() <= 4e-6 * scale, i


# 33,752,070 voxels: above 2^25, so the prox trial takes its one-pass kernels and a
# second reduction level; two voxels after the last group of four
LARGE = syn.Geometry(331, 330, 309, 0.1, 0.1, 0.1, 64, 64, 0.15, 0.15, 500.0, 1000.0, 4)


@pytest.mark.parametrize("shape", ["odd", "large"])
def test_step_parity(fbl, orc, shape):
    import torch
    g = ODD if shape == "odd" else LARGE
    print("case step parity %s (%d voxels)" % (shape, g.d), flush=True)
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 0.03, g.vol_shape).astype(np.float32)
    x[rng.random(g.vol_shape) < 0.2] = 0.0
    grad = rng.standard_normal(g.vol_shape).astype(np.float32) * 3.0
    settings = ((1e-3, 0.0, 0.0, math.inf), (2.5e-3, 0.7, 0.0, 0.03), (1e-4, 2.0, 0.001, 0.025))
    with fbl.Plan(g) as plan:
        for alpha, mu, lo, hi in (settings if shape == "odd" else settings[1:2]):
            red = torch.zeros(3, dtype=torch.float64, device="cuda")
            xb, red = fbl.fb_lisa_step(plan, _t(x), _t(grad), alpha, mu, lo, hi, red=red)
            xb = xb.cpu().numpy()
            red = red.cpu().numpy()
            xr, inner, sq, gg = orc.prox_step(x, grad, alpha, mu, lo, hi, storage=np.float32)
            ulp = np.spacing(np.abs(xr).astype(np.float32)).astype(np.float64)
            assert np.all(np.abs(xb.astype(np.float64) - xr) <= ulp)
            frac_exact = np.mean(xb.astype(np.float64) == xr)
            assert frac_exact > 0.999
            assert red[0] == pytest.approx(inner, rel=1e-9)
            assert red[1] == pytest.approx(sq, rel=1e-9)
            assert red[2] == pytest.approx(gg, rel=1e-12)



def test_reductions_over_many_partials(fbl, orc):
    # More than 2048 per-block partials, so the final one-block sum takes its batched
    # path: the prox trial at 128^3 runs 2048 blocks, and a 512^2 detector gives
    # 64 forward blocks per view (2560 for 40 views).
    import torch
    g = syn.config_geometry("c4")
    assert g.d == 128 ** 3
    rng = np.random.default_rng(41)
    x = rng.uniform(0, 0.02, g.vol_shape).astype(np.float32)
    grad = (rng.standard_normal(g.vol_shape) * 3.0).astype(np.float32)
    with fbl.Plan(g) as plan:
        red = torch.zeros(3, dtype=torch.float64, device="cuda")
        xb, red = fbl.fb_lisa_step(plan, _t(x), _t(grad), 1e-3, 0.5, 0.0, 0.03, red=red)
        xr, inner, sq, gg = orc.prox_step(x, grad, 1e-3, 0.5, 0.0, 0.03, storage=np.float32)
        red = red.cpu().numpy()
        assert red[0] == pytest.approx(inner, rel=1e-9)
        assert red[1] == pytest.approx(sq, rel=1e-9)
        assert red[2] == pytest.approx(gg, rel=1e-12)
        xb = xb.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(xb - xr) <= np.spacing(np.abs(xr).astype(np.float32)).astype(np.float64))
    # 0.5 mm voxels and pixels: rows 0.5 voxels apart at the centre (a wide detector,
    # most of whose rays miss the volume, still runs 64 forward blocks per view)
    g2 = syn.Geometry(64, 64, 64, 0.5, 0.5, 0.5, 512, 512, 0.5, 0.5, 500.0, 1000.0, 40)
    x2 = rng.uniform(0, 0.02, g2.vol_shape).astype(np.float32)
    views = np.arange(40, dtype=np.int32)
    with fbl.Plan(g2, max_batch=40) as plan:
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        y = fbl.fb_lisa_forward(plan, _t(x2), views, loss=loss, loss_scale=0.5)
        yy = y.cpu().numpy().astype(np.float64)
        assert float(loss[0]) == pytest.approx(0.5 * np.sum(yy * yy), rel=1e-12)

def test_chunked_batches_and_duplicates(fbl, orc):
    # more views than one launch carries (256), duplicates and B = 1
    g = syn.Geometry(12, 10, 8, 1.0, 1.0, 1.0, 16, 12, 1.5, 1.5, 300.0, 600.0, 300)
    rng = np.random.default_rng(10)
    x = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    views = rng.integers(0, 300, 290).astype(np.int32)
    views[5] = views[4]
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    y_ref = orc.forward(g, x.astype(np.float64), views)
    g_ref = orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x), views).cpu().numpy()
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
        y1 = fbl.fb_lisa_forward(plan, _t(x), views[:1]).cpu().numpy()
    _cmp_views(y, y_ref, what="forward chunked")
    assert np.array_equal(y[4], y[5])
    _cmp_vol(gg, g_ref, what="backprojection chunked")
    assert np.array_equal(y1[0], y[0])


def test_host_checks_launch_nothing(fbl):
    import torch
    g = syn.tiny_geometry(n=8, det=12, views=16)
    with fbl.Plan(g, max_batch=4) as plan:
        x = torch.zeros(g.vol_shape, dtype=torch.float32, device="cuda")
        with pytest.raises(fbl.FblError) as e:
            fbl.fb_lisa_forward(plan, x, [0, 1, 2, 3, 4])
        assert e.value.code == 3
        with pytest.raises(fbl.FblError) as e:
            fbl.fb_lisa_forward(plan, x, [16])
        assert e.value.code == 3
        with pytest.raises(fbl.FblError) as e:
            fbl.fb_lisa_step(plan, x, torch.zeros_like(x), alpha=-1.0)
        assert e.value.code == 1
        with pytest.raises(fbl.FblError) as e:
            fbl.fb_lisa_step(plan, x, torch.zeros_like(x), alpha=1.0, lo=0.5, hi=0.1)
        assert e.value.code == 1
    with pytest.raises(fbl.FblError) as e:
        fbl.Plan(g, max_batch=17)
    assert e.value.code == 3
    with pytest.raises(fbl.FblError) as e:
        fbl.Plan(g, vol_dtype="f32", proj_dtype="f32", max_batch=0)
    assert e.value.code == 3


def test_launch_timing_records_every_kernel(fbl):
    import torch
    g = syn.tiny_geometry(n=8, det=12, views=16)
    x = _t(syn.random_volume(g, seed=3).astype(np.float32))
    b = torch.zeros((g.n_views, g.nv, g.nu), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    with fbl.Plan(g) as plan:
        views = list(range(g.n_views))   # includes views that march x = const slices
        plan.timing(True)
        r = fbl.fb_lisa_forward(plan, x, views, b, loss=loss)
        gr = fbl.fb_lisa_backproject(plan, r, views)
        fbl.fb_lisa_step(plan, x, gr, 1e-3)
        kt = plan.timing_read()
        assert {k: n for k, (_, n) in kt.items()} == {"forward": 1, "transpose": 1, "finalize": 2, "prescale": 1,
                                                       "backproject": 1, "step": 1}
        assert all(ms > 0 for ms, n in kt.values())
        assert all(n == 0 for _, n in plan.timing_read().values())   # read clears
        plan.timing(False)
        fbl.fb_lisa_forward(plan, x, views)
        assert all(n == 0 for _, n in plan.timing_read().values())
        # a selection brackets only the chosen kernels
        plan.timing(True, kernels=("forward", "backproject"))
        r = fbl.fb_lisa_forward(plan, x, views, b, loss=loss)
        fbl.fb_lisa_backproject(plan, r, views)
        fbl.fb_lisa_step(plan, x, gr, 1e-3)
        kt = plan.timing_read()
        assert {k: n for k, (_, n) in kt.items()} == {"forward": 1, "transpose": 0, "finalize": 0, "prescale": 0,
                                                       "backproject": 1, "step": 0}
        plan.timing(False)
        torch.cuda.synchronize()


def test_timing_default_selects_every_kernel(fbl):
    # through the C ABI with no fbl_timing_select: the documented default brackets every
    # kernel the calls launch
    import ctypes
    import torch
    from paper_2605_12085_amd import _lib
    g = syn.tiny_geometry(n=8, det=12, views=16)
    x = _t(syn.random_volume(g, seed=3).astype(np.float32))
    b = torch.zeros((g.n_views, g.nv, g.nu), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    with fbl.Plan(g) as plan:
        _lib._check(_lib.lib.fbl_timing_enable(plan.handle, 1))
        views = list(range(g.n_views))
        r = fbl.fb_lisa_forward(plan, x, views, b, loss=loss)
        gr = fbl.fb_lisa_backproject(plan, r, views)
        fbl.fb_lisa_step(plan, x, gr, 1e-3)
        ms = (ctypes.c_double * len(_lib.KERNELS))()
        n = (ctypes.c_int64 * len(_lib.KERNELS))()
        _lib._check(_lib.lib.fbl_timing_read(plan.handle, ms, n))
        _lib._check(_lib.lib.fbl_timing_enable(plan.handle, 0))
        assert dict(zip(_lib.KERNELS, list(n))) == {"forward": 1, "transpose": 1, "finalize": 2, "prescale": 1,
                                                     "backproject": 1, "step": 1}
        assert all(v > 0 for v in ms)
        torch.cuda.synchronize()


def _forward_line_entries(g, rows_per_thread=16):
    """The forward's per-thread line length for a geometry, from the plan's rule: the
    z-span of 16 rows on the slice farthest from the source, plus three entries."""
    taus = []
    for v in range(g.n_views):
        th = g.angles[v]
        c, s = math.cos(th), math.sin(th)
        for iu in range(g.nu):
            u = (iu - 0.5 * (g.nu - 1)) * g.du
            src = np.array([g.sod * c, g.sod * s])
            q = np.array([(g.sod - g.sdd) * c - u * s, (g.sod - g.sdd) * s + u * c])
            h = np.array([g.hx, g.hy])
            n = np.array([g.nx, g.ny])
            P, D = src / h + 0.5 * (n - 1), (q - src) / h
            a = 0 if abs(D[0]) >= abs(D[1]) else 1
            taus += [(0.0 - P[a]) / D[a], (n[a] - 1.0 - P[a]) / D[a]]
    span = max(taus) * (rows_per_thread - 1) * (g.dv / g.hz)
    need = math.floor(span + 0.01) + 3
    return next(sz for sz in (12, 16, 24, 32, 48) if need <= sz)


@pytest.mark.parametrize("dv,kb", [(3.2, 32), (4.8, 48)])
def test_coarse_detector_rows_long_forward_lines(fbl, orc, dv, kb):
    # detector rows 1.6-2.4 voxels apart at the volume: a thread's 16 rows span 25-37
    # voxels in z, which selects the forward's 32- and 48-entry line buffers
    g = syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 12, 1.5, dv, 300.0, 600.0, 12)
    assert _forward_line_entries(g) == kb
    rng = np.random.default_rng(40 + kb)
    views = np.arange(g.n_views, dtype=np.int32)
    x = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
    y_ref = orc.forward(g, x.astype(np.float64), views)
    g_ref = orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x), views).cpu().numpy()
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
    _cmp_views(y, y_ref, what="forward, %d-entry lines" % kb)
    _cmp_vol(gg, g_ref, what="backprojection, coarse rows")


def test_exact_dominant_axis_tie(fbl, orc):
    # theta = 0, isotropic voxels, outermost columns at u = +-SDD: their rays run at 45
    # degrees, |D_x| = |D_y| exactly in FP64, and the tie goes to x on both sides.  SOD is
    # small enough (18 mm for a 20 mm volume) that these rays cross the volume's corners.
    g = syn.Geometry(20, 20, 4, 1.0, 1.0, 1.0, 5, 6, 18.0, 2.0, 18.0, 36.0, 1, angles=[0.0])
    views = np.array([0], dtype=np.int32)
    for iu in (0, 4):
        u = (iu - 2) * 18.0
        dx, dy = (-18.0 - 18.0) / 1.0, u / 1.0
        assert abs(dx) == abs(dy)
    axes = orc.dominant_axes(g, 0)
    assert np.all(axes == 0)
    rng = np.random.default_rng(44)
    x = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    r = rng.standard_normal((1, g.nv, g.nu)).astype(np.float32)
    y_ref = orc.forward(g, x.astype(np.float64), views)
    assert np.all(y_ref[0][:, [0, 4]] > 0)   # the tie rays cross the volume
    g_ref = orc.backproject(g, r.astype(np.float64), views)
    with fbl.Plan(g) as plan:
        y = fbl.fb_lisa_forward(plan, _t(x), views).cpu().numpy()
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
    _cmp_views(y, y_ref, what="forward, exact axis tie")
    for iu in (0, 4):
        col = y[0][:, iu].astype(np.float64)
        assert np.abs(col - y_ref[0][:, iu]).max() <= TOL * np.abs(y_ref[0][:, iu]).max()
    _cmp_vol(gg, g_ref, what="backprojection, exact axis tie")


@pytest.mark.parametrize("cfg", ["c2", "c3", "c5"])
def test_full_size_sampled_parity(fbl, orc, cfg):
    # Full-size geometry and the batch size the benchmark times; rays and voxels are
    # sampled because the oracle evaluates them one by one.
    import torch
    g = syn.config_geometry(cfg)
    c = syn.CONFIGS[cfg]
    print("case full-size", cfg, flush=True)
    if cfg == "c5":
        # 1024^3 FP32 (4 GiB, byte offsets up to 2^32): seeded uniform values instead of a
        # voxelised phantom, which would take minutes on the host
        x32 = syn.random_volume(g, seed=2000)
    else:
        ells, xt = syn.phantom(g, c["k"], seed=2000, hi=c["hi"], sub=2 if cfg == "c2" else 1)
        x32 = xt.astype(np.float32)
        del xt
    views = syn.view_permutations(g.n_views, 1, seed=2002)[0][:c["batch"]]
    rng = np.random.default_rng(11)
    with fbl.Plan(g, max_batch=c["batch"]) as plan:
        xd = _t(x32)
        y = fbl.fb_lisa_forward(plan, xd, views).cpu().numpy()
        r = rng.standard_normal((len(views), g.nv, g.nu)).astype(np.float32)
        gg = fbl.fb_lisa_backproject(plan, _t(r), views, grad_scale=1.0).cpu().numpy()
    nr = 3000
    rays = np.stack([rng.integers(0, len(views), nr), rng.integers(0, g.nv, nr), rng.integers(0, g.nu, nr)], 1)
    rays_v = rays.copy()
    rays_v[:, 0] = views[rays[:, 0]]
    ref = orc.forward_rays(g, x32.astype(np.float64), rays_v)
    got = y[rays[:, 0], rays[:, 1], rays[:, 2]].astype(np.float64)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got - ref).max() <= TOL * scale
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)
    # voxels: inside the field of view and at the volume's edges and corners (the oracle
    # sums over every ray of the batch per voxel, so fewer are taken at the larger sizes)
    nvx = {"c2": 96, "c3": 64, "c5": 64}[cfg]
    vox = rng.integers(0, g.d, nvx)
    vox[:8] = [0, g.nx - 1, g.nx * (g.ny - 1), g.d - 1, g.d // 2, g.d // 2 + 1, g.d // 2 + g.nx, g.d // 3]
    # near the rotation axis at the top and bottom of the volume, where the rows reaching a
    # backprojection tile span the tallest windows, and at tile boundaries in z
    cx, cy = g.nx // 2, g.ny // 2
    for n_, (k, dx, dy) in enumerate([(0, 0, 0), (1, 5, -7), (15, -3, 2), (16, 9, 4),
                                      (g.nz - 17, 1, 1), (g.nz - 16, -6, 8), (g.nz - 2, 2, -2), (g.nz - 1, -1, 0)]):
        vox[8 + n_] = (cx + dx) + g.nx * ((cy + dy) + g.ny * k)
    gref = orc.backproject_voxels(g, r.astype(np.float64), views, vox)
    ggot = gg.reshape(-1)[vox].astype(np.float64)
    gscale = np.abs(gref).max()
    assert gscale > 0
    assert np.abs(ggot - gref).max() <= TOL * gscale


def test_grouped_forward_reads_agree_bit_for_bit(fbl):
    # A launch of 8192 waves or more reads four rays' line taps together before their
    # lerps, a smaller one two.  One call over 256 views of a 128^3 / 192^2 geometry (9
    # blocks of 4 waves per view: 9216 waves) takes the first form, the same views in two
    # calls of 128 (4608 waves each) the second; both must give the same bits.  (The
    # compiler-scheduled form, taken by split marches and long lines, is checked against
    # the oracle on the small and coarse-row geometries.)
    import dataclasses
    import torch
    g = dataclasses.replace(syn.config_geometry("c4"), n_views=256, angles=None)
    print("case grouped forward reads 128^3, 256 views", flush=True)
    views = np.random.default_rng(40).permutation(256).astype(np.int32)
    x = syn.random_volume(g, seed=41)
    b = np.random.default_rng(42).standard_normal((g.n_views, g.nv, g.nu)).astype(np.float32)
    with fbl.Plan(g, max_batch=256) as plan:
        xd, bd = _t(x), _t(b)
        l_all = torch.zeros(1, dtype=torch.float64, device="cuda")
        y_all = fbl.fb_lisa_forward(plan, xd, views, b=bd, loss=l_all, loss_scale=1.0).cpu().numpy()
        l_two = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2)]
        y_two = np.concatenate([fbl.fb_lisa_forward(plan, xd, views[i:i + 128], b=bd, loss=l_two[i // 128],
                                                    loss_scale=1.0).cpu().numpy() for i in (0, 128)])
    assert np.array_equal(y_all, y_two)
    assert np.any(y_all != 0)
    # the loss sums the same squares in another order: equal to FP64 rounding
    assert float(l_all) == pytest.approx(float(l_two[0]) + float(l_two[1]), rel=1e-12)
