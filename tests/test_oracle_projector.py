"""Pins of the FP64 oracle's projector pair against closed forms and brute force.

Each test checks the oracle against something other than itself:
  * exact chord lengths (all-ones volume, uniform ball, ellipsoids, Gaussian blob)
    computed from the continuous objects in ``synthetic``;
  * the hat-function weight of a single hot voxel, derived from a line/plane
    intersection in millimetres;
  * explicit matrices assembled column by column (forward) and row by row
    (backprojection), and the adjoint identity <Ax, y> = <x, A^T y>.
"""
import math

import numpy as np
import pytest

import synthetic as syn


def _endpoints_mm(g, view, iu, iv):
    src, pix = syn.ray_endpoints(g, [view])
    return src[0], pix[0, iv, iu]


def test_all_ones_volume_gives_slab_chord(orc):
    # A ray that enters and leaves the slab of slices through the two faces normal
    # to its dominant axis, with every tap interior, sees exactly N_a slices of value
    # 1: its value is the chord length N_a h_a / |cos(angle to axis a)|.
    g = syn.tiny_geometry(n=12, det=16, views=7)
    x = np.ones(g.vol_shape)
    views = np.arange(g.n_views)
    y = orc.forward(g, x, views)
    src, pix = syn.ray_endpoints(g, views)
    n = np.array([g.nx, g.ny, g.nz])
    h = np.array([g.hx, g.hy, g.hz])
    checked = 0
    for b in range(len(views)):
        for iv in range(g.nv):
            for iu in range(g.nu):
                s, q = src[b], pix[b, iv, iu]
                D = (q - s) / h
                a = int(np.argmax(np.abs(D)))
                # index coordinates of the ray on the first and last slice planes
                P = s / h + 0.5 * (n - 1)
                ok = True
                for m in (0, n[a] - 1):
                    t = (m - P[a]) / D[a]
                    p = P + t * D
                    for o in range(3):
                        if o != a and not (0.0 <= p[o] <= n[o] - 1):
                            ok = False
                if not ok:
                    continue
                expect = n[a] * h[a] * np.linalg.norm(q - s) / abs(q[a] - s[a])
                assert y[b, iv, iu] == pytest.approx(expect, rel=1e-13)
                checked += 1
    assert checked > 100


def test_rays_missing_the_volume_are_zero(orc):
    g = syn.tiny_geometry(n=8, det=12, views=4, du=12.0)  # wide detector: outer rays miss
    x = np.ones(g.vol_shape)
    y = orc.forward(g, x, [0, 1, 2, 3])
    src, pix = syn.ray_endpoints(g, [0, 1, 2, 3])
    # distance of each ray from the origin; beyond the volume's half-diagonal + 1 voxel -> no taps
    d = pix - src[:, None, None, :]
    dn = d / np.linalg.norm(d, axis=-1, keepdims=True)
    w = -src[:, None, None, :]
    perp = w - (w * dn).sum(-1, keepdims=True) * dn
    dist = np.linalg.norm(perp, axis=-1)
    far = dist > math.sqrt(3) * 4 * g.hx + 2
    assert far.any()
    assert np.all(y[far] == 0.0)
    assert np.all(y[~far] >= 0.0)


def test_hot_voxel_hat_weights_anisotropic(orc):
    # Non-cubic volume with anisotropic voxels, so a swap of the two in-slice axes,
    # of strides or of voxel sizes fails.  The expected entry is derived from the
    # intersection of the ray (in mm) with the plane through the voxel centre normal
    # to the ray's dominant axis, and the hat function of the in-plane offsets.
    g = syn.Geometry(7, 9, 5, 1.0, 0.8, 1.3, 14, 10, 1.9, 2.1, 300.0, 700.0, 5)
    rng = np.random.default_rng(3)
    for _ in range(6):
        vi, vj, vk = rng.integers(1, g.nx - 1), rng.integers(1, g.ny - 1), rng.integers(1, g.nz - 1)
        x = np.zeros(g.vol_shape)
        x[vk, vj, vi] = 1.0
        view = int(rng.integers(0, g.n_views))
        y = orc.forward(g, x, [view])[0]
        h = np.array([g.hx, g.hy, g.hz])
        n = np.array([g.nx, g.ny, g.nz])
        centre = (np.array([vi, vj, vk]) - 0.5 * (n - 1)) * h
        expect = np.zeros((g.nv, g.nu))
        src, pix = syn.ray_endpoints(g, [view])
        for iv in range(g.nv):
            for iu in range(g.nu):
                s, q = src[0], pix[0, iv, iu]
                dmm = q - s
                a = int(np.argmax(np.abs(dmm / h)))
                t = (centre[a] - s[a]) / dmm[a]
                p = s + t * dmm
                wgt = 1.0
                for o in range(3):
                    if o != a:
                        wgt *= max(0.0, 1.0 - abs(p[o] - centre[o]) / h[o])
                seg = h[a] * np.linalg.norm(dmm) / abs(dmm[a])
                expect[iv, iu] = seg * wgt
        assert np.max(np.abs(y - expect)) <= 1e-12 * max(1.0, np.abs(expect).max())
        assert np.abs(expect).max() > 0


def _refine_errors(make, levels):
    errs = []
    for g, x, ref in make(levels):
        errs.append(float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel())))
    return errs


def test_gaussian_blob_second_order(orc):
    # Smooth object: bilinear Joseph converges as O(h^2).  The blob is off-centre so a
    # wrong angle direction, detector axis or centring fails.
    centre = (3.0, -2.0, 1.5)
    sigma = 3.0
    errs = []
    for n in (16, 32, 64):
        h = 32.0 / n
        g = syn.Geometry(n, n, n, h, h, h, 3 * n // 2, 3 * n // 2, 48.0 / (3 * n // 2), 48.0 / (3 * n // 2),
                         250.0, 500.0, 6)
        views = [0, 1, 3, 5]
        x = syn.gaussian_volume(g, sigma, centre)
        y = orc.forward(g, x, views)
        ref = syn.gaussian_line_integrals(g, views, sigma, centre)
        errs.append(float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel())))
    assert errs[-1] < 5e-3
    r1, r2 = errs[1] / errs[0], errs[2] / errs[1]
    assert 0.15 < r1 < 0.35 and 0.15 < r2 < 0.35, errs


def test_ball_and_ellipsoids_first_order(orc):
    # Piecewise-constant objects: discontinuities give O(h) convergence in the l2 norm
    # of the sinogram error.
    errs_ball, errs_ell = [], []
    for n in (16, 32, 64):
        h = 32.0 / n
        g = syn.Geometry(n, n, n, h, h, h, 3 * n // 2, 3 * n // 2, 48.0 / (3 * n // 2), 48.0 / (3 * n // 2),
                         250.0, 500.0, 5)
        views = [0, 2, 4]
        ball = [syn.Ellipsoid(np.zeros(3), np.full(3, 7.0), np.eye(3), 1.0)]
        xb = syn.voxelize_ellipsoids(g, ball, sub=4)
        yb = orc.forward(g, xb, views)
        rb = syn.ball_line_integrals(g, views, 7.0)
        errs_ball.append(float(np.linalg.norm((yb - rb).ravel()) / np.linalg.norm(rb.ravel())))
        ells = syn.random_ellipsoids(g, 6, seed=11)
        xe = syn.voxelize_ellipsoids(g, ells, sub=4)
        ye = orc.forward(g, xe, views)
        re = syn.ellipsoid_line_integrals(g, ells, views)
        errs_ell.append(float(np.linalg.norm((ye - re).ravel()) / np.linalg.norm(re.ravel())))
    for errs in (errs_ball, errs_ell):
        assert errs[-1] < 0.1, errs
        assert errs[1] < 0.8 * errs[0] and errs[2] < 0.8 * errs[1], errs


def test_ball_projection_is_view_independent(orc):
    g = syn.Geometry(32, 32, 32, 1.0, 1.0, 1.0, 40, 40, 1.2, 1.2, 250.0, 500.0, 8)
    ball = [syn.Ellipsoid(np.zeros(3), np.full(3, 9.0), np.eye(3), 1.0)]
    x = syn.voxelize_ellipsoids(g, ball, sub=4)
    # views 0, 2, 4, 6 are multiples of 90 degrees: the cube's symmetry makes them equal
    y = orc.forward(g, x, [0, 2, 4, 6])
    for b in range(1, 4):
        assert np.allclose(y[b], y[0], rtol=0, atol=1e-9 * y.max())


def test_explicit_matrix_transpose_8cubed(orc):
    # Brute force: A assembled by forward projection of unit voxels equals the
    # transpose of A^T assembled by backprojection of unit rays, entry by entry.
    g = syn.tiny_geometry(n=8, det=12, views=16)
    views = np.arange(16)
    A = orc.assemble_matrix(g, views)
    AT = orc.assemble_matrix_transpose(g, views)
    assert A.shape == (16 * 144, 512)
    assert np.max(np.abs(A - AT.T)) <= 1e-14 * np.abs(A).max()
    # every voxel is seen by some ray of this geometry
    assert np.all(np.abs(A).sum(axis=0) > 0)
    # spot-check matrix_entry
    rng = np.random.default_rng(0)
    for _ in range(50):
        row = int(rng.integers(0, A.shape[0]))
        col = int(rng.integers(0, 512))
        b, p = divmod(row, 144)
        iv, iu = divmod(p, 12)
        assert orc.matrix_entry(g, int(views[b]), iu, iv, col) == pytest.approx(A[row, col], abs=1e-15)


def test_adjoint_identity_odd_sizes(orc):
    g = syn.Geometry(29, 41, 37, 0.9, 1.1, 1.0, 50, 33, 1.7, 1.9, 400.0, 900.0, 9,
                     angles=[0.0, np.pi / 4, np.pi / 2, np.pi, 0.3, 1.7, 2.9, 4.0, 5.5])
    rng = np.random.default_rng(7)
    x = rng.standard_normal(g.vol_shape)
    views = np.array([0, 1, 2, 3, 6, 8])
    yr = rng.standard_normal((len(views), g.nv, g.nu))
    lhs = float(np.dot(orc.forward(g, x, views).ravel(), yr.ravel()))
    rhs = float(np.dot(x.ravel(), orc.backproject(g, yr, views).ravel()))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_voxel_evaluator_matches_scatter(orc):
    g = syn.Geometry(13, 11, 9, 1.0, 1.0, 1.0, 20, 16, 1.5, 1.5, 300.0, 600.0, 10)
    rng = np.random.default_rng(5)
    views = np.array([1, 4, 7, 9])
    r = rng.standard_normal((len(views), g.nv, g.nu))
    full = orc.backproject(g, r, views).ravel()
    vox = rng.choice(g.d, 60, replace=False)
    part = orc.backproject_voxels(g, r, views, vox)
    assert np.allclose(part, full[vox], rtol=1e-12, atol=1e-12 * np.abs(full).max())


def test_ray_subset_matches_full(orc):
    g = syn.Geometry(13, 11, 9, 1.0, 1.0, 1.0, 20, 16, 1.5, 1.5, 300.0, 600.0, 10)
    x = syn.random_volume(g, 1).astype(np.float64)
    views = np.array([2, 3, 8])
    y = orc.forward(g, x, views)
    rays = np.array([[b, iv, iu] for b in range(3) for iv in (0, 5, 15) for iu in (0, 7, 19)])
    rays_v = rays.copy()
    rays_v[:, 0] = views[rays[:, 0]]
    vals = orc.forward_rays(g, x, rays_v)
    assert np.allclose(vals, y[rays[:, 0], rays[:, 1], rays[:, 2]], rtol=0, atol=0)


def test_dominant_axis_rule(orc):
    g = syn.Geometry(16, 16, 16, 1.0, 1.0, 1.0, 24, 24, 1.0, 1.0, 200.0, 400.0, 4)
    assert np.all(orc.dominant_axes(g, 0) == 0)     # theta = 0: rays along -x
    assert np.all(orc.dominant_axes(g, 1) == 1)     # theta = pi/2: rays along -y
    # a huge cone angle makes the outer rows z-dominant
    wide = syn.Geometry(16, 16, 16, 1.0, 1.0, 1.0, 4, 64, 1.0, 20.0, 200.0, 400.0, 4)
    ax = orc.dominant_axes(wide, 0)
    assert (ax == 2).any() and (ax == 0).any()
    assert np.all(ax[0] == 2) and np.all(ax[wide.nv // 2] == 0)


def test_dominant_axis_exact_ties_go_to_lowest_axis(orc):
    # theta = 0, SOD 4, SDD 8 and a column with u = SDD: q - s = (-8, 8, v), an exact
    # |D_x| = |D_y| tie, which the convention resolves to x.  A row with |v| = 8 ties
    # all three axes.  Every other ray is compared with numpy's first-maximum argmax.
    g = syn.Geometry(2, 2, 2, 1.0, 1.0, 1.0, 3, 3, 8.0, 8.0, 4.0, 8.0, 1, angles=[0.0])
    ax = orc.dominant_axes(g, 0)
    src, pix = syn.ray_endpoints(g, [0])
    D = (pix[0] - src[0][None, None, :]) / np.array([g.hx, g.hy, g.hz])
    assert abs(D[1, 2, 0]) == abs(D[1, 2, 1])        # the constructed tie
    assert abs(D[2, 2, 0]) == abs(D[2, 2, 2])
    expect = np.argmax(np.abs(D), axis=-1)
    assert np.array_equal(ax, expect)
    assert ax[1, 2] == 0 and ax[2, 2] == 0
    # centre column, outer rows: |D_x| = 8 = |D_z|, again resolved to x
    assert abs(D[2, 1, 0]) == abs(D[2, 1, 2]) and ax[2, 1] == 0 and ax[0, 1] == 0
