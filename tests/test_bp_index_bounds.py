"""CPU replay of the backprojection kernel's index arithmetic (bp_kernel in
csrc/backproject.hip): for every test and workload geometry, the per-tile detector column
ranges, pair-table slots, residual row windows, staging addresses and fallback addresses
the kernel forms, with its FP32 arithmetic emulated in numpy.

Checked:
  * no slice of a tile needs more detector columns than the kernel's pair table holds
    (the kernel clamps to that size, which would drop pairs silently);
  * every detector column whose ray plane meets the tile's slice within one voxel is
    among the slice's pairs;
  * every detector row with nonzero weight on a half tile lies inside the staged row
    window of that half;
  * every staged or fallback residual address lies inside the view's residual rows;
  * each voxel column's gather range is exactly the run of its slice's pairs within one
    voxel of it;
  * an empty (slice, column) pass is skipped before any window is formed.
The larger workloads are checked on tiles sampled at the corners, the centre and the top
and bottom of the volume, where the row windows are tallest."""
import math

import numpy as np
import pytest

import synthetic as syn

TQ, TK, KH = 16, 16, 8          # tile extents and z-entries per half pass (kernel constants)
WIN_ROWS, WIN_EXTRA = 28, 16    # staged rows per column; extra window columns over the pair table
COL_TOL = 0.01                  # the kernel's tolerance on computed detector columns
F32 = np.float32


def _columns(g):
    """FP64 ray parameters of every (view, column), as the plan forms them on the host."""
    th = np.asarray(g.angles, dtype=np.float64)[:, None]
    c, s = np.cos(th), np.sin(th)
    u = (np.arange(g.nu, dtype=np.float64)[None, :] - 0.5 * (g.nu - 1)) * g.du
    dc = g.sod - g.sdd
    sx, sy = g.sod * c, g.sod * s
    qx, qy = dc * c + u * (-s), dc * s + u * c
    P = [sx / g.hx + 0.5 * (g.nx - 1), sy / g.hy + 0.5 * (g.ny - 1)]
    D = [(qx - sx) / g.hx, (qy - sy) / g.hy]
    P = [np.broadcast_to(P[0], D[0].shape), np.broadcast_to(P[1], D[1].shape)]
    axis = np.where(np.abs(D[0]) >= np.abs(D[1]), 0, 1)
    Pa, Pb = np.where(axis == 0, P[0], P[1]), np.where(axis == 0, P[1], P[0])
    Da, Db = np.where(axis == 0, D[0], D[1]), np.where(axis == 0, D[1], D[0])
    t1, t0 = 1.0 / Da, -Pa / Da
    r = Db / Da
    return dict(axis=axis, t0=t0, t1=t1, xi0=Pb - Pa * r, xi1=r, Pa=Pa, Da=Da)


def _plan_sizes(g, cols):
    """The plan's pair-table width WP and the per-view axis split, from its host rules."""
    axis = cols["axis"]
    split = np.full(g.n_views, g.nu)
    for v in range(g.n_views):
        ch = np.nonzero(axis[v, 1:] != axis[v, :-1])[0]
        assert len(ch) <= 1
        if len(ch):
            split[v] = ch[0] + 1
    return split


def _col_of(g, c, s, X, Y):
    lat = (-X * s + Y * c).astype(F32)
    dep = (F32(g.sod) - (X * c + Y * s)).astype(F32)
    return (F32(g.sdd) * lat * (F32(1.0) / (dep * F32(g.du))) + F32(0.5 * (g.nu - 1))).astype(F32)


def _wp_of_plan(g, cols, split):
    """Plan: the largest number of columns crossing one slice of a tile, over every view,
    class, slice and in-slice tile position, plus two columns of margin, rounded up to
    32, 48 or 64."""
    cxv, cyv = F32(0.5 * (g.nx - 1)), F32(0.5 * (g.ny - 1))
    max_n = 0
    for v in range(g.n_views):
        c, s = F32(math.cos(g.angles[v])), F32(math.sin(g.angles[v]))
        a0 = cols["axis"][v, 0]
        for cls in range(2):
            axis = a0 if cls == 0 else 1 - a0
            cl0, cl1 = (0, split[v] - 1) if cls == 0 else (split[v], g.nu - 1)
            if cl0 > cl1:
                continue
            na, nq = (g.nx, g.ny) if axis == 0 else (g.ny, g.nx)
            q0 = np.arange(0, nq, TQ)[:, None].astype(F32)
            fm = np.arange(na)[None, :].astype(F32)
            if axis == 0:
                X = ((fm - cxv) * F32(g.hx)).astype(F32)
                u0 = _col_of(g, c, s, X, ((q0 - 1 - cyv) * F32(g.hy)).astype(F32))
                u1 = _col_of(g, c, s, X, ((q0 + TQ - cyv) * F32(g.hy)).astype(F32))
            else:
                Y = ((fm - cyv) * F32(g.hy)).astype(F32)
                u0 = _col_of(g, c, s, ((q0 - 1 - cxv) * F32(g.hx)).astype(F32), Y)
                u1 = _col_of(g, c, s, ((q0 + TQ - cxv) * F32(g.hx)).astype(F32), Y)
            a = np.maximum(cl0, np.floor(np.minimum(u0, u1)).astype(np.int64) - 1)
            b = np.minimum(cl1, np.ceil(np.maximum(u0, u1)).astype(np.int64) + 1)
            max_n = max(max_n, int((b - a + 1).max()))
    need = max_n + 2
    return next((sz for sz in (32, 48, 64) if need <= sz), None)


def _check_gather_ranges(g, cols, v, c, s, axis, ms, q0, a, n, cxv, cyv, stats):
    """Each voxel column (slice m, in-slice index q) gathers the pairs of slice m between
    the floor and the ceiling of the detector columns through (m, q - 1) and (m, q + 1),
    clamped to the slice's range, after dropping up to two columns at either end whose
    stored xi (FP32) lies a voxel or more from q.  Checked: the valid pairs (|xi - q| < 1)
    form one run inside the candidate range with at most two spare columns at either end,
    so the kernel's range is exactly that run."""
    q = np.arange(TQ, dtype=F32)[None, :]
    fm = ms.astype(F32)[:, None]
    lo_q = ((F32(q0 - 1) + q) - (cyv if axis == 0 else cxv)).astype(F32)
    hi_q = ((F32(q0 + 1) + q) - (cyv if axis == 0 else cxv)).astype(F32)
    if axis == 0:
        X = np.broadcast_to(((fm - cxv) * F32(g.hx)).astype(F32), (len(ms), TQ))
        u0 = _col_of(g, c, s, X, np.broadcast_to((lo_q * F32(g.hy)).astype(F32), X.shape))
        u1 = _col_of(g, c, s, X, np.broadcast_to((hi_q * F32(g.hy)).astype(F32), X.shape))
    else:
        Y = np.broadcast_to(((fm - cyv) * F32(g.hy)).astype(F32), (len(ms), TQ))
        u0 = _col_of(g, c, s, np.broadcast_to((lo_q * F32(g.hx)).astype(F32), Y.shape), Y)
        u1 = _col_of(g, c, s, np.broadcast_to((hi_q * F32(g.hx)).astype(F32), Y.shape), Y)
    f = np.maximum(a[:, None], np.floor(np.maximum(np.minimum(u0, u1), -4.0)).astype(np.int64))
    l = np.minimum((a + n - 1)[:, None], np.ceil(np.minimum(np.maximum(u0, u1), g.nu + 4.0)).astype(np.int64))
    for im, m in enumerate(ms):
        if n[im] == 0:
            assert np.all(f[im] > l[im])
            continue
        cc = np.arange(a[im], a[im] + n[im])
        xi = (cols["xi0"][v, cc] + float(m) * cols["xi1"][v, cc] - q0).astype(F32)
        valid = np.abs(xi[None, :] - np.arange(TQ, dtype=F32)[:, None]) < F32(1.0)   # [q][column]
        cnt = valid.sum(axis=1)
        none = cnt == 0
        assert np.all(l[im][none] - f[im][none] + 1 <= 4), (v, m)
        first = cc[np.argmax(valid, axis=1)]
        last = cc[n[im] - 1 - np.argmax(valid[:, ::-1], axis=1)]
        some = ~none
        assert np.all((last - first + 1)[some] == cnt[some]), (v, m)             # one run
        assert np.all(f[im][some] <= first[some]) and np.all(l[im][some] >= last[some]), (v, m)
        spare = np.maximum(first - f[im], l[im] - last)[some]
        if spare.size:
            assert spare.max() <= 2, (v, m, int(spare.max()))
            stats["gather_spare_max"] = max(stats.get("gather_spare_max", 0), int(spare.max()))


def _check_tiles(g, cols, split, WP, tiles, views, check_cover=True):
    """Replay bp_kernel's set-up for the given tiles (list of (i0, j0, k0)) and views."""
    cxv, cyv = F32(0.5 * (g.nx - 1)), F32(0.5 * (g.ny - 1))
    cz, cv = 0.5 * (g.nz - 1), F32(0.5 * (g.nv - 1))
    dvz = g.dv / g.hz
    npix = g.nu * g.nv
    stats = {"passes": 0, "staged": 0, "fallback": 0, "skipped_empty": 0}
    gathered = set()
    for bi, v in enumerate(views):
        c, s = F32(math.cos(g.angles[v])), F32(math.sin(g.angles[v]))
        a0 = cols["axis"][v, 0]
        for (i0, j0, k0) in tiles:
            corners = []
            for q in range(4):
                X = F32((i0 + TQ if q & 1 else i0 - 1) - cxv) * F32(g.hx)
                Y = F32((j0 + TQ if q & 2 else j0 - 1) - cyv) * F32(g.hy)
                corners.append(float(_col_of(g, c, s, np.asarray(X, F32), np.asarray(Y, F32))))
            umin, umax = min(corners), max(corners)
            cT0 = max(0, int(math.floor(max(umin, -4.0))) - 1)
            cT1 = min(g.nu - 1, int(math.ceil(min(umax, g.nu + 4.0))) + 1)
            if cT0 > cT1:
                continue
            # the view is skipped when no detector row within two of the detector reaches the
            # tile's z-range at any depth of the grown square: check that none really does
            deps = []
            for q in range(4):
                X = F32((i0 + TQ if q & 1 else i0 - 1) - cxv) * F32(g.hx)
                Y = F32((j0 + TQ if q & 2 else j0 - 1) - cyv) * F32(g.hy)
                deps.append(float(F32(g.sod) - (X * c + Y * s)))
            e0, e1 = F32(k0 - 1 - cz), F32(k0 + TK - cz)
            sc = [F32(g.sdd) / (F32(d) * F32(dvz)) for d in (min(deps), max(deps))]
            cand = [e * t for e in (e0, e1) for t in sc]
            if min(cand) + cv > g.nv + 1 or max(cand) + cv < -2:
                stats["skipped_z"] = stats.get("skipped_z", 0) + 1
                for cls in range(2):
                    ax = a0 if cls == 0 else 1 - a0
                    lo_c = cT0 if cls == 0 else max(cT0, split[v])
                    hi_c = min(cT1, split[v] - 1) if cls == 0 else cT1
                    if lo_c > hi_c:
                        continue
                    cc = np.arange(lo_c, hi_c + 1)
                    na_ = g.nx if ax == 0 else g.ny
                    mt = i0 if ax == 0 else j0
                    ms_ = np.arange(mt, min(mt + TQ, na_))
                    qt = j0 if ax == 0 else i0
                    # only (slice, column) pairs whose column crosses the tile
                    xi = cols["xi0"][v, cc][None, :] + ms_[:, None] * cols["xi1"][v, cc][None, :] - qt
                    crosses = (xi > -1.0) & (xi < TQ)
                    tau = ms_[:, None] * cols["t1"][v, cc][None, :] + cols["t0"][v, cc][None, :]
                    r_a = (k0 - 1 - cz) / (tau * dvz) + (g.nv - 1) / 2.0
                    r_b = (min(k0 + TK, g.nz) - cz) / (tau * dvz) + (g.nv - 1) / 2.0
                    first = np.maximum(np.floor(np.minimum(r_a, r_b)) + 1, 0)
                    last = np.minimum(np.ceil(np.maximum(r_a, r_b)) - 1, g.nv - 1)
                    assert np.all((first > last) | ~crosses), (v, i0, j0, k0)
                continue
            for cls in range(2):
                axis = a0 if cls == 0 else 1 - a0
                cl0 = cT0 if cls == 0 else max(cT0, split[v])
                cl1 = min(cT1, split[v] - 1) if cls == 0 else cT1
                if cl0 > cl1:
                    continue
                na = g.nx if axis == 0 else g.ny
                mt0, q0 = (i0, j0) if axis == 0 else (j0, i0)
                ms = np.arange(mt0, min(mt0 + TQ, na))
                fm = ms.astype(F32)
                if axis == 0:
                    X = ((fm - cxv) * F32(g.hx)).astype(F32)
                    u0 = _col_of(g, c, s, X, np.full_like(X, F32(q0 - 1 - cyv) * F32(g.hy)))
                    u1 = _col_of(g, c, s, X, np.full_like(X, F32(q0 + TQ - cyv) * F32(g.hy)))
                else:
                    Y = ((fm - cyv) * F32(g.hy)).astype(F32)
                    u0 = _col_of(g, c, s, np.full_like(Y, F32(q0 - 1 - cxv) * F32(g.hx)), Y)
                    u1 = _col_of(g, c, s, np.full_like(Y, F32(q0 + TQ - cxv) * F32(g.hx)), Y)
                lo, hi = np.minimum(u0, u1), np.maximum(u0, u1)
                a = np.maximum(cl0, np.floor(np.maximum(lo, F32(-4.0)) - F32(COL_TOL)).astype(np.int64) + 1)
                b = np.minimum(cl1, np.ceil(np.minimum(hi, F32(g.nu + 4.0)) + F32(COL_TOL)).astype(np.int64) - 1)
                # the table holds WP pairs per slice: a wider range would be cut silently
                assert np.all(b - a + 1 <= WP), (v, i0, j0, k0, int((b - a + 1).max()), WP)
                n = np.minimum(WP, np.maximum(0, b - a + 1))
                if not np.any(n > 0):
                    stats["skipped_empty"] += 1      # the kernel continues before any window
                    continue
                c0 = int(a[n > 0].min())
                c1 = int((a + n - 1)[n > 0].max())
                nC = c1 - c0 + 1
                stats["passes"] += 1
                # columns whose plane meets a slice within one voxel of the tile are pairs
                if check_cover:
                    cc = np.arange(cl0, cl1 + 1)
                    xi = cols["xi0"][v, cc][None, :] + ms[:, None] * cols["xi1"][v, cc][None, :] - q0
                    near = (xi > -1.0) & (xi < TQ)
                    inside = (cc[None, :] >= a[:, None]) & (cc[None, :] < (a + n)[:, None])
                    assert np.all(inside | ~near), (v, i0, j0, k0)
                    if (v, i0, j0, cls) not in gathered:   # the gather ranges do not depend on z
                        gathered.add((v, i0, j0, cls))
                        _check_gather_ranges(g, cols, v, c, s, axis, ms, q0, a, n, cxv, cyv, stats)
                # row windows of the two halves, from the class's outermost columns
                mA, mB = float(mt0), float(min(mt0 + TQ - 1, na - 1))
                ts = [mA * cols["t1"][v, cl] + cols["t0"][v, cl] for cl in (cl0, cl1)] + \
                     [mB * cols["t1"][v, cl] + cols["t0"][v, cl] for cl in (cl0, cl1)]
                imin = F32(1.0) / F32(max(ts) * dvz)
                imax = F32(1.0) / F32(min(ts) * dvz)
                for h in range(2):
                    kb = k0 + h * KH
                    if kb >= g.nz:
                        continue
                    e0, e1 = F32(kb - 1 - cz), F32(kb + KH - cz)
                    cand = [e0 * imin, e0 * imax, e1 * imin, e1 * imax]
                    rlo, rhi = min(cand) + cv, max(cand) + cv
                    r0 = max(0, int(math.floor(rlo)) - 1)
                    nR = min(g.nv - 1, int(math.ceil(rhi)) + 1) - r0 + 1
                    staged = 0 < nR <= WIN_ROWS and nC <= WP + WIN_EXTRA
                    if nR <= 0:
                        continue                      # no row reaches the half: no profiles
                    base = bi * npix
                    if staged:
                        stats["staged"] += 1
                        # staging reads rows r0 .. r0+nR-1 of columns c0 .. c1 (clamped)
                        lo_addr = base + r0 * g.nu + c0
                        hi_addr = base + (r0 + nR - 1) * g.nu + c1
                        assert base <= lo_addr and hi_addr < base + npix
                    else:
                        stats["fallback"] += 1
                        # the tap loop reads rows min(t, nv-1) of columns c0 + pcr in [c0, c1]
                        assert c0 >= 0 and c1 < g.nu
                    if not (check_cover and staged):
                        continue
                    # every row with nonzero weight on z in [kb, kb + KH) lies in the window:
                    # eta_r = cz + tau (r - cv) dvz within (kb - 1, kb + KH), for every column
                    # of the window [c0, c1] (each slice's pairs lie within it)
                    cc = np.arange(c0, c1 + 1)
                    tau = ms[:, None] * cols["t1"][v, cc][None, :] + cols["t0"][v, cc][None, :]
                    r_lo = (kb - 1 - cz) / (tau * dvz) + (g.nv - 1) / 2.0
                    r_hi = (min(kb + KH, g.nz) - cz) / (tau * dvz) + (g.nv - 1) / 2.0
                    first = np.maximum(np.floor(r_lo) + 1, 0)          # first row with eta > kb - 1
                    last = np.minimum(np.ceil(r_hi) - 1, g.nv - 1)     # last row with eta < kb + KH
                    need = first <= last
                    assert np.all(first[need] >= r0) and np.all(last[need] <= r0 + nR - 1), (v, i0, j0, k0, h)
    return stats


def _tiles_all(g):
    return [(i, j, k) for k in range(0, g.nz, TK) for j in range(0, g.ny, TQ) for i in range(0, g.nx, TQ)]


def _tiles_sampled(g, seed=0, n_random=24):
    ti, tj, tk = range(0, g.nx, TQ), range(0, g.ny, TQ), range(0, g.nz, TK)
    pick = set()
    for k in (tk[0], tk[1], tk[len(tk) // 2], tk[-2], tk[-1]):
        for i in (ti[0], ti[len(ti) // 2 - 1], ti[len(ti) // 2], ti[-1]):
            for j in (tj[0], tj[len(tj) // 2 - 1], tj[len(tj) // 2], tj[-1]):
                pick.add((i, j, k))
    rng = np.random.default_rng(seed)
    for _ in range(n_random):
        pick.add((int(rng.choice(ti)), int(rng.choice(tj)), int(rng.choice(tk))))
    return sorted(pick)


ODD = syn.Geometry(29, 41, 37, 0.9, 1.1, 1.0, 50, 33, 1.7, 1.9, 400.0, 900.0, 12,
                   angles=[0.0, np.pi / 4, np.pi / 2, np.pi, 3 * np.pi / 2, 0.3, 1.7, 2.9, 4.0, 5.5, 0.05, 6.2])

SMALL = {
    "odd": ODD,
    "fine_rows": syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 60, 1.5, 0.6, 300.0, 600.0, 12),
    "fine_columns": syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 77, 30, 0.7, 1.5, 300.0, 600.0, 8),
    "many_views": syn.Geometry(12, 10, 8, 1.0, 1.0, 1.0, 16, 12, 1.5, 1.5, 300.0, 600.0, 300),
    "coarse_rows_32": syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 12, 1.5, 3.2, 300.0, 600.0, 12),
    "coarse_rows_48": syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 12, 1.5, 4.8, 300.0, 600.0, 12),
    "axis_tie": syn.Geometry(20, 20, 4, 1.0, 1.0, 1.0, 5, 6, 18.0, 2.0, 18.0, 36.0, 1, angles=[0.0]),
    "smoke": syn.Geometry(24, 24, 20, 1.0, 1.0, 1.0, 36, 30, 1.5, 1.5, 300.0, 600.0, 24),
    "tiny8": syn.tiny_geometry(n=8, det=12, views=16),
    "c1": syn.config_geometry("c1"),
    "c4": syn.config_geometry("c4"),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_small_geometries_every_tile(name):
    g = SMALL[name]
    cols = _columns(g)
    split = _plan_sizes(g, cols)
    WP = _wp_of_plan(g, cols, split)
    assert WP is not None
    st = _check_tiles(g, cols, split, WP, _tiles_all(g), list(range(g.n_views)))
    assert st["passes"] > 0


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_workload_geometries_sampled_tiles(name):
    g = syn.config_geometry(name)
    cols = _columns(g)
    split = _plan_sizes(g, cols)
    WP = _wp_of_plan(g, cols, split)
    assert WP is not None
    B = syn.CONFIGS[name]["batch"]
    views = list(syn.view_permutations(g.n_views, 1, seed=1000 * int(name[1:]) + 2)[0][:B])
    views += [0, g.n_views // 8, g.n_views // 4, g.n_views // 2]     # axis-aligned and diagonal views
    st = _check_tiles(g, cols, split, WP, _tiles_sampled(g), views)
    assert st["staged"] > 0


def test_fine_rows_geometry_takes_the_fallback():
    # the fine-row geometry of the GPU tests really reaches the device-memory fallback
    g = SMALL["fine_rows"]
    cols = _columns(g)
    split = _plan_sizes(g, cols)
    st = _check_tiles(g, cols, split, _wp_of_plan(g, cols, split), _tiles_all(g), list(range(g.n_views)))
    assert st["fallback"] > 0 and st["staged"] > 0


def test_empty_passes_are_skipped():
    # a tile outside every ray plane of a view (the tie geometry's single view sees only a
    # band of the volume): the pass is skipped before a window is formed
    g = SMALL["axis_tie"]
    cols = _columns(g)
    split = _plan_sizes(g, cols)
    st = _check_tiles(g, cols, split, _wp_of_plan(g, cols, split), _tiles_all(g), [0])
    assert st["passes"] > 0
