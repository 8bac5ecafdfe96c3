"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module produces *inputs* only: scan geometries, ellipsoid phantoms, their
exact (continuous-object) line integrals, measurement noise and the random view
draws of the stochastic method.  It holds none of the method's arithmetic: no
discretised projector, no gradient, no prox and no line search.  Both the FP64
oracle and the HIP path consume what it returns, and neither is imported here.

Geometry convention (circular cone beam, z is the rotation axis, millimetres):
  * voxel (i, j, k) has its centre at ((i-(nx-1)/2)hx, (j-(ny-1)/2)hy, (k-(nz-1)/2)hz),
    linear index i + nx*(j + ny*k), i.e. a C array [nz][ny][nx];
  * view j has angle theta_j (default 2*pi*j/n_views, uniform over [0, 2*pi) as in
    the paper's experimental section);
  * source s = SOD*(cos t, sin t, 0); detector centre (SOD-SDD)*(cos t, sin t, 0);
    detector axes e_u = (-sin t, cos t, 0), e_v = (0, 0, 1);
  * pixel (iu, iv) has its centre at c + (iu-(nu-1)/2)du e_u + (iv-(nv-1)/2)dv e_v,
    projections are stored [view][nv][nu];
  * one ray per pixel, from the source to the pixel centre.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Geometry", "Ellipsoid", "CONFIGS", "config_geometry", "tiny_geometry",
    "random_ellipsoids", "voxelize_ellipsoids", "ellipsoid_line_integrals",
    "ball_line_integrals", "gaussian_line_integrals", "gaussian_volume",
    "ray_endpoints", "add_noise", "view_permutations", "random_volume",
    "random_projections", "fov_radius",
]


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    nu: int
    nv: int
    du: float
    dv: float
    sod: float
    sdd: float
    n_views: int
    angles: Optional[np.ndarray] = field(default=None, compare=False)

    def __post_init__(self):
        if self.angles is None:
            a = 2.0 * np.pi * np.arange(self.n_views, dtype=np.float64) / float(self.n_views)
            object.__setattr__(self, "angles", a)
        else:
            a = np.ascontiguousarray(np.asarray(self.angles, dtype=np.float64))
            if a.shape != (self.n_views,):
                raise ValueError("angles must have n_views entries")
            object.__setattr__(self, "angles", a)

    @property
    def d(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_p(self) -> int:
        return self.nu * self.nv

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    def proj_shape(self, n_views: Optional[int] = None):
        return (self.n_views if n_views is None else n_views, self.nv, self.nu)

    def with_angles(self, angles) -> "Geometry":
        angles = np.asarray(angles, dtype=np.float64)
        return replace(self, n_views=int(angles.shape[0]), angles=angles)


@dataclass(frozen=True)
class Ellipsoid:
    center: np.ndarray  # (3,) mm
    axes: np.ndarray    # (3,) semi-axes, mm
    rot: np.ndarray     # (3,3); columns are the ellipsoid's principal directions
    rho: float          # attenuation, 1/mm


# Physical extents shared by every configuration: a 64 mm cube, a 96 mm square
# detector, SOD 500 mm and SDD 1000 mm; voxel and pixel sizes scale with the
# counts so that line integrals keep their magnitude across configurations.
_VOL_MM = 64.0
_DET_MM = 96.0
_SOD = 500.0
_SDD = 1000.0

CONFIGS = {
    # name: (N voxels per side, views, detector pixels per side, batch, epochs, lo, hi, K ellipsoids)
    "c1": dict(n=64, views=60, det=96, batch=6, epochs=10, lo=0.0, hi=math.inf, k=10),
    "c2": dict(n=256, views=360, det=384, batch=20, epochs=20, lo=0.0, hi=0.03, k=30),
    "c3": dict(n=512, views=720, det=768, batch=40, epochs=1, lo=0.0, hi=math.inf, k=30),
    "c4": dict(n=128, views=180, det=192, batch=10, epochs=10, lo=0.0, hi=math.inf, k=10),
    "c5": dict(n=1024, views=1440, det=1536, batch=40, epochs=10, lo=0.0, hi=math.inf, k=30),
}


def config_geometry(name: str) -> Geometry:
    c = CONFIGS[name]
    n, det = c["n"], c["det"]
    h = _VOL_MM / n
    p = _DET_MM / det
    return Geometry(n, n, n, h, h, h, det, det, p, p, _SOD, _SDD, c["views"])


def tiny_geometry(n=8, det=12, views=16, h=1.0, du=None, sod=_SOD, sdd=_SDD, angles=None,
                  nx=None, ny=None, nz=None, nu=None, nv=None) -> Geometry:
    """A small geometry whose detector sees the whole volume (used for explicit-A work)."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    nu = det if nu is None else nu
    nv = det if nv is None else nv
    if du is None:
        # cover the volume's half-diagonal at the near face, magnified, plus margin
        half = 0.5 * math.sqrt((nx * h) ** 2 + (ny * h) ** 2 + (nz * h) ** 2)
        mag = sdd / (sod - half)
        du = 2.0 * half * mag * 1.05 / max(nu, nv)
    g = Geometry(nx, ny, nz, h, h, h, nu, nv, du, du, sod, sdd, views, angles)
    return g


def fov_radius(g: Geometry) -> float:
    """Radius of the ball in the central plane seen by every view."""
    half_u = 0.5 * g.nu * g.du
    return g.sod * math.sin(math.atan(half_u / g.sdd))


# ----------------------------------------------------------------------------------
# ray endpoints (for the analytic references only)
# ----------------------------------------------------------------------------------

def ray_endpoints(g: Geometry, views: Sequence[int]):
    """Source (B,3) and pixel centres (B,nv,nu,3) in mm for the listed views."""
    views = np.asarray(views, dtype=np.int64)
    th = g.angles[views]
    c, s = np.cos(th), np.sin(th)
    src = np.stack([g.sod * c, g.sod * s, np.zeros_like(c)], axis=-1)
    u = (np.arange(g.nu, dtype=np.float64) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv, dtype=np.float64) - 0.5 * (g.nv - 1)) * g.dv
    dc = g.sod - g.sdd
    qx = dc * c[:, None, None] + u[None, None, :] * (-s)[:, None, None]
    qy = dc * s[:, None, None] + u[None, None, :] * c[:, None, None]
    qz = np.broadcast_to(v[None, :, None], (len(views), g.nv, g.nu))
    qx = np.broadcast_to(qx, (len(views), g.nv, g.nu))
    qy = np.broadcast_to(qy, (len(views), g.nv, g.nu))
    pix = np.stack([qx, qy, qz], axis=-1)
    return src, pix


# ----------------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_ellipsoids(g: Geometry, k: int, seed: int, rho_max: float = 0.02) -> List[Ellipsoid]:
    """k seeded random ellipsoids inside 0.95 of the field-of-view ball."""
    rng = np.random.default_rng(seed)
    R = 0.95 * fov_radius(g)
    out = []
    for _ in range(k):
        w = rng.standard_normal(3)
        w /= np.linalg.norm(w)
        c = 0.5 * R * rng.uniform() ** (1.0 / 3.0) * w
        a = rng.uniform(0.1 * R, 0.45 * R, size=3)
        reach = np.linalg.norm(c) + a.max()
        if reach > R:
            a = a * (R - np.linalg.norm(c)) / a.max()
        rot = _random_rotation(rng)
        rho = float(rng.uniform(0.0, rho_max))
        out.append(Ellipsoid(c, a, rot, rho))
    return out


def _voxel_centres_1d(n, h):
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * h


def voxelize_ellipsoids(g: Geometry, ells: Sequence[Ellipsoid], sub: int = 4,
                        hi: float = math.inf) -> np.ndarray:
    """x_true = sum of rho * (fraction of sub^3 sub-samples inside), FP64 [nz][ny][nx].

    If the sum exceeds the box bound ``hi`` somewhere, every density is scaled by
    hi / max so that the phantom is feasible for the box prox.
    """
    x = np.zeros(g.vol_shape, dtype=np.float64)
    cx, cy, cz = (_voxel_centres_1d(g.nx, g.hx), _voxel_centres_1d(g.ny, g.hy),
                  _voxel_centres_1d(g.nz, g.hz))
    offs = (np.arange(sub, dtype=np.float64) + 0.5) / sub - 0.5
    for e in ells:
        # axis-aligned half extent of the ellipsoid
        ext = np.sqrt(((e.rot * e.axes[None, :]) ** 2).sum(axis=1))
        lo = e.center - ext
        hi_ = e.center + ext
        ranges = []
        for cc, h, l, u in ((cx, g.hx, lo[0], hi_[0]), (cy, g.hy, lo[1], hi_[1]), (cz, g.hz, lo[2], hi_[2])):
            idx = np.nonzero((cc + 0.5 * h >= l) & (cc - 0.5 * h <= u))[0]
            ranges.append(idx)
        if any(len(r) == 0 for r in ranges):
            continue
        ix, iy, iz = ranges
        M = (e.rot / e.axes[None, :]).T  # maps (p - c) to the unit-sphere frame
        frac = np.zeros((len(iz), len(iy), len(ix)), dtype=np.float64)
        for oz in offs:
            pz = cz[iz] + oz * g.hz - e.center[2]
            for oy in offs:
                py = cy[iy] + oy * g.hy - e.center[1]
                for ox in offs:
                    px = cx[ix] + ox * g.hx - e.center[0]
                    u0 = M[0, 0] * px[None, None, :] + M[0, 1] * py[None, :, None] + M[0, 2] * pz[:, None, None]
                    u1 = M[1, 0] * px[None, None, :] + M[1, 1] * py[None, :, None] + M[1, 2] * pz[:, None, None]
                    u2 = M[2, 0] * px[None, None, :] + M[2, 1] * py[None, :, None] + M[2, 2] * pz[:, None, None]
                    frac += (u0 * u0 + u1 * u1 + u2 * u2) <= 1.0
        x[np.ix_(iz, iy, ix)] += e.rho * frac / sub ** 3
    if math.isfinite(hi):
        mx = x.max()
        if mx > hi:
            x *= hi / mx
    return x


def rescale_ellipsoids(ells: Sequence[Ellipsoid], factor: float) -> List[Ellipsoid]:
    return [Ellipsoid(e.center, e.axes, e.rot, e.rho * factor) for e in ells]


def phantom(g: Geometry, k: int, seed: int, hi: float = math.inf, sub: int = 4):
    """Seeded ellipsoid phantom: (ellipsoids, voxelised FP64 x_true), densities box-feasible."""
    ells = random_ellipsoids(g, k, seed)
    x = voxelize_ellipsoids(g, ells, sub=sub)
    if math.isfinite(hi) and x.max() > hi:
        f = hi / x.max()
        ells = rescale_ellipsoids(ells, f)
        x = x * f
    return ells, x


# ----------------------------------------------------------------------------------
# exact line integrals of continuous objects (independent of any discretisation)
# ----------------------------------------------------------------------------------

def ellipsoid_line_integrals(g: Geometry, ells: Sequence[Ellipsoid], views: Sequence[int]) -> np.ndarray:
    """Exact line integrals (FP64, [B][nv][nu]) of a sum of uniform ellipsoids.

    Each ray is solved as a quadratic in the ellipsoid's unit-sphere frame; the chord
    length in mm times rho is accumulated.  Rays are culled per view and ellipsoid to
    the detector rectangle covering the ellipsoid's bounding sphere.
    """
    views = np.asarray(views, dtype=np.int64)
    out = np.zeros((len(views), g.nv, g.nu), dtype=np.float64)
    u = (np.arange(g.nu, dtype=np.float64) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv, dtype=np.float64) - 0.5 * (g.nv - 1)) * g.dv
    for bi, vw in enumerate(views):
        th = g.angles[vw]
        c, s = math.cos(th), math.sin(th)
        src = np.array([g.sod * c, g.sod * s, 0.0])
        dc = g.sod - g.sdd
        nrm = np.array([c, s, 0.0])
        eu = np.array([-s, c, 0.0])
        for e in ells:
            rb = float(e.axes.max())
            # bounding-sphere footprint on the detector
            p = e.center - src
            dpar = -p @ nrm
            lat_u = p @ eu
            lat_v = p[2]
            if dpar - rb <= 0:
                iu0, iu1, iv0, iv1 = 0, g.nu, 0, g.nv
            else:
                mag_hi = g.sdd / (dpar - rb)
                umin = min((lat_u - rb) * g.sdd / (dpar - rb), (lat_u - rb) * g.sdd / (dpar + rb))
                umax = max((lat_u + rb) * g.sdd / (dpar - rb), (lat_u + rb) * g.sdd / (dpar + rb))
                vmin = min((lat_v - rb) * g.sdd / (dpar - rb), (lat_v - rb) * g.sdd / (dpar + rb))
                vmax = max((lat_v + rb) * g.sdd / (dpar - rb), (lat_v + rb) * g.sdd / (dpar + rb))
                del mag_hi
                iu0 = max(0, int(math.floor(umin / g.du + 0.5 * (g.nu - 1))) - 1)
                iu1 = min(g.nu, int(math.ceil(umax / g.du + 0.5 * (g.nu - 1))) + 2)
                iv0 = max(0, int(math.floor(vmin / g.dv + 0.5 * (g.nv - 1))) - 1)
                iv1 = min(g.nv, int(math.ceil(vmax / g.dv + 0.5 * (g.nv - 1))) + 2)
            if iu0 >= iu1 or iv0 >= iv1:
                continue
            uu = u[iu0:iu1]
            vv = v[iv0:iv1]
            qx = dc * c + uu * (-s)
            qy = dc * s + uu * c
            dx = np.broadcast_to((qx - src[0])[None, :], (len(vv), len(uu)))
            dy = np.broadcast_to((qy - src[1])[None, :], (len(vv), len(uu)))
            dz = np.broadcast_to((vv - src[2])[:, None], (len(vv), len(uu)))
            M = (e.rot / e.axes[None, :]).T
            o = M @ (src - e.center)
            d0 = M[0, 0] * dx + M[0, 1] * dy + M[0, 2] * dz
            d1 = M[1, 0] * dx + M[1, 1] * dy + M[1, 2] * dz
            d2 = M[2, 0] * dx + M[2, 1] * dy + M[2, 2] * dz
            A = d0 * d0 + d1 * d1 + d2 * d2
            Bq = 2.0 * (o[0] * d0 + o[1] * d1 + o[2] * d2)
            Cq = float(o @ o) - 1.0
            disc = Bq * Bq - 4.0 * A * Cq
            dt = np.sqrt(np.maximum(disc, 0.0)) / A
            length = dt * np.sqrt(dx * dx + dy * dy + dz * dz)
            out[bi, iv0:iv1, iu0:iu1] += e.rho * length
    return out



def ellipsoid_line_integrals_torch(g: Geometry, ells: Sequence[Ellipsoid], views: Sequence[int], device="cuda",
                                   out=None):
    """ellipsoid_line_integrals with torch on `device`, for data sets too large for the host
    loop (FP64, [B][nv][nu]; written into `out` when given, of any float dtype).

    The same FP64 operations in the same order, per view and ellipsoid, over the whole
    detector instead of the culled rectangle: a ray outside it misses the ellipsoid, its
    discriminant is not positive and it adds exactly zero.
    """
    import torch
    views = np.asarray(views, dtype=np.int64)
    f64 = torch.float64
    if out is None:
        out = torch.empty((len(views), g.nv, g.nu), dtype=f64, device=device)
    u = (torch.arange(g.nu, dtype=f64, device=device) - 0.5 * (g.nu - 1)) * g.du
    v = (torch.arange(g.nv, dtype=f64, device=device) - 0.5 * (g.nv - 1)) * g.dv
    dc = g.sod - g.sdd
    for bi, vw in enumerate(views):
        th = g.angles[vw]
        c, s = math.cos(th), math.sin(th)
        src = np.array([g.sod * c, g.sod * s, 0.0])
        qx = dc * c + u * (-s)
        qy = dc * s + u * c
        dx = (qx - src[0])[None, :].expand(g.nv, g.nu)
        dy = (qy - src[1])[None, :].expand(g.nv, g.nu)
        dz = (v - src[2])[:, None].expand(g.nv, g.nu)
        ray_len = torch.sqrt(dx * dx + dy * dy + dz * dz)
        acc = torch.zeros((g.nv, g.nu), dtype=f64, device=device)
        for e in ells:
            M = (e.rot / e.axes[None, :]).T
            o = M @ (src - e.center)
            d0 = M[0, 0] * dx + M[0, 1] * dy + M[0, 2] * dz
            d1 = M[1, 0] * dx + M[1, 1] * dy + M[1, 2] * dz
            d2 = M[2, 0] * dx + M[2, 1] * dy + M[2, 2] * dz
            A = d0 * d0 + d1 * d1 + d2 * d2
            Bq = 2.0 * (o[0] * d0 + o[1] * d1 + o[2] * d2)
            Cq = float(o @ o) - 1.0
            disc = Bq * Bq - 4.0 * A * Cq
            dt = torch.sqrt(torch.clamp(disc, min=0.0)) / A
            acc += e.rho * (dt * ray_len)
        out[bi] = acc
    return out


def add_noise_torch(y_clean, level: float, seed: int):
    """add_noise in place on a torch tensor on its own device, with torch's seeded generator
    (another random stream than add_noise's): y + sigma N(0, 1), sigma = level ||y|| / sqrt(n)."""
    import torch
    gen = torch.Generator(device=y_clean.device).manual_seed(seed)
    sigma = level * float(torch.linalg.vector_norm(y_clean.double())) / math.sqrt(y_clean.numel())
    for i in range(y_clean.shape[0]):   # one view at a time: no second full-size array
        y_clean[i].add_(torch.empty_like(y_clean[i]).normal_(generator=gen).mul_(sigma))
    return y_clean

def _ray_distance_to_point(g: Geometry, views, point):
    src, pix = ray_endpoints(g, views)
    d = pix - src[:, None, None, :]
    dn = d / np.linalg.norm(d, axis=-1, keepdims=True)
    w = point[None, None, None, :] - src[:, None, None, :]
    proj = (w * dn).sum(-1, keepdims=True)
    perp = w - proj * dn
    return np.linalg.norm(perp, axis=-1)


def ball_line_integrals(g: Geometry, views, radius: float, rho: float = 1.0,
                        center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Exact chord lengths times rho through a uniform ball."""
    dist = _ray_distance_to_point(g, views, np.asarray(center, dtype=np.float64))
    return rho * 2.0 * np.sqrt(np.maximum(radius * radius - dist * dist, 0.0))


def gaussian_volume(g: Geometry, sigma: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Isotropic unit-peak Gaussian blob sampled at voxel centres (FP64)."""
    cx = _voxel_centres_1d(g.nx, g.hx) - center[0]
    cy = _voxel_centres_1d(g.ny, g.hy) - center[1]
    cz = _voxel_centres_1d(g.nz, g.hz) - center[2]
    r2 = cx[None, None, :] ** 2 + cy[None, :, None] ** 2 + cz[:, None, None] ** 2
    return np.exp(-r2 / (2.0 * sigma * sigma))


def gaussian_line_integrals(g: Geometry, views, sigma: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Line integral of exp(-|p-c|^2/(2 sigma^2)) along each ray: sigma sqrt(2 pi) exp(-d^2/(2 sigma^2))."""
    dist = _ray_distance_to_point(g, views, np.asarray(center, dtype=np.float64))
    return sigma * math.sqrt(2.0 * math.pi) * np.exp(-dist * dist / (2.0 * sigma * sigma))


# ----------------------------------------------------------------------------------
# noise, random draws, random test tensors
# ----------------------------------------------------------------------------------

def add_noise(y_clean: np.ndarray, level: float, seed: int) -> np.ndarray:
    """b = y + sigma * N(0, 1), sigma = level * ||y||_2 / sqrt(n) (negative b allowed)."""
    rng = np.random.default_rng(seed)
    sigma = level * float(np.linalg.norm(y_clean.ravel())) / math.sqrt(y_clean.size)
    return y_clean + sigma * rng.standard_normal(y_clean.shape)


def view_permutations(n_views: int, n_iters: int, seed: int) -> np.ndarray:
    """One uniform random permutation of the views per iteration, int32 [n_iters][n_views].

    The method's mini-batch at iteration k of size N is the first N entries of row k:
    a uniform draw of N distinct view indices, independent across iterations.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n_iters, n_views), dtype=np.int32)
    for k in range(n_iters):
        out[k] = rng.permutation(n_views)
    return out


def random_volume(g: Geometry, seed: int, lo=0.0, hi=0.02, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=g.vol_shape).astype(dtype)


def random_projections(g: Geometry, n: int, seed: int, scale=1.0, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal((n, g.nv, g.nu))).astype(dtype)


def mlp_params(seed: int, n_in: int = 5, n_hidden: int = 64) -> np.ndarray:
    """Seeded initial parameters of the step-proposal perceptron, flat FP32 in the order
    W1[h][n_in], b1[h], W2[h][h], b2[h], w3[h], b3: weights uniform in +-sqrt(6/fan_in),
    biases zero."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (n_hidden, n_in)) * math.sqrt(6.0 / n_in), np.zeros(n_hidden),
             rng.uniform(-1, 1, (n_hidden, n_hidden)) * math.sqrt(6.0 / n_hidden), np.zeros(n_hidden),
             rng.uniform(-1, 1, n_hidden) * math.sqrt(6.0 / n_hidden), np.zeros(1)]
    return np.concatenate([q.ravel() for q in parts]).astype(np.float32)

