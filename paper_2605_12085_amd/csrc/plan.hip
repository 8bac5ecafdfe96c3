// Host side of libfblisa: geometry validation, FP64 ray set-up into the plan's device
// tables, argument checks, and the C ABI declared in include/fblisa.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

using namespace fbl;

namespace {
thread_local std::string g_err;
}

namespace fbl {

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int clear_error()
{
    g_err.clear();
    return FBL_OK;
}

int check_step_buffers(const void *x, const float *g, double alpha, double mu, double lo, double hi, const void *xbar,
                       const double *red_dev)
{
    auto al16 = [](const void *q) { return ((uintptr_t)q & 15u) == 0; };
    if (!x || !g || !xbar || !red_dev) return set_error(FBL_E_INVALID, "x, g, xbar and red_dev must be non-NULL");
    if (!al16(x) || !al16(g) || !al16(xbar) || ((uintptr_t)red_dev & 7u) != 0)
        return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned and red_dev 8-byte aligned");
    if (xbar == x || (const void *)xbar == (const void *)g) return set_error(FBL_E_INVALID, "xbar may not alias x or g");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return set_error(FBL_E_INVALID, "alpha must be finite and > 0");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return set_error(FBL_E_INVALID, "mu must be finite and >= 0");
    if (!(lo >= 0.0) || !std::isfinite(lo) || !(hi >= lo))
        return set_error(FBL_E_INVALID, "bounds must satisfy 0 <= lo <= hi (lo finite)");
    return FBL_OK;
}

}  // namespace fbl

namespace {

int ok() { return clear_error(); }

int hip_fail(hipError_t e, const char *what)
{
    return set_error(FBL_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

double view_angle(const fbl_geometry &g, int64_t v)
{
    if (g.angles) return g.angles[v];
    return 2.0 * M_PI * (double)v / (double)g.n_views;
}

// FP64 ray geometry of one detector column, evaluated without fused multiply-adds in
// the order of the conventions (source, pixel centre, index coordinates P and D), so the
// dominant-axis decision is reproducible bit for bit.
#pragma clang fp contract(off)
struct ColumnGeom {
    double s[2], q[2];
    double P[2], D[2];
};

ColumnGeom column_geom(const fbl_geometry &g, int64_t v, int64_t iu)
{
    ColumnGeom cg;
    const double th = view_angle(g, v);
    const double c = std::cos(th), sn = std::sin(th);
    const double dc = g.sod - g.sdd;
    const double u = ((double)iu - 0.5 * (double)(g.nu - 1)) * g.du;
    cg.s[0] = g.sod * c;
    cg.s[1] = g.sod * sn;
    cg.q[0] = dc * c + u * (-sn);
    cg.q[1] = dc * sn + u * c;
    const double h[2] = {g.hx, g.hy};
    const int64_t n[2] = {g.nx, g.ny};
    for (int k = 0; k < 2; ++k) {
        cg.P[k] = cg.s[k] / h[k] + 0.5 * (double)(n[k] - 1);
        cg.D[k] = (cg.q[k] - cg.s[k]) / h[k];
    }
    return cg;
}

// Largest |D_z| over the detector rows: |(v - 0) / hz| with v the row centre height.
double max_abs_dz(const fbl_geometry &g)
{
    double m = 0.0;
    for (int64_t iv = 0; iv < g.nv; ++iv) {
        const double v = ((double)iv - 0.5 * (double)(g.nv - 1)) * g.dv;
        const double dz = std::fabs((v - 0.0) / g.hz);
        if (dz > m) m = dz;
    }
    return m;
}
#pragma clang fp contract(on)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_geometry(const fbl_geometry *g)
{
    if (!g) return set_error(FBL_E_INVALID, "geometry is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nu < 1 || g->nv < 1 || g->n_views < 1)
        return set_error(FBL_E_GEOMETRY, "every count must be >= 1 (nx=%lld ny=%lld nz=%lld nu=%lld nv=%lld n_views=%lld)",
                    (long long)g->nx, (long long)g->ny, (long long)g->nz, (long long)g->nu, (long long)g->nv,
                    (long long)g->n_views);
    if (g->nx < 2 || g->ny < 2)
        return set_error(FBL_E_GEOMETRY, "nx and ny must be >= 2 (the in-slice interpolation needs two taps)");
    if (g->nx > (1 << 24) || g->ny > (1 << 24) || g->nz > (1 << 24) || g->nu > (1 << 24) || g->nv > (1 << 24))
        return set_error(FBL_E_GEOMETRY, "a dimension exceeds 2^24");
    if ((double)g->nx * (double)g->ny * (double)g->nz >= 2147483648.0)
        return set_error(FBL_E_GEOMETRY, "nx*ny*nz must be below 2^31");
    if ((double)g->nu * (double)g->nv > 268435456.0) return set_error(FBL_E_GEOMETRY, "nu*nv must not exceed 2^28");
    if (g->n_views > (1 << 24)) return set_error(FBL_E_GEOMETRY, "n_views exceeds 2^24");
    if (!finite_pos(g->hx) || !finite_pos(g->hy) || !finite_pos(g->hz) || !finite_pos(g->du) || !finite_pos(g->dv))
        return set_error(FBL_E_GEOMETRY, "voxel and pixel sizes must be finite and positive");
    if (!finite_pos(g->sod) || !std::isfinite(g->sdd)) return set_error(FBL_E_GEOMETRY, "SOD must be finite and positive");
    if (!(g->sdd > g->sod)) return set_error(FBL_E_GEOMETRY, "SDD (%g) must exceed SOD (%g)", g->sdd, g->sod);
    // half-diagonal of the volume grown by two voxels on every side (the backprojection
    // projects points up to that far out)
    const double ex = 0.5 * (double)(g->nx + 4) * g->hx, ey = 0.5 * (double)(g->ny + 4) * g->hy,
                 ez = 0.5 * (double)(g->nz + 4) * g->hz;
    const double half = std::sqrt(ex * ex + ey * ey + ez * ez);
    if (!(g->sod > half) || !(g->sdd - g->sod > half))
        return set_error(FBL_E_GEOMETRY,
                    "the volume must lie strictly between source and detector: SOD=%g and SDD-SOD=%g must exceed "
                    "the padded half-diagonal %g",
                    g->sod, g->sdd - g->sod, half);
    if (g->angles)
        for (int64_t v = 0; v < g->n_views; ++v)
            if (!std::isfinite(g->angles[v])) return set_error(FBL_E_GEOMETRY, "angle %lld is not finite", (long long)v);
    const double dz = max_abs_dz(*g);
    for (int64_t v = 0; v < g->n_views; ++v)
        for (int64_t iu = 0; iu < g->nu; ++iu) {
            const ColumnGeom cg = column_geom(*g, v, iu);
            const double mxy = std::fmax(std::fabs(cg.D[0]), std::fabs(cg.D[1]));
            if (!(mxy >= dz))
                return set_error(FBL_E_GEOMETRY,
                            "view %lld column %lld has rays whose dominant axis is z (cone angle too large)",
                            (long long)v, (long long)iu);
        }
    return FBL_OK;
}

template <typename T>
int dev_upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
    if (e != hipSuccess) return set_error(FBL_E_NOMEM, "hipMalloc of %zu bytes: %s", src.size() * sizeof(T), hipGetErrorString(e));
    e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of plan table");
    return FBL_OK;
}

void free_plan(fbl_plan *p)
{
    if (!p) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (p->device >= 0 && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipFree(p->d_col);
    (void)hipFree(p->d_col64);
    (void)hipFree(p->d_rowV);
    (void)hipFree(p->d_rowV2);
    (void)hipFree(p->d_view);
    (void)hipFree(p->d_bp_order);
    (void)hipFree(p->d_partials);
    (void)hipFree(p->d_rw);
    (void)hipFree(p->d_xt);
    for (auto &t : p->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (hipEvent_t ev : p->event_pool) (void)hipEventDestroy(ev);
    if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
    delete[] p->angles_host;
    delete[] p->view_axis0;
    delete p;
}

int check_call(const fbl_plan *p, const int32_t *views, int32_t B)
{
    if (!p) return set_error(FBL_E_INVALID, "plan is NULL");
    if (!views) return set_error(FBL_E_INVALID, "views is NULL");
    if (B < 1 || B > p->max_batch)
        return set_error(FBL_E_RANGE, "batch size %d outside [1, %d]", (int)B, (int)p->max_batch);
    for (int32_t k = 0; k < B; ++k)
        if (views[k] < 0 || views[k] >= p->geom.n_views)
            return set_error(FBL_E_RANGE, "views[%d] = %d outside [0, %lld)", (int)k, (int)views[k],
                        (long long)p->geom.n_views);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device)
        return set_error(FBL_E_INVALID, "the current device (%d) is not the plan's device (%d)", cur, p->device);
    return FBL_OK;
}

hipError_t pooled_event(fbl_plan *p, hipEvent_t *ev)
{
    if (!p->event_pool.empty()) {
        *ev = p->event_pool.back();
        p->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

// Enqueue one kernel through `launch`, bracketed by timing events while timing is on.
template <typename F>
hipError_t timed(fbl_plan *p, int kernel, hipStream_t st, F &&launch)
{
    if (!p->timing_on || !((p->timing_mask >> kernel) & 1u)) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = pooled_event(p, &a);
    if (e == hipSuccess) e = pooled_event(p, &b);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    p->timed.push_back({kernel, a, b});
    return hipSuccess;
}

ViewList chunk(const int32_t *views, int first, int nb)
{
    ViewList vl;
    std::memset(&vl, 0, sizeof vl);
    for (int k = 0; k < nb; ++k) vl.v[k] = views[first + k];
    return vl;
}

// Argument checks shared by the prox-trial entry points (the plan is non-NULL).
int check_step_args(const fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo, double hi,
                    const void *xbar, const double *red_dev)
{
    const int rc = check_step_buffers(x, g, alpha, mu, lo, hi, xbar, red_dev);
    if (rc != FBL_OK) return rc;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device) return set_error(FBL_E_INVALID, "the current device is not the plan's device");
    return FBL_OK;
}

int step_call(fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo, double hi,
              bool stochastic, uint64_t key, void *xbar, double *red_dev, void *stream)
{
    if (!p) return set_error(FBL_E_INVALID, "plan is NULL");
    int rc = check_step_args(p, x, g, alpha, mu, lo, hi, xbar, red_dev);
    if (rc != FBL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    int64_t nparts = 0;
    double *parts = nullptr;
    e = timed(p, FBL_K_STEP, st,
              [&] { return launch_step(p, x, g, alpha, mu, lo, hi, stochastic, key, xbar, &parts, &nparts, st); });
    if (e != hipSuccess) return hip_fail(e, "step launch");
    e = timed(p, FBL_K_FINALIZE, st, [&] { return launch_finalize_sum(parts, nparts, 3, 1.0, red_dev, st); });
    if (e != hipSuccess) return hip_fail(e, "step reduction launch");
    return ok();
}


}  // namespace

extern "C" {

const char *fbl_last_error(void) { return g_err.c_str(); }

int fbl_geometry_check(const fbl_geometry *g)
{
    int rc = check_geometry(g);
    return rc == FBL_OK ? ok() : rc;
}

int fbl_plan_create(const fbl_geometry *g, int32_t vol_dtype, int32_t proj_dtype, int32_t max_batch, fbl_plan **out)
{
    if (!out) return set_error(FBL_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_geometry(g);
    if (rc != FBL_OK) return rc;
    if (vol_dtype != FBL_F32 && vol_dtype != FBL_BF16 && vol_dtype != FBL_F16)
        return set_error(FBL_E_DTYPE, "vol_dtype %d is not FBL_F32, FBL_BF16 or FBL_F16", (int)vol_dtype);
    if (proj_dtype != FBL_F32 && proj_dtype != FBL_BF16 && proj_dtype != FBL_F16)
        return set_error(FBL_E_DTYPE, "proj_dtype %d is not FBL_F32, FBL_BF16 or FBL_F16", (int)proj_dtype);
    if (max_batch < 1 || max_batch > g->n_views)
        return set_error(FBL_E_RANGE, "max_batch %d outside [1, n_views=%lld]", (int)max_batch, (long long)g->n_views);

    // value-initialisation zeroes every plain field (the struct has no user-provided
    // constructor) and constructs the vectors; defaults that are not zero follow
    fbl_plan *p = new fbl_plan();
    p->timing_mask = (1u << FBL_K_COUNT) - 1u;   // documented default: every kernel
    p->device = -1;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "hipGetDevice");
    }
    p->geom = *g;
    p->angles_host = new double[g->n_views];
    for (int64_t v = 0; v < g->n_views; ++v) p->angles_host[v] = view_angle(*g, v);
    p->geom.angles = p->angles_host;
    p->vol_dtype = vol_dtype;
    p->proj_dtype = proj_dtype;
    p->max_batch = max_batch;

    Geo &G = p->geo;
    G.nx = (int)g->nx; G.ny = (int)g->ny; G.nz = (int)g->nz;
    G.nu = (int)g->nu; G.nv = (int)g->nv;
    G.hx = (float)g->hx; G.hy = (float)g->hy; G.hz = (float)g->hz;
    G.du = (float)g->du; G.dv = (float)g->dv;
    G.sod = (float)g->sod; G.sdd = (float)g->sdd;
    G.cz = 0.5 * (double)(g->nz - 1);
    G.cu = (float)(0.5 * (double)(g->nu - 1));
    G.cv = (float)(0.5 * (double)(g->nv - 1));
    G.dvz = (float)(g->dv / g->hz);
    G.np = g->nu * g->nv;

    std::vector<ColParam> col((size_t)g->n_views * (size_t)g->nu);
    std::vector<ColParam64> col64(col.size());
    p->view_axis0 = new unsigned char[g->n_views];
    double tau_max = 0.0, tau_min = 1.0;
    for (int64_t v = 0; v < g->n_views; ++v) {
        p->view_axis0[v] = 0;
        for (int64_t iu = 0; iu < g->nu; ++iu) {
            const ColumnGeom cg = column_geom(p->geom, v, iu);
            ColParam &cp = col[(size_t)v * (size_t)g->nu + (size_t)iu];
            const int a = std::fabs(cg.D[0]) >= std::fabs(cg.D[1]) ? 0 : 1;
            if (a == 0) p->view_axis0[v] = 1;
            {
                // largest ray parameter on the first and last slice (tau is affine in m)
                const double na = (double)(a == 0 ? g->nx : g->ny);
                const double ta = (0.0 - cg.P[a]) / cg.D[a], tb = (na - 1.0 - cg.P[a]) / cg.D[a];
                tau_max = std::fmax(tau_max, std::fmax(ta, tb));
                tau_min = std::fmin(tau_min, std::fmin(ta, tb));
            }
            const int b = 1 - a;
            const double ha = a == 0 ? g->hx : g->hy;
            // slice m is crossed at t = (m - P_a)/D_a; there xi = P_b + t D_b
            const double t1 = 1.0 / cg.D[a], t0 = -cg.P[a] / cg.D[a];
            const double r = cg.D[b] / cg.D[a];
            cp.t1 = t1;
            cp.t0 = t0;
            cp.xi1 = r;
            cp.xi0 = cg.P[b] - cg.P[a] * r;
            const double ex = cg.q[0] - cg.s[0], ey = cg.q[1] - cg.s[1];
            cp.wa = (float)(ha / std::fabs(cg.q[a] - cg.s[a]));
            cp.l2 = (float)(ex * ex + ey * ey);
            col64[(size_t)v * (size_t)g->nu + (size_t)iu] = ColParam64{ha / std::fabs(cg.q[a] - cg.s[a]), ex * ex + ey * ey};
            cp.axis = a;
            cp.pad = 0;
        }
    }
    // Forward: a thread's rows span at most tau_max * (rows-1) * dv/hz voxels in z on a
    // slice.  Its LDS line runs from floor(first - 1e-3) to floor(last) + 1, i.e. at most
    // floor(span + 1e-3) + 3 entries; the bound below keeps a margin for FP32 rounding.
    // Every entry beyond the need costs two tap loads and a lerp per slice: the benchmark
    // geometries need 11, and 12-entry lines ran 7% slower there, so 11 is compiled too.
    {
        const double span = tau_max * (double)(forward_rows_per_thread() - 1) * (g->dv / g->hz);
        const double need = std::floor(span + 0.01) + 3.0;
        const int sizes[] = {11, 12, 16, 24, 32, 48};
        p->fp_line = 0;
        for (int sz : sizes)
            if (p->fp_line == 0 && need <= (double)sz) p->fp_line = sz;
        if (p->fp_line == 0) {
            free_plan(p);
            return set_error(FBL_E_GEOMETRY,
                        "detector rows are too coarse for the voxel size: %d rows span %.1f voxels in z (max 45)",
                        forward_rows_per_thread(), span);
        }
    }
    std::vector<ViewParam> vp((size_t)g->n_views);
    for (int64_t v = 0; v < g->n_views; ++v) {
        const double th = p->angles_host[v];
        vp[(size_t)v].c = (float)std::cos(th);
        vp[(size_t)v].s = (float)std::sin(th);
        // columns change dominant axis at most once along a detector row
        const ColParam *cv = &col[(size_t)v * (size_t)g->nu];
        int split = (int)g->nu, changes = 0;
        for (int64_t iu = 1; iu < g->nu; ++iu)
            if (cv[iu].axis != cv[iu - 1].axis) {
                if (changes == 0) split = (int)iu;
                ++changes;
            }
        if (changes > 1) {
            free_plan(p);
            return set_error(FBL_E_GEOMETRY, "view %lld: the detector row changes dominant axis %d times (fan too wide)",
                        (long long)v, changes);
        }
        vp[(size_t)v].axis_first = cv[0].axis;
        vp[(size_t)v].split = split;
    }
    // Backprojection: the largest number of detector columns crossing one slice of a tile
    // (kernel arithmetic replayed in FP32 over every view, class, slice and tile), which
    // sizes the tile's LDS pair table; and the number of detector rows within one voxel
    // of a z-position, ceil(2 / (row spacing in voxels)), which sizes the profile gather.
    {
        const double rowz_min = tau_min * (g->dv / g->hz);
        // rows with eta in an open interval of length 2: at most ceil(2 / spacing)
        const double cand = std::ceil(2.0 / rowz_min + 1e-4);
        p->bp_cand = cand <= 3.0 ? 3 : cand <= 4.0 ? 4 : cand <= 5.0 ? 5 : cand <= 6.0 ? 6 : cand <= 8.0 ? 8 : 0;
        if (p->bp_cand == 0) {
            free_plan(p);
            return set_error(FBL_E_GEOMETRY, "detector rows are too fine for the voxel size (%.3f voxels apart, min 0.34)",
                        rowz_min);
        }
        const int TQ = backproject_tile();
        const float cxv = 0.5f * (float)(g->nx - 1), cyv = 0.5f * (float)(g->ny - 1);
        const float fsod = (float)g->sod, fsdd = (float)g->sdd, fdu = (float)g->du, fcu = (float)(0.5 * (double)(g->nu - 1));
        const float fhx = (float)g->hx, fhy = (float)g->hy;
        auto col_of = [&](float c, float s, float X, float Y) {
            const float lat = -X * s + Y * c;
            const float dep = fsod - (X * c + Y * s);
            return fsdd * lat / dep / fdu + fcu;
        };
        int max_n = 0;
        for (int64_t v = 0; v < g->n_views; ++v) {
            const float c = vp[(size_t)v].c, s = vp[(size_t)v].s;
            for (int cls = 0; cls < 2; ++cls) {
                const int axis = cls == 0 ? vp[(size_t)v].axis_first : 1 - vp[(size_t)v].axis_first;
                const int cl0 = cls == 0 ? 0 : vp[(size_t)v].split;
                const int cl1 = cls == 0 ? vp[(size_t)v].split - 1 : (int)g->nu - 1;
                if (cl0 > cl1) continue;
                const int na = (int)(axis == 0 ? g->nx : g->ny), nq = (int)(axis == 0 ? g->ny : g->nx);
                for (int q0 = 0; q0 < nq; q0 += TQ)
                    for (int mg = 0; mg < na; ++mg) {
                        const float fm = (float)mg;
                        float u0, u1;
                        if (axis == 0) {
                            const float X = (fm - cxv) * fhx;
                            u0 = col_of(c, s, X, ((float)(q0 - 1) - cyv) * fhy);
                            u1 = col_of(c, s, X, ((float)(q0 + TQ) - cyv) * fhy);
                        } else {
                            const float Y = (fm - cyv) * fhy;
                            u0 = col_of(c, s, ((float)(q0 - 1) - cxv) * fhx, Y);
                            u1 = col_of(c, s, ((float)(q0 + TQ) - cxv) * fhx, Y);
                        }
                        const int a = std::max(cl0, (int)std::floor(std::fmin(u0, u1)) - 1);
                        const int b = std::min(cl1, (int)std::ceil(std::fmax(u0, u1)) + 1);
                        max_n = std::max(max_n, b - a + 1);
                    }
            }
        }
        // two columns of margin: the device forms the same ranges with FP contraction and
        // a hardware reciprocal, which can move each end by one column
        const int need = max_n + 2;
        const int sizes[] = {32, 48, 64};
        p->bp_pairs = 0;
        for (int sz : sizes)
            if (p->bp_pairs == 0 && need <= sz) p->bp_pairs = sz;
        if (p->bp_pairs == 0) {
            free_plan(p);
            return set_error(FBL_E_GEOMETRY,
                        "detector columns are too fine for the voxel size: %d columns cross one %d-voxel tile slice",
                        max_n, TQ);
        }
    }
    std::vector<double> rowV((size_t)g->nv);
    std::vector<float> rowV2((size_t)g->nv);
    for (int64_t iv = 0; iv < g->nv; ++iv) {
        const double v = ((double)iv - 0.5 * (double)(g->nv - 1)) * g->dv;
        rowV[(size_t)iv] = v / g->hz;
        rowV2[(size_t)iv] = (float)(v * v);
    }
    // Backprojection launch order: most work first, the least at the end of the launch,
    // where it shortens the tail.  A tile's work grows with the views whose rays reach
    // it: every view's fan covers the tiles near the rotation axis and fewer cover those
    // towards the corners, and a view's cone reaches a tile high or low in the volume only
    // where the tile lies far from its source.  The estimate counts, over up to 64 views
    // spread over the orbit, those whose fan holds the tile's centre and whose rows reach
    // its height there; ties go by distance from the axis.
    std::vector<int> bp_order;
    {
        const int TQ = backproject_tile(), TK = backproject_tile_z();
        const int tx = (int)((g->nx + TQ - 1) / TQ), ty = (int)((g->ny + TQ - 1) / TQ), tz = (int)((g->nz + TK - 1) / TK);
        const int64_t nxy = (int64_t)tx * ty;
        const int nsv = (int)std::min<int64_t>(64, g->n_views);
        const double vmax = 0.5 * (double)(g->nv - 1) * (g->dv / g->hz);   // largest row slope, index units
        const double czz = 0.5 * (double)(g->nz - 1);
        std::vector<double> r2((size_t)nxy);
        std::vector<std::vector<double>> reach((size_t)nxy);   // per xy tile: |z - cz| each view reaches
        for (int j = 0; j < ty; ++j)
            for (int i = 0; i < tx; ++i) {
                const double X = ((double)i * TQ + 0.5 * (TQ - 1) - 0.5 * (double)(g->nx - 1)) * g->hx;
                const double Y = ((double)j * TQ + 0.5 * (TQ - 1) - 0.5 * (double)(g->ny - 1)) * g->hy;
                const size_t t = (size_t)j * tx + i;
                r2[t] = X * X + Y * Y;
                for (int k = 0; k < nsv; ++k) {
                    const double th = p->angles_host[(int64_t)k * g->n_views / nsv];
                    const double c = std::cos(th), sn = std::sin(th);
                    const double dep = g->sod - (X * c + Y * sn);
                    const double u = g->sdd * (-X * sn + Y * c) / (dep * g->du) + 0.5 * (double)(g->nu - 1);
                    if (u < -1.0 || u > (double)g->nu) continue;   // outside the fan
                    reach[t].push_back(dep / g->sdd * vmax);
                }
                std::sort(reach[t].begin(), reach[t].end());
            }
        std::vector<int> work((size_t)nxy * tz);
        for (int64_t t = 0; t < nxy; ++t)
            for (int k = 0; k < tz; ++k) {
                const double zc = std::fabs((double)k * TK + 0.5 * (TK - 1) - czz) - 0.5 * TK;
                const auto &rv = reach[(size_t)t];
                work[(size_t)k * nxy + t] = (int)(rv.end() - std::lower_bound(rv.begin(), rv.end(), zc));
            }
        bp_order.resize((size_t)nxy * tz);
        for (size_t t = 0; t < bp_order.size(); ++t) bp_order[t] = (int)t;
        std::stable_sort(bp_order.begin(), bp_order.end(), [&](int a, int b) {
            if (work[(size_t)a] != work[(size_t)b]) return work[(size_t)a] > work[(size_t)b];
            return r2[(size_t)(a % nxy)] < r2[(size_t)(b % nxy)];
        });
    }
    p->fp_blocks_max = forward_blocks_per_view(G, 4);
    const int64_t np_fp = (int64_t)max_batch * p->fp_blocks_max;
    const int64_t np_step = step_partials_needed((int64_t)G.nx * G.ny * G.nz);
    p->n_partials = np_fp > np_step ? np_fp : np_step;

    if ((rc = dev_upload(&p->d_col, col)) != FBL_OK || (rc = dev_upload(&p->d_col64, col64)) != FBL_OK ||
        (rc = dev_upload(&p->d_rowV, rowV)) != FBL_OK ||
        (rc = dev_upload(&p->d_rowV2, rowV2)) != FBL_OK || (rc = dev_upload(&p->d_view, vp)) != FBL_OK ||
        (rc = dev_upload(&p->d_bp_order, bp_order)) != FBL_OK) {
        std::string msg = g_err;
        free_plan(p);
        g_err = msg;
        return rc;
    }
    e = hipMalloc((void **)&p->d_partials, (size_t)p->n_partials * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_rw, (size_t)max_batch * (size_t)G.np * sizeof(float));
    if (e == hipSuccess)
        e = hipMalloc(&p->d_xt, (size_t)g->nx * (size_t)g->ny * (size_t)g->nz * (vol_dtype == FBL_F32 ? 4u : 2u));
    if (e != hipSuccess) {
        free_plan(p);
        return set_error(FBL_E_NOMEM, "hipMalloc of plan workspace: %s", hipGetErrorString(e));
    }
    *out = p;
    return ok();
}

void fbl_plan_destroy(fbl_plan *plan) { free_plan(plan); }

int fb_lisa_forward(fbl_plan *p, const void *x, const int32_t *views, int32_t B, const void *b, float *y,
                    double *loss_dev, double loss_scale, void *stream)
{
    int rc = check_call(p, views, B);
    if (rc != FBL_OK) return rc;
    if (!x || !y) return set_error(FBL_E_INVALID, "x and y must be non-NULL");
    if (!aligned16(x) || !aligned16(y) || (b && !aligned16(b)) || (loss_dev && !aligned8(loss_dev)))
        return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned and loss_dev 8-byte aligned");
    if (loss_dev && !std::isfinite(loss_scale)) return set_error(FBL_E_INVALID, "loss_scale must be finite");
    hipStream_t st = (hipStream_t)stream;
    bool need_xt = false;
    for (int32_t k = 0; k < B; ++k) need_xt = need_xt || p->view_axis0[views[k]];
    if (need_xt) {
        // views that march x = const slices read a y-fastest copy of x
        hipError_t e = timed(p, FBL_K_TRANSPOSE, st, [&] { return launch_transpose(p, x, st); });
        if (e != hipSuccess) return hip_fail(e, "volume transpose launch");
    }
    const int parts = forward_parts(p->geo, B);
    for (int first = 0; first < B; first += kViewsPerLaunch) {
        const int nb = B - first < kViewsPerLaunch ? B - first : kViewsPerLaunch;
        const ViewList vl = chunk(views, first, nb);
        hipError_t e = timed(p, FBL_K_FORWARD, st, [&] {
            return launch_forward(p, x, vl, nb, first, b, y, loss_dev != nullptr, parts, st);
        });
        if (e != hipSuccess) return hip_fail(e, "forward projection launch");
    }
    if (loss_dev) {
        const int64_t n = (int64_t)B * forward_blocks_per_view(p->geo, parts);
        hipError_t e = timed(p, FBL_K_FINALIZE, st,
                             [&] { return launch_finalize_sum(p->d_partials, n, 1, loss_scale, loss_dev, st); });
        if (e != hipSuccess) return hip_fail(e, "loss reduction launch");
    }
    return ok();
}

int fb_lisa_backproject(fbl_plan *p, const float *r, const int32_t *views, int32_t B, double grad_scale, float *g,
                        void *stream)
{
    int rc = check_call(p, views, B);
    if (rc != FBL_OK) return rc;
    if (!r || !g) return set_error(FBL_E_INVALID, "r and g must be non-NULL");
    if (!aligned16(r) || !aligned16(g)) return set_error(FBL_E_INVALID, "device buffers must be 16-byte aligned");
    if (!std::isfinite(grad_scale)) return set_error(FBL_E_INVALID, "grad_scale must be finite");
    hipStream_t st = (hipStream_t)stream;
    for (int first = 0; first < B; first += kViewsPerLaunch) {
        const int nb = B - first < kViewsPerLaunch ? B - first : kViewsPerLaunch;
        const ViewList vl = chunk(views, first, nb);
        hipError_t e = timed(p, FBL_K_PRESCALE, st,
                             [&] { return launch_prescale(p, r, vl, nb, first, grad_scale, p->d_rw, st); });
        if (e != hipSuccess) return hip_fail(e, "residual weighting launch");
    }
    for (int first = 0; first < B; first += kViewsPerLaunch) {
        const int nb = B - first < kViewsPerLaunch ? B - first : kViewsPerLaunch;
        const ViewList vl = chunk(views, first, nb);
        hipError_t e = timed(p, FBL_K_BACKPROJECT, st,
                             [&] { return launch_backproject(p, p->d_rw, vl, nb, first, first > 0, g, st); });
        if (e != hipSuccess) return hip_fail(e, "backprojection launch");
    }
    return ok();
}


int fb_lisa_forward_f64(fbl_plan *p, const double *x, const int32_t *views, int32_t B, double *y, void *stream)
{
    int rc = check_call(p, views, B);
    if (rc != FBL_OK) return rc;
    if (!x || !y) return set_error(FBL_E_INVALID, "x and y must be non-NULL");
    if (!aligned16(x) || !aligned16(y)) return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    for (int first = 0; first < B; first += kViewsPerLaunch) {
        const int nb = B - first < kViewsPerLaunch ? B - first : kViewsPerLaunch;
        const ViewList vl = chunk(views, first, nb);
        hipError_t e = launch_forward64(p, x, vl, nb, y + (int64_t)first * p->geo.np, st);
        if (e != hipSuccess) return hip_fail(e, "FP64 forward projection launch");
    }
    return ok();
}

int fb_lisa_backproject_f64(fbl_plan *p, const double *r, const int32_t *views, int32_t B, double grad_scale,
                            double *g, void *stream)
{
    int rc = check_call(p, views, B);
    if (rc != FBL_OK) return rc;
    if (!r || !g) return set_error(FBL_E_INVALID, "r and g must be non-NULL");
    if (!aligned16(r) || !aligned16(g)) return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned");
    if (!std::isfinite(grad_scale)) return set_error(FBL_E_INVALID, "grad_scale must be finite");
    hipStream_t st = (hipStream_t)stream;
    for (int first = 0; first < B; first += kViewsPerLaunch) {
        const int nb = B - first < kViewsPerLaunch ? B - first : kViewsPerLaunch;
        const ViewList vl = chunk(views, first, nb);
        hipError_t e = launch_backproject64(p, r + (int64_t)first * p->geo.np, vl, nb, grad_scale, first > 0, g, st);
        if (e != hipSuccess) return hip_fail(e, "FP64 backprojection launch");
    }
    return ok();
}

int fb_lisa_step(fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo, double hi, void *xbar,
                 double *red_dev, void *stream)
{
    return step_call(p, x, g, alpha, mu, lo, hi, false, 0, xbar, red_dev, stream);
}

int fb_lisa_step_mixed(fbl_plan *p, const float *x, const float *g, double alpha, double mu, double lo, double hi,
                       float *xbar, void *xbar16, double *red_dev, void *stream)
{
    if (!p) return set_error(FBL_E_INVALID, "plan is NULL");
    if (p->vol_dtype == FBL_F32)
        return set_error(FBL_E_DTYPE, "fb_lisa_step_mixed needs a plan with 16-bit volume storage (BF16 or F16)");
    if (!xbar16) return set_error(FBL_E_INVALID, "xbar16 must be non-NULL");
    if (!aligned16(xbar16)) return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned");
    if (xbar16 == (void *)x || xbar16 == (void *)g || xbar16 == (void *)xbar)
        return set_error(FBL_E_INVALID, "xbar16 may not alias x, g or xbar");
    int rc = check_step_args(p, x, g, alpha, mu, lo, hi, xbar, red_dev);
    if (rc != FBL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    int64_t nparts = 0;
    double *parts = nullptr;
    hipError_t e = timed(p, FBL_K_STEP, st, [&] {
        return launch_step_mixed(p, x, g, alpha, mu, lo, hi, xbar, xbar16, &parts, &nparts, st);
    });
    if (e != hipSuccess) return hip_fail(e, "mixed step launch");
    e = timed(p, FBL_K_FINALIZE, st, [&] { return launch_finalize_sum(parts, nparts, 3, 1.0, red_dev, st); });
    if (e != hipSuccess) return hip_fail(e, "step reduction launch");
    return ok();
}

int fb_lisa_step_sr(fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo, double hi,
                    uint64_t key, void *xbar, double *red_dev, void *stream)
{
    return step_call(p, x, g, alpha, mu, lo, hi, true, key, xbar, red_dev, stream);
}

size_t fbl_mlp_workspace_bytes(int64_t n) { return n < 1 ? 0 : mlp_workspace_bytes(n); }

int fbl_mlp_forward(const float *params, const float *X, int64_t n, float *out, void *stream)
{
    if (!params || !X || !out) return set_error(FBL_E_INVALID, "params, X and out must be non-NULL");
    if (n < 1 || n > ((int64_t)1 << 31)) return set_error(FBL_E_RANGE, "n = %lld outside [1, 2^31]", (long long)n);
    if (!aligned16(params) || !aligned16(X) || !aligned16(out))
        return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned");
    hipError_t e = launch_mlp_forward(params, X, n, out, (hipStream_t)stream);
    return e == hipSuccess ? ok() : hip_fail(e, "MLP forward launch");
}

int fbl_mlp_loss_grad(const float *params, const float *X, const float *t, int64_t n, float *grad, double *loss_dev,
                      void *work, void *stream)
{
    if (!params || !X || !t || !grad || !work) return set_error(FBL_E_INVALID, "params, X, t, grad and work must be non-NULL");
    if (n < 1 || n > ((int64_t)1 << 31)) return set_error(FBL_E_RANGE, "n = %lld outside [1, 2^31]", (long long)n);
    if (!aligned16(params) || !aligned16(X) || !aligned16(t) || !aligned16(grad) || (loss_dev && !aligned8(loss_dev)))
        return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned and loss_dev 8-byte aligned");
    if (((uintptr_t)work & 255u) != 0) return set_error(FBL_E_INVALID, "work must be 256-byte aligned");
    hipError_t e = launch_mlp_loss_grad(params, X, t, n, grad, loss_dev, work, (hipStream_t)stream);
    return e == hipSuccess ? ok() : hip_fail(e, "MLP gradient launch");
}

int fbl_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, double lr, double beta1,
                 double beta2, double eps, void *stream)
{
    if (!params || !grad || !m || !v) return set_error(FBL_E_INVALID, "params, grad, m and v must be non-NULL");
    if (step < 1) return set_error(FBL_E_RANGE, "step must be >= 1");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0) ||
        !std::isfinite(lr) || !std::isfinite(eps))
        return set_error(FBL_E_INVALID, "need lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
    if (!aligned16(params) || !aligned16(grad) || !aligned16(m) || !aligned16(v))
        return set_error(FBL_E_INVALID, "arrays must be 16-byte aligned");
    hipError_t e = launch_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    return e == hipSuccess ? ok() : hip_fail(e, "Adam launch");
}

int fbl_timing_enable(fbl_plan *p, int on)
{
    if (!p) return set_error(FBL_E_INVALID, "plan is NULL");
    if (on) {
        double ms[FBL_K_COUNT];
        int64_t n[FBL_K_COUNT];
        int rc = fbl_timing_read(p, ms, n);  // waits for and drops any earlier record
        if (rc != FBL_OK) return rc;
    }
    p->timing_on = on != 0;
    return ok();
}

int fbl_timing_select(fbl_plan *p, uint32_t mask)
{
    if (!p) return set_error(FBL_E_INVALID, "plan is NULL");
    if (mask >> FBL_K_COUNT) return set_error(FBL_E_INVALID, "mask 0x%x has bits beyond FBL_K_COUNT", (unsigned)mask);
    p->timing_mask = mask;
    return ok();
}

int fbl_timing_read(fbl_plan *p, double ms[FBL_K_COUNT], int64_t launches[FBL_K_COUNT])
{
    if (!p || !ms || !launches) return set_error(FBL_E_INVALID, "plan, ms and launches must be non-NULL");
    for (int k = 0; k < FBL_K_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    hipError_t first_err = hipSuccess;
    for (auto &t : p->timed) {
        float dt = 0.0f;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&dt, t.start, t.stop);
        if (e == hipSuccess) {
            ms[t.kernel] += dt;
            launches[t.kernel] += 1;
        } else if (first_err == hipSuccess) {
            first_err = e;
        }
        p->event_pool.push_back(t.start);
        p->event_pool.push_back(t.stop);
    }
    p->timed.clear();
    if (first_err != hipSuccess) return hip_fail(first_err, "reading launch timing events");
    return ok();
}

}  // extern "C"
