/*
 * FP64 CPU oracle for the FB-LISA hot path.  TEST INFRASTRUCTURE ONLY: the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use it; the product
 * library never links or calls it, and it shares no code with the HIP path.
 *
 * What it computes (paper: "A Line-Search-Based Stochastic Gradient Method for 3D
 * Computed Tomography", arXiv 2605.12085):
 *   - the per-view cone-beam operator blocks A_i of the data term of problem (2.1),
 *     split over projection angles as in (2.4), discretised with Joseph's ray-driven
 *     bilinear interpolation (the paper's projector is unspecified; this reading is
 *     listed in the design notes);
 *   - the restricted forward operator A_N x over a mini-batch N of whole views, as in
 *     the mini-batch objective (2.5);
 *   - its exact transpose A_N^T r (matched adjoint), by scatter and by a per-voxel
 *     evaluator that sums the matrix entries of every ray of the batch.
 *
 * Everything is FP64, evaluated in the order written (built with -ffp-contract=off
 * so no fused multiply-adds change the dominant-axis decision).  Parallel loops use a
 * static schedule and reduce per-thread partial volumes in thread order, so results
 * are deterministic for a given thread count.
 *
 * Conventions (continuous index coordinates):
 *   P = s/h + (n-1)/2 and D = (q-s)/h componentwise, for source s and pixel centre q;
 *   dominant axis a = argmax |D_a|, ties to the lowest axis (x < y < z);
 *   slice m = 0..n_a-1 is crossed at t = (m - P_a)/D_a, where the two other index
 *   coordinates (increasing axis order) are xi = P_b + t D_b, eta = P_c + t D_c;
 *   the sample is the bilinear interpolation of the slice at (xi, eta), taps outside
 *   the volume count as zero;
 *   the ray value is w * (sum of samples), w = h_a |q-s| / |q_a - s_a| (mm per slice).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t nx, ny, nz;
    double hx, hy, hz;
    int64_t nu, nv;
    double du, dv;
    double sod, sdd;
    int64_t n_views;
    const double *angles; /* n_views entries; NULL means 2*pi*j/n_views */
} orc_geom;

typedef struct {
    int64_t n[3];
    int64_t stride[3];
    double h[3];
} orc_vol;

static orc_vol vol_of(const orc_geom *g)
{
    orc_vol v;
    v.n[0] = g->nx; v.n[1] = g->ny; v.n[2] = g->nz;
    v.stride[0] = 1; v.stride[1] = g->nx; v.stride[2] = g->nx * g->ny;
    v.h[0] = g->hx; v.h[1] = g->hy; v.h[2] = g->hz;
    return v;
}

static double view_angle(const orc_geom *g, int64_t j)
{
    if (g->angles) return g->angles[j];
    return 2.0 * M_PI * (double)j / (double)g->n_views;
}

/* Source s and pixel centre q (mm) of ray (view j, column iu, row iv). */
void orc_ray_endpoints(const orc_geom *g, int64_t j, int64_t iu, int64_t iv, double s[3], double q[3])
{
    double th = view_angle(g, j);
    double c = cos(th), sn = sin(th);
    double dc = g->sod - g->sdd;
    double u = ((double)iu - 0.5 * (double)(g->nu - 1)) * g->du;
    double v = ((double)iv - 0.5 * (double)(g->nv - 1)) * g->dv;
    s[0] = g->sod * c;
    s[1] = g->sod * sn;
    s[2] = 0.0;
    q[0] = dc * c + u * (-sn);
    q[1] = dc * sn + u * c;
    q[2] = v;
}

/* Per-ray Joseph set-up: dominant axis, the two other axes, P, D and the weight w. */
typedef struct {
    int a, b, c;
    double P[3], D[3];
    double w;
} orc_ray;

static void ray_setup(const orc_geom *g, const orc_vol *V, int64_t j, int64_t iu, int64_t iv, orc_ray *r)
{
    double s[3], q[3];
    orc_ray_endpoints(g, j, iu, iv, s, q);
    for (int k = 0; k < 3; ++k) {
        r->P[k] = s[k] / V->h[k] + 0.5 * (double)(V->n[k] - 1);
        r->D[k] = (q[k] - s[k]) / V->h[k];
    }
    double ax = fabs(r->D[0]), ay = fabs(r->D[1]), az = fabs(r->D[2]);
    if (ax >= ay && ax >= az) { r->a = 0; r->b = 1; r->c = 2; }
    else if (ay >= az)        { r->a = 1; r->b = 0; r->c = 2; }
    else                      { r->a = 2; r->b = 0; r->c = 1; }
    double e0 = q[0] - s[0], e1 = q[1] - s[1], e2 = q[2] - s[2];
    double len = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    r->w = V->h[r->a] * len / fabs(q[r->a] - s[r->a]);
}

/* Position (xi, eta) where the ray crosses slice m of its dominant axis. */
static void ray_at_slice(const orc_ray *r, int64_t m, double *xi, double *eta)
{
    double t = ((double)m - r->P[r->a]) / r->D[r->a];
    *xi = r->P[r->b] + t * r->D[r->b];
    *eta = r->P[r->c] + t * r->D[r->c];
}

/* Joseph line integral of one ray through volume x (FP64 [nz][ny][nx]). */
double orc_ray_value(const orc_geom *g, const double *x, int64_t j, int64_t iu, int64_t iv)
{
    orc_vol V = vol_of(g);
    orc_ray r;
    ray_setup(g, &V, j, iu, iv, &r);
    const int64_t na = V.n[r.a], nb = V.n[r.b], nc = V.n[r.c];
    const int64_t sa = V.stride[r.a], sb = V.stride[r.b], sc = V.stride[r.c];
    double sum = 0.0;
    for (int64_t m = 0; m < na; ++m) {
        double xi, eta;
        ray_at_slice(&r, m, &xi, &eta);
        if (!(xi > -2.0 && xi < (double)nb + 1.0 && eta > -2.0 && eta < (double)nc + 1.0)) continue;
        double fxi = floor(xi), feta = floor(eta);
        int64_t i0 = (int64_t)fxi, j0 = (int64_t)feta;
        double wx = xi - fxi, wy = eta - feta;
        double tap[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj) {
                int64_t ii = i0 + di, jj = j0 + dj;
                if (ii >= 0 && ii < nb && jj >= 0 && jj < nc)
                    tap[di][dj] = x[m * sa + ii * sb + jj * sc];
            }
        sum += (1.0 - wx) * (1.0 - wy) * tap[0][0] + wx * (1.0 - wy) * tap[1][0]
             + (1.0 - wx) * wy * tap[0][1] + wx * wy * tap[1][1];
    }
    return r.w * sum;
}

/* Transpose of orc_ray_value: out += val * (column of the ray's matrix row). */
static void ray_adjoint(const orc_geom *g, const orc_vol *V, int64_t j, int64_t iu, int64_t iv,
                        double val, double *out)
{
    orc_ray r;
    ray_setup(g, V, j, iu, iv, &r);
    const int64_t na = V->n[r.a], nb = V->n[r.b], nc = V->n[r.c];
    const int64_t sa = V->stride[r.a], sb = V->stride[r.b], sc = V->stride[r.c];
    const double wv = r.w * val;
    for (int64_t m = 0; m < na; ++m) {
        double xi, eta;
        ray_at_slice(&r, m, &xi, &eta);
        if (!(xi > -2.0 && xi < (double)nb + 1.0 && eta > -2.0 && eta < (double)nc + 1.0)) continue;
        double fxi = floor(xi), feta = floor(eta);
        int64_t i0 = (int64_t)fxi, j0 = (int64_t)feta;
        double wx = xi - fxi, wy = eta - feta;
        double wt[2][2] = {{(1.0 - wx) * (1.0 - wy), (1.0 - wx) * wy}, {wx * (1.0 - wy), wx * wy}};
        for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj) {
                int64_t ii = i0 + di, jj = j0 + dj;
                if (ii >= 0 && ii < nb && jj >= 0 && jj < nc)
                    out[m * sa + ii * sb + jj * sc] += wv * wt[di][dj];
            }
    }
}

/*
 * Forward projection of the mini-batch (2.5): y[b][iv][iu] = (A_{views[b]} x)[iv][iu].
 */
void orc_forward(const orc_geom *g, const double *x, const int32_t *views, int64_t B, double *y)
{
    const int64_t np = g->nu * g->nv;
    const int64_t total = B * np;
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < total; ++idx) {
        int64_t b = idx / np, p = idx % np;
        int64_t iv = p / g->nu, iu = p % g->nu;
        y[idx] = orc_ray_value(g, x, views[b], iu, iv);
    }
}

/* Forward values of an explicit list of rays: rays[3*i] = (view, iv, iu). */
void orc_forward_rays(const orc_geom *g, const double *x, const int64_t *rays, int64_t n, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        y[i] = orc_ray_value(g, x, rays[3 * i], rays[3 * i + 2], rays[3 * i + 1]);
}

/*
 * Backprojection (exact transpose of orc_forward): out = A_N^T r, overwritten.
 * Each thread scatters its static share of rays into a private volume; the private
 * volumes are then added in thread order.
 */
int orc_backproject(const orc_geom *g, const double *r, const int32_t *views, int64_t B, double *out)
{
    orc_vol V = vol_of(g);
    const int64_t d = g->nx * g->ny * g->nz;
    const int64_t np = g->nu * g->nv;
    const int64_t total = B * np;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nth * (size_t)d, sizeof(double));
    if (!priv) return -1;
#pragma omp parallel num_threads(nth)
    {
        int tid = 0, T = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        T = omp_get_num_threads();
#endif
        double *acc = priv + (size_t)tid * (size_t)d;
        int64_t lo = total * tid / T, hi = total * (tid + 1) / T;
        for (int64_t idx = lo; idx < hi; ++idx) {
            double val = r[idx];
            if (val == 0.0) continue;
            int64_t b = idx / np, p = idx % np;
            ray_adjoint(g, &V, views[b], p % g->nu, p / g->nu, val, acc);
        }
#pragma omp barrier
#pragma omp for schedule(static)
        for (int64_t v = 0; v < d; ++v) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += priv[(size_t)t * (size_t)d + (size_t)v];
            out[v] = s;
        }
    }
    free(priv);
    return 0;
}

/*
 * Matrix entry A[(view, iu, iv)][voxel]: the Joseph weight with which the ray taps
 * the voxel.  A ray taps voxel (i0..) only on the slice of its dominant axis that
 * holds the voxel, so the entry is w * (bilinear weight of the voxel at that slice).
 */
static double ray_voxel_weight(const orc_ray *r, const orc_vol *V, const int64_t vox[3])
{
    int64_t m = vox[r->a];
    double xi, eta;
    ray_at_slice(r, m, &xi, &eta);
    if (!(xi > -2.0 && xi < (double)V->n[r->b] + 1.0 && eta > -2.0 && eta < (double)V->n[r->c] + 1.0))
        return 0.0;
    double fxi = floor(xi), feta = floor(eta);
    int64_t i0 = (int64_t)fxi, j0 = (int64_t)feta;
    double wx = xi - fxi, wy = eta - feta;
    double ab, ac;
    if (vox[r->b] == i0) ab = 1.0 - wx;
    else if (vox[r->b] == i0 + 1) ab = wx;
    else return 0.0;
    if (vox[r->c] == j0) ac = 1.0 - wy;
    else if (vox[r->c] == j0 + 1) ac = wy;
    else return 0.0;
    return r->w * ab * ac;
}

double orc_matrix_entry(const orc_geom *g, int64_t view, int64_t iu, int64_t iv, int64_t voxel)
{
    orc_vol V = vol_of(g);
    orc_ray r;
    ray_setup(g, &V, view, iu, iv, &r);
    int64_t vox[3] = {voxel % g->nx, (voxel / g->nx) % g->ny, voxel / (g->nx * g->ny)};
    return ray_voxel_weight(&r, &V, vox);
}

/*
 * Per-voxel backprojection: out[i] = sum over every ray of the batch of
 * A[ray][voxels[i]] * r[ray].  Brute force over all rays; used to check sampled
 * voxels of the GPU gradient at sizes where the full scatter is too slow.
 */
void orc_backproject_voxels(const orc_geom *g, const double *r, const int32_t *views, int64_t B,
                            const int64_t *voxels, int64_t nvox, double *out)
{
    orc_vol V = vol_of(g);
    const int64_t np = g->nu * g->nv;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nvox; ++i) {
        int64_t vx = voxels[i];
        int64_t vox[3] = {vx % g->nx, (vx / g->nx) % g->ny, vx / (g->nx * g->ny)};
        double s = 0.0;
        for (int64_t b = 0; b < B; ++b)
            for (int64_t p = 0; p < np; ++p) {
                double val = r[b * np + p];
                if (val == 0.0) continue;
                orc_ray ray;
                ray_setup(g, &V, views[b], p % g->nu, p / g->nu, &ray);
                double a = ray_voxel_weight(&ray, &V, vox);
                if (a != 0.0) s += a * val;
            }
        out[i] = s;
    }
}

/* Dominant axis of every ray of one view, [nv][nu] (0 = x, 1 = y, 2 = z). */
void orc_dominant_axes(const orc_geom *g, int64_t view, int32_t *axes)
{
    orc_vol V = vol_of(g);
    for (int64_t iv = 0; iv < g->nv; ++iv)
        for (int64_t iu = 0; iu < g->nu; ++iu) {
            orc_ray r;
            ray_setup(g, &V, view, iu, iv, &r);
            axes[iv * g->nu + iu] = r.a;
        }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
