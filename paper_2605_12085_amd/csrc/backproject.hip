// Matched backprojection g = s * A_N^T r, voxel-driven (gather, no atomics).
//
// The transpose of the Joseph forward: voxel (i, j, k) receives, from every ray of the
// batch whose dominant-axis slice holds it, the ray's weighted residual times the same
// bilinear weight the forward projection applied to the voxel.  A column c of a view
// taps voxel (i, j) only on slice m = (i if its slices are x = const, else j), where its
// horizontal index coordinate xi_c(m) lies within one voxel of the voxel's other index;
// the rays of the column then tap voxel k where |eta - k| < 1.
#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

// rw = grad_scale * w * r: the per-ray path length per slice folded into the residual.
__global__ __launch_bounds__(256) void prescale_kernel(const float *__restrict__ r, Geo geo, DeviceTables tab,
                                                       ViewList vl, int first, double grad_scale,
                                                       float *__restrict__ rw)
{
    const int bi = blockIdx.y;
    const int view = vl.v[bi];
    const float gs = (float)grad_scale;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < geo.np; p += (int64_t)gridDim.x * 256) {
        const int iv = (int)(p / geo.nu), iu = (int)(p % geo.nu);
        const ColParam cp = tab.col[(int64_t)view * geo.nu + iu];
        const float w = cp.wa * sqrtf(cp.l2 + tab.rowV2[iv]);
        const int64_t o = (int64_t)(first + bi) * geo.np + p;
        rw[o] = gs * (w * r[o]);
    }
}

__global__ __launch_bounds__(256) void bp_kernel(const float *__restrict__ rw, Geo geo, DeviceTables tab,
                                                 ViewList vl, int nb, int first, int accumulate,
                                                 float *__restrict__ g)
{
    const int64_t d = (int64_t)geo.nx * geo.ny * geo.nz;
    const int64_t vox = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (vox >= d) return;
    const int i = (int)(vox % geo.nx);
    const int j = (int)((vox / geo.nx) % geo.ny);
    const int k = (int)(vox / ((int64_t)geo.nx * geo.ny));
    const float px = ((float)i - 0.5f * (float)(geo.nx - 1)) * geo.hx;
    const float py = ((float)j - 0.5f * (float)(geo.ny - 1)) * geo.hy;
    const float fk = (float)k;
    float acc = 0.0f;
    for (int bi = 0; bi < nb; ++bi) {
        const int view = vl.v[bi];
        const ViewParam vp = tab.view[view];
        const float *__restrict__ rwv = rw + (int64_t)(first + bi) * geo.np;
        const ColParam *__restrict__ cols = tab.col + (int64_t)view * geo.nu;
        // detector columns whose ray plane passes within one voxel: project the corners
        // of the 2h x 2h square around the voxel centre
        float umin = 3.0e38f, umax = -3.0e38f;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const float qx = px + ((cc & 1) ? geo.hx : -geo.hx);
            const float qy = py + ((cc & 2) ? geo.hy : -geo.hy);
            const float lat = -qx * vp.s + qy * vp.c;
            const float dep = geo.sod - (qx * vp.c + qy * vp.s);
            const float uf = geo.sdd * lat / dep / geo.du + geo.cu;
            umin = fminf(umin, uf);
            umax = fmaxf(umax, uf);
        }
        // clamp before converting so no extreme value can wrap the integer range
        const int c0 = max(0, (int)floorf(fmaxf(umin, -4.0f)) - 1);
        const int c1 = min(geo.nu - 1, (int)ceilf(fminf(umax, (float)geo.nu + 4.0f)) + 1);
        for (int c = c0; c <= c1; ++c) {
            const ColParam cp = cols[c];
            const int m = cp.axis == 0 ? i : j;
            const int pb = cp.axis == 0 ? j : i;
            // positions in FP64 (index coordinates reach thousands), weights in FP32
            const double fm = (double)m;
            const double xi = fma(fm, cp.xi1, cp.xi0);
            const float hxi = (float)(1.0 - fabs(xi - (double)pb));
            if (hxi <= 0.0f) continue;
            const double tau = fma(fm, cp.t1, cp.t0);
            const float inv = (float)(1.0 / (tau * (double)geo.dvz));
            const float czf = (float)geo.cz;
            const float lo = (fk - 1.0f - czf) * inv + geo.cv;
            const float hi = (fk + 1.0f - czf) * inv + geo.cv;
            const int r0 = max(0, (int)floorf(fmaxf(lo, -4.0f)) - 1);
            const int r1 = min(geo.nv - 1, (int)ceilf(fminf(hi, (float)geo.nv + 4.0f)) + 1);
            float part = 0.0f;
            for (int iv = r0; iv <= r1; ++iv) {
                const double eta = fma(tau, tab.rowV[iv], geo.cz);
                const float heta = (float)(1.0 - fabs(eta - (double)k));
                if (heta > 0.0f) part = fmaf(heta, rwv[(int64_t)iv * geo.nu + c], part);
            }
            acc = fmaf(hxi, part, acc);
        }
    }
    g[vox] = accumulate ? g[vox] + acc : acc;
}

}  // namespace

hipError_t launch_prescale(const fbl_plan *p, const float *r, const ViewList &vl, int nb, int first,
                           double grad_scale, float *rw, hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    int64_t blocks = (p->geo.np + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(prescale_kernel, dim3((unsigned)blocks, nb), dim3(256), 0, st, r, p->geo, tab, vl, first,
                       grad_scale, rw);
    return hipGetLastError();
}

hipError_t launch_backproject(const fbl_plan *p, const float *rw, const ViewList &vl, int nb, int first,
                              bool accumulate, float *g, hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    hipLaunchKernelGGL(bp_kernel, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, rw, p->geo, tab, vl, nb,
                       first, accumulate ? 1 : 0, g);
    return hipGetLastError();
}

}  // namespace fbl
