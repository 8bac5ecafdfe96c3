// FP64 instantiation of the projector pair, for checks: the same discretised operator A
// (Joseph, bilinear, zero padding, path length per slice) with every position, weight and
// sum in FP64, so that finite differences and the adjoint identity can be tested to
// near FP64 rounding.  These kernels favour plainness over speed: one thread per ray,
// positions formed directly per slice, and the transpose as a scatter with FP64 atomic
// additions (the summation order varies between launches only at FP64 rounding level).
#include "common.h"

namespace fbl {

namespace {

// Path length per slice of ray (view, iv, iu): h_a |q - s| / |q_a - s_a|.
__device__ __forceinline__ double path_length64(const Geo &geo, const ColParam64 *__restrict__ c64, double dv_mm,
                                                int view, int iv, int iu)
{
    const ColParam64 w = c64[(int64_t)view * geo.nu + iu];
    const double v = ((double)iv - 0.5 * (double)(geo.nv - 1)) * dv_mm;   // row height above the source, mm
    return w.wa * sqrt(w.l2 + v * v);
}

// Visit the bilinear taps of ray (view, iv, iu) on every slice of its dominant axis:
// f(voxel linear index, tap weight) for each tap inside the volume.
template <typename F>
__device__ __forceinline__ void march64(const Geo &geo, const DeviceTables &tab, int view, int iv, int iu, F &&f)
{
    const ColParam cp = tab.col[(int64_t)view * geo.nu + iu];
    const double V = tab.rowV[iv];                               // eta slope: (iv - cv) dv / hz
    const int na = cp.axis == 0 ? geo.nx : geo.ny;
    const int nb = cp.axis == 0 ? geo.ny : geo.nx;
    const int64_t plane = (int64_t)geo.nx * geo.ny;
    for (int m = 0; m < na; ++m) {
        const double xi = cp.xi0 + (double)m * cp.xi1;
        const double tau = cp.t0 + (double)m * cp.t1;
        const double eta = geo.cz + tau * V;
        const double fx = floor(xi), fz = floor(eta);
        const double ax = xi - fx, az = eta - fz;
        const int64_t i0 = (int64_t)fx, k0 = (int64_t)fz;
#pragma unroll
        for (int dq = 0; dq < 2; ++dq) {
            const int64_t q = i0 + dq;
            if (q < 0 || q >= nb) continue;
            const double wq = dq ? ax : 1.0 - ax;
#pragma unroll
            for (int dk = 0; dk < 2; ++dk) {
                const int64_t k = k0 + dk;
                if (k < 0 || k >= geo.nz) continue;
                const double wk = dk ? az : 1.0 - az;
                // slices along x (axis 0): voxel (m, q, k); along y: voxel (q, m, k)
                const int64_t vox = cp.axis == 0 ? (int64_t)m + (int64_t)geo.nx * q + plane * k
                                                 : q + (int64_t)geo.nx * m + plane * k;
                f(vox, wq * wk);
            }
        }
    }
}

__global__ __launch_bounds__(256) void fp64_kernel(const double *__restrict__ x, Geo geo, DeviceTables tab,
                                                   const ColParam64 *__restrict__ c64, double dv, ViewList vl,
                                                   int nb, double *__restrict__ y)
{
    const int64_t n = (int64_t)nb * geo.np;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const int b = (int)(t / geo.np);
        const int64_t p = t % geo.np;
        const int iv = (int)(p / geo.nu), iu = (int)(p % geo.nu);
        double s = 0.0;
        march64(geo, tab, vl.v[b], iv, iu, [&](int64_t vox, double wt) { s += wt * x[vox]; });
        y[t] = path_length64(geo, c64, dv, vl.v[b], iv, iu) * s;
    }
}

__global__ __launch_bounds__(256) void bp64_kernel(const double *__restrict__ r, Geo geo, DeviceTables tab,
                                                   const ColParam64 *__restrict__ c64, double dv, ViewList vl,
                                                   int nb, double scale, double *__restrict__ g)
{
    const int64_t n = (int64_t)nb * geo.np;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const int b = (int)(t / geo.np);
        const int64_t p = t % geo.np;
        const int iv = (int)(p / geo.nu), iu = (int)(p % geo.nu);
        const double rv = r[t];
        if (rv == 0.0) continue;
        const double c = scale * path_length64(geo, c64, dv, vl.v[b], iv, iu) * rv;
        march64(geo, tab, vl.v[b], iv, iu, [&](int64_t vox, double wt) { atomicAdd(g + vox, c * wt); });
    }
}

__global__ __launch_bounds__(256) void fill64_kernel(double *__restrict__ g, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) g[i] = 0.0;
}

int grid_for(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_forward64(const fbl_plan *p, const double *x, const ViewList &vl, int nb, double *y,
                            hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    hipLaunchKernelGGL(fp64_kernel, dim3(grid_for((int64_t)nb * p->geo.np)), dim3(256), 0, st, x, p->geo, tab,
                       (const ColParam64 *)p->d_col64, p->geom.dv, vl, nb, y);
    return hipGetLastError();
}

hipError_t launch_backproject64(const fbl_plan *p, const double *r, const ViewList &vl, int nb, double scale,
                                bool accumulate, double *g, hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    if (!accumulate) {
        hipLaunchKernelGGL(fill64_kernel, dim3(grid_for(d)), dim3(256), 0, st, g, d);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bp64_kernel, dim3(grid_for((int64_t)nb * p->geo.np)), dim3(256), 0, st, r, p->geo, tab,
                       (const ColParam64 *)p->d_col64, p->geom.dv, vl, nb, scale, g);
    return hipGetLastError();
}

}  // namespace fbl
