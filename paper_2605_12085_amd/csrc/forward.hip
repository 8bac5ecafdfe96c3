// Forward projection A_N x (Joseph, bilinear) with the residual and FP64 loss epilogue.
#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kTileU = 64;   // one wavefront spans 64 adjacent detector columns of a row
constexpr int kTileV = 4;    // four rows per 256-thread block
constexpr int kChunk = 16;   // slices per FP64 position refresh and per FP32 partial sum

template <typename TV>
__device__ __forceinline__ float tap(const TV *__restrict__ x, int base, int ib, int jz, int nb, int nz, int sb,
                                     int sz)
{
    return ((unsigned)ib < (unsigned)nb && (unsigned)jz < (unsigned)nz) ? to_f32(x[base + ib * sb + jz * sz])
                                                                         : 0.0f;
}

template <typename TV, typename TB>
__global__ __launch_bounds__(256) void fp_kernel(const TV *__restrict__ x, Geo geo, DeviceTables tab, ViewList vl,
                                                 int first, const TB *__restrict__ b, float *__restrict__ y,
                                                 double *__restrict__ partials, int blocks_per_view, int want_loss)
{
    __shared__ double red[4];
    const int bi = blockIdx.y;
    const int view = vl.v[bi];
    const int tiles_u = (geo.nu + kTileU - 1) / kTileU;
    const int iu = (blockIdx.x % tiles_u) * kTileU + (threadIdx.x & (kTileU - 1));
    const int iv = (blockIdx.x / tiles_u) * kTileV + (threadIdx.x / kTileU);
    double sq = 0.0;
    if (iu < geo.nu && iv < geo.nv) {
        const ColParam cp = tab.col[(int64_t)view * geo.nu + iu];
        const double V = tab.rowV[iv];
        // slices along x (axis 0) or y (axis 1); xi runs along the other horizontal axis
        const int na = cp.axis == 0 ? geo.nx : geo.ny;
        const int nb = cp.axis == 0 ? geo.ny : geo.nx;
        const int sa = cp.axis == 0 ? 1 : geo.nx;
        const int sb = cp.axis == 0 ? geo.nx : 1;
        const int sz = geo.nx * geo.ny;
        const float xs = (float)cp.xi1;          // xi per slice
        const float es = (float)(cp.t1 * V);     // eta per slice
        float acc = 0.0f;
        for (int m0 = 0; m0 < na; m0 += kChunk) {
            // FP64 position at the chunk's first slice, split into index + FP32 offset
            const double xb = fma((double)m0, cp.xi1, cp.xi0);
            const double eb = fma(fma((double)m0, cp.t1, cp.t0), V, geo.cz);
            const double fxb = floor(xb), feb = floor(eb);
            const int ib = (int)fxb, jb = (int)feb;
            const float xf = (float)(xb - fxb), ef = (float)(eb - feb);
            const int m1 = min(m0 + kChunk, na);
            float part = 0.0f;
            for (int m = m0; m < m1; ++m) {
                const float fl = (float)(m - m0);
                const float xl = fmaf(fl, xs, xf), el = fmaf(fl, es, ef);
                const float fxl = floorf(xl), fel = floorf(el);
                const int i0 = ib + (int)fxl, j0 = jb + (int)fel;
                const float ax = xl - fxl, ay = el - fel;
                const int base = m * sa;
                const float t00 = tap(x, base, i0, j0, nb, geo.nz, sb, sz);
                const float t10 = tap(x, base, i0 + 1, j0, nb, geo.nz, sb, sz);
                const float t01 = tap(x, base, i0, j0 + 1, nb, geo.nz, sb, sz);
                const float t11 = tap(x, base, i0 + 1, j0 + 1, nb, geo.nz, sb, sz);
                const float lo = fmaf(ax, t10 - t00, t00);
                const float hi = fmaf(ax, t11 - t01, t01);
                part += fmaf(ay, hi - lo, lo);
            }
            acc += part;
        }
        const float w = cp.wa * sqrtf(cp.l2 + tab.rowV2[iv]);
        float val = w * acc;
        if (b) val -= to_f32(b[(int64_t)view * geo.np + (int64_t)iv * geo.nu + iu]);
        y[(int64_t)(first + bi) * geo.np + (int64_t)iv * geo.nu + iu] = val;
        sq = (double)val * (double)val;
    }
    if (want_loss) {
        const double s = block_sum_256(sq, red);
        if (threadIdx.x == 0) partials[(int64_t)(first + bi) * blocks_per_view + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ partials, int64_t n, int ncomp,
                                                       double scale, double *__restrict__ out)
{
    __shared__ double red[4];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += 256) s += partials[i * ncomp + c];
        const double tot = block_sum_256(s, red);
        if (threadIdx.x == 0) out[c] = scale * tot;
    }
}

}  // namespace

int forward_blocks_per_view(const Geo &g)
{
    return ((g.nu + kTileU - 1) / kTileU) * ((g.nv + kTileV - 1) / kTileV);
}

template <typename TV, typename TB>
static hipError_t launch_fp_t(const fbl_plan *p, const void *x, const ViewList &vl, int nb, int first,
                              const void *b, float *y, bool want_loss, hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    dim3 grid(p->fp_blocks_per_view, nb);
    hipLaunchKernelGGL((fp_kernel<TV, TB>), grid, dim3(256), 0, st, (const TV *)x, p->geo, tab, vl, first,
                       (const TB *)b, y, p->d_partials, p->fp_blocks_per_view, want_loss ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_forward(const fbl_plan *p, const void *x, const ViewList &vl, int nb, int first, const void *b,
                          float *y, bool want_loss, hipStream_t st)
{
    const bool bh = p->proj_dtype == FBL_F16;
    switch (p->vol_dtype) {
    case FBL_F32:
        return bh ? launch_fp_t<float, __half>(p, x, vl, nb, first, b, y, want_loss, st)
                  : launch_fp_t<float, float>(p, x, vl, nb, first, b, y, want_loss, st);
    case FBL_BF16:
        return bh ? launch_fp_t<__hip_bfloat16, __half>(p, x, vl, nb, first, b, y, want_loss, st)
                  : launch_fp_t<__hip_bfloat16, float>(p, x, vl, nb, first, b, y, want_loss, st);
    default:
        return bh ? launch_fp_t<__half, __half>(p, x, vl, nb, first, b, y, want_loss, st)
                  : launch_fp_t<__half, float>(p, x, vl, nb, first, b, y, want_loss, st);
    }
}

hipError_t launch_finalize_sum(double *partials, int64_t n, int ncomp, double scale, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, st, (const double *)partials, n, ncomp, scale, out);
    return hipGetLastError();
}

}  // namespace fbl
