// Matched backprojection g = s * A_N^T r: the exact transpose of the forward Joseph
// operator, voxel-tile driven, free of atomics and deterministic.
//
// The forward projection of one view factors per detector column c and slice m into a
// horizontal interpolation at xi_c(m) (taps p, p+1 with weights 1-a, a) and, per ray,
// a vertical interpolation at eta.  Its transpose factors the same way:
//   Z_{c,m}(k) = sum over the column's rays of hat(eta_r(m) - k) * rw_r,
//   g(m, q, k) += sum over columns of hat(xi_c(m) - q) * Z_{c,m}(k),
// with rw = s * w * r (the per-ray path length per slice folded into the residual) and
// hat(t) = max(0, 1 - |t|), which equals the forward's tap weights (zero padding
// included: voxels outside the volume are never written).
//
// A workgroup owns a 16 x 16 x 16 voxel tile and loops over the batch's views.  For a
// view, each axis class of its columns and each half of the tile's slices it
//   1. finds, per slice, the detector columns whose ray plane crosses the tile;
//   2. stages the weighted residual of those columns and of the rows that reach the
//      tile's z-range in LDS, and lets one lane per (slice, column) pair gather that
//      pair's 16-entry z-profile from the few rows within one voxel of each k (rows
//      are equally spaced in eta, so the candidates are consecutive);
//   3. lets each thread gather its 16 voxels from the profiles of the columns whose
//      xi lies within one voxel (binary search: xi is monotone along the row).
#include <climits>

#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kTQ = 16;        // tile extent along x and along y
constexpr int kTK = 16;        // tile extent along z (voxels per thread)
constexpr int kSP = 8;         // slices per pass (two passes cover the tile)
constexpr int kThreads = 256;
constexpr int kRowPad = 8;     // zero rows above and below the staged residual window
constexpr int kWinRows = 48;   // staged rows per column (longer spans read global memory)

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

// Detector column index (fractional) of the ray through the point (X, Y) mm (any z).
__device__ __forceinline__ float column_of(const Geo &geo, const ViewParam &vp, float X, float Y)
{
    const float lat = -X * vp.s + Y * vp.c;
    const float dep = geo.sod - (X * vp.c + Y * vp.s);
    return geo.sdd * lat / dep / geo.du + geo.cu;
}

// z-profile of one (slice, column) pair: Z(kk) = sum_t hat(e_t - kk) * val(t), where row t
// of the pair's source has e_t = a0 + rowz * t (eta relative to the tile's first z).  The
// NC = ceil(2 / rowz) candidates of each kk start at the first row with e_t > kk - 1.
template <int NC, typename Fetch>
__device__ __forceinline__ void pair_profile(float a0, float rowz, int t_lo, int t_hi, Fetch fetch, float *zout,
                                             int zstride)
{
    const float inv = 1.0f / rowz;
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) {
        const float rho = ((float)kk - 1.0f - a0) * inv;   // e_t = kk - 1 at t = rho
        int tf = (int)floorf(rho) + 1;
        tf = min(max(tf, t_lo), t_hi);
        float d = fmaf(rowz, (float)tf, a0 - (float)kk);
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const float w = fmaxf(1.0f - fabsf(d), 0.0f);
            s = fmaf(w, fetch(tf + t), s);
            d += rowz;
        }
        zout[kk * zstride] = s;
    }
}

template <int WP, int NC>
__global__ __launch_bounds__(kThreads, WP <= 48 ? 3 : 2) void bp_kernel(const float *__restrict__ rw, Geo geo, DeviceTables tab,
                                                      ViewList vl, int nb, int first, int accumulate,
                                                      float *__restrict__ g)
{
    constexpr int NPAIR = kSP * WP;
    constexpr int kWinCols = WP + 3 * kSP;          // column union of a pass (per-slice ranges shift)
    constexpr int kWinStride = kWinRows + 2 * kRowPad + 1;   // odd: staging writes avoid bank conflicts
    static_assert(NPAIR <= 2 * kThreads, "a thread owns at most two pairs");
    __shared__ float Z[kTK * NPAIR];                // Z[k][pair]: z-profile of each (slice, column) pair
    __shared__ float xiq[NPAIR];                    // xi of the pair's column on its slice, relative to q0
    __shared__ float win[kWinCols * kWinStride];    // residual window, column-major, zero-padded rows
    __shared__ int colA[kSP], colN[kSP];            // first column and column count per slice
    __shared__ float dirS[kSP];                     // +1 if xi increases along the slice's columns, else -1

    const int tid = threadIdx.x;
    const int tiles_x = (geo.nx + kTQ - 1) / kTQ, tiles_y = (geo.ny + kTQ - 1) / kTQ;
    const int tile = blockIdx.x;
    const int i0 = (tile % tiles_x) * kTQ;
    const int j0 = ((tile / tiles_x) % tiles_y) * kTQ;
    const int k0 = (tile / (tiles_x * tiles_y)) * kTK;
    const int ti = tid % kTQ, tj = tid / kTQ;
    const float cxv = 0.5f * (float)(geo.nx - 1), cyv = 0.5f * (float)(geo.ny - 1);
    const double dvz = (double)geo.dvz;

    float acc[kTK];
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) acc[kk] = 0.0f;

    for (int bi = 0; bi < nb; ++bi) {
        const int view = vl.v[bi];
        const ViewParam vp = tab.view[view];
        const ColParam *__restrict__ cols = tab.col + (int64_t)view * geo.nu;
        const float *__restrict__ rwv = rw + (int64_t)(first + bi) * geo.np;
        // columns whose ray plane crosses the tile's xy square grown by one voxel
        float umin = 3.0e38f, umax = -3.0e38f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float X = ((float)((q & 1) ? i0 + kTQ : i0 - 1) - cxv) * geo.hx;
            const float Y = ((float)((q & 2) ? j0 + kTQ : j0 - 1) - cyv) * geo.hy;
            const float u = column_of(geo, vp, X, Y);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
        const int cT0 = max(0, (int)floorf(fmaxf(umin, -4.0f)) - 1);
        const int cT1 = min(geo.nu - 1, (int)ceilf(fminf(umax, (float)geo.nu + 4.0f)) + 1);
        if (cT0 > cT1) continue;   // uniform across the block
        // columns [0, split) march slices of axis_first, the rest the other axis
        for (int cls = 0; cls < 2; ++cls) {
            const int axis = cls == 0 ? vp.axis_first : 1 - vp.axis_first;
            const int cl0 = cls == 0 ? cT0 : max(cT0, vp.split);
            const int cl1 = cls == 0 ? min(cT1, vp.split - 1) : cT1;
            if (cl0 > cl1) continue;
            const int na = axis == 0 ? geo.nx : geo.ny;
            const int mt0 = axis == 0 ? i0 : j0;       // first slice of the tile
            const int q0 = axis == 0 ? j0 : i0;        // first in-slice index of the tile
            for (int half = 0; half < kTQ / kSP; ++half) {
                __syncthreads();   // the previous pass's readers are done with the shared arrays
                // 1. per-slice column ranges
                if (tid < kSP) {
                    const int mg = mt0 + half * kSP + tid;
                    int a = 0, n = 0;
                    if (mg < na) {
                        const float fm = (float)mg;
                        float u0, u1;
                        if (axis == 0) {
                            const float X = (fm - cxv) * geo.hx;
                            u0 = column_of(geo, vp, X, ((float)(q0 - 1) - cyv) * geo.hy);
                            u1 = column_of(geo, vp, X, ((float)(q0 + kTQ) - cyv) * geo.hy);
                        } else {
                            const float Y = (fm - cyv) * geo.hy;
                            u0 = column_of(geo, vp, ((float)(q0 - 1) - cxv) * geo.hx, Y);
                            u1 = column_of(geo, vp, ((float)(q0 + kTQ) - cxv) * geo.hx, Y);
                        }
                        const float lo = fminf(u0, u1), hi = fmaxf(u0, u1);
                        a = max(cl0, (int)floorf(fmaxf(lo, -4.0f)) - 1);
                        const int b = min(cl1, (int)ceilf(fminf(hi, (float)geo.nu + 4.0f)) + 1);
                        n = min(WP, max(0, b - a + 1));
                    }
                    colA[tid] = a;
                    colN[tid] = n;
                }
                __syncthreads();
                // 2a. the pass's detector window: columns [c0, c1] (union of the slices'
                //     ranges) and every row that can reach z in (k0 - 1, k0 + kTK).  The
                //     ray parameter tau is monotone along a detector row (it is inversely
                //     proportional to the column's D_a, which is affine in the column) and
                //     affine in the slice index, so its extremes over the pass sit at the
                //     corner (first/last column, first/last slice) pairs; the detector row
                //     of a given height is monotone in tau.
                int c0 = INT_MAX, c1 = -1;
#pragma unroll
                for (int m = 0; m < kSP; ++m)
                    if (colN[m] > 0) {
                        c0 = min(c0, colA[m]);
                        c1 = max(c1, colA[m] + colN[m] - 1);
                    }
                if (c1 < 0) continue;   // uniform across the block
                int r0, nR;
                {
                    const int mA = mt0 + half * kSP, mB = min(mA + kSP - 1, na - 1);
                    const ColParam ca = cols[c0], cb = cols[c1];
                    const double t00 = fma((double)mA, ca.t1, ca.t0), t01 = fma((double)mB, ca.t1, ca.t0);
                    const double t10 = fma((double)mA, cb.t1, cb.t0), t11 = fma((double)mB, cb.t1, cb.t0);
                    // bounds in FP32 (rounding is far below the one-row margins)
                    const float imin = 1.0f / (float)(fmax(fmax(t00, t01), fmax(t10, t11)) * dvz);
                    const float imax = 1.0f / (float)(fmin(fmin(t00, t01), fmin(t10, t11)) * dvz);
                    const float e0 = (float)((double)(k0 - 1) - geo.cz), e1 = (float)((double)(k0 + kTK) - geo.cz);
                    const float a = e0 * imin, b = e0 * imax, c = e1 * imin, d = e1 * imax;
                    const float rlo = fminf(fminf(a, b), fminf(c, d)) + geo.cv;
                    const float rhi = fmaxf(fmaxf(a, b), fmaxf(c, d)) + geo.cv;
                    r0 = max(0, (int)floorf(rlo) - 1);
                    nR = min(geo.nv - 1, (int)ceilf(rhi) + 1) - r0 + 1;
                }
                if (nR <= 0) continue;   // uniform
                const int nC = c1 - c0 + 1;
                const bool staged = nR <= kWinRows && nC <= kWinCols;
                // staging: every load is issued before the LDS writes; consecutive lanes
                // read consecutive columns (contiguous in memory); addresses are clamped
                // into the detector and entries outside the window are written as 0
                constexpr int kWinSize = kWinCols * kWinStride;
                constexpr int kIt = (kWinSize + kThreads - 1) / kThreads;
                float stv[kIt];
                if (staged) {
#pragma unroll
                    for (int it = 0; it < kIt; ++it) {
                        const int e = tid + it * kThreads;
                        const int col = e % kWinCols, row = e / kWinCols;
                        const int r = min(max(r0 + row - kRowPad, 0), geo.nv - 1);
                        const int cc = min(c0 + col, geo.nu - 1);
                        stv[it] = rwv[(int64_t)r * geo.nu + cc];
                    }
                }
                // 2b. pair geometry: xi for step 3 and the ray parameter for the profile
                double ptau[2] = {0.0, 0.0};
                int pcol[2] = {0, 0};
                bool pin[2] = {false, false};
#pragma unroll
                for (int sI = 0; sI < 2; ++sI) {
                    const int pr = tid + sI * kThreads;
                    if (pr < NPAIR) {
                        const int ml = pr % kSP, cl = pr / kSP;
                        float xl = 3.0e38f;
                        if (cl < colN[ml]) {
                            const int c = colA[ml] + cl;
                            const ColParam cp = cols[c];
                            const double fm = (double)(mt0 + half * kSP + ml);
                            xl = (float)(fma(fm, cp.xi1, cp.xi0) - (double)q0);
                            if (xl > -1.0f && xl < (float)kTQ) {
                                pin[sI] = true;
                                pcol[sI] = c;
                                ptau[sI] = fma(fm, cp.t1, cp.t0);
                            }
                        }
                        xiq[pr] = xl;
                    }
                }
                if (staged) {
#pragma unroll
                    for (int it = 0; it < kIt; ++it) {
                        const int e = tid + it * kThreads;
                        if (e < kWinSize) {
                            const int col = e % kWinCols, row = e / kWinCols;
                            const bool inside = row >= kRowPad && row < kRowPad + nR && col < nC;
                            win[col * kWinStride + row] = inside ? stv[it] : 0.0f;
                        }
                    }
                }
                __syncthreads();
                if (tid < kSP) {
                    const int n = colN[tid];
                    dirS[tid] = (n >= 2 && xiq[(n - 1) * kSP + tid] < xiq[tid]) ? -1.0f : 1.0f;
                }
                // 2c. one lane per pair gathers the pair's z-profile
#pragma unroll
                for (int sI = 0; sI < 2; ++sI) {
                    const int pr = tid + sI * kThreads;
                    if (pr < NPAIR && pin[sI]) {
                        const double rowz = ptau[sI] * dvz;
                        const float rz = (float)rowz;
                        if (staged) {
                            // source row t = window row (t - kRowPad) = detector row r0 + t - kRowPad
                            const float a0 = (float)(geo.cz + ptau[sI] * ((double)(r0 - kRowPad) - (double)geo.cv) * dvz -
                                                     (double)k0);
                            const float *__restrict__ wc = win + (pcol[sI] - c0) * kWinStride;
                            pair_profile<NC>(a0, rz, 0, kWinStride - NC, [&](int t) { return wc[t]; }, Z + pr, NPAIR);
                        } else {
                            // detector row t directly (rows outside [0, nv) do not exist)
                            const float a0 = (float)(geo.cz + ptau[sI] * (0.0 - (double)geo.cv) * dvz - (double)k0);
                            const float *__restrict__ src = rwv + pcol[sI];
                            const int64_t nu = geo.nu;
                            pair_profile<NC>(a0, rz, 0, max(0, geo.nv - NC),
                                             [&](int t) {
                                                 const float v = src[(int64_t)min(t, geo.nv - 1) * nu];
                                                 return t < geo.nv ? v : 0.0f;
                                             },
                                             Z + pr, NPAIR);
                        }
                    }
                }
                __syncthreads();
                // 3. each thread gathers its voxel column (m, q) from the columns near q
                const int ml = (axis == 0 ? ti : tj) - half * kSP;
                if (ml >= 0 && ml < kSP) {
                    const float q = (float)(axis == 0 ? tj : ti);
                    const int n = colN[ml];
                    const float s = dirS[ml];
                    // first pair with s*xi > s*q - 1 (s*xi increases with the pair index)
                    int lo = 0, hi = n;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s * xiq[mid * kSP + ml] > s * q - 1.0f) hi = mid;
                        else lo = mid + 1;
                    }
                    for (int p = lo; p < n; ++p) {
                        const float xv = xiq[p * kSP + ml];
                        if (!(s * xv < s * q + 1.0f)) break;
                        const float w = 1.0f - fabsf(xv - q);
                        if (w > 0.0f) {
                            const float *__restrict__ zp = Z + (p * kSP + ml);
#pragma unroll
                            for (int kk = 0; kk < kTK; ++kk) acc[kk] = fmaf(w, zp[kk * NPAIR], acc[kk]);
                        }
                    }
                }
            }
        }
    }
    const int i = i0 + ti, j = j0 + tj;
    if (i < geo.nx && j < geo.ny) {
        const int64_t base = (int64_t)j * geo.nx + i;
        const int64_t zs = (int64_t)geo.nx * geo.ny;
#pragma unroll
        for (int kk = 0; kk < kTK; ++kk) {
            const int k = k0 + kk;
            if (k < geo.nz) {
                const int64_t o = base + (int64_t)k * zs;
                g[o] = accumulate ? g[o] + acc[kk] : acc[kk];
            }
        }
    }
}

}  // namespace

int backproject_tile() { return kTQ; }

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

template <int WP, int NC>
static hipError_t launch_bp_t(const fbl_plan *p, const float *rw, const ViewList &vl, int nb, int first,
                              bool accumulate, float *g, hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    const int tiles = ((p->geo.nx + kTQ - 1) / kTQ) * ((p->geo.ny + kTQ - 1) / kTQ) * ((p->geo.nz + kTK - 1) / kTK);
    hipLaunchKernelGGL((bp_kernel<WP, NC>), dim3(tiles), dim3(kThreads), 0, st, rw, p->geo, tab, vl, nb, first,
                       accumulate ? 1 : 0, g);
    return hipGetLastError();
}

template <int WP>
static hipError_t launch_bp_w(const fbl_plan *p, const float *rw, const ViewList &vl, int nb, int first,
                              bool accumulate, float *g, hipStream_t st)
{
    switch (p->bp_cand) {
    case 3: return launch_bp_t<WP, 3>(p, rw, vl, nb, first, accumulate, g, st);
    case 4: return launch_bp_t<WP, 4>(p, rw, vl, nb, first, accumulate, g, st);
    case 5: return launch_bp_t<WP, 5>(p, rw, vl, nb, first, accumulate, g, st);
    case 6: return launch_bp_t<WP, 6>(p, rw, vl, nb, first, accumulate, g, st);
    default: return launch_bp_t<WP, 8>(p, rw, vl, nb, first, accumulate, g, st);
    }
}

hipError_t launch_backproject(const fbl_plan *p, const float *rw, const ViewList &vl, int nb, int first,
                              bool accumulate, float *g, hipStream_t st)
{
    switch (p->bp_pairs) {
    case 48: return launch_bp_w<48>(p, rw, vl, nb, first, accumulate, g, st);
    case 64: return launch_bp_w<64>(p, rw, vl, nb, first, accumulate, g, st);
    default: return launch_bp_w<32>(p, rw, vl, nb, first, accumulate, g, st);
    }
}

}  // namespace fbl
