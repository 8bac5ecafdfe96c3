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
// view and each axis class of its columns it
//   1. finds, per slice of the tile, the detector columns whose ray plane crosses the
//      tile, and lists the (slice, column) pairs with their xi and ray parameter;
// then, for each half of the tile's z-range,
//   2. reads the weighted residual of those columns on the rows that reach the half's
//      z-range and keeps, per column, two prefix sums over its rows in LDS: of the
//      residual and of the residual times the row index;
//   3. forms each pair's 8-entry z-profile from those prefix sums (below);
//   4. lets every thread add to its voxel column (m, q) the profiles of the columns whose
//      xi lies within one voxel (a contiguous run of the slice's pairs, located from the
//      columns through (m, q - 1) and (m, q + 1)).
//
// Profiles from prefix sums.  The hat is the second difference of the ramp
// ramp(t) = max(0, t):  hat(e - k) = ramp(k + 1 - e) - 2 ramp(k - e) + ramp(k - 1 - e).
// So Z(k) = H(k + 1) - 2 H(k) + H(k - 1) with H(y) = sum over rows with e_s < y of
// (y - e_s) v_s, and since a pair's rows are equally spaced (e_s = a + b s),
//   H(y) = (y - a) P(T) - b Q(T),  P(T) = sum_{s<T} v_s,  Q(T) = sum_{s<T} s v_s,
// where T(y) is the number of rows below y.  Ten look-ups give the 8 entries of a half;
// the column's two prefix arrays are shared by the pairs of all 16 slices.  A row whose
// position is within rounding of y enters H(y) with weight y - e_s ~ 0, so T needs no
// exact rounding, and rows below the window add an affine function of y to H, which
// the second difference removes.  The cancellation in that difference is why the sums
// are exact: each column's residuals are scaled by a power of two to at most 2^22 in
// magnitude and rounded to integers (a relative change of at most 2^-23 of the
// column's largest entry, the size of one FP32 rounding of it), their prefix sums are
// exact 32-bit integers, and H and its second difference are taken in FP64.
#include <climits>
#include <type_traits>

#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kTQ = 16;        // tile extent along x and along y (and slices per class pass)
constexpr int kTK = 16;        // tile extent along z (voxels per thread)
constexpr int kKH = 8;         // z-entries per half pass
constexpr int kKQ = 4;         // z-entries per work item of the fallback tap loop
static_assert(kKH == 2 * kKQ, "the fallback tap loop has two items per pair and half pass");
constexpr int kThreads = 256;
constexpr int kWinRows = 28;   // staged rows per column (longer spans read global memory)
constexpr int kSegRows = kWinRows / 4;     // rows per lane: four lanes share a column
static_assert(kWinRows % 4 == 0, "a column's rows split evenly over four lanes");
// Prefix entries per column (odd: adjacent columns use distinct banks).  A stride of 31,
// which spreads a wave's look-ups over more banks, was measured 28% slower: the block's
// LDS then exceeds a third of the compute unit's in allocation granules, and only two
// blocks fit per compute unit instead of three.
constexpr int kPreStride = kWinRows + 1;
constexpr int kRowCen = kWinRows / 2;      // row origin of the moment prefix (keeps it within 32 bits)
constexpr int kQuantBits = 22;             // residuals are scaled to at most 2^22 in magnitude
constexpr float kRoundMagic = 12582912.0f; // 1.5 * 2^23
constexpr int kBufferFlags = 0x00020000;   // word 3 of a raw gfx9 buffer resource (32-bit data)
// A buffer offset past the end of every residual window: the plan admits at most 2^28 detector
// pixels, i.e. 2^30 bytes per view, and offsets stay far below 2^32.
constexpr int kOutOfRange = 1 << 30;
constexpr int kWinExtra = 16;  // columns the 16 slices' ranges may add to one slice's
// Bound on the error of a detector column computed by column_of (FP32, hardware
// reciprocal; a few 1e-4 columns at 1536 columns), with margin.
constexpr float kColTol = 0.01f;

// Lane exchanges within a wave64.  A row is 16 consecutive lanes; DPP moves stay within a
// row, and gfx950's permlane swaps exchange whole rows.
constexpr int kDppRowShr1 = 0x111;         // row_shr:n is kDppRowShr1 - 1 + n
constexpr int kDppXor1 = 0xB1;             // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;             // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;   // lane i <-> 7 - i within each half row
constexpr int kDppRowMirror = 0x140;       // lane i <-> 15 - i within the row

template <int kCtrl>
__device__ __forceinline__ int dpp(int x)
{
    // bound_ctrl: a source lane outside the row reads 0
    return __builtin_amdgcn_update_dpp(0, x, kCtrl, 0xF, 0xF, true);
}

// Inclusive prefix sum over the 16 lanes of each row.
__device__ __forceinline__ int row_inclusive_sum(int x)
{
    x += dpp<kDppRowShr1>(x);
    x += dpp<kDppRowShr1 + 1>(x);
    x += dpp<kDppRowShr1 + 3>(x);
    x += dpp<kDppRowShr1 + 7>(x);
    return x;
}

// Minimum and maximum over the 16 lanes of each row, in every lane of the row.
__device__ __forceinline__ int row_min(int x)
{
    x = min(x, dpp<kDppXor1>(x));
    x = min(x, dpp<kDppXor2>(x));
    x = min(x, dpp<kDppRowHalfMirror>(x));
    return min(x, dpp<kDppRowMirror>(x));
}
__device__ __forceinline__ int row_max(int x)
{
    x = max(x, dpp<kDppXor1>(x));
    x = max(x, dpp<kDppXor2>(x));
    x = max(x, dpp<kDppRowHalfMirror>(x));
    return max(x, dpp<kDppRowMirror>(x));
}

// Maximum over the four lanes l, l ^ 16, l ^ 32, l ^ 48 (the same lane of every row), NaN
// if any of them is NaN.
// permlane16_swap(x, x) returns x of the even row of each row pair in its first element
// and x of the odd row in its second, in both rows; permlane32_swap likewise returns the
// lower and the upper half's x.
__device__ __forceinline__ float rows_max(float x)
{
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __builtin_elementwise_maximum(__uint_as_float(a[0]), __uint_as_float(a[1]));
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __builtin_elementwise_maximum(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

// Sum of x over the lanes of rows 0 .. row - 1 at this lane's position in the row.
__device__ __forceinline__ int rows_exclusive_sum(int x, int row)
{
    const auto a = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
    const int even = (int)a[0], pair = (int)a[0] + (int)a[1];   // even row's x; the row pair's sum
    const auto b = __builtin_amdgcn_permlane32_swap((unsigned)pair, (unsigned)pair, false, false);
    return ((row & 1) ? even : 0) + (row >= 2 ? (int)b[0] : 0);
}

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
// Column ranges are built from its floor and ceiling, which tolerate any error below one
// column, so the hardware reciprocal (within a few units in the last place) serves
// instead of a division.
__device__ __forceinline__ float column_of(const Geo &geo, const ViewParam &vp, float X, float Y)
{
    const float lat = -X * vp.s + Y * vp.c;
    const float dep = geo.sod - (X * vp.c + Y * vp.s);
    return fmaf(geo.sdd * lat, __builtin_amdgcn_rcpf(dep * geo.du), geo.cu);
}

// Part of the z-profile of one (slice, column) pair, tap by tap (the path for windows
// too tall to stage): Z(kk) = sum_t hat(e_t - kk) * val(t) for kk = kk0 .. kk0 + kKQ - 1,
// where row t of the pair's source has e_t = a0 + rowz * t (eta relative to the pass's
// first z) and inv = 1 / rowz.  The NC candidates of each kk start at the first row with
// e_t > kk - 1 as computed in FP32, clamped to [t_lo, t_hi]; NC = ceil(2 / rowz) + 1, one
// more than the rows in reach, covers a start one row early by rounding.  store(kk, Z)
// receives each entry.
template <int NC, typename Fetch, typename Store>
__device__ __forceinline__ void pair_profile(float a0, float rowz, float inv, int kk0, float t_lo, float t_hi,
                                             Fetch fetch, Store store)
{
    const float c1 = fmaf(-1.0f - a0, inv, 1.0f);
#pragma unroll
    for (int j = 0; j < kKQ; ++j) {
        // e_t = kk - 1 at t = rho; the first candidate is floor(rho) + 1 = floor(rho + 1)
        const float rho1 = fmaf((float)(kk0 + j), inv, c1);
        const float tf = __builtin_amdgcn_fmed3f(floorf(rho1), t_lo, t_hi);
        const int t0 = (int)tf;
        float d = fmaf(rowz, tf, a0 - (float)(kk0 + j));
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const float w = fmaxf(1.0f - fabsf(d), 0.0f);
            s = fmaf(w, fetch(t0 + t), s);
            d += rowz;
        }
        store(kk0 + j, s);
    }
}

template <int WP, int NC>
__global__ __launch_bounds__(kThreads, WP <= 48 ? 3 : 2) void bp_kernel(const float *__restrict__ rw, Geo geo,
                                                                        DeviceTables tab, ViewList vl, int nb,
                                                                        int first, int accumulate,
                                                                        const int *__restrict__ order,
                                                                        float *__restrict__ g)
{
    constexpr int NPM = kTQ * WP;                     // pair slots: 16 slices x WP columns
    constexpr int kWinCols = WP + kWinExtra;          // column union of the 16 slices
    constexpr int kColSweeps = (kWinCols + 63) / 64;  // window columns: 16 per wave and sweep
    constexpr int kPairIters = (NPM + kThreads - 1) / kThreads;
    __shared__ float Z[kKH * NPM];                    // Z[k][pair]: half-pass z-profile of each pair
    __shared__ float xiq[NPM];                        // xi of the pair's column on its slice, minus q0
    __shared__ float prz[NPM];                        // row spacing in eta there; 0 if xi misses the tile
    __shared__ float pa0[2][NPM];                     // per half: eta of the pair's source row 0, minus the
                                                      // half's first z (window row 0 if staged, else detector row 0)
    __shared__ short pcr[NPM];                        // the pair's column minus the class window's c0
    __shared__ int2 pre[kWinCols * kPreStride];       // per window column and T: (P(T), Q(T)), integers
    __shared__ double psc[kWinCols];                  // per window column: 2^-(residual scale exponent),
                                                      // NaN for a column with a non-finite entry

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (geo.nx + kTQ - 1) / kTQ, tiles_y = (geo.ny + kTQ - 1) / kTQ;
    const int tile = order[blockIdx.x];   // a permutation of the tiles (launch order)
    const int i0 = (tile % tiles_x) * kTQ;
    const int j0 = ((tile / tiles_x) % tiles_y) * kTQ;
    const int k0 = (tile / (tiles_x * tiles_y)) * kTK;
    const int ti = tid % kTQ, tj = tid / kTQ;
    const float cxv = 0.5f * (float)(geo.nx - 1), cyv = 0.5f * (float)(geo.ny - 1);
    const double dvz = (double)geo.dvz;

    float acc[kTK];
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) acc[kk] = 0.0f;

    ViewParam vp_next = tab.view[vl.v[0]];   // loaded a view ahead
    for (int bi = 0; bi < nb; ++bi) {
        const int view = vl.v[bi];
        const ViewParam vp = vp_next;
        if (bi + 1 < nb) vp_next = tab.view[vl.v[bi + 1]];
        const ColParam *__restrict__ cols = tab.col + (int64_t)view * geo.nu;
        const float *__restrict__ rwv = rw + (int64_t)(first + bi) * geo.np;
        // columns whose ray plane crosses the tile's xy square grown by one voxel (with a
        // column of margin): they bound the row windows below
        // and the depths of its corners from the source along the central ray
        float umin = 3.0e38f, umax = -3.0e38f, dmin = 3.0e38f, dmax = -3.0e38f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float X = ((float)((q & 1) ? i0 + kTQ : i0 - 1) - cxv) * geo.hx;
            const float Y = ((float)((q & 2) ? j0 + kTQ : j0 - 1) - cyv) * geo.hy;
            const float u = column_of(geo, vp, X, Y);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            const float dep = geo.sod - (X * vp.c + Y * vp.s);
            dmin = fminf(dmin, dep);
            dmax = fmaxf(dmax, dep);
        }
        const int cT0 = max(0, (int)floorf(fmaxf(umin, -4.0f)) - 1);
        const int cT1 = min(geo.nu - 1, (int)ceilf(fminf(umax, (float)geo.nu + 4.0f)) + 1);
        if (cT0 > cT1) continue;   // uniform across the block
        {
            // A ray's parameter at a point is the point's depth over SDD (the detector is
            // flat and faces the source), so inside the square it lies in
            // [dmin, dmax] / SDD, and detector row r reaches the vertical index coordinate
            // eta there at r = cv + (eta - cz) / (tau dv/hz).  No row within two of the
            // detector reaching eta in (k0 - 1, k0 + kTK): the view adds nothing to the tile.
            const float e0 = (float)((double)(k0 - 1) - geo.cz), e1 = (float)((double)(k0 + kTK) - geo.cz);
            const float s0 = geo.sdd * __builtin_amdgcn_rcpf(dmin * geo.dvz);   // 1 / (tau dv/hz)
            const float s1 = geo.sdd * __builtin_amdgcn_rcpf(dmax * geo.dvz);
            const float rlo = fminf(fminf(e0 * s0, e0 * s1), fminf(e1 * s0, e1 * s1)) + geo.cv;
            const float rhi = fmaxf(fmaxf(e0 * s0, e0 * s1), fmaxf(e1 * s0, e1 * s1)) + geo.cv;
            if (rlo > (float)(geo.nv + 1) || rhi < -2.0f) continue;   // uniform across the block
        }
        // columns [0, split) march slices of axis_first, the rest the other axis (a view
        // whose fan crosses a diagonal has two classes, any other view one)
        for (int cls = 0; cls < 2; ++cls) {
            const int axis = cls == 0 ? vp.axis_first : 1 - vp.axis_first;
            const int cl0 = cls == 0 ? cT0 : max(cT0, vp.split);
            const int cl1 = cls == 0 ? min(cT1, vp.split - 1) : cT1;
            if (cl0 > cl1) continue;
            const int na = axis == 0 ? geo.nx : geo.ny;
            const int mt0 = axis == 0 ? i0 : j0;       // first slice of the tile
            const int q0 = axis == 0 ? j0 : i0;        // first in-slice index of the tile
            // 1. per-slice column ranges: lane l of every 16-lane row holds slice l & 15, so
            //    every row of every wave holds all 16 slices.  Each slice's first pair (a
            //    prefix sum over the row) and the class window's columns [c0, c1] (the union
            //    of the slices' ranges, a reduction over the row) come from row-local DPP
            //    moves; every wave computes the same values from the same inputs and keeps
            //    them in its own registers, so none pass through LDS.
            int sa, sn, sp, c0, c1, NP;
            {
                const int mg = mt0 + (lane & 15);
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
                    // the columns strictly between u0 and u1 cross the slice within one voxel
                    // of the tile; u is within kColTol of its exact value, so the columns
                    // above lo - kColTol and below hi + kColTol hold them all
                    const float lo = fminf(u0, u1), hi = fmaxf(u0, u1);
                    a = max(cl0, (int)floorf(fmaxf(lo, -4.0f) - kColTol) + 1);
                    const int b = min(cl1, (int)ceilf(fminf(hi, (float)geo.nu + 4.0f) + kColTol) - 1);
                    n = min(WP, max(0, b - a + 1));
                }
                const int incl = row_inclusive_sum(n);
                const int lo = row_min(n > 0 ? a : INT_MAX), hi = row_max(n > 0 ? a + n - 1 : -1);
                sa = a;
                sn = n;
                sp = incl - n;
                c0 = __builtin_amdgcn_readlane(lo, 0);
                c1 = __builtin_amdgcn_readlane(hi, 0);
                NP = __builtin_amdgcn_readlane(incl, kTQ - 1);
            }
            if (c1 < 0) continue;   // no ray of the class crosses the tile (uniform across the block)
            const int nC = c1 - c0 + 1;
            // Every pair lies within the class's columns [cl0, cl1], and the ray parameter is
            // monotone along a detector row, so bounds taken at these two columns hold for
            // all pairs.
            const ColParam ca = cols[cl0], cb = cols[cl1];
            // Pair tables: thread tid takes the pairs of its lane's slice tid & 15 (whose
            // range it holds) at column offsets tid / 16 + 16 i (kPairIters = WP / 16 rounds
            // cover the slice's at most WP).  Their column parameters are loaded with the two
            // above, so that the latencies overlap.
            static_assert(kThreads == kTQ * 16 && WP % 16 == 0, "16 threads per slice");
            const int sm = lane & 15, si = tid >> 4;
            ColParam pc[kPairIters];
#pragma unroll
            for (int i = 0; i < kPairIters; ++i)
                if (si + 16 * i < sn) pc[i] = cols[sa + si + 16 * i];
            __syncthreads();   // the previous class's readers are done with the shared arrays
            // bounds of the ray parameter over the class's pairs: tau is monotone along a
            // detector row (inversely proportional to the column's D_a, which is affine in
            // the column) and affine in the slice, so over columns [cl0, cl1] and the tile's
            // slices they sit at the corners; a detector row of a given height is monotone in
            // tau.  Bounds are taken in FP32 with the hardware reciprocal (rounding is far
            // below the one-row margins).
            float imin, imax;
            {
                const int mA = mt0, mB = min(mt0 + kTQ - 1, na - 1);
                const double t00 = fma((double)mA, ca.t1, ca.t0), t01 = fma((double)mB, ca.t1, ca.t0);
                const double t10 = fma((double)mA, cb.t1, cb.t0), t11 = fma((double)mB, cb.t1, cb.t0);
                imin = __builtin_amdgcn_rcpf((float)(fmax(fmax(t00, t01), fmax(t10, t11)) * dvz));
                imax = __builtin_amdgcn_rcpf((float)(fmin(fmin(t00, t01), fmin(t10, t11)) * dvz));
            }
            // per half: detector rows that can reach z in (kb - 1, kb + kKH), kb = k0 + h kKH
            int r0h[2], nRh[2];
            bool stg[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int kb = k0 + h * kKH;
                const float e0 = (float)((double)(kb - 1) - geo.cz), e1 = (float)((double)(kb + kKH) - geo.cz);
                const float a = e0 * imin, b = e0 * imax, c = e1 * imin, d = e1 * imax;
                const float rlo = fminf(fminf(a, b), fminf(c, d)) + geo.cv;
                const float rhi = fmaxf(fmaxf(a, b), fmaxf(c, d)) + geo.cv;
                r0h[h] = max(0, (int)floorf(rlo) - 1);
                nRh[h] = min(geo.nv - 1, (int)ceilf(rhi) + 1) - r0h[h] + 1;
                stg[h] = nRh[h] > 0 && nRh[h] <= kWinRows && nC <= kWinCols;
            }
            // no detector row reaches the tile's z-range (a tile above or below the view's
            // cone): nothing to add (uniform across the block)
            if (nRh[0] <= 0 && nRh[1] <= 0) continue;
            // The pairs' column parameters and the first half's residual window are loaded
            // together, before either is used; the second half's window is loaded after
            // the first half's profiles, so that it arrives during that half's gather.
            // Window row t is detector row r0 + t (zero for t >= nR).  Four lanes share a
            // window column (lanes c, c + 16, c + 32, c + 48 of a wave), each holding
            // kSegRows consecutive rows.
            const int wcol = (lane & 15) + 16 * wave, wseg = lane >> 4;
            float wv[kColSweeps][kSegRows];
            // Loads are unconditional buffer loads, so that they issue back to back without
            // branches or address arithmetic and stay in flight until the prefix sums use
            // them; the buffer's bounds make every entry outside the window 0 (so a
            // non-finite value outside it never reaches the prefix sums).
            auto load_window = [&](int h) {
                // The view's residual up to the window's last row as one buffer: rows below the
                // window read past its end, and a lane whose window column lies past the
                // window's columns reads at kOutOfRange, so every entry outside the window
                // loads as 0.  Rows step by a uniform offset (scalar registers).
                const __amdgpu_buffer_rsrc_t win = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)rwv, (short)0, (r0h[h] + nRh[h]) * geo.nu * 4, kBufferFlags);
#pragma unroll
                for (int cs = 0; cs < kColSweeps; ++cs) {
                    const int col = wcol + 64 * cs;
                    const int vo = col < nC ? ((r0h[h] + wseg * kSegRows) * geo.nu + c0 + col) * 4 : kOutOfRange;
#pragma unroll
                    for (int j = 0; j < kSegRows; ++j)
                        wv[cs][j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(win, vo, j * geo.nu * 4, 0));
                }
            };
            // Prefix sums of the loaded window: the column's scale exponent from its largest
            // magnitude (two exchanges among its four lanes), each lane's running sums over
            // its rows, then the sums of the lanes below it added (an inclusive scan over the
            // four lanes).  |q| <= 2^22 keeps |P| < 2^27 and |Q| < 196 * 2^22 < 2^31.
            auto build_prefix = [&](int h) {
#pragma unroll
                for (int cs = 0; cs < kColSweeps; ++cs) {
                    const int col = wcol + 64 * cs;
                    // largest magnitude, NaN if any entry is NaN (IEEE maximum propagates it)
                    float mx = 0.0f;
#pragma unroll
                    for (int j = 0; j < kSegRows; ++j) mx = __builtin_elementwise_maximum(mx, fabsf(wv[cs][j]));
                    mx = rows_max(mx);
                    const bool fin = mx <= 3.4028235e38f;   // false for inf and NaN
                    int ex;
                    (void)frexpf(fin ? mx : 1.0f, &ex);      // mx < 2^ex
                    // 2^kx, kept a normal FP32 number: only a column whose entries all lie
                    // below 2^-105 in magnitude is quantised more coarsely than 2^-22 of its
                    // largest (at 2^-127 absolute)
                    const int kx = min(kQuantBits - ex, 127);
                    const float scl = ldexpf(1.0f, kx);
                    int P = 0, Q = 0, ps[kSegRows], qs[kSegRows];
#pragma unroll
                    for (int j = 0; j < kSegRows; ++j) {
                        // round(v 2^kx) for |v 2^kx| < 2^22: adding 1.5 2^23 leaves it in
                        // [2^23, 2^24], where FP32 steps by one, so the bits count the integer
                        // (entries of a non-finite column give garbage; the column is marked)
                        const int q = __float_as_int(fmaf(wv[cs][j], scl, kRoundMagic)) - __float_as_int(kRoundMagic);
                        P += q;
                        // |row - kRowCen| <= 14 and |q| <= 2^22 both fit 24 bits: a 24-bit product
                        Q += __mul24(wseg * kSegRows + j - kRowCen, q);
                        ps[j] = P;
                        qs[j] = Q;
                    }
                    // sums of the rows below this lane's (the lanes of rows 0 .. wseg - 1)
                    const int oP = rows_exclusive_sum(P, wseg), oQ = rows_exclusive_sum(Q, wseg);
                    if (col < nC) {
                        int2 *__restrict__ dst = pre + col * kPreStride;
                        if (wseg == 0) {
                            dst[0] = make_int2(0, 0);
                            psc[col] = fin ? ldexp(1.0, -kx) : __builtin_nan("");
                        }
#pragma unroll
                        for (int j = 0; j < kSegRows; ++j)
                            dst[wseg * kSegRows + j + 1] = make_int2(ps[j] + oP, qs[j] + oQ);
                    }
                }
            };
            if (stg[0]) load_window(0);
            // 2. pair geometry: xi for the voxel gather, the ray parameter for the profile
#pragma unroll
            for (int i = 0; i < kPairIters; ++i) {
                const int cl = si + 16 * i;
                if (cl < sn) {
                    const int p = sp + cl;
                    const ColParam &cp = pc[i];
                    const double fm = (double)(mt0 + sm);
                    const float xl = (float)(fma(fm, cp.xi1, cp.xi0) - (double)q0);
                    xiq[p] = xl;
                    const bool in = xl > -1.0f && xl < (float)kTQ;
                    const double B = fma(fm, cp.t1, cp.t0) * dvz;   // tau dv/hz: eta per detector row
                    prz[p] = in ? (float)B : 0.0f;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double row0 = stg[h] ? (double)r0h[h] : 0.0;
                        pa0[h][p] = (float)fma(B, row0 - (double)geo.cv, geo.cz - (double)(k0 + h * kKH));
                    }
                    pcr[p] = (short)(sa + cl - c0);
                }
            }
            if (stg[0]) build_prefix(0);
            __syncthreads();   // pair tables and the first half's prefix sums complete
            // This thread's voxel column (slice m, in-slice index q) takes the pairs of slice m
            // whose xi lies within one voxel of q; both halves use them.  The detector column
            // through a point is monotone along the slice, so those pairs are the columns
            // between the ones through (m, q - 1) and (m, q + 1): the floor and ceiling of
            // those two (in FP32, far within a column of the exact values) bound them with at
            // most two columns to spare at either end, and the spare ones, whose xi as stored
            // lies a voxel or more from q, are dropped after reading the two outermost of
            // each end (xi is monotone along a slice's pairs).
            const float gq = (float)(axis == 0 ? tj : ti);
            int gfirst = 0, gcnt = 0;
            {
                int ga = sa, gn = sn, gp = sp;   // axis 0: the slice is this lane's own, ti
                if (axis != 0) {                 // axis 1: slice tj, held by lane tj of every row
                    ga = __shfl(sa, tj);
                    gn = __shfl(sn, tj);
                    gp = __shfl(sp, tj);
                }
                const float fm = (float)(mt0 + (axis == 0 ? ti : tj));
                float u0, u1;
                if (axis == 0) {
                    const float X = (fm - cxv) * geo.hx;
                    u0 = column_of(geo, vp, X, ((float)(q0 - 1) + gq - cyv) * geo.hy);
                    u1 = column_of(geo, vp, X, ((float)(q0 + 1) + gq - cyv) * geo.hy);
                } else {
                    const float Y = (fm - cyv) * geo.hy;
                    u0 = column_of(geo, vp, ((float)(q0 - 1) + gq - cxv) * geo.hx, Y);
                    u1 = column_of(geo, vp, ((float)(q0 + 1) + gq - cxv) * geo.hx, Y);
                }
                int f = max(ga, (int)floorf(fmaxf(fminf(u0, u1), -4.0f)));
                int l = min(ga + gn - 1, (int)ceilf(fminf(fmaxf(u0, u1), (float)geo.nu + 4.0f)));
                if (f <= l) {
                    const float *__restrict__ xs = xiq + (gp - ga);   // xs[c]: xi of column c's pair
                    const float xf0 = xs[f], xf1 = xs[min(f + 1, l)];
                    const float xl0 = xs[l], xl1 = xs[max(l - 1, f)];
                    f += fabsf(xf0 - gq) < 1.0f ? 0 : fabsf(xf1 - gq) < 1.0f ? 1 : 2;
                    l -= fabsf(xl0 - gq) < 1.0f ? 0 : fabsf(xl1 - gq) < 1.0f ? 1 : 2;
                }
                gfirst = gp + (f - ga);
                gcnt = max(0, l - f + 1);
            }

            // 3. profiles of the pairs that meet the tile, for half h
            auto profiles = [&](auto hc) {
                constexpr int h = decltype(hc)::value;
                if (stg[h]) {
                    for (int p = tid; p < NP; p += kThreads) {
                        // A pair whose xi misses the tile (rz = 0) is read by no voxel; its
                        // profile is formed anyway (with rz = 1, so that every look-up stays in
                        // the window) rather than branched around: a wave skips a pair only if
                        // all its lanes do, and the branch would wait on rz before reading the
                        // pair's other entries.
                        const float rz0 = prz[p];
                        const float a0 = pa0[h][p];
                        const int col = pcr[p];
                        const float rz = rz0 == 0.0f ? 1.0f : rz0;
                        const int2 *__restrict__ pc = pre + col * kPreStride;
                        // T(y) = ceil((y - a0) / rz) clamped to the window, taken as the
                        // truncation of (y - a0) / rz + 1 (one more only where a row sits
                        // exactly at y); that and the approximate reciprocal only move rows
                        // at zero weight (see the file's head)
                        const float inv = __builtin_amdgcn_rcpf(rz);
                        const float ub = fmaf(-a0, inv, 1.0f);
                        // H is formed scaled by the column's sc = 2^-kx (psc), which undoes
                        // its quantisation scale (scaling by a power of two commutes with FP64
                        // rounding, so it costs no accuracy, and the entries need no
                        // rescaling).  A column with a non-finite entry has sc = NaN, hence
                        // NaN entries.
                        const double sc = psc[col];
                        const double rzs = -(double)rz * sc;
                        // -(eta of row kRowCen), scaled: H(y) = (y - that) P - rz Q with the
                        // moment prefix taken about row kRowCen
                        const double nam = -fma((double)rz, (double)kRowCen, (double)a0) * sc;
                        int2 e[kKH + 2];
#pragma unroll
                        for (int i = 0; i < kKH + 2; ++i) {
                            const float u = fmaf((float)(i - 1), inv, ub);
                            const int T = (int)__builtin_amdgcn_fmed3f(u, 0.0f, (float)kWinRows + 0.5f);
                            e[i] = pc[T];
                        }
                        // all ten look-ups are in flight before the first is used
                        __builtin_amdgcn_sched_barrier(0);
                        // coefficient of P at y = i - 1, scaled: (y + nam) sc, as a running sum
                        // (each step rounds at most at 2^-52 of a value below 2^7, far below
                        // the FP32 rounding of the entries)
                        double cy = nam - sc;
                        double H[kKH + 2];
#pragma unroll
                        for (int i = 0; i < kKH + 2; ++i) {
                            H[i] = fma(cy, (double)e[i].x, rzs * (double)e[i].y);
                            cy += sc;
                        }
#pragma unroll
                        for (int kk = 0; kk < kKH; ++kk) {
                            const double zd = (H[kk + 2] + H[kk]) - 2.0 * H[kk + 1];
                            Z[kk * NPM + p] = (float)zd;
                        }
                    }
                } else {
                    const int nItems = (kKH / kKQ) * NP;
                    for (int it = tid; it < nItems; it += kThreads) {
                        int pr = it, kq = 0;
                        if (pr >= NP) { pr -= NP; kq = 1; }
                        const float rz = prz[pr];
                        if (rz == 0.0f) continue;
                        // detector rows directly (rows outside [0, nv) do not exist)
                        const float *__restrict__ src = rwv + c0 + pcr[pr];
                        const int64_t nu = geo.nu;
                        pair_profile<NC + 1>(pa0[h][pr], rz, 1.0f / rz, kq * kKQ, 0.0f,
                                             (float)max(0, geo.nv - (NC + 1)),
                                             [&](int t) {
                                                 const float v = src[(int64_t)min(t, geo.nv - 1) * nu];
                                                 return t < geo.nv ? v : 0.0f;
                                             },
                                             [&](int kk, float z) { Z[kk * NPM + pr] = z; });
                    }
                }
            };
            // 4. each thread adds to its voxel column the profiles of the pairs found above
            auto gather = [&](auto hc) {
                constexpr int h = decltype(hc)::value;
                // (the search admits only pairs with |xi - q| < 1; the clamp keeps a weight
                // rounded at that edge from turning negative)
#pragma unroll 1
                for (int j = 0; j < gcnt; ++j) {
                    const int pp = gfirst + j;
                    const float w = fmaxf(1.0f - fabsf(xiq[pp] - gq), 0.0f);
#pragma unroll
                    for (int kk = 0; kk < kKH; ++kk)
                        acc[h * kKH + kk] = fmaf(w, Z[kk * NPM + pp], acc[h * kKH + kk]);
                }
            };
            using H0 = std::integral_constant<int, 0>;
            using H1 = std::integral_constant<int, 1>;
            if (nRh[0] > 0) profiles(H0{});   // uniform across the block, as are nRh and stg
            if (stg[1]) load_window(1);
            __syncthreads();   // half-0 profiles complete; the prefix sums' readers are done
            if (nRh[0] > 0) gather(H0{});
            if (nRh[1] > 0) {
                if (stg[1]) build_prefix(1);
                __syncthreads();   // half-1 prefix sums complete; the half-0 gather is done with Z
                profiles(H1{});
                __syncthreads();
                gather(H1{});
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
int backproject_tile_z() { return kTK; }

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
                       accumulate ? 1 : 0, p->d_bp_order, g);
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
