// Forward projection A_N x (Joseph, bilinear) with the residual and FP64 loss epilogue.
//
// Structure on gfx950.  All rays of one detector column share their dominant axis,
// the slice plane they cross and their horizontal index coordinate xi on it, so the
// bilinear sample factors into one horizontal interpolation of the slice's z-line at xi
// (shared by every row of the column) and one vertical interpolation per ray.
//   - A thread owns one column and kRows consecutive rows; a wavefront spans 64
//     adjacent columns, so the horizontal tap pairs it loads are contiguous in memory
//     (x-fastest volume for views whose slices are y = const, a y-fastest transposed
//     copy for views whose slices are x = const).
//   - Per slice the thread interpolates the z-range its rays cover into a private LDS
//     line (interleaved [k][thread] so the 64 lanes never conflict), then each ray
//     reads its two vertical taps with one ds_read2st64 and does one lerp.
//   - Ray positions are refreshed in FP64 every kChunk slices and stepped in FP32
//     inside the chunk; per-chunk FP32 partial sums keep the 256-1024-term sums accurate.
//   - When a launch has too few rays to fill the chip, the waves of a block split the
//     slice march of the same rays (PARTS parts of whole chunks) and add their sums in a
//     fixed order at the end.
//   - Launch order: the block index runs over detector column tiles fastest, then views,
//     then row tiles.  A row tile's rays cross one horizontal band of the volume, so the
//     blocks resident at one time (every view's column tiles of a few row tiles) read the
//     same band, which the last-level cache then serves to all views of the batch instead
//     of each view reading the volume from HBM.  Within runs of 64 blocks, the 8 blocks
//     that land on one XCD take 8 consecutive tiles, so neighbouring column tiles (whose
//     tap rows share cache lines at their edges) read through the same L2.
#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kCols = 64;     // columns per block (one per lane)
constexpr int kWaves = 4;     // row groups per block (one per wavefront)
constexpr int kRows = 16;     // rays (rows) per thread
constexpr int kChunk = 16;    // slices per FP64 position refresh and per FP32 partial sum
constexpr int kThreads = kCols * kWaves;
constexpr int kFillWaves = 2048;  // two waves per SIMD: below this a launch splits the slice march

// Launch-order index of workgroup b of a grid of n.  The dispatcher deals consecutive
// workgroups to the chip's 8 XCDs in turn, each with its own L2.  Within every whole run
// of 64 workgroups this gives the 8 that share an XCD 8 consecutive indices, so tiles
// that are neighbours in the launch order (and read overlapping cache lines) share an
// L2, while the 8 XCDs still work on the same 64-tile stretch of the order.  A bijection
// on [0, n): runs are permuted within themselves and a final partial run is unchanged.
__device__ __forceinline__ int xcd_grouped_block(int b, int n)
{
    if (b >= (n & ~63)) return b;
    const int w = b & 63;
    return (b & ~63) + (w & 7) * 8 + (w >> 3);
}

// Horizontal pair of taps (p, p+1) of one z-row: both at consecutive addresses.
template <typename TV>
__device__ __forceinline__ void load_pair(const TV *__restrict__ base, int64_t off, float &a, float &b)
{
    a = to_f32(base[off]);
    b = to_f32(base[off + 1]);
}

// Per-slice horizontal state of a thread: tap column p with weights (wa, wb), and the
// z-line it fills: line entry kk holds z = kz + kk; ka is the line origin in the
// thread's ray coordinates.
struct SliceState {
    int sp;          // element offset of (slice, p, z = 0); 32 bits hold every offset into
                     // the volume (the plan admits fewer than 2^31 voxels)
    float wa, wb;
    int ka, kz;
    bool inside;     // z = kz .. kz+KB-1 all inside the volume
};

template <typename TB, int KB>
struct LineRegs {
    float a[KB], b[KB];
};

// Waves per SIMD the register budget is held to: short lines fit four (<= 128 VGPRs).
constexpr int fp_waves(int kb) { return kb <= 16 ? 4 : kb <= 32 ? 3 : 2; }

// PARTS: parts of the slice march per ray (the block's waves are kWaves / PARTS row
// groups of PARTS parts each).  RB: rays whose two line reads are issued together before
// their lerps (1: as the compiler schedules them, which keeps one or two reads in flight
// at this register budget).  Reading four rays' taps at once hides more LDS latency in
// launches whose waves run in several rounds (1024^3: -2.4%, 512^3: -1.9%); where all
// waves are resident at once (256^3) two at a time is best (-1.3%, four: +0.5%).  The
// results are the same to the bit.
template <typename TV, typename TB, int KB, int PARTS, int RB = 1>
__global__ __launch_bounds__(kThreads, fp_waves(KB)) void fp_kernel(
    const TV *__restrict__ x, const TV *__restrict__ xt, Geo geo, DeviceTables tab, ViewList vl, int first,
    const TB *__restrict__ b, float *__restrict__ y, double *__restrict__ partials, int blocks_per_view,
    int want_loss)
{
    // the line buffer also carries the march parts' sums to part 0
    constexpr int kLineFloats = KB * kThreads > (PARTS - 1) * (kWaves / PARTS) * kRows * kCols
                                    ? KB * kThreads : (PARTS - 1) * (kWaves / PARTS) * kRows * kCols;
    __shared__ float line[kLineFloats];
    __shared__ double red[4];
    const int tiles_u = (geo.nu + kCols - 1) / kCols;
    const int lb = xcd_grouped_block((int)blockIdx.x, (int)gridDim.x);
    // linear block index -> (row tile, view, column tile), column tiles fastest
    const int nbv = (int)gridDim.x / blocks_per_view;          // views in this launch
    const int rt = lb / (nbv * tiles_u);
    const int rem = lb - rt * nbv * tiles_u;
    const int bi = rem / tiles_u;
    const int tile = rt * tiles_u + (rem - bi * tiles_u);    // tile within the view (column fastest)
    const int view = vl.v[bi];
    const int tid = threadIdx.x;
    const int lane = tid & (kCols - 1), wave = tid / kCols;
    constexpr int kGroups = kWaves / PARTS;
    static_assert(kGroups * PARTS == kWaves, "PARTS divides the waves of a block");
    static_assert((PARTS - 1) * kGroups * kRows * kCols <= kLineFloats, "the line buffer holds the parts' sums");
    const int grp = wave % kGroups, part = wave / kGroups;
    const int c = (tile % tiles_u) * kCols + lane;
    const int r0 = ((tile / tiles_u) * kGroups + grp) * kRows;
    const int nrows = max(0, min(kRows, geo.nv - r0));
    const bool active = c < geo.nu && nrows > 0;

    float acc[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = 0.0f;

    // Inactive lanes (past the detector edge) run the loop on a clamped column and row
    // so that every lane takes part in the wave-wide decisions; their sums are dropped.
    const int cc = min(c, geo.nu - 1);
    const int rr0 = min(r0, geo.nv - 1);
    const ColParam cp = tab.col[(int64_t)view * geo.nu + cc];
    // slices along x (axis 0, read from the transposed copy) or y (axis 1)
    const int na = cp.axis == 0 ? geo.nx : geo.ny;
    const int nb = cp.axis == 0 ? geo.ny : geo.nx;
    const TV *__restrict__ vol = cp.axis == 0 ? xt : x;
    const int zstride = geo.nx * geo.ny;
    const int sstride = cp.axis == 0 ? geo.ny : geo.nx;
    const float xs = (float)cp.xi1;
    // Rows are equally spaced in eta: row rr0 + r sits at eta = cz + tau * (V0 + r * dvz),
    // with V0 the vertical index slope of row rr0.  Per slice the thread keeps the first
    // row's line coordinate A and the row-to-row step D = tau * dvz; ray r is at A + r D.
    const double V0 = tab.rowV[rr0];
    const float es0 = (float)(cp.t1 * V0);              // dA per slice
    const float ds = (float)(cp.t1 * (double)geo.dvz);  // dD per slice
    float *__restrict__ my = line + tid;
    // the longest slice march in the block decides the trip count of every lane
    int na_max = na;
    for (int off = 32; off > 0; off >>= 1) na_max = max(na_max, __shfl_xor(na_max, off, 64));

    // this wave's part of the march: whole chunks [mb, mb + seg) (the wave's columns, and
    // with them na_max, are the same in every part)
    const int seg = ((na_max + PARTS - 1) / PARTS + kChunk - 1) / kChunk * kChunk;
    const int mb = part * seg, me = min(na, mb + seg);
    for (int m0 = mb; m0 < min(na_max, mb + seg); m0 += kChunk) {
        const int sc = min(kChunk, me - m0);   // slices of this lane in the chunk (may be <= 0)
        // FP64 positions at the chunk's first slice.  Integer bases are taken below the
        // smallest value reached in the chunk, so all in-chunk offsets are >= 0 and
        // truncation equals floor.
        const double xb = fma((double)m0, cp.xi1, cp.xi0);
        const double xmin = fmin(xb, xb + (double)(kChunk - 1) * cp.xi1);
        const int ib = (int)floor(xmin) - 1;
        const float xf = (float)(xb - (double)ib);
        const double tb = fma((double)m0, cp.t1, cp.t0);
        const double e0 = fma(tb, V0, geo.cz);
        const double emin = fmin(e0, e0 + (double)(kChunk - 1) * cp.t1 * V0);
        const int k0 = (int)floor(emin) - 1;
        const float eb0 = (float)(e0 - (double)k0);       // A at the chunk's first slice
        const float db = (float)(tb * (double)geo.dvz);   // D at the chunk's first slice
        float part[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) part[r] = 0.0f;

        auto slice_state = [&](int s) {
            SliceState S;
            const float fl = (float)s;
            const float xl = fmaf(fl, xs, xf);
            const int i0 = ib + (int)xl;
            const float ax = __builtin_amdgcn_fractf(xl);
            int p = i0;
            S.wa = 1.0f - ax;
            S.wb = ax;
            if (i0 < 0 || i0 > nb - 2) {
                if (i0 == -1) { p = 0; S.wa = ax; S.wb = 0.0f; }
                else if (i0 == nb - 1) { p = nb - 2; S.wa = 0.0f; S.wb = 1.0f - ax; }
                else { p = 0; S.wa = 0.0f; S.wb = 0.0f; }
            }
            const float ef = fmaf(fl, es0, eb0);
            S.ka = (int)(ef - 1e-3f);
            S.kz = k0 + S.ka;
            S.inside = S.kz >= 0 && S.kz + KB <= geo.nz;
            // a lane whose march ended (fewer slices than the block's longest) keeps
            // addressing its last slice; its ray pass is skipped
            S.sp = min(m0 + s, na - 1) * sstride + p;
            return S;
        };
        auto load_line = [&](const SliceState &S, LineRegs<TB, KB> &L) {
            const TV *__restrict__ q = vol + (S.sp + S.kz * zstride);   // inside: kz >= 0
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
                L.a[kk] = to_f32(q[0]);
                L.b[kk] = to_f32(q[1]);
                q += zstride;
            }
        };

        LineRegs<TB, KB> L;
        SliceState P = slice_state(0);
        bool fastP = __all(P.inside);
        if (fastP) load_line(P, L);
        for (int s = 0; s < kChunk; ++s) {
            // horizontal interpolation of the z-line at the column's xi
            if (fastP) {
#pragma unroll
                for (int kk = 0; kk < KB; ++kk) my[kk * kThreads] = fmaf(P.wb, L.b[kk], P.wa * L.a[kk]);
            } else {
                for (int kk = 0; kk < KB; ++kk) {
                    const int k = P.kz + kk;
                    float v = 0.0f;
                    if ((unsigned)k < (unsigned)geo.nz) {
                        const TV *__restrict__ q = vol + (P.sp + k * zstride);
                        v = fmaf(P.wb, to_f32(q[1]), P.wa * to_f32(q[0]));
                    }
                    my[kk * kThreads] = v;
                }
            }
            // prefetch the next slice's taps before the ray pass of this one
            SliceState Q = P;
            bool fastQ = false;
            if (s + 1 < kChunk) {
                Q = slice_state(s + 1);
                fastQ = __all(Q.inside);
                if (fastQ) load_line(Q, L);
            }
            // vertical interpolation per ray from the thread's line
            if (s < sc) {
                const float fl = (float)s;
                const float A = fmaf(fl, es0, eb0);
                const float D = fmaf(fl, ds, db);
                float *__restrict__ base = my - P.ka * kThreads;
                if constexpr (RB == 1) {
#pragma unroll
                    for (int r = 0; r < kRows; ++r) {
                        const float e = fmaf((float)r, D, A);
                        const int j = (int)e;
                        const float ay = __builtin_amdgcn_fractf(e);
                        const float t0 = base[j * kThreads];
                        const float t1 = base[(j + 1) * kThreads];
                        part[r] += fmaf(ay, t1 - t0, t0);
                    }
                } else {
                    static_assert(kRows % RB == 0, "whole groups of rays");
#pragma unroll
                    for (int r0 = 0; r0 < kRows; r0 += RB) {
                        float t0[RB], t1[RB], ay[RB];
#pragma unroll
                        for (int rr = 0; rr < RB; ++rr) {
                            const float e = fmaf((float)(r0 + rr), D, A);
                            const int j = (int)e;
                            ay[rr] = __builtin_amdgcn_fractf(e);
                            t0[rr] = base[j * kThreads];
                            t1[rr] = base[(j + 1) * kThreads];
                        }
                        __builtin_amdgcn_sched_barrier(0);   // the group's reads are issued before its lerps
#pragma unroll
                        for (int rr = 0; rr < RB; ++rr) part[r0 + rr] += fmaf(ay[rr], t1[rr] - t0[rr], t0[rr]);
                    }
                }
            }
            P = Q;
            fastP = fastQ;
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) acc[r] += part[r];
    }

    if constexpr (PARTS > 1) {
        // parts 1..S-1 hand their sums to part 0 through the line buffer
        __syncthreads();
        float *__restrict__ xfer = line;
        if (part > 0) {
#pragma unroll
            for (int r = 0; r < kRows; ++r) xfer[(((part - 1) * kGroups + grp) * kRows + r) * kCols + lane] = acc[r];
        }
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int q = 1; q < PARTS; ++q) {
#pragma unroll
                for (int r = 0; r < kRows; ++r) acc[r] += xfer[(((q - 1) * kGroups + grp) * kRows + r) * kCols + lane];
            }
        }
    }
    double sq = 0.0;
    if (active && part == 0) {
        const int64_t row0 = (int64_t)(first + bi) * geo.np;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            if (r < nrows) {
                const int iv = r0 + r;
                const float w = cp.wa * sqrtf(cp.l2 + tab.rowV2[iv]);
                float val = w * acc[r];
                if (b) val -= to_f32(b[(int64_t)view * geo.np + (int64_t)iv * geo.nu + c]);
                y[row0 + (int64_t)iv * geo.nu + c] = val;
                sq += (double)val * (double)val;
            }
        }
    }
    if (want_loss) {
        const double s = block_sum_256(sq, red);
        if (tid == 0) partials[(int64_t)(first + bi) * blocks_per_view + tile] = s;
    }
}

// xt[k][i][j] = x[k][j][i]: y-fastest copy read by views whose slices are x = const.
// A block moves a 32 x 32 tile of kTrZ consecutive z-slices: every load is issued before
// the first store, and each block moves kTrZ times 4 KB (FP32).
constexpr int kTrZ = 4;
template <typename TV>
__global__ __launch_bounds__(256) void transpose_xy_kernel(const TV *__restrict__ x, TV *__restrict__ xt, int nx,
                                                           int ny, int nz)
{
    __shared__ TV tile[kTrZ][32][33];
    const int tiles_x = (nx + 31) / 32;
    const int ti = blockIdx.x % tiles_x, tj = blockIdx.x / tiles_x;
    const int k0 = blockIdx.y * kTrZ;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int64_t plane = (int64_t)nx * ny;
    TV v[kTrZ][4];
#pragma unroll
    for (int z = 0; z < kTrZ; ++z)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = tj * 32 + ty + 8 * q, i = ti * 32 + tx;
            if (i < nx && j < ny && k0 + z < nz) v[z][q] = x[(int64_t)(k0 + z) * plane + (int64_t)j * nx + i];
        }
#pragma unroll
    for (int z = 0; z < kTrZ; ++z)
#pragma unroll
        for (int q = 0; q < 4; ++q) tile[z][ty + 8 * q][tx] = v[z][q];
    __syncthreads();
#pragma unroll
    for (int z = 0; z < kTrZ; ++z)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = ti * 32 + ty + 8 * q, j = tj * 32 + tx;
            if (i < nx && j < ny && k0 + z < nz) xt[(int64_t)(k0 + z) * plane + (int64_t)i * ny + j] = tile[z][tx][ty + 8 * q];
        }
}

// out[c] = scale * sum_i partials[i * NC + c].  Thread t adds entries t, t + 256, ... in
// that order, then the block sums the 256 thread sums in a fixed order.  Each thread
// issues eight rounds of loads (all NC components of each) before adding them, so the
// loads overlap instead of forming one dependent chain per component.
template <int NC>
__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ partials, int64_t n, double scale,
                                                       double *__restrict__ out)
{
    constexpr int kU = 8;
    __shared__ double red[4];
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] = 0.0;
    int64_t i = threadIdx.x;
    for (; i + (kU - 1) * 256 < n; i += kU * 256) {
        double v[kU][NC];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c) v[u][c] = partials[(i + u * 256) * NC + c];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c) s[c] += v[u][c];
    }
    for (; i < n; i += 256)
#pragma unroll
        for (int c = 0; c < NC; ++c) s[c] += partials[i * NC + c];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double tot = block_sum_256(s[c], red);
        if (threadIdx.x == 0) out[c] = scale * tot;
    }
}

}  // namespace

int forward_blocks_per_view(const Geo &g, int parts)
{
    const int rows = (kWaves / parts) * kRows;
    return ((g.nu + kCols - 1) / kCols) * ((g.nv + rows - 1) / rows);
}

int forward_parts(const Geo &g, int B)
{
    for (int parts = 1; parts < kWaves; parts *= 2)
        if ((int64_t)kWaves * forward_blocks_per_view(g, parts) * B >= kFillWaves) return parts;
    return kWaves;
}

int forward_rows_per_thread() { return kRows; }

template <typename TV, typename TB, int KB, int S, int RB = 1>
static hipError_t launch_fp_s(const fbl_plan *p, const void *x, const void *xt, const ViewList &vl, int nb,
                              int first, const void *b, float *y, bool want_loss, hipStream_t st)
{
    DeviceTables tab{p->d_col, p->d_rowV, p->d_rowV2, p->d_view};
    const int bpv = forward_blocks_per_view(p->geo, S);
    dim3 grid(bpv * nb);
    hipLaunchKernelGGL((fp_kernel<TV, TB, KB, S, RB>), grid, dim3(kThreads), 0, st, (const TV *)x, (const TV *)xt,
                       p->geo, tab, vl, first, (const TB *)b, y, p->d_partials, bpv, want_loss ? 1 : 0);
    return hipGetLastError();
}

// Launches with at least this many waves (two rounds of four per SIMD) read four rays'
// taps at a time (RB = 4), smaller ones two (RB = 2); split marches keep the compiler's
// schedule.
constexpr int64_t kGroupedReadWaves = 8192;

template <typename TV, typename TB, int KB>
static hipError_t launch_fp_kb(const fbl_plan *p, const void *x, const void *xt, const ViewList &vl, int nb,
                               int first, const void *b, float *y, bool want_loss, int parts, hipStream_t st)
{
    if constexpr (KB <= 12) {   // longer lines spill registers with four rays' taps in flight
        if (parts == 1) {
            if ((int64_t)forward_blocks_per_view(p->geo, 1) * nb * kWaves >= kGroupedReadWaves)
                return launch_fp_s<TV, TB, KB, 1, 4>(p, x, xt, vl, nb, first, b, y, want_loss, st);
            return launch_fp_s<TV, TB, KB, 1, 2>(p, x, xt, vl, nb, first, b, y, want_loss, st);
        }
    }
    switch (parts) {
    case 1: return launch_fp_s<TV, TB, KB, 1>(p, x, xt, vl, nb, first, b, y, want_loss, st);
    case 2: return launch_fp_s<TV, TB, KB, 2>(p, x, xt, vl, nb, first, b, y, want_loss, st);
    default: return launch_fp_s<TV, TB, KB, 4>(p, x, xt, vl, nb, first, b, y, want_loss, st);
    }
}

template <typename TV>
static hipError_t launch_transpose_t(const fbl_plan *p, const void *x, hipStream_t st)
{
    const int tiles = ((p->geo.nx + 31) / 32) * ((p->geo.ny + 31) / 32);
    hipLaunchKernelGGL((transpose_xy_kernel<TV>), dim3(tiles, (p->geo.nz + kTrZ - 1) / kTrZ), dim3(256), 0, st, (const TV *)x,
                       (TV *)p->d_xt, p->geo.nx, p->geo.ny, p->geo.nz);
    return hipGetLastError();
}

hipError_t launch_transpose(const fbl_plan *p, const void *x, hipStream_t st)
{
    switch (p->vol_dtype) {
    case FBL_F32: return launch_transpose_t<float>(p, x, st);
    case FBL_BF16: return launch_transpose_t<__hip_bfloat16>(p, x, st);
    default: return launch_transpose_t<__half>(p, x, st);
    }
}

template <typename TV, typename TB>
static hipError_t launch_fp_t(const fbl_plan *p, const void *x, const ViewList &vl, int nb, int first,
                              const void *b, float *y, bool want_loss, int parts, hipStream_t st)
{
    const void *xt = p->d_xt;
    switch (p->fp_line) {
    case 11: return launch_fp_kb<TV, TB, 11>(p, x, xt, vl, nb, first, b, y, want_loss, parts, st);
    case 12: return launch_fp_kb<TV, TB, 12>(p, x, xt, vl, nb, first, b, y, want_loss, parts, st);
    case 16: return launch_fp_kb<TV, TB, 16>(p, x, xt, vl, nb, first, b, y, want_loss, parts, st);
    case 24: return launch_fp_kb<TV, TB, 24>(p, x, xt, vl, nb, first, b, y, want_loss, parts, st);
    case 32: return launch_fp_kb<TV, TB, 32>(p, x, xt, vl, nb, first, b, y, want_loss, parts, st);
    default: return launch_fp_kb<TV, TB, 48>(p, x, xt, vl, nb, first, b, y, want_loss, parts, st);
    }
}

template <typename TV>
static hipError_t launch_fp_b(const fbl_plan *p, const void *x, const ViewList &vl, int nb, int first,
                              const void *b, float *y, bool want_loss, int parts, hipStream_t st)
{
    switch (p->proj_dtype) {
    case FBL_F32: return launch_fp_t<TV, float>(p, x, vl, nb, first, b, y, want_loss, parts, st);
    case FBL_BF16: return launch_fp_t<TV, __hip_bfloat16>(p, x, vl, nb, first, b, y, want_loss, parts, st);
    default: return launch_fp_t<TV, __half>(p, x, vl, nb, first, b, y, want_loss, parts, st);
    }
}

hipError_t launch_forward(const fbl_plan *p, const void *x, const ViewList &vl, int nb, int first, const void *b,
                          float *y, bool want_loss, int parts, hipStream_t st)
{
    switch (p->vol_dtype) {
    case FBL_F32: return launch_fp_b<float>(p, x, vl, nb, first, b, y, want_loss, parts, st);
    case FBL_BF16: return launch_fp_b<__hip_bfloat16>(p, x, vl, nb, first, b, y, want_loss, parts, st);
    default: return launch_fp_b<__half>(p, x, vl, nb, first, b, y, want_loss, parts, st);
    }
}

hipError_t launch_finalize_sum(double *partials, int64_t n, int ncomp, double scale, double *out, hipStream_t st)
{
    if (ncomp == 3)
        hipLaunchKernelGGL(finalize_kernel<3>, dim3(1), dim3(256), 0, st, (const double *)partials, n, scale, out);
    else if (ncomp == 1)
        hipLaunchKernelGGL(finalize_kernel<1>, dim3(1), dim3(256), 0, st, (const double *)partials, n, scale, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fbl
