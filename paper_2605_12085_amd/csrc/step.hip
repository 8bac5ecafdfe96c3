// Prox-gradient trial and the FP64 inner products of the sufficient-decrease test.
#include <mutex>

#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kStepBlocks = 2048;   // grid-stride trial: 8 blocks per compute unit

// Blocks of the grid-stride prox trial for d voxels.
int blocks_for(int64_t d)
{
    const int64_t need = (d + 255) / 256;
    return (int)(need < kStepBlocks ? need : kStepBlocks);
}

// V consecutive values of one array as a single 2-, 4-, 8- or 16-byte access.  Every
// access is non-temporal: each voxel of x, g and xbar is touched once per launch, and
// streaming them past the caches measured 6% faster at 1024^3 (2.52 -> 2.37 ms, FP32).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int BYTES> struct Chunk;
template <> struct Chunk<2> { using type = uint16_t; };
template <> struct Chunk<4> { using type = uint32_t; };
template <> struct Chunk<8> { using type = u32x2; };
template <> struct Chunk<16> { using type = u32x4; };

// Groups of 32 bytes (eight FP32 values) are two 16-byte accesses.
template <int V, typename T>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, int64_t q, T (&v)[V])
{
    constexpr int B = V * (int)sizeof(T);
    constexpr int N = B > 16 ? B / 16 : 1;
    using C = typename Chunk<B / N>::type;
    C t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = __builtin_nontemporal_load(reinterpret_cast<const C *>(p) + N * q + i);
    __builtin_memcpy(v, t, sizeof(t));
}

template <int V, typename T>
__device__ __forceinline__ void store_vec(T *__restrict__ p, int64_t q, const T (&v)[V])
{
    constexpr int B = V * (int)sizeof(T);
    constexpr int N = B > 16 ? B / 16 : 1;
    using C = typename Chunk<B / N>::type;
    C t[N];
    __builtin_memcpy(t, v, sizeof(t));
#pragma unroll
    for (int i = 0; i < N; ++i) __builtin_nontemporal_store(t[i], reinterpret_cast<C *>(p) + N * q + i);
}

// The grid-stride prox trial: a loop over at most kStepBlocks blocks, used for volumes of
// up to kFlatMinVoxels (below) and by the allocation-free entry point, whose FP64 partials
// must fit a fixed scratch array.  Voxels per thread and pass: with 16-bit storage four
// voxels share one 8-byte access of x and of x-bar (and one 16-byte access of g), 5-20%
// faster than one voxel per pass at 128^3 to 1024^3; with FP32 storage one voxel per pass
// (16-byte accesses lost 9-14% in this loop at 512^3 and 1024^3).
template <typename TV> constexpr int step_vec() { return sizeof(TV) == 2 ? 4 : 1; }

// SR: round the trial point stochastically (counter-based, keyed) instead of to nearest.
// Each thread takes V consecutive voxels per pass, then the last d mod V one by one.
template <typename TV, bool SR>
__global__ __launch_bounds__(256) void step_kernel(const TV *__restrict__ x, const float *__restrict__ g,
                                                   double alpha, double amu, double lo, double hi, uint64_t key,
                                                   TV *__restrict__ xbar, int64_t d, double *__restrict__ partials)
{
    // the trial point is formed exactly as written, (x - alpha g) - alpha mu, without
    // fused multiply-adds, so it rounds like an FP64 evaluation of the prox on the host
#pragma clang fp contract(off)
    constexpr int V = step_vec<TV>();
    __shared__ double red[4];
    double s_inner = 0.0, s_sq = 0.0, s_gg = 0.0;
    auto trial = [&](float xf, float gf, int64_t i) -> TV {
        const double xv = (double)xf;
        const double gv = (double)gf;
        double v = (xv - alpha * gv) - amu;
        v = fmin(fmax(v, lo), hi);
        const TV out = SR ? round_stochastic<TV>(v, key, (uint64_t)i) : from_f64<TV>(v);
        const double dl = (double)to_f32(out) - xv;
        s_inner += gv * dl;
        s_sq += dl * dl;
        s_gg += gv * gv;
        return out;
    };
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t dv = d / V;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < dv; q += stride) {
        TV xv[V], out[V];
        float gv[V];
        load_vec<V>(x, q, xv);
        load_vec<V>(g, q, gv);
#pragma unroll
        for (int k = 0; k < V; ++k) out[k] = trial(to_f32(xv[k]), gv[k], V * q + k);
        store_vec<V>(xbar, q, out);
    }
    for (int64_t i = V * dv + (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += stride)
        xbar[i] = trial(to_f32(x[i]), g[i], i);
    const double a = block_sum_256(s_inner, red);
    const double b = block_sum_256(s_sq, red);
    const double c = block_sum_256(s_gg, red);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = a;
        partials[3 * blockIdx.x + 1] = b;
        partials[3 * blockIdx.x + 2] = c;
    }
}

// Mixed storage: an FP32 master iterate x (read) and trial point xbar (written), plus a
// 16-bit copy xbar16 = round-to-nearest(xbar) for the projector to read.  The inner
// products are those of the FP32 master values.  Two voxels per thread and pass: 8-byte
// accesses of x, g and xbar, a 4-byte access of xbar16.
template <typename TS>
__global__ __launch_bounds__(256) void step_mixed_kernel(const float *__restrict__ x, const float *__restrict__ g,
                                                         double alpha, double amu, double lo, double hi,
                                                         float *__restrict__ xbar, TS *__restrict__ xbar16,
                                                         int64_t d, double *__restrict__ partials)
{
#pragma clang fp contract(off)
    constexpr int V = 2;
    __shared__ double red[4];
    double s_inner = 0.0, s_sq = 0.0, s_gg = 0.0;
    auto trial = [&](float xf, float gf, float &out, TS &out16) {
        const double xv = (double)xf;
        const double gv = (double)gf;
        double v = (xv - alpha * gv) - amu;
        v = fmin(fmax(v, lo), hi);
        out = (float)v;
        out16 = from_f64<TS>((double)out);   // exact input: one rounding to nearest
        const double dl = (double)out - xv;
        s_inner += gv * dl;
        s_sq += dl * dl;
        s_gg += gv * gv;
    };
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t dv = d / V;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < dv; q += stride) {
        float xv[V], gv[V], out[V];
        TS o16[V];
        load_vec<V>(x, q, xv);
        load_vec<V>(g, q, gv);
#pragma unroll
        for (int k = 0; k < V; ++k) trial(xv[k], gv[k], out[k], o16[k]);
        store_vec<V>(xbar, q, out);
        store_vec<V>(xbar16, q, o16);
    }
    for (int64_t i = V * dv + (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += stride)
        trial(x[i], g[i], xbar[i], xbar16[i]);
    const double a = block_sum_256(s_inner, red);
    const double b = block_sum_256(s_sq, red);
    const double c = block_sum_256(s_gg, red);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = a;
        partials[3 * blockIdx.x + 1] = b;
        partials[3 * blockIdx.x + 2] = c;
    }
}

// The three sums of a block of 256 threads, in a fixed order, written by thread 0 to
// out[0..2]: each wave adds its lanes (a butterfly of lane exchanges), then thread 0 adds
// the four waves' sums.  One barrier (the kernel ends after it).
__device__ __forceinline__ void block_sums3_256(double a, double b, double c, double *__restrict__ out)
{
    __shared__ double red3[3][4];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
        c += __shfl_xor(c, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red3[0][wave] = a;
        red3[1][wave] = b;
        red3[2][wave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] = ((red3[k][0] + red3[k][1]) + red3[k][2]) + red3[k][3];
    }
}

// The prox trial as one pass over the volume: thread t of the launch takes voxels
// [Vt, Vt + V), V = 4 with FP32 storage and 8 with 16-bit storage (16-byte accesses of x
// and x-bar either way; g in one or two), and the thread just past the last whole group
// takes the d mod V voxels left.  Every thread touches one group and exits, so
// consecutive blocks sweep the arrays in order: at 1024^3 FP32 this streams at 6.5 TB/s,
// where a grid-stride loop over 2048 blocks (however many loads it keeps in flight)
// reached 5.4 TB/s.  Each block writes its three FP64 sums; reduce_partials_kernel and
// finalize_kernel add them in a fixed order.
constexpr int kFlatV = 4;   // voxels per thread of the FP32 and mixed forms
template <typename TV> constexpr int flat_vec() { return sizeof(TV) == 2 ? 8 : kFlatV; }
// Up to this many voxels the grid-stride kernels are used instead: at 256^3 their arrays
// sit in the 256 MB last-level cache, where they ran faster (FP32 32.9 against 35.2 us,
// BF16 27 against 35 us); from 512^3 up the one-pass kernels win (1024^3 FP32: 2.48 ->
// 2.00 ms).
constexpr int64_t kFlatMinVoxels = (int64_t)1 << 25;

template <typename TV, bool SR>
__global__ __launch_bounds__(256) void step_flat_kernel(const TV *__restrict__ x, const float *__restrict__ g,
                                                        double alpha, double amu, double lo, double hi,
                                                        uint64_t key, TV *__restrict__ xbar, int64_t d,
                                                        double *__restrict__ partials)
{
#pragma clang fp contract(off)
    constexpr int V = flat_vec<TV>();
    double s_inner = 0.0, s_sq = 0.0, s_gg = 0.0;
    auto trial = [&](float xf, float gf, int64_t i) -> TV {
        const double xv = (double)xf;
        const double gv = (double)gf;
        double v = (xv - alpha * gv) - amu;
        v = fmin(fmax(v, lo), hi);
        const TV out = SR ? round_stochastic<TV>(v, key, (uint64_t)i) : from_f64<TV>(v);
        const double dl = (double)to_f32(out) - xv;
        s_inner += gv * dl;
        s_sq += dl * dl;
        s_gg += gv * gv;
        return out;
    };
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t dv = d / V;
    if (q < dv) {
        TV xv[V], out[V];
        float gv[V];
        load_vec<V>(x, q, xv);
        load_vec<V>(g, q, gv);
#pragma unroll
        for (int k = 0; k < V; ++k) out[k] = trial(to_f32(xv[k]), gv[k], V * q + k);
        store_vec<V>(xbar, q, out);
    } else if (q == dv) {
        for (int64_t i = V * dv; i < d; ++i) xbar[i] = trial(to_f32(x[i]), g[i], i);
    }
    block_sums3_256(s_inner, s_sq, s_gg, partials + 3 * blockIdx.x);
}

// Mixed storage in one pass: an FP32 master iterate x (read) and trial point xbar
// (written), plus a 16-bit copy xbar16 = round-to-nearest(xbar) for the projector to read;
// the inner products are those of the FP32 master values.  Four voxels per thread: 16-byte
// accesses of x, g and xbar, an 8-byte access of xbar16.
template <typename TS>
__global__ __launch_bounds__(256) void step_mixed_flat_kernel(const float *__restrict__ x, const float *__restrict__ g,
                                                              double alpha, double amu, double lo, double hi,
                                                              float *__restrict__ xbar, TS *__restrict__ xbar16,
                                                              int64_t d, double *__restrict__ partials)
{
#pragma clang fp contract(off)
    constexpr int V = kFlatV;
    double s_inner = 0.0, s_sq = 0.0, s_gg = 0.0;
    auto trial = [&](float xf, float gf, float &out, TS &out16) {
        const double xv = (double)xf;
        const double gv = (double)gf;
        double v = (xv - alpha * gv) - amu;
        v = fmin(fmax(v, lo), hi);
        out = (float)v;
        out16 = from_f64<TS>((double)out);   // exact input: one rounding to nearest
        const double dl = (double)out - xv;
        s_inner += gv * dl;
        s_sq += dl * dl;
        s_gg += gv * gv;
    };
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t dv = d / V;
    if (q < dv) {
        float xv[V], gv[V], out[V];
        TS o16[V];
        load_vec<V>(x, q, xv);
        load_vec<V>(g, q, gv);
#pragma unroll
        for (int k = 0; k < V; ++k) trial(xv[k], gv[k], out[k], o16[k]);
        store_vec<V>(xbar, q, out);
        store_vec<V>(xbar16, q, o16);
    } else if (q == dv) {
        for (int64_t i = V * dv; i < d; ++i) trial(x[i], g[i], xbar[i], xbar16[i]);
    }
    block_sums3_256(s_inner, s_sq, s_gg, partials + 3 * blockIdx.x);
}

// Second reduction level: block r adds the three sums of blocks [1024 r, 1024 r + 1024)
// of the first level (each thread four consecutive ones, in order, then the block's fixed
// tree) into out[3 r + c].
constexpr int kReduceSpan = 1024;
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *__restrict__ in, int64_t n,
                                                              double *__restrict__ out)
{
    __shared__ double red[4];
    double s[3] = {0.0, 0.0, 0.0};
    const int64_t i0 = (int64_t)blockIdx.x * kReduceSpan + 4 * threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n) {
#pragma unroll
            for (int c = 0; c < 3; ++c) s[c] += in[3 * (i0 + k) + c];
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double t = block_sum_256(s[c], red);
        if (threadIdx.x == 0) out[3 * blockIdx.x + c] = t;
    }
}

// Blocks of the one-pass prox trial for d voxels at V voxels per thread (at most those of
// V = kFlatV, which size the partials), and the entries its reduction writes.
int64_t flat_blocks(int64_t d, int V = kFlatV) { return (d / V + 1 + 255) / 256; }
int64_t reduce_blocks(int64_t first_level) { return (first_level + kReduceSpan - 1) / kReduceSpan; }

// After the first level's partials[0, 3 nb): a second level when there are many, then the
// pointer and count the final sum (finalize_kernel) takes.
hipError_t reduce_step_partials(double *partials, int64_t nb, double **final_partials, int64_t *n_final,
                                hipStream_t st)
{
    if (nb <= 2 * kReduceSpan) {
        *final_partials = partials;
        *n_final = nb;
        return hipSuccess;
    }
    const int64_t r = reduce_blocks(nb);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)r), dim3(256), 0, st, (const double *)partials, nb,
                       partials + 3 * nb);
    *final_partials = partials + 3 * nb;
    *n_final = r;
    return hipGetLastError();
}

}  // namespace

int64_t step_partials_needed(int64_t d)
{
    if (d <= kFlatMinVoxels) return 3 * (int64_t)kStepBlocks;
    const int64_t nb = flat_blocks(d);
    return 3 * (nb + reduce_blocks(nb));
}

hipError_t launch_step_mixed(const fbl_plan *p, const float *x, const float *g, double alpha, double mu, double lo,
                             double hi, float *xbar, void *xbar16, double **final_partials, int64_t *n_final,
                             hipStream_t st)
{
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    const double amu = alpha * mu;
    if (d <= kFlatMinVoxels) {
        const int blocks = blocks_for(d);
        if (p->vol_dtype == FBL_BF16)
            hipLaunchKernelGGL(step_mixed_kernel<__hip_bfloat16>, dim3(blocks), dim3(256), 0, st, x, g, alpha, amu,
                               lo, hi, xbar, (__hip_bfloat16 *)xbar16, d, p->d_partials);
        else if (p->vol_dtype == FBL_F16)
            hipLaunchKernelGGL(step_mixed_kernel<__half>, dim3(blocks), dim3(256), 0, st, x, g, alpha, amu, lo, hi,
                               xbar, (__half *)xbar16, d, p->d_partials);
        else
            return hipErrorInvalidValue;
        *final_partials = p->d_partials;
        *n_final = blocks;
        return hipGetLastError();
    }
    const int64_t blocks = flat_blocks(d);
    if (p->vol_dtype == FBL_BF16)
        hipLaunchKernelGGL(step_mixed_flat_kernel<__hip_bfloat16>, dim3((unsigned)blocks), dim3(256), 0, st, x, g,
                           alpha, amu, lo, hi, xbar, (__hip_bfloat16 *)xbar16, d, p->d_partials);
    else if (p->vol_dtype == FBL_F16)
        hipLaunchKernelGGL(step_mixed_flat_kernel<__half>, dim3((unsigned)blocks), dim3(256), 0, st, x, g, alpha,
                           amu, lo, hi, xbar, (__half *)xbar16, d, p->d_partials);
    else
        return hipErrorInvalidValue;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_step_partials(p->d_partials, blocks, final_partials, n_final, st);
}




template <typename TV, bool SR>
static hipError_t launch_step_t(int64_t d, const void *x, const float *g, double alpha, double amu, double lo,
                                double hi, uint64_t key, void *xbar, double *partials, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL((step_kernel<TV, SR>), dim3(blocks), dim3(256), 0, st, (const TV *)x, g, alpha, amu, lo, hi,
                       key, (TV *)xbar, d, partials);
    return hipGetLastError();
}

template <bool SR>
static hipError_t launch_step_r(int32_t vol_dtype, int64_t d, const void *x, const float *g, double alpha,
                                double amu, double lo, double hi, uint64_t key, void *xbar, double *partials,
                                int blocks, hipStream_t st)
{
    switch (vol_dtype) {
    case FBL_F32: return launch_step_t<float, SR>(d, x, g, alpha, amu, lo, hi, key, xbar, partials, blocks, st);
    case FBL_BF16:
        return launch_step_t<__hip_bfloat16, SR>(d, x, g, alpha, amu, lo, hi, key, xbar, partials, blocks, st);
    default: return launch_step_t<__half, SR>(d, x, g, alpha, amu, lo, hi, key, xbar, partials, blocks, st);
    }
}

// Launches the one-pass trial and returns its block count in *blocks.
template <typename TV, bool SR>
static hipError_t launch_flat_t(int64_t d, const void *x, const float *g, double alpha, double amu, double lo,
                                double hi, uint64_t key, void *xbar, double *partials, int64_t *blocks, hipStream_t st)
{
    *blocks = flat_blocks(d, flat_vec<TV>());
    hipLaunchKernelGGL((step_flat_kernel<TV, SR>), dim3((unsigned)*blocks), dim3(256), 0, st, (const TV *)x, g,
                       alpha, amu, lo, hi, key, (TV *)xbar, d, partials);
    return hipGetLastError();
}

template <bool SR>
static hipError_t launch_flat_r(int32_t vol_dtype, int64_t d, const void *x, const float *g, double alpha,
                                double amu, double lo, double hi, uint64_t key, void *xbar, double *partials,
                                int64_t *blocks, hipStream_t st)
{
    switch (vol_dtype) {
    case FBL_F32: return launch_flat_t<float, SR>(d, x, g, alpha, amu, lo, hi, key, xbar, partials, blocks, st);
    case FBL_BF16:
        return launch_flat_t<__hip_bfloat16, SR>(d, x, g, alpha, amu, lo, hi, key, xbar, partials, blocks, st);
    default: return launch_flat_t<__half, SR>(d, x, g, alpha, amu, lo, hi, key, xbar, partials, blocks, st);
    }
}

hipError_t launch_step(const fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo,
                       double hi, bool stochastic, uint64_t key, void *xbar, double **final_partials,
                       int64_t *n_final, hipStream_t st)
{
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    const double amu = alpha * mu;
    if (d <= kFlatMinVoxels) {
        const int blocks = blocks_for(d);
        *final_partials = p->d_partials;
        *n_final = blocks;
        return stochastic
                   ? launch_step_r<true>(p->vol_dtype, d, x, g, alpha, amu, lo, hi, key, xbar, p->d_partials, blocks,
                                         st)
                   : launch_step_r<false>(p->vol_dtype, d, x, g, alpha, amu, lo, hi, key, xbar, p->d_partials, blocks,
                                          st);
    }
    int64_t blocks = 0;
    const hipError_t e =
        stochastic
            ? launch_flat_r<true>(p->vol_dtype, d, x, g, alpha, amu, lo, hi, key, xbar, p->d_partials, &blocks, st)
            : launch_flat_r<false>(p->vol_dtype, d, x, g, alpha, amu, lo, hi, key, xbar, p->d_partials, &blocks, st);
    if (e != hipSuccess) return e;
    return reduce_step_partials(p->d_partials, blocks, final_partials, n_final, st);
}

// ---- the allocation-free prox trial ---------------------------------------------------
//
// Its FP64 block partials live in a file-scope device array instead of a plan: at most
// kStepBlocks blocks each write three sums, whatever the volume size.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for the symbol):
// the device address is taken once per device with hipGetSymbolAddress and kept.
constexpr int kScratchDoubles = 3 * kStepBlocks;   // 48 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices];

static hipError_t scratch_of_current_device(double **out, int *dev_out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    *dev_out = dev;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace fbl

extern "C" int fb_lisa_step_noalloc(int64_t n_voxels, int32_t vol_dtype, const void *x, const float *g, double alpha,
                                    double mu, double lo, double hi, void *xbar, double *red_dev, void *stream)
{
    using namespace fbl;
    if (vol_dtype != FBL_F32 && vol_dtype != FBL_BF16 && vol_dtype != FBL_F16)
        return set_error(FBL_E_DTYPE, "vol_dtype %d is not FBL_F32, FBL_BF16 or FBL_F16", (int)vol_dtype);
    if (n_voxels < 1 || n_voxels >= ((int64_t)1 << 31))
        return set_error(FBL_E_RANGE, "n_voxels = %lld outside [1, 2^31): the allocation-free prox trial holds "
                                      "at most %d blocks' partial sums for volumes below 2^31 voxels",
                         (long long)n_voxels, kStepBlocks);
    const int rc = check_step_buffers(x, g, alpha, mu, lo, hi, xbar, red_dev);
    if (rc != FBL_OK) return rc;
    double *partials = nullptr;
    int dev = -1;
    hipError_t e = scratch_of_current_device(&partials, &dev);
    if (e != hipSuccess)
        return set_error(FBL_E_HIP, "device scratch of the allocation-free prox trial (device %d): %s", dev,
                         hipGetErrorString(e));
    const int blocks = blocks_for(n_voxels);
    hipStream_t st = (hipStream_t)stream;
    e = launch_step_r<false>(vol_dtype, n_voxels, x, g, alpha, alpha * mu, lo, hi, 0, xbar, partials, blocks, st);
    if (e != hipSuccess) return set_error(FBL_E_HIP, "step launch: %s", hipGetErrorString(e));
    e = launch_finalize_sum(partials, blocks, 3, 1.0, red_dev, st);
    if (e != hipSuccess) return set_error(FBL_E_HIP, "step reduction launch: %s", hipGetErrorString(e));
    return clear_error();
}
