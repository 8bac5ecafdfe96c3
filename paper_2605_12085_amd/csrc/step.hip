// Prox-gradient trial and the FP64 inner products of the sufficient-decrease test.
#include <mutex>

#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kStepBlocks = 2048;   // 8 blocks per compute unit, grid-stride over the volume

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

template <int V, typename T>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, int64_t q, T (&v)[V])
{
    using C = typename Chunk<V * sizeof(T)>::type;
    const C t = __builtin_nontemporal_load(reinterpret_cast<const C *>(p) + q);
    __builtin_memcpy(v, &t, sizeof(t));
}

template <int V, typename T>
__device__ __forceinline__ void store_vec(T *__restrict__ p, int64_t q, const T (&v)[V])
{
    using C = typename Chunk<V * sizeof(T)>::type;
    C t;
    __builtin_memcpy(&t, v, sizeof(t));
    __builtin_nontemporal_store(t, reinterpret_cast<C *>(p) + q);
}

// Voxels per thread and pass.  With 16-bit storage four voxels share one 8-byte access
// of x and of x-bar (and one 16-byte access of g); that measured 5-20% faster than one
// voxel per pass at 128^3 to 1024^3.  With FP32 storage one voxel per pass streamed
// faster at 512^3 and 1024^3 (16-byte accesses lost 9-14% there) and equally at 256^3.
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

}  // namespace

hipError_t launch_step_mixed(const fbl_plan *p, const float *x, const float *g, double alpha, double mu, double lo,
                             double hi, float *xbar, void *xbar16, int64_t *n_partials_used, hipStream_t st)
{
    const int blocks = step_blocks(p);
    *n_partials_used = blocks;
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    const double amu = alpha * mu;
    if (p->vol_dtype == FBL_BF16)
        hipLaunchKernelGGL(step_mixed_kernel<__hip_bfloat16>, dim3(blocks), dim3(256), 0, st, x, g, alpha, amu, lo,
                           hi, xbar, (__hip_bfloat16 *)xbar16, d, p->d_partials);
    else if (p->vol_dtype == FBL_F16)
        hipLaunchKernelGGL(step_mixed_kernel<__half>, dim3(blocks), dim3(256), 0, st, x, g, alpha, amu, lo, hi,
                           xbar, (__half *)xbar16, d, p->d_partials);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}


static int blocks_for(int64_t d)
{
    const int64_t need = (d + 255) / 256;
    return (int)(need < kStepBlocks ? need : kStepBlocks);
}

int step_blocks(const fbl_plan *p) { return blocks_for((int64_t)p->geo.nx * p->geo.ny * p->geo.nz); }

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

hipError_t launch_step(const fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo,
                       double hi, bool stochastic, uint64_t key, void *xbar, int64_t *n_partials_used,
                       hipStream_t st)
{
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    const int blocks = blocks_for(d);
    *n_partials_used = blocks;
    const double amu = alpha * mu;
    return stochastic
               ? launch_step_r<true>(p->vol_dtype, d, x, g, alpha, amu, lo, hi, key, xbar, p->d_partials, blocks, st)
               : launch_step_r<false>(p->vol_dtype, d, x, g, alpha, amu, lo, hi, key, xbar, p->d_partials, blocks,
                                      st);
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
