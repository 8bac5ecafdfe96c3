// Prox-gradient trial and the FP64 inner products of the sufficient-decrease test.
#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kStepBlocks = 2048;   // 8 blocks per compute unit, grid-stride over the volume

// Four consecutive storage values as one 16-byte (FP32) or 8-byte (16-bit) access.
template <typename TV>
__device__ __forceinline__ void load4(const TV *__restrict__ p, int64_t q, TV (&v)[4])
{
    if constexpr (sizeof(TV) == 4) {
        const float4 t = reinterpret_cast<const float4 *>(p)[q];
        __builtin_memcpy(v, &t, sizeof(t));
    } else {
        const uint2 t = reinterpret_cast<const uint2 *>(p)[q];
        __builtin_memcpy(v, &t, sizeof(t));
    }
}

template <typename TV>
__device__ __forceinline__ void store4(TV *__restrict__ p, int64_t q, const TV (&v)[4])
{
    if constexpr (sizeof(TV) == 4) {
        float4 t;
        __builtin_memcpy(&t, v, sizeof(t));
        reinterpret_cast<float4 *>(p)[q] = t;
    } else {
        uint2 t;
        __builtin_memcpy(&t, v, sizeof(t));
        reinterpret_cast<uint2 *>(p)[q] = t;
    }
}

// SR: round the trial point stochastically (counter-based, keyed) instead of to nearest.
// Each thread takes four consecutive voxels per pass (one wide access per array), then
// the last d mod 4 voxels one by one.
template <typename TV, bool SR>
__global__ __launch_bounds__(256) void step_kernel(const TV *__restrict__ x, const float *__restrict__ g,
                                                   double alpha, double amu, double lo, double hi, uint64_t key,
                                                   TV *__restrict__ xbar, int64_t d, double *__restrict__ partials)
{
    // the trial point is formed exactly as written, (x - alpha g) - alpha mu, without
    // fused multiply-adds, so it rounds like an FP64 evaluation of the prox on the host
#pragma clang fp contract(off)
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
    const int64_t d4 = d >> 2;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < d4; q += stride) {
        TV xv[4], out[4];
        load4(x, q, xv);
        const float4 g4 = reinterpret_cast<const float4 *>(g)[q];
        const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = trial(to_f32(xv[k]), gv[k], 4 * q + k);
        store4(xbar, q, out);
    }
    for (int64_t i = 4 * d4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += stride)
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

}  // namespace

int step_blocks(const fbl_plan *p)
{
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    const int64_t need = (d + 255) / 256;
    return (int)(need < kStepBlocks ? need : kStepBlocks);
}

template <typename TV, bool SR>
static hipError_t launch_step_t(const fbl_plan *p, const void *x, const float *g, double alpha, double amu,
                                double lo, double hi, uint64_t key, void *xbar, int blocks, hipStream_t st)
{
    const int64_t d = (int64_t)p->geo.nx * p->geo.ny * p->geo.nz;
    hipLaunchKernelGGL((step_kernel<TV, SR>), dim3(blocks), dim3(256), 0, st, (const TV *)x, g, alpha, amu, lo, hi,
                       key, (TV *)xbar, d, p->d_partials);
    return hipGetLastError();
}

template <bool SR>
static hipError_t launch_step_r(const fbl_plan *p, const void *x, const float *g, double alpha, double amu,
                                double lo, double hi, uint64_t key, void *xbar, int blocks, hipStream_t st)
{
    switch (p->vol_dtype) {
    case FBL_F32: return launch_step_t<float, SR>(p, x, g, alpha, amu, lo, hi, key, xbar, blocks, st);
    case FBL_BF16: return launch_step_t<__hip_bfloat16, SR>(p, x, g, alpha, amu, lo, hi, key, xbar, blocks, st);
    default: return launch_step_t<__half, SR>(p, x, g, alpha, amu, lo, hi, key, xbar, blocks, st);
    }
}

hipError_t launch_step(const fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo,
                       double hi, bool stochastic, uint64_t key, void *xbar, int64_t *n_partials_used,
                       hipStream_t st)
{
    const int blocks = step_blocks(p);
    *n_partials_used = blocks;
    const double amu = alpha * mu;
    return stochastic ? launch_step_r<true>(p, x, g, alpha, amu, lo, hi, key, xbar, blocks, st)
                      : launch_step_r<false>(p, x, g, alpha, amu, lo, hi, key, xbar, blocks, st);
}

}  // namespace fbl
