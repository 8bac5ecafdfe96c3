// Device helpers: storage-type conversions and deterministic block reductions.
#pragma once

#include "common.h"

namespace fbl {

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__hip_bfloat16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float to_f32(__half v) { return __half2float(v); }

// Round an FP64 value once to the storage type (round to nearest, ties to even).
// For the 16-bit types the value is first rounded to FP32 with round-to-odd (24 bits,
// at least two more than the target keeps), which makes the second rounding exact.
__device__ __forceinline__ uint32_t f64_to_f32_round_odd_bits(double v)
{
    float f = (float)v;
    uint32_t u = __float_as_uint(f);
    double df = (double)f;
    if (df != v && v == v) {
        if (fabs(df) > fabs(v)) u -= 1u;   // step back toward zero: truncation
        u |= 1u;                           // sticky bit
    }
    return u;
}

template <typename T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ __half from_f64<__half>(double v)
{
    return __float2half_rn(__uint_as_float(f64_to_f32_round_odd_bits(v)));
}
template <> __device__ __forceinline__ __hip_bfloat16 from_f64<__hip_bfloat16>(double v)
{
    uint32_t u = f64_to_f32_round_odd_bits(v);
    unsigned short bits;
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
        bits = (unsigned short)((u >> 16) | 0x40u);          // NaN stays NaN
    } else {
        u += 0x7FFFu + ((u >> 16) & 1u);                     // nearest, ties to even
        bits = (unsigned short)(u >> 16);
    }
    __hip_bfloat16 r;
    __builtin_memcpy(&r, &bits, sizeof(bits));
    return r;
}

// Sum of a double over a 256-thread block; the result is valid in thread 0.  The
// order of additions is fixed (butterfly within each wave, then the four wave sums in
// order), so repeated launches give identical bits.
__device__ __forceinline__ double block_sum_256(double v, double *lds4)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds4[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
    __syncthreads();
    return s;
}

}  // namespace fbl
