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

// Output number c+1 of SplitMix64 (Steele, Lea and Flood, 2014) seeded with `key`: the
// state after c+1 steps is key + (c+1) * gamma, mixed by the generator's finaliser.  A
// counter-based draw: element c of an array takes output c+1.
__device__ __forceinline__ uint64_t splitmix64(uint64_t key, uint64_t c)
{
    uint64_t z = key + (c + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T> struct StoragePrecision;
template <> struct StoragePrecision<float> { static constexpr int bits = 24, emin = -126; };
template <> struct StoragePrecision<__hip_bfloat16> { static constexpr int bits = 8, emin = -126; };
template <> struct StoragePrecision<__half> { static constexpr int bits = 11, emin = -14; };

// Stochastic rounding of an FP64 value to the storage type: between the adjacent
// representable numbers a <= v < a + q it returns a + q with probability (v - a) / q,
// decided by the 53-bit uniform of splitmix64(key, i).  Every step is exact in FP64 (q
// is a power of two, a a multiple of q within one q of v), so the choice depends only on
// v, key and i; the chosen value is representable and converts exactly.
template <typename T>
__device__ __forceinline__ T round_stochastic(double v, uint64_t key, uint64_t i)
{
    if (v == 0.0 || !isfinite(v)) return from_f64<T>(v);
    int e;
    (void)frexp(v, &e);   // |v| in [2^(e-1), 2^e)
    const int qe = max(e - 1, StoragePrecision<T>::emin) - (StoragePrecision<T>::bits - 1);
    const double vs = ldexp(v, -qe);   // v in units of the quantum q = 2^qe (exact)
    const double a = floor(vs);
    const double p = vs - a;
    const double r = (double)(splitmix64(key, i) >> 11) * 0x1.0p-53;
    return from_f64<T>(ldexp(r < p ? a + 1.0 : a, qe));
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
