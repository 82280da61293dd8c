// Device helpers shared by the gfx950 kernels of the local-GP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lagp {

constexpr int kWave = 64;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Squared Euclidean distance summed left to right over the coordinates with
// every product and sum rounded separately (no fused multiply-add), so that
// candidate pools are reproducible bit for bit.
__device__ __forceinline__ double sqdist_strict(const double *a, int astride, const double *b,
                                                int bstride, int p)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int k = 0; k < p; k++) {
        double t = a[k * astride] - b[k * bstride];
        s = s + t * t;
    }
    return s;
}

// Isotropic Gaussian correlation exp(-r2 / d) (Sec. 2.1), float64.
__device__ __forceinline__ double corr64(double r2, double d)
{
    return exp(-r2 / d);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Broadcast lane `l` (wave-uniform) of a double.
__device__ __forceinline__ double readlane(double v, int l)
{
    unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
    unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Score candidate ordering: larger score wins, equal scores go to the smaller
// design index.  Invalid entries carry score -1 and index INT32_MAX.
template <typename T>
__device__ __forceinline__ bool beats(T s1, int i1, T s2, int i2)
{
    return s1 > s2 || (s1 == s2 && i1 < i2);
}

// Wave-wide argmax of (score, design index, slot).
template <typename T>
__device__ __forceinline__ void wave_argmax(T &s, int &idx, int &slot)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T s2 = __shfl_xor(s, o, kWave);
        int i2 = __shfl_xor(idx, o, kWave);
        int k2 = __shfl_xor(slot, o, kWave);
        if (beats(s2, i2, s, idx)) {
            s = s2;
            idx = i2;
            slot = k2;
        }
    }
}

}  // namespace lagp
