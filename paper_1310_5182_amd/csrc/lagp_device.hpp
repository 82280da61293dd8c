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

// Score candidate ordering: larger score wins, equal scores go to the smaller
// design index.  Invalid entries carry score -1 and index INT32_MAX.
template <typename T>
__device__ __forceinline__ bool beats(T s1, int i1, T s2, int i2)
{
    return s1 > s2 || (s1 == s2 && i1 < i2);
}

// ---- lane exchanges on the VALU (no LDS crossbar), for full-wave reductions.
// Stage S pairs every lane with one partner; after stages 0..5 every lane has
// combined all 64 lanes.  xchg<S>(v) returns (a, b): for stages 0-3 (DPP) a is
// the lane's own word and b its partner's; for stages 4-5 (permlane swaps) a is
// the even row's (lower half's) word and b the odd row's (upper half's), the
// same pair in both lanes.  A combine(a, b) that is symmetric in its operands
// (IEEE addition, a strict-order argmax) therefore gives every lane of a pair
// the same bits, so results are identical across lanes and runs.
struct Pair32 {
    unsigned a, b;
};

template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

template <int S>
__device__ __forceinline__ Pair32 xchg(unsigned v)
{
    if constexpr (S == 0) {
        return {v, dpp_u32<0xB1>(v)};  // quad_perm [1,0,3,2]: lane ^ 1
    } else if constexpr (S == 1) {
        return {v, dpp_u32<0x4E>(v)};  // quad_perm [2,3,0,1]: lane ^ 2
    } else if constexpr (S == 2) {
        return {v, dpp_u32<0x141>(v)};  // row_half_mirror: i <-> 7 - i in each 8
    } else if constexpr (S == 3) {
        return {v, dpp_u32<0x140>(v)};  // row_mirror: i <-> 15 - i in each 16
    } else if constexpr (S == 4) {
        auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);  // rows 0<->1, 2<->3
        return {r[0], r[1]};
    } else {
        auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);  // halves
        return {r[0], r[1]};
    }
}

struct PairF64 {
    double a, b;
};

template <int S>
__device__ __forceinline__ PairF64 xchg(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const Pair32 lo = xchg<S>((unsigned)u), hi = xchg<S>((unsigned)(u >> 32));
    return {__builtin_bit_cast(double, ((unsigned long long)hi.a << 32) | lo.a),
            __builtin_bit_cast(double, ((unsigned long long)hi.b << 32) | lo.b)};
}

template <int S>
__device__ __forceinline__ float xsum(float v)
{
    const Pair32 p = xchg<S>(__builtin_bit_cast(unsigned, v));
    return __builtin_bit_cast(float, p.a) + __builtin_bit_cast(float, p.b);
}

template <int S>
__device__ __forceinline__ double xsum(double v)
{
    const PairF64 p = xchg<S>(v);
    return p.a + p.b;
}

template <int S>
__device__ __forceinline__ double xmax(double v)
{
    const PairF64 p = xchg<S>(v);
    return fmax(p.a, p.b);
}

template <int S>
__device__ __forceinline__ float xmax(float v)
{
    const Pair32 p = xchg<S>(__builtin_bit_cast(unsigned, v));
    return fmaxf(__builtin_bit_cast(float, p.a), __builtin_bit_cast(float, p.b));
}

// Sum over the four 16-lane rows (lanes l, l^16, l^32, l^48 hold partials).
template <typename T>
__device__ __forceinline__ T row_sum4(T v)
{
    return xsum<5>(xsum<4>(v));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v = xsum<0>(v);
    v = xsum<1>(v);
    v = xsum<2>(v);
    v = xsum<3>(v);
    v = xsum<4>(v);
    return xsum<5>(v);
}

// Broadcast lane `l` (wave-uniform) of a double.
__device__ __forceinline__ double readlane(double v, int l)
{
    unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
    unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Lane 0's value, as a wave-uniform quantity.
__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(unsigned, v)));
}

__device__ __forceinline__ double uniform(double v)
{
    return readlane(v, 0);
}

template <int S>
__device__ __forceinline__ void argmax_stage(float &s, int &idx, int &slot)
{
    const Pair32 ps = xchg<S>(__builtin_bit_cast(unsigned, s));
    const Pair32 pi = xchg<S>((unsigned)idx), pk = xchg<S>((unsigned)slot);
    const float sa = __builtin_bit_cast(float, ps.a), sb = __builtin_bit_cast(float, ps.b);
    const bool take_b = beats(sb, (int)pi.b, sa, (int)pi.a);
    s = take_b ? sb : sa;
    idx = (int)(take_b ? pi.b : pi.a);
    slot = (int)(take_b ? pk.b : pk.a);
}

template <int S>
__device__ __forceinline__ void argmax_stage(double &s, int &idx, int &slot)
{
    const PairF64 ps = xchg<S>(s);
    const Pair32 pi = xchg<S>((unsigned)idx), pk = xchg<S>((unsigned)slot);
    const bool take_b = beats(ps.b, (int)pi.b, ps.a, (int)pi.a);
    s = take_b ? ps.b : ps.a;
    idx = (int)(take_b ? pi.b : pi.a);
    slot = (int)(take_b ? pk.b : pk.a);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    v = xmax<0>(v);
    v = xmax<1>(v);
    v = xmax<2>(v);
    v = xmax<3>(v);
    v = xmax<4>(v);
    return xmax<5>(v);
}

template <int S>
__device__ __forceinline__ int xmin_i32(int v)
{
    const Pair32 p = xchg<S>((unsigned)v);
    const int a = (int)p.a, b = (int)p.b;
    return a < b ? a : b;
}

__device__ __forceinline__ int wave_min_i32(int v)
{
    v = xmin_i32<0>(v);
    v = xmin_i32<1>(v);
    v = xmin_i32<2>(v);
    v = xmin_i32<3>(v);
    v = xmin_i32<4>(v);
    return xmin_i32<5>(v);
}

// Wave-wide argmax of (score, design index, slot) for scores that are never
// NaN: the largest score first, then, only if several lanes hold exactly that
// score, the smallest design index among them.  Every lane gets the result.
__device__ __forceinline__ void wave_argmax_ballot(double &s, int &idx, int &slot)
{
    const double m = wave_max(s);
    unsigned long long b = __ballot(s == m);
    if (b & (b - 1)) {
        const int v = wave_min_i32(s == m ? idx : INT32_MAX);
        b = __ballot(s == m && idx == v);
    }
    const int l = __builtin_ctzll(b);
    s = m;
    idx = __builtin_amdgcn_readlane(idx, l);
    slot = __builtin_amdgcn_readlane(slot, l);
}

// Wave-wide argmax of (score, design index, slot); every lane gets the result.
template <typename T>
__device__ __forceinline__ void wave_argmax(T &s, int &idx, int &slot)
{
    argmax_stage<0>(s, idx, slot);
    argmax_stage<1>(s, idx, slot);
    argmax_stage<2>(s, idx, slot);
    argmax_stage<3>(s, idx, slot);
    argmax_stage<4>(s, idx, slot);
    argmax_stage<5>(s, idx, slot);
}

}  // namespace lagp
