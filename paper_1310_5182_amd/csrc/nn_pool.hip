// Nearest-neighbour candidate pools on gfx950 (Sec. 2.2 NN sub-design,
// Sec. 3.1: the ALC search runs over the N' nearest neighbours of x).
//
// One workgroup per predictive location streams the design once.  Each row's
// squared distance is summed left to right in float64 without fused
// multiply-adds; its bit pattern (non-negative doubles order like unsigned
// integers) together with the row index forms a unique composite key.  Rows
// whose key is below the running threshold are appended to an LDS buffer;
// when the buffer could overflow it is bitonic-sorted and cut to the Np
// smallest, and the threshold becomes the Np-th key.  The final sort gives
// the pool in ascending (distance, index) order, so the result is exact and
// independent of scheduling.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

namespace lagp {

constexpr int kNnBlock = 256;
constexpr int kNnItems = 4;
constexpr int kNnChunk = kNnBlock * kNnItems;

__device__ __forceinline__ bool key_less(uint64_t k1, int32_t i1, uint64_t k2, int32_t i2)
{
    return k1 < k2 || (k1 == k2 && i1 < i2);
}

template <int CAP>
__device__ void bitonic_sort(uint64_t *keys, int32_t *idx)
{
    for (int k = 2; k <= CAP; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < CAP; i += kNnBlock) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint64_t ka = keys[i], kb = keys[ixj];
                    int32_t ia = idx[i], ib = idx[ixj];
                    bool up = (i & k) == 0;
                    bool swap = up ? key_less(kb, ib, ka, ia) : key_less(ka, ia, kb, ib);
                    if (swap) {
                        keys[i] = kb;
                        keys[ixj] = ka;
                        idx[i] = ib;
                        idx[ixj] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int CAP>
__device__ void pad_and_sort(uint64_t *keys, int32_t *idx, int count)
{
    for (int i = count + threadIdx.x; i < CAP; i += kNnBlock) {
        keys[i] = ~0ull;
        idx[i] = INT32_MAX;
    }
    __syncthreads();
    bitonic_sort<CAP>(keys, idx);
}

// PF > 0: p known at compile time (coordinates of x in registers).
template <int CAP, int PF>
__global__ __launch_bounds__(kNnBlock) void nn_pool_kernel(const double *__restrict__ X, int64_t N,
                                                           int p_rt, const double *__restrict__ XX,
                                                           int Np, int32_t *__restrict__ pool)
{
    const int p = PF > 0 ? PF : p_rt;
    __shared__ uint64_t keys[CAP];
    __shared__ int32_t idxs[CAP];
    __shared__ double xs[kMaxP];
    __shared__ int count;
    __shared__ uint64_t thr_k;
    __shared__ int32_t thr_i;

    const int64_t m = blockIdx.x;
    if (threadIdx.x < p) xs[threadIdx.x] = XX[m * p + threadIdx.x];
    if (threadIdx.x == 0) {
        count = 0;
        thr_k = ~0ull;
        thr_i = INT32_MAX;
    }
    __syncthreads();

    double xr[PF > 0 ? PF : 1];
    if (PF > 0) {
#pragma unroll
        for (int k = 0; k < (PF > 0 ? PF : 1); k++) xr[k] = xs[k];
    }

    for (int64_t base = 0; base < N; base += kNnChunk) {
        if (count + kNnChunk > CAP) {  // uniform: count is only written before barriers
            pad_and_sort<CAP>(keys, idxs, count);
            if (threadIdx.x == 0) {
                count = Np;
                thr_k = keys[Np - 1];
                thr_i = idxs[Np - 1];
            }
            __syncthreads();
        }
        const uint64_t tk = thr_k;
        const int32_t ti = thr_i;
#pragma unroll
        for (int it = 0; it < kNnItems; it++) {
            const int64_t i = base + it * kNnBlock + threadIdx.x;
            if (i < N) {
                double s;
                if (PF > 0)
                    s = sqdist_strict(X + i * PF, 1, xr, 1, PF);
                else
                    s = sqdist_strict(X + i * p, 1, xs, 1, p);
                const uint64_t key = __builtin_bit_cast(uint64_t, s);
                if (key_less(key, (int32_t)i, tk, ti)) {
                    int pos = atomicAdd(&count, 1);
                    keys[pos] = key;
                    idxs[pos] = (int32_t)i;
                }
            }
        }
        __syncthreads();
    }
    pad_and_sort<CAP>(keys, idxs, count);
    for (int r = threadIdx.x; r < Np; r += kNnBlock) pool[m * Np + r] = idxs[r];
}

template <int CAP>
static hipError_t launch_cap(const double *X, int64_t N, int p, const double *XX, int64_t M,
                             int Np, int32_t *pool, hipStream_t st)
{
    dim3 grid((unsigned)M), block(kNnBlock);
    switch (p) {
    case 2:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, 2>), grid, block, 0, st, X, N, p, XX, Np, pool);
        break;
    case 4:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, 4>), grid, block, 0, st, X, N, p, XX, Np, pool);
        break;
    case 8:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, 8>), grid, block, 0, st, X, N, p, XX, Np, pool);
        break;
    default:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, 0>), grid, block, 0, st, X, N, p, XX, Np, pool);
    }
    return hipGetLastError();
}

int nn_pool_cap(int Np)
{
    if (Np + kNnChunk <= 2048) return 2048;
    if (Np + kNnChunk <= 4096) return 4096;
    return 0;
}

hipError_t launch_nn_pool(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                          int32_t *pool, hipStream_t st)
{
    if (M == 0) return hipSuccess;
    switch (nn_pool_cap(Np)) {
    case 2048:
        return launch_cap<2048>(X, N, p, XX, M, Np, pool, st);
    case 4096:
        return launch_cap<4096>(X, N, p, XX, M, Np, pool, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace lagp
