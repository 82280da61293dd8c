// Nearest-neighbour candidate pools on gfx950 (Sec. 2.2 NN sub-design,
// Sec. 3.1: the ALC search runs over the N' nearest neighbours of x).
//
// One workgroup per predictive location streams the design once.  Each row's
// squared distance is summed left to right in float64 without fused
// multiply-adds; its bit pattern (non-negative doubles order like unsigned
// integers) followed by the row index forms a unique 96-bit composite key.
// Rows whose key is below the running threshold are appended to an LDS
// buffer.  When the buffer could overflow, an exact radix select on the
// composite key finds the Np-th smallest key, the buffer is cut to exactly
// the Np smallest and the threshold becomes that key.  A final bitonic sort
// of the Np survivors gives the pool in ascending (distance, index) order:
// exact, and independent of scheduling.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

namespace lagp {

constexpr int kNnBlock = 256;
constexpr int kNnWaves = kNnBlock / kWave;
constexpr int kNnItems = 4;
constexpr int kNnChunk = kNnBlock * kNnItems;
constexpr int kNnMaxNp = 2048;

__device__ __forceinline__ bool key_less(uint64_t k1, int32_t i1, uint64_t k2, int32_t i2)
{
    return k1 < k2 || (k1 == k2 && i1 < i2);
}

struct NnShared {
    uint32_t hist[256];
    int16_t holes[kNnMaxNp];
    uint64_t wmin[kNnWaves], wmax[kNnWaves];
    int count, nholes, nmove;
    uint64_t thr_k;
    int32_t thr_i;
    // radix-select state
    uint64_t sel_k;
    int32_t sel_i;
    int rank, bin, bin_count;
};

// 256-bin histogram scan by one wave: finds bin b with cum(<b) <= rank < cum(<=b).
__device__ void hist_pick(NnShared &S, int lane)
{
    uint32_t h[4];
    uint32_t local = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        h[q] = S.hist[lane * 4 + q];
        local += h[q];
    }
    // inclusive scan of `local` over the wave
    uint32_t incl = local;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    uint32_t before = incl - local;
    const uint32_t r = (uint32_t)S.rank;
    if (r >= before && r < incl) {
        uint32_t c = before;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (r >= c && r < c + h[q]) {
                S.bin = lane * 4 + q;
                S.bin_count = (int)h[q];
                S.rank = (int)(r - c);
            }
            c += h[q];
        }
    }
}

// Keeps exactly the Np smallest composite keys of keys/idxs[0, count) in
// [0, Np) (unordered) and sets the threshold to the largest kept key.
__device__ void select_keep(uint64_t *keys, int32_t *idxs, NnShared &S, int count, int Np)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // common prefix of all keys: min and max
    uint64_t lo = ~0ull, hi = 0;
    for (int i = tid; i < count; i += kNnBlock) {
        lo = min(lo, keys[i]);
        hi = max(hi, keys[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (uint64_t)__shfl_xor((unsigned long long)lo, o, kWave));
        hi = max(hi, (uint64_t)__shfl_xor((unsigned long long)hi, o, kWave));
    }
    if (lane == 0) {
        S.wmin[w] = lo;
        S.wmax[w] = hi;
    }
    if (tid == 0) S.rank = Np - 1;
    __syncthreads();
    lo = S.wmin[0];
    hi = S.wmax[0];
    for (int q = 1; q < kNnWaves; q++) {
        lo = min(lo, S.wmin[q]);
        hi = max(hi, S.wmax[q]);
    }
    // digits of the key below the common prefix, then digits of the index
    uint64_t kpref = lo;  // key bits fixed so far (bits above `kshift`)
    int kshift = lo == hi ? 0 : 64 - __builtin_clzll(lo ^ hi);  // bits [kshift, 64) shared
    uint32_t ipref = 0;
    int ishift = 32;
    bool done = false;
    while (!done) {
        const bool on_key = kshift > 0;
        const int width = on_key ? min(8, kshift) : min(8, ishift);
        const int sh = on_key ? kshift - width : ishift - width;
        for (int b = tid; b < 256; b += kNnBlock) S.hist[b] = 0;
        __syncthreads();
        for (int i = tid; i < count; i += kNnBlock) {
            const uint64_t k = keys[i];
            if (on_key) {
                if (kshift == 64 || (k >> kshift) == (kpref >> kshift))
                    atomicAdd(&S.hist[(uint32_t)(k >> sh) & 0xFFu], 1u);
            } else {
                const uint32_t ix = (uint32_t)idxs[i];
                if (k == kpref && (ishift == 32 || (ix >> ishift) == (ipref >> ishift)))
                    atomicAdd(&S.hist[(ix >> sh) & 0xFFu], 1u);
            }
        }
        __syncthreads();
        if (w == 0) hist_pick(S, lane);
        __syncthreads();
        const uint64_t b = (uint64_t)S.bin;
        if (on_key) {
            const uint64_t keep = kshift == 64 ? 0 : (kpref >> kshift) << kshift;
            kpref = keep | (b << sh);
            kshift = sh;
        } else {
            const uint32_t keep = ishift == 32 ? 0 : (ipref >> ishift) << ishift;
            ipref = keep | ((uint32_t)b << sh);
            ishift = sh;
        }
        done = S.bin_count == 1 || (kshift == 0 && ishift == 0);
    }
    // the selected element: unique match of the fixed prefix bits
    for (int i = tid; i < count; i += kNnBlock) {
        const uint64_t k = keys[i];
        const uint32_t ix = (uint32_t)idxs[i];
        const bool key_ok = kshift == 64 ? true : (k >> kshift) == (kpref >> kshift);
        const bool idx_ok = kshift > 0 || ishift == 32 || (ix >> ishift) == (ipref >> ishift);
        if (key_ok && idx_ok && (kshift > 0 || k == kpref)) {
            S.sel_k = k;
            S.sel_i = (int32_t)ix;
        }
    }
    if (tid == 0) {
        S.nholes = 0;
        S.nmove = 0;
    }
    __syncthreads();
    const uint64_t ks = S.sel_k;
    const int32_t is = S.sel_i;
    // holes: positions < Np holding keys above the selection
    for (int i = tid; i < Np; i += kNnBlock)
        if (key_less(ks, is, keys[i], idxs[i])) S.holes[atomicAdd(&S.nholes, 1)] = (int16_t)i;
    __syncthreads();
    // movers: positions >= Np holding keys at or below the selection fill the
    // holes (sources and holes are disjoint, and as many as each other)
    const int nholes = S.nholes;
    for (int i = Np + tid; i < count; i += kNnBlock) {
        const uint64_t k = keys[i];
        const int32_t ix = idxs[i];
        if (!key_less(ks, is, k, ix)) {
            const int mv = atomicAdd(&S.nmove, 1);
            if (mv < nholes) {
                const int h = S.holes[mv];
                keys[h] = k;
                idxs[h] = ix;
            }
        }
    }
    if (tid == 0) {
        S.count = Np;
        S.thr_k = ks;
        S.thr_i = is;
    }
    __syncthreads();
}

template <int SORTN>
__device__ void bitonic_sort(uint64_t *keys, int32_t *idx)
{
    for (int k = 2; k <= SORTN; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < SORTN; i += kNnBlock) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t ka = keys[i], kb = keys[ixj];
                    const int32_t ia = idx[i], ib = idx[ixj];
                    const bool up = (i & k) == 0;
                    const bool swap = up ? key_less(kb, ib, ka, ia) : key_less(ka, ia, kb, ib);
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

// CAP: LDS buffer entries (>= Np + chunk); SORTN: power of two >= Np.
// PF > 0: p known at compile time (coordinates of x in registers).
template <int CAP, int SORTN, int PF>
__global__ __launch_bounds__(kNnBlock) void nn_pool_kernel(const double *__restrict__ X, int64_t N,
                                                           int p_rt, const double *__restrict__ XX,
                                                           int Np, int32_t *__restrict__ pool)
{
    static_assert(CAP >= SORTN + kNnChunk, "room for one chunk above the kept set");
    const int p = PF > 0 ? PF : p_rt;
    __shared__ uint64_t keys[CAP];
    __shared__ int32_t idxs[CAP];
    __shared__ double xs[kMaxP];
    __shared__ NnShared S;

    const int64_t m = blockIdx.x;
    if (threadIdx.x < p) xs[threadIdx.x] = XX[m * p + threadIdx.x];
    if (threadIdx.x == 0) {
        S.count = 0;
        S.thr_k = ~0ull;
        S.thr_i = INT32_MAX;
    }
    __syncthreads();

    double xr[PF > 0 ? PF : 1];
    if (PF > 0) {
#pragma unroll
        for (int k = 0; k < (PF > 0 ? PF : 1); k++) xr[k] = xs[k];
    }

    for (int64_t base = 0; base < N; base += kNnChunk) {
        const int count = S.count;  // written only before barriers
        if (count + kNnChunk > CAP) select_keep(keys, idxs, S, count, Np);
        const uint64_t tk = S.thr_k;
        const int32_t ti = S.thr_i;
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
                    const int pos = atomicAdd(&S.count, 1);
                    keys[pos] = key;
                    idxs[pos] = (int32_t)i;
                }
            }
        }
        __syncthreads();
    }
    if (S.count > Np) select_keep(keys, idxs, S, S.count, Np);
    for (int i = Np + threadIdx.x; i < SORTN; i += kNnBlock) {
        keys[i] = ~0ull;
        idxs[i] = INT32_MAX;
    }
    __syncthreads();
    bitonic_sort<SORTN>(keys, idxs);
    for (int r = threadIdx.x; r < Np; r += kNnBlock) pool[m * Np + r] = idxs[r];
}

template <int CAP, int SORTN>
static hipError_t launch_cap(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                             int32_t *pool, hipStream_t st)
{
    dim3 grid((unsigned)M), block(kNnBlock);
    switch (p) {
    case 2:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, SORTN, 2>), grid, block, 0, st, X, N, p, XX, Np, pool);
        break;
    case 4:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, SORTN, 4>), grid, block, 0, st, X, N, p, XX, Np, pool);
        break;
    case 8:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, SORTN, 8>), grid, block, 0, st, X, N, p, XX, Np, pool);
        break;
    default:
        hipLaunchKernelGGL((nn_pool_kernel<CAP, SORTN, 0>), grid, block, 0, st, X, N, p, XX, Np, pool);
    }
    return hipGetLastError();
}

int nn_pool_cap(int Np)
{
    if (Np <= 512) return 2048;
    if (Np <= 1024) return 4096;
    if (Np <= kNnMaxNp) return 4096 + 1024;
    return 0;
}

hipError_t launch_nn_pool(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                          int32_t *pool, hipStream_t st)
{
    if (M == 0) return hipSuccess;
    if (Np <= 512) return launch_cap<2048, 512>(X, N, p, XX, M, Np, pool, st);
    if (Np <= 1024) return launch_cap<4096, 1024>(X, N, p, XX, M, Np, pool, st);
    if (Np <= kNnMaxNp) return launch_cap<4096 + 1024, 2048>(X, N, p, XX, M, Np, pool, st);
    return hipErrorInvalidValue;
}

}  // namespace lagp
