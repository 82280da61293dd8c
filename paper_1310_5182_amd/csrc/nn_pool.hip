// Nearest-neighbour candidate pools on gfx950 (Sec. 2.2 NN sub-design,
// Sec. 3.1: the ALC search runs over the N' nearest neighbours of x).
//
// One workgroup serves G predictive locations and streams the design once
// for all of them: each float64 row is loaded once, rounded to float32 once
// and compared with the G locations in float32.  A row can only be among a
// location's nearest if its float32 squared distance, less a rigorous bound
// on the float32 error, is below the location's running threshold; only such
// rows get the exact key.  The exact squared distance is summed left to right
// in float64 without fused multiply-adds; its bit pattern (non-negative
// doubles order like unsigned integers) followed by the row index forms a
// unique 96-bit composite key.  Rows whose key is below the running threshold
// are appended to the location's LDS buffer.  When a buffer could overflow,
// an exact radix select on the composite key finds the Np-th smallest key,
// the buffer is cut to exactly the Np smallest and the threshold becomes that
// key.  A final bitonic sort of the Np survivors (in registers, lane
// exchanges within a wave, LDS between waves) gives the pool in ascending
// (distance, index) order: exact, and independent of scheduling.
//
// Float32 error bound.  With u = 2^-24, coordinates bounded by B in
// magnitude, t = x_k - c_k: rounding x_k and c_k to float32 and subtracting
// errs by at most ~4uB, squaring adds ~20uB^2 per coordinate in all, and the
// float32 sum of p terms errs by at most (p-1)u times its value, so
// |d32 - d| <= 40 p u B^2 + 2 p u d32 (twice the first-order terms).  B is the
// larger of the row's and the location's largest coordinate magnitude; taken
// from the float32 values, it is short of the exact one by a factor of at most
// 1 - u, far inside the bound's slack.
//
// With a float32 copy of X (made once per call into caller workspace), the
// stream reads half the bytes and the float64 row is fetched only for the rows
// that pass the float32 test.
//
// Grid-pruned pools (with caller workspace).  The design is bucketed once per
// call into C <= 1024 cells of a regular grid over its bounding box (the bits
// of the cell index spread over the first dimensions) by a counting sort,
// which leaves float32 and float64 copies of the rows cell by cell, their design indices,
// and the exact float64 bounding box of each cell's rows.  Each location
// sorts the cells by the squared distance from x to their boxes and streams
// the rows nearest cell first; a cell whose box is farther than the running
// threshold (with a relative margin of 2^-20, far above the rounding of
// either side) holds no row below it, and since the cells come in order of
// that distance, the first such chunk ends the stream.  Every row that is
// streamed goes through the same screen and exact key as above, so the pools
// are identical to the unpruned ones.  In the grid kernel the rows that pass
// the float32 screen are first gathered into a per-wave list and their exact
// keys are then computed 64 at a time, so that the float64 arithmetic and the
// gathers of float64 rows run on full waves rather than on the few lanes of a
// block that passed; the float64 row comes from the bucketed copy, loaded
// beside its design index rather than through it.  The locations are bucketed into the
// same cells, and the workgroups of each XCD (the dispatcher hands out
// consecutive workgroups to the XCDs in turn) take a contiguous run of them in
// cell order, so that the workgroups resident on one XCD read mostly the same
// cells through its L2.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <mutex>

namespace lagp {

constexpr int kNnBlock = 256;
constexpr int kNnWaves = kNnBlock / kWave;
constexpr int kNnItems = 4;
constexpr int kNnChunk = kNnBlock * kNnItems;
// items whose row loads are in flight together (p <= 8; one at a time above,
// where the registers of a second row would spill)
constexpr int kNnBatchPmax = 8;
constexpr int kNnMaxNp = 2048;

__device__ __forceinline__ bool key_less(uint64_t k1, int32_t i1, uint64_t k2, int32_t i2)
{
    return k1 < k2 || (k1 == k2 && i1 < i2);
}

// Selection scratch, shared by the locations of a workgroup (one select at a time).
struct NnShared {
    uint32_t hist[256];
    // holes of a selection; between selections, the grid kernel's per-wave
    // lists of the rows that passed the float32 screen in the current chunk
    union {
        int16_t holes[kNnMaxNp];
        int32_t surv[kNnMaxNp / 2];
    };
    uint64_t wmin[kNnWaves], wmax[kNnWaves];
    int nholes, nmove;
    // radix-select state
    uint64_t sel_k;
    int32_t sel_i;
    int rank, bin, bin_count;
};

// Buffer fill and threshold of one location.  full[c & 1] is set when an
// append of chunk c finds the buffer full.  Every thread reads it after the
// chunk's barrier, and nothing writes it again before the end of chunk c + 1
// (the flag of chunk c + 1 is the other one, and a selection clears it before
// its last barrier), so all threads take the same decision even when some of
// them are already appending rows of chunk c + 1, which moves the count.
struct NnGroup {
    int count;
    int full[2];
    int cut;  // grid kernel: first stream position out of the threshold's reach
    uint64_t thr_k;
    int32_t thr_i;
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
__device__ void select_keep(uint64_t *keys, int32_t *idxs, NnShared &S, NnGroup &grp, int count, int Np)
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
        grp.count = Np;
        grp.full[0] = grp.full[1] = 0;
        grp.thr_k = ks;
        grp.thr_i = is;
    }
    __syncthreads();
}

// Ascending sort of SORTN composite keys, E = SORTN / kNnBlock per thread in
// registers (thread t holds elements t E .. t E + E - 1), by the bitonic
// network: steps between elements of one thread in registers, between threads
// of one wave by lane exchanges (every lane keeps the smaller or the larger of
// its element and its partner's), between waves through LDS (kv, iv; the first
// such step waits for every thread to have read what it needs from them).
// Step (KK, J) compares elements i and i ^ J in blocks of KK; the steps are
// instantiated one by one so that every register index is a constant.
template <int SORTN, int KK, int J>
__device__ __forceinline__ void bitonic_step(uint64_t (&k)[SORTN / kNnBlock], int32_t (&ix)[SORTN / kNnBlock],
                                             uint64_t *kv, int32_t *iv)
{
    constexpr int E = SORTN / kNnBlock;
    const int tid = threadIdx.x;
    if constexpr (J < E) {
#pragma unroll
        for (int q = 0; q < E; q++) {
            const int l = q ^ J;
            if (l > q) {
                const bool up = ((tid * E + q) & KK) == 0;
                const bool sw = up ? key_less(k[l], ix[l], k[q], ix[q]) : key_less(k[q], ix[q], k[l], ix[l]);
                if (sw) {
                    const uint64_t tk = k[q];
                    const int32_t tix = ix[q];
                    k[q] = k[l];
                    ix[q] = ix[l];
                    k[l] = tk;
                    ix[l] = tix;
                }
            }
        }
    } else {
        uint64_t pk[E];
        int32_t pi[E];
        if constexpr (J < kWave * E) {
            constexpr int lm = J / E;
#pragma unroll
            for (int q = 0; q < E; q++) {
                const uint32_t lo = __shfl_xor((uint32_t)k[q], lm, kWave);
                const uint32_t hi = __shfl_xor((uint32_t)(k[q] >> 32), lm, kWave);
                pk[q] = ((uint64_t)hi << 32) | lo;
                pi[q] = __shfl_xor(ix[q], lm, kWave);
            }
        } else {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < E; q++) {
                kv[tid * E + q] = k[q];
                iv[tid * E + q] = ix[q];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < E; q++) {
                pk[q] = kv[(tid * E + q) ^ J];
                pi[q] = iv[(tid * E + q) ^ J];
            }
        }
#pragma unroll
        for (int q = 0; q < E; q++) {
            const int i = tid * E + q;
            const bool keep_min = ((i & J) == 0) == ((i & KK) == 0);
            const bool pless = key_less(pk[q], pi[q], k[q], ix[q]);
            if (keep_min == pless) {
                k[q] = pk[q];
                ix[q] = pi[q];
            }
        }
    }
    if constexpr (J > 1)
        bitonic_step<SORTN, KK, J / 2>(k, ix, kv, iv);
    else if constexpr (KK < SORTN)
        bitonic_step<SORTN, 2 * KK, KK>(k, ix, kv, iv);
}

template <int SORTN>
__device__ __forceinline__ void bitonic_sort_regs(uint64_t (&k)[SORTN / kNnBlock], int32_t (&ix)[SORTN / kNnBlock],
                                                  uint64_t *kv, int32_t *iv)
{
    static_assert(SORTN % kNnBlock == 0 && (SORTN & (SORTN - 1)) == 0, "whole elements per thread");
    bitonic_step<SORTN, 2, 1>(k, ix, kv, iv);
}

// Ascending sort of n (a power of two <= the buffers) composite keys.
__device__ void bitonic_sort_n(uint64_t *keys, int32_t *idx, int n)
{
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += kNnBlock) {
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

// G: locations per workgroup; CAP: LDS buffer entries per location
// (>= SORTN + chunk); SORTN: power of two >= Np; PF: p at compile time;
// F32: stream the float32 copy X32 (else X).
// Waves per SIMD that the LDS of one-location workgroups allows (five at
// CAP = 2048, three at 3072): registers are held to that occupancy.
template <int G, int CAP>
constexpr int nn_waves()
{
    return G != 1 ? 1 : CAP <= 2048 ? 5 : CAP <= 3072 ? 3 : 1;
}

template <int G, int CAP, int SORTN, int PF, bool F32>
__global__ __launch_bounds__(kNnBlock) __attribute__((amdgpu_waves_per_eu(nn_waves<G, CAP>()))) void nn_pool_kernel(const double *__restrict__ X,
                                                           const float *__restrict__ X32, int64_t N,
                                                           const double *__restrict__ XX, int64_t M,
                                                           int Np, int32_t *__restrict__ pool)
{
    static_assert(CAP >= SORTN + kNnChunk, "room for one chunk above the kept set");
    static_assert(PF >= 1 && PF <= kMaxP, "compile-time dimension");
    constexpr int p = PF;
    constexpr float kU = 5.9604645e-8f;  // 2^-24
    __shared__ uint64_t keys[G][CAP];
    __shared__ int32_t idxs[G][CAP];
    __shared__ double xs[G][PF];
    __shared__ NnGroup grp[G];
    __shared__ NnShared S;

    const int64_t m0 = (int64_t)blockIdx.x * G;
    const int ng = (int)(M - m0 < G ? M - m0 : G);  // locations of this workgroup
    for (int t = threadIdx.x; t < G * PF; t += kNnBlock) {
        const int g = t / PF, k = t - g * PF;
        xs[g][k] = g < ng ? XX[(m0 + g) * p + k] : 0.0;
    }
    if (threadIdx.x < G) {
        grp[threadIdx.x].count = 0;
        grp[threadIdx.x].full[0] = grp[threadIdx.x].full[1] = 0;
        grp[threadIdx.x].thr_k = ~0ull;
        grp[threadIdx.x].thr_i = INT32_MAX;
    }
    __syncthreads();

    // float32 copies of the locations and their error-bound constants
    float xf[G][PF], lmax[G];
#pragma unroll
    for (int g = 0; g < G; g++) {
        lmax[g] = 0.0f;
#pragma unroll
        for (int k = 0; k < PF; k++) {
            xf[g][k] = (float)xs[g][k];
            lmax[g] = fmaxf(lmax[g], fabsf(xf[g][k]));
        }
    }
    constexpr float kSlope = 1.0f - 2.0f * PF * kU;  // d32 (1 - 2pu) - 40 p u B^2 < thr
    constexpr float kConst = 40.0f * PF * kU;

    for (int64_t base = 0; base < N; base += kNnChunk) {
        const int par = (int)((base / kNnChunk) & 1);
        uint64_t tk[G];
        int32_t ti[G];
        float tf[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            tk[g] = grp[g].thr_k;
            ti[g] = grp[g].thr_i;
            // the threshold distance, rounded up to float32 (+inf before the first select)
            const double td = tk[g] == ~0ull ? INFINITY : __builtin_bit_cast(double, tk[g]);
            const float f = (float)td;  // td >= 0: the next float up is the next bit pattern
            tf[g] = (double)f < td ? __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u) : f;
        }
        // bit g * kNnItems + it: the row of item `it` passed for location g but
        // found the buffer full; it is tried again after the next selection
        uint32_t pend = 0;
        // rows are loaded kNnBatch items at a time, all loads in flight together
        // (a row index past the design reads the last row and is not used)
        constexpr int kNnBatch = PF <= kNnBatchPmax ? 2 : 1;
#pragma unroll
        for (int it0 = 0; it0 < kNnItems; it0 += kNnBatch) {
        double xb[kNnBatch][F32 ? 1 : PF];
        float xbf[kNnBatch][F32 ? PF : 1];
#pragma unroll
        for (int b = 0; b < kNnBatch; b++) {
            const int64_t i = base + (it0 + b) * kNnBlock + threadIdx.x;
            const int64_t ic = i < N ? i : N - 1;
#pragma unroll
            for (int k = 0; k < PF; k++) {
                if constexpr (F32)
                    xbf[b][k] = X32[ic * PF + k];
                else
                    xb[b][k] = X[ic * PF + k];
            }
        }
#pragma unroll
        for (int b = 0; b < kNnBatch; b++) {
            const int it = it0 + b;
            const int64_t i = base + it * kNnBlock + threadIdx.x;
            if (i < N) {
                double xr[PF];
                float xrf[PF];
                float rmax = 0.0f;
                if constexpr (F32) {
#pragma unroll
                    for (int k = 0; k < PF; k++) xrf[k] = xbf[b][k];
                } else {
#pragma unroll
                    for (int k = 0; k < PF; k++) {
                        xr[k] = xb[b][k];
                        xrf[k] = (float)xr[k];
                    }
                }
                bool have64 = !F32;
#pragma unroll
                for (int k = 0; k < PF; k++) rmax = fmaxf(rmax, fabsf(xrf[k]));
#pragma unroll
                for (int g = 0; g < G; g++) {
                    float d32 = 0.0f;
#pragma unroll
                    for (int k = 0; k < PF; k++) {
                        const float t = xrf[k] - xf[g][k];
                        d32 = fmaf(t, t, d32);
                    }
                    const float B = fmaxf(rmax, lmax[g]);
                    if (d32 * kSlope - kConst * B * B < tf[g] && g < ng) {
                        if (!have64) {
#pragma unroll
                            for (int k = 0; k < PF; k++) xr[k] = X[i * PF + k];
                            have64 = true;
                        }
                        const double s = sqdist_strict(xr, 1, xs[g], 1, p);
                        const uint64_t key = __builtin_bit_cast(uint64_t, s);
                        if (key_less(key, (int32_t)i, tk[g], ti[g])) {
                            const int pos = atomicAdd(&grp[g].count, 1);
                            if (pos < CAP) {
                                keys[g][pos] = key;
                                idxs[g][pos] = (int32_t)i;
                            } else {
                                pend |= 1u << (g * kNnItems + it);
                                grp[g].full[par] = 1;
                            }
                        }
                    }
                }
            }
        }
        }
        __syncthreads();
        // A full buffer: keep the Np smallest of its CAP keys, then insert the
        // rows that did not fit and still beat the new threshold (at most one
        // chunk, and CAP >= Np + chunk).  The decision reads this chunk's flag,
        // the same for every thread (the count may already be moving).
#pragma unroll 1
        for (int g = 0; g < G; g++) {
            if (grp[g].full[par]) {
                select_keep(keys[g], idxs[g], S, grp[g], CAP, Np);
                const uint64_t nk = grp[g].thr_k;
                const int32_t ni = grp[g].thr_i;
#pragma unroll
                for (int it = 0; it < kNnItems; it++) {
                    if ((pend >> (g * kNnItems + it)) & 1u) {
                        const int64_t i = base + it * kNnBlock + threadIdx.x;
                        const double s = sqdist_strict(X + i * PF, 1, xs[g], 1, p);
                        const uint64_t key = __builtin_bit_cast(uint64_t, s);
                        if (key_less(key, (int32_t)i, nk, ni)) {
                            const int pos = atomicAdd(&grp[g].count, 1);
                            keys[g][pos] = key;
                            idxs[g][pos] = (int32_t)i;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
#pragma unroll 1
    for (int g = 0; g < ng; g++) {
        if (grp[g].count > Np) select_keep(keys[g], idxs[g], S, grp[g], grp[g].count, Np);
        constexpr int E = SORTN / kNnBlock;
        uint64_t kr[E];
        int32_t ir[E];
#pragma unroll
        for (int qq = 0; qq < E; qq++) {
            const int e = threadIdx.x * E + qq;
            kr[qq] = e < Np ? keys[g][e] : ~0ull;
            ir[qq] = e < Np ? idxs[g][e] : INT32_MAX;
        }
        bitonic_sort_regs<SORTN>(kr, ir, keys[g], idxs[g]);
#pragma unroll
        for (int qq = 0; qq < E; qq++) {
            const int e = threadIdx.x * E + qq;
            if (e < Np) pool[(m0 + g) * Np + e] = ir[qq];
        }
        __syncthreads();
    }
}

// Locations per workgroup: more share each pass over X; fewer keep more
// workgroups resident (each location holds CAP keys in LDS).
template <int G, int CAP, int SORTN>
static hipError_t launch_cap(const double *X, const float *X32, int64_t N, int p, const double *XX, int64_t M,
                             int Np, int32_t *pool, hipStream_t st)
{
    dim3 grid((unsigned)((M + G - 1) / G)), block(kNnBlock);
    switch (p) {
#define LAGP_NN_CASE(P)                                                                                    \
    case P:                                                                                                \
        if (X32)                                                                                           \
            hipLaunchKernelGGL((nn_pool_kernel<G, CAP, SORTN, P, true>), grid, block, 0, st, X, X32, N, XX, M, \
                               Np, pool);                                                                  \
        else                                                                                               \
            hipLaunchKernelGGL((nn_pool_kernel<G, CAP, SORTN, P, false>), grid, block, 0, st, X, X32, N, XX, M, \
                               Np, pool);                                                                  \
        break;
        LAGP_NN_CASE(1)
        LAGP_NN_CASE(2)
        LAGP_NN_CASE(3)
        LAGP_NN_CASE(4)
        LAGP_NN_CASE(5)
        LAGP_NN_CASE(6)
        LAGP_NN_CASE(7)
        LAGP_NN_CASE(8)
        LAGP_NN_CASE(9)
        LAGP_NN_CASE(10)
        LAGP_NN_CASE(11)
        LAGP_NN_CASE(12)
        LAGP_NN_CASE(13)
        LAGP_NN_CASE(14)
        LAGP_NN_CASE(15)
        LAGP_NN_CASE(16)
#undef LAGP_NN_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ grid pruning
constexpr int kGridCmax = 1024;  // cells
constexpr int kGridParts = 256;  // workgroups of the bounding-box pass

struct NnGrid {
    float *x32;      // [N x p] float32 rows, cell by cell
    double *x64;     // [N x p] the same rows in float64
    int32_t *perm;   // [N] design index of each of those rows
    int32_t *cid;    // [N] cell of each design row
    int32_t *cnt;    // [C] rows per cell
    int32_t *cur;    // [C] scatter cursors
    int32_t *off;    // [C + 1] first row of each cell
    double *box;     // [C][p][2] smallest and largest coordinate of each cell's rows
    double *part;    // [kGridParts + 1][p][2] partial bounds, then the design's bounds
    int32_t *lcid;   // [M] cell of each location
    int32_t *lcnt, *lcur, *loff;  // [C], [C], [C + 1] as above, for the locations
    int32_t *lperm;  // [M] locations in cell order
    int C;
    int bits[kMaxP];  // cell-index bits of each dimension
};

// Cells of 256 rows or more (up to kGridCmax cells): finer cells prune more
// rows, coarser ones keep the blocks of a chunk within one cell more often
// (measured: 256 beats 512, 128 and 64 at N = 1e5 and 2e5).
static int grid_cells(int64_t N)
{
    int C = 1;
    while (C < kGridCmax && (int64_t)C * 2 * 256 <= N) C *= 2;
    return C;
}

static size_t align256(size_t v)
{
    return (v + 255) & ~(size_t)255;
}

size_t nn_pool_workspace(int64_t N, int p, int64_t M)
{
    return align256((size_t)N * p * 4) + align256((size_t)N * p * 8) + 2 * align256((size_t)N * 4) +
           3 * align256((kGridCmax + 1) * 4) +
           align256((size_t)kGridCmax * p * 16) + align256((size_t)(kGridParts + 1) * p * 16) +
           2 * align256((size_t)M * 4) + 3 * align256((kGridCmax + 1) * 4);
}

static NnGrid grid_layout(void *ws, int64_t N, int p, int64_t M)
{
    NnGrid g{};
    char *b = (char *)ws;
    g.x32 = (float *)b;
    b += align256((size_t)N * p * 4);
    g.x64 = (double *)b;
    b += align256((size_t)N * p * 8);
    g.perm = (int32_t *)b;
    b += align256((size_t)N * 4);
    g.cid = (int32_t *)b;
    b += align256((size_t)N * 4);
    g.cnt = (int32_t *)b;
    b += align256((kGridCmax + 1) * 4);
    g.cur = (int32_t *)b;
    b += align256((kGridCmax + 1) * 4);
    g.off = (int32_t *)b;
    b += align256((kGridCmax + 1) * 4);
    g.box = (double *)b;
    b += align256((size_t)kGridCmax * p * 16);
    g.part = (double *)b;
    b += align256((size_t)(kGridParts + 1) * p * 16);
    g.lcid = (int32_t *)b;
    b += align256((size_t)M * 4);
    g.lperm = (int32_t *)b;
    b += align256((size_t)M * 4);
    g.lcnt = (int32_t *)b;
    b += align256((kGridCmax + 1) * 4);
    g.lcur = (int32_t *)b;
    b += align256((kGridCmax + 1) * 4);
    g.loff = (int32_t *)b;
    g.C = grid_cells(N);
    int cb = 0;
    while ((1 << cb) < g.C) cb++;
    for (int k = 0; k < kMaxP; k++) g.bits[k] = k < p ? cb / p + (k < cb % p ? 1 : 0) : 0;
    return g;
}

// Partial bounds of the design per workgroup; non-finite coordinates widen
// the bounds to the whole line.
__global__ __launch_bounds__(256) void grid_minmax(const double *__restrict__ X, int64_t N, int p, NnGrid g)
{
    __shared__ double slo[256], shi[256];
    double lo[kMaxP], hi[kMaxP];
#pragma unroll
    for (int k = 0; k < kMaxP; k++) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int k = 0; k < kMaxP; k++)
            if (k < p) {
                const double v = X[i * p + k];
                lo[k] = isfinite(v) ? fmin(lo[k], v) : -INFINITY;
                hi[k] = isfinite(v) ? fmax(hi[k], v) : INFINITY;
            }
#pragma unroll
    for (int k = 0; k < kMaxP; k++) {
        if (k >= p) break;
        slo[threadIdx.x] = lo[k];
        shi[threadIdx.x] = hi[k];
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (threadIdx.x < s2) {
                slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s2]);
                shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s2]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            g.part[((size_t)blockIdx.x * p + k) * 2] = slo[0];
            g.part[((size_t)blockIdx.x * p + k) * 2 + 1] = shi[0];
        }
        __syncthreads();
    }
}

// The design's bounds from the partials; cell counters cleared.
__global__ __launch_bounds__(256) void grid_final(int p, int parts, NnGrid g)
{
    if (threadIdx.x < p) {
        const int k = threadIdx.x;
        double lo = INFINITY, hi = -INFINITY;
        for (int b = 0; b < parts; b++) {
            lo = fmin(lo, g.part[((size_t)b * p + k) * 2]);
            hi = fmax(hi, g.part[((size_t)b * p + k) * 2 + 1]);
        }
        g.part[((size_t)kGridParts * p + k) * 2] = lo;
        g.part[((size_t)kGridParts * p + k) * 2 + 1] = hi;
    }
    for (int c = threadIdx.x; c < kGridCmax + 1; c += 256) {
        g.cnt[c] = 0;
        g.lcnt[c] = 0;
    }
}

__device__ __forceinline__ int grid_cell_of(const double *__restrict__ X, int64_t i, int p, const NnGrid &g)
{
    int cell = 0;
#pragma unroll
    for (int k = 0; k < kMaxP; k++) {
        if (k >= p) break;
        const int b = g.bits[k];
        if (b == 0) continue;
        const double lo = g.part[((size_t)kGridParts * p + k) * 2], hi = g.part[((size_t)kGridParts * p + k) * 2 + 1];
        const int s = 1 << b;
        int q = 0;
        const double v = X[i * p + k];
        if (hi > lo && isfinite(hi - lo) && isfinite(v)) {
            const double t = floor((v - lo) / (hi - lo) * s);
            q = t < 0.0 ? 0 : t >= (double)s ? s - 1 : (int)t;
        }
        cell = (cell << b) | q;
    }
    return cell;
}

// Cell of each of the n points P (the design rows, or the locations) and the
// points per cell.
__global__ __launch_bounds__(256) void grid_count(const double *__restrict__ P, int64_t n, int p, NnGrid g,
                                                  int32_t *cid, int32_t *cnt)
{
    __shared__ int32_t h[kGridCmax];
    for (int c = threadIdx.x; c < g.C; c += 256) h[c] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int c = grid_cell_of(P, i, p, g);
        cid[i] = c;
        atomicAdd(&h[c], 1);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < g.C; c += 256)
        if (h[c]) atomicAdd(&cnt[c], h[c]);
}

// Exclusive scan of the counts (one workgroup, four cells per thread).
__global__ __launch_bounds__(256) void grid_scan(int64_t n, int C, const int32_t *cnt, int32_t *off, int32_t *cur)
{
    __shared__ int32_t part[256];
    const int t = threadIdx.x;
    int32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int c = 4 * t + q;
        v[q] = c < C ? cnt[c] : 0;
        sum += v[q];
    }
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int32_t add = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int c = 4 * t + q;
        if (c < C) {
            off[c] = run;
            cur[c] = run;
        }
        run += v[q];
    }
    if (t == 0) off[C] = (int32_t)n;
}

// The locations in cell order.
__global__ __launch_bounds__(256) void grid_order(int64_t M, NnGrid g)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256)
        g.lperm[atomicAdd(&g.lcur[g.lcid[i]], 1)] = (int32_t)i;
}

__global__ __launch_bounds__(256) void grid_scatter(const double *__restrict__ X, int64_t N, int p, NnGrid g)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const int pos = atomicAdd(&g.cur[g.cid[i]], 1);
        g.perm[pos] = (int32_t)i;
        for (int k = 0; k < p; k++) {
            const double v = X[i * p + k];
            g.x64[(size_t)pos * p + k] = v;
            g.x32[(size_t)pos * p + k] = (float)v;
        }
    }
}

// Exact float64 bounds of each cell's rows (one workgroup per cell; an empty
// cell gets +inf / -inf, which puts it out of reach).
__global__ __launch_bounds__(256) void grid_box(const double *__restrict__ X, int p, NnGrid g)
{
    __shared__ double slo[256], shi[256];
    const int c = blockIdx.x;
    const int r0 = g.off[c], r1 = g.off[c + 1];
    for (int k = 0; k < p; k++) {
        double lo = INFINITY, hi = -INFINITY;
        for (int r = r0 + threadIdx.x; r < r1; r += 256) {
            const double v = X[(int64_t)g.perm[r] * p + k];
            lo = isfinite(v) ? fmin(lo, v) : -INFINITY;
            hi = isfinite(v) ? fmax(hi, v) : INFINITY;
        }
        slo[threadIdx.x] = lo;
        shi[threadIdx.x] = hi;
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (threadIdx.x < s2) {
                slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s2]);
                shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s2]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            g.box[((size_t)c * p + k) * 2] = slo[0];
            g.box[((size_t)c * p + k) * 2 + 1] = shi[0];
        }
        __syncthreads();
    }
}

// Largest rank r >= r0 with pre[r] <= v, for pre[r0] <= v < pre[C] (pre
// ascending): a forward walk, short because cells hold 256 rows or more.
__device__ __forceinline__ int rank_from(const int32_t *pre, int r0, int64_t v)
{
    while (pre[r0 + 1] <= v) r0++;
    return r0;
}

// A non-negative float kept in 16 bits, its top half (truncation toward zero):
// a lower bound of the value, +inf for +inf.
__device__ __forceinline__ uint16_t f16_down(float f)
{
    return (uint16_t)(__builtin_bit_cast(uint32_t, f) >> 16);
}
__device__ __forceinline__ float f16_value(uint16_t h)
{
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

constexpr double kGridMargin = 1.0 - 1.0 / (1 << 20);

// The first stream position that lies in a cell out of the reach of the
// threshold distance td: pre[R] for the smallest rank R whose lower bound on
// the box distance, less the margin, exceeds td (the bounds ascend with the
// rank), or N = pre[C] if there is none.
__device__ int grid_cut(const uint16_t *mind, const int32_t *pre, int C, double td)
{
    int lo = 0, hi = C;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((double)f16_value(mind[mid]) * kGridMargin > td)
            hi = mid;
        else
            lo = mid + 1;
    }
    return pre[lo];
}

__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// The cells of the grid in order of the squared distance from x to their boxes
// (ties by cell index) for the grid kernel: E ranks per thread (thread t gets
// ranks t E .. t E + E - 1, C <= E kNnBlock), sorted in registers with the
// entries past C padded by the largest key; then the lower bound of each
// cell's distance (mindr), the rows before it in rank order (pre, with
// pre[C] = N) and its row offset (rbase).  kv, iv: LDS scratch of E kNnBlock
// entries for the sort; hist: kNnBlock words for the scan; box, off: the
// grid's cell bounds and row offsets.
template <int E, int PF>
__device__ __forceinline__ void grid_rank_cells(const double *box, const int32_t *off, const double *xs, int C,
                                                int64_t N, uint64_t *kv, int32_t *iv, uint32_t *hist, int32_t *pre,
                                                int32_t *rbase, uint16_t *mindr)
{
    static_assert((E == 1 || E == 2 || E == 4) && 4 * kNnBlock >= kGridCmax, "up to four ranks per thread");
    const int tid = threadIdx.x;
    uint64_t kr[E];
    int32_t cr[E];
#pragma unroll
    for (int qq = 0; qq < E; qq++) {
        const int c = tid * E + qq;
        kr[qq] = ~0ull;
        cr[qq] = c;
        if (c < C) {
            double sd = 0.0;
#pragma unroll
            for (int k = 0; k < PF; k++) {
                const double lo = box[((size_t)c * PF + k) * 2], hi = box[((size_t)c * PF + k) * 2 + 1];
                const double gap = fmax(fmax(lo - xs[k], xs[k] - hi), 0.0);
                sd = fma(gap, gap, sd);
            }
            kr[qq] = __builtin_bit_cast(uint64_t, sd);  // >= 0 (or NaN for a NaN location: after the others)
        }
    }
    bitonic_sort_regs<E * kNnBlock>(kr, cr, kv, iv);
    int32_t csum[E], coff[E], tot = 0;
#pragma unroll
    for (int qq = 0; qq < E; qq++) {
        const int r = tid * E + qq;
        csum[qq] = 0;
        coff[qq] = 0;
        if (r < C) {
            const int c = cr[qq];
            const double md = __builtin_bit_cast(double, kr[qq]);
            float f = (float)md;  // rounded down to a float below md
            if (!(md >= 0.0)) f = INFINITY;
            else if ((double)f > md) f = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) - 1u);
            mindr[r] = f16_down(f);
            coff[qq] = off[c];
            csum[qq] = off[c + 1] - coff[qq];
        }
        tot += csum[qq];
    }
    // exclusive scan of the cell sizes in rank order: pre[r]
    hist[tid] = (uint32_t)tot;
    __syncthreads();
    for (int o = 1; o < kNnBlock; o <<= 1) {
        const uint32_t add = tid >= o ? hist[tid - o] : 0u;
        __syncthreads();
        hist[tid] += add;
        __syncthreads();
    }
    int32_t run = (int32_t)hist[tid] - tot;
#pragma unroll
    for (int qq = 0; qq < E; qq++) {
        const int r = tid * E + qq;
        if (r < C) {
            pre[r] = run;
            rbase[r] = coff[qq] - run;
        }
        run += csum[qq];
    }
    if (tid == 0) pre[C] = (int32_t)N;
    __syncthreads();
}

// One location per workgroup, rows streamed cell by cell (nearest first).
//
// Stream position v (0 <= v < N) is row v + rbase[r] of the bucketed design,
// where r is the rank of the cell with pre[r] <= v < pre[r + 1].  A chunk is
// kNnChunk positions; wave w takes kNnItems blocks of 64 consecutive positions
// from it.  Each wave keeps a cursor on the cell of its current block (its
// positions only grow), so a block inside one cell costs one add per lane;
// lanes of a block that crosses into later cells walk pre[] on their own.
// Since the box bounds ascend with the rank, every position below `cut` is in
// a cell within reach of the threshold and every position from `cut` on is
// not: the stream ends at the first chunk that starts at or past it.  Rows
// that pass the float32 screen go to a per-wave list, and the exact keys are
// then computed for the list, 64 rows at a time, so that the float64 work and
// its gathers run on full waves; a wave appends its new keys with one atomic.
template <int CAP, int SORTN, int PF>
__global__ __launch_bounds__(kNnBlock) void nn_grid_kernel(const double *__restrict__ X, int64_t N,
                                                           const double *__restrict__ XX, int64_t M, int Np,
                                                           int32_t *__restrict__ pool, NnGrid gr)
{
    static_assert(CAP >= SORTN + kNnChunk && CAP >= kGridCmax, "room for one chunk above the kept set");
    static_assert(kNnWaves * kNnItems * kWave <= kNnMaxNp / 2, "the survivor lists fit in the holes' space");
    static_assert(kNnItems <= 32, "pending bits in one word");
    constexpr int p = PF;
    constexpr float kU = 5.9604645e-8f;  // 2^-24
    __shared__ uint64_t keys[CAP];
    __shared__ int32_t idxs[CAP];
    __shared__ double xs[PF];
    __shared__ NnGroup grp;
    __shared__ NnShared S;
    __shared__ int32_t pre[kGridCmax + 1];  // rows in the cells of rank < r
    __shared__ int32_t rbase[kGridCmax];    // first row of the cell of rank r (nearest first), less pre[r]
    __shared__ uint16_t mindr[kGridCmax];   // <= squared distance from x to the box of that cell

    const int tid = threadIdx.x, C = gr.C;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & (kWave - 1);
    // the XCD of this workgroup (blockIdx.x mod 8) takes the slots
    // [x q, (x + 1) q) of the locations in cell order; the grid is 8 q wide
    const int64_t q8 = (M + 7) / 8, slot = (int64_t)(blockIdx.x & 7) * q8 + (blockIdx.x >> 3);
    if (slot >= M) return;  // the whole workgroup, before any barrier
    const int64_t m = gr.lperm[slot];
    if (tid < PF) xs[tid] = XX[m * p + tid];
    if (tid == 0) {
        grp.count = 0;
        grp.full[0] = grp.full[1] = 0;
        grp.cut = (int)N;  // no threshold yet: every cell is in reach
        grp.thr_k = ~0ull;
        grp.thr_i = INT32_MAX;
    }
    __syncthreads();
    float xf[PF], lmax = 0.0f;
#pragma unroll
    for (int k = 0; k < PF; k++) {
        xf[k] = (float)xs[k];
        lmax = fmaxf(lmax, fabsf(xf[k]));
    }
    constexpr float kSlope = 1.0f - 2.0f * PF * kU;
    constexpr float kConst = 40.0f * PF * kU;
    // The screen's bound B on the magnitude of every coordinate, the row's and
    // x's, from the design's bounding box (rounded up to float32, so that it is
    // at least every float32 row coordinate) instead of each row's own maximum:
    // a larger B only lets more rows through to the exact test.
    float bd = 0.0f;
#pragma unroll
    for (int k = 0; k < PF; k++) {
        const double lo = gr.part[((size_t)kGridParts * p + k) * 2], hi = gr.part[((size_t)kGridParts * p + k) * 2 + 1];
        const double mk = fmax(fabs(lo), fabs(hi));
        float f = (float)mk;
        if ((double)f < mk) f = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u);
        bd = fmaxf(bd, f);
    }
    const float bB = fmaxf(bd, lmax);
    const float cB = kConst * bB * bB;

    // ---- cells in order of the squared distance from x to their boxes
    if (C <= kNnBlock)
        grid_rank_cells<1, PF>(gr.box, gr.off, xs, C, N, keys, idxs, S.hist, pre, rbase, mindr);
    else if (C <= 2 * kNnBlock)
        grid_rank_cells<2, PF>(gr.box, gr.off, xs, C, N, keys, idxs, S.hist, pre, rbase, mindr);
    else
        grid_rank_cells<4, PF>(gr.box, gr.off, xs, C, N, keys, idxs, S.hist, pre, rbase, mindr);

    // ---- the rows, nearest cell first
    int32_t *surv = S.surv + w * (kNnItems * kWave);  // this wave's list
    int cr = 0;                                        // this wave's cursor: a cell rank,
    int cend = __builtin_amdgcn_readfirstlane(pre[1]);  // the position where that cell ends,
    int cbase = __builtin_amdgcn_readfirstlane(rbase[0]);  // and its row offset
    for (int64_t vb = 0; vb < N; vb += kNnChunk) {
        const int par = (int)((vb / kNnChunk) & 1);
        const uint64_t tk = grp.thr_k;
        const int32_t ti = grp.thr_i;
        const int cut = __builtin_amdgcn_readfirstlane(grp.cut);
        if (vb >= cut) break;
        const double td = tk == ~0ull ? INFINITY : __builtin_bit_cast(double, tk);
        float tf;
        {
            const float f = (float)td;
            tf = (double)f < td ? __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u) : f;
        }
        // screen: bit it of okm is set if the lane's row of block it passed
        uint32_t okm = 0;
        int32_t rowi[kNnItems];
        constexpr int kB = PF <= kNnBatchPmax ? 4 : 1;
#pragma unroll
        for (int it0 = 0; it0 < kNnItems; it0 += kB) {
            int nval[kB];
#pragma unroll
            for (int b = 0; b < kB; b++) {
                const int64_t vi = vb + (int64_t)(w * kNnItems + it0 + b) * kWave;  // the block's first position
                const int64_t nv = (int64_t)cut - vi;
                nval[b] = (int)(nv < 0 ? 0 : nv > kWave ? kWave : nv);  // its positions in reach (and < N)
                int row = 0;
                if (nval[b] > 0) {
                    while (vi >= cend) {  // wave-uniform: move the cursor to the block's first cell
                        cr++;
                        cend = __builtin_amdgcn_readfirstlane(pre[cr + 1]);
                        cbase = __builtin_amdgcn_readfirstlane(rbase[cr]);
                    }
                    if (lane < nval[b]) {
                        const int v = (int)vi + lane;
                        int rb = cbase;
                        if (v >= cend) {  // past the cursor's cell: this lane's own walk
                            int r = cr + 1;
                            while (v >= pre[r + 1]) r++;
                            rb = rbase[r];
                        }
                        row = v + rb;
                    }
                }
                rowi[it0 + b] = row;
            }
            float xb[kB][PF];
#pragma unroll
            for (int b = 0; b < kB; b++) {
#pragma unroll
                for (int k = 0; k < PF; k++) xb[b][k] = gr.x32[(int64_t)rowi[it0 + b] * PF + k];
            }
#pragma unroll
            for (int b = 0; b < kB; b++) {
                float d32 = 0.0f;
#pragma unroll
                for (int k = 0; k < PF; k++) {
                    const float t = xb[b][k] - xf[k];
                    d32 = fmaf(t, t, d32);
                }
                if (lane < nval[b] && d32 * kSlope - cB < tf) okm |= 1u << (it0 + b);
            }
        }
        // this wave's list of the rows that passed
        int ns = 0;
#pragma unroll
        for (int it = 0; it < kNnItems; it++) {
            const bool ok = (okm >> it) & 1u;
            const uint64_t bal = __ballot(ok);
            if (ok) surv[ns + lanes_below(bal)] = rowi[it];
            ns += __popcll(bal);
        }
        __builtin_amdgcn_wave_barrier();
        // exact keys of the list, 64 at a time; keys below the threshold are appended
        uint32_t pend = 0;
        int32_t iq[kNnItems];
#pragma unroll
        for (int qq = 0; qq < kNnItems; qq++) {
            iq[qq] = 0;
            if (qq * kWave >= ns) continue;
            const int j = qq * kWave + lane;
            bool app = false;
            uint64_t key = 0;
            if (j < ns) {
                const int row = surv[j];
                const int32_t i = gr.perm[row];  // loaded beside the row's float64 copy
                iq[qq] = i;
                const double sd = sqdist_strict(gr.x64 + (int64_t)row * PF, 1, xs, 1, p);
                key = __builtin_bit_cast(uint64_t, sd);
                app = key_less(key, i, tk, ti);
            }
            const uint64_t am = __ballot(app);
            if (am) {
                const int lead = (int)__builtin_ctzll(am);
                int base = 0;
                if (lane == lead) base = atomicAdd(&grp.count, __popcll(am));
                base = __shfl(base, lead, kWave);
                if (app) {
                    const int pos = base + lanes_below(am);
                    if (pos < CAP) {
                        keys[pos] = key;
                        idxs[pos] = iq[qq];
                    } else {
                        pend |= 1u << qq;
                        grp.full[par] = 1;
                    }
                }
            }
        }
        __syncthreads();
        // a full buffer: as in nn_pool_kernel (the decision reads the chunk's flag)
        if (grp.full[par]) {
            select_keep(keys, idxs, S, grp, CAP, Np);
            const uint64_t nk = grp.thr_k;
            const int32_t ni = grp.thr_i;
            if (tid == 0) grp.cut = grid_cut(mindr, pre, C, __builtin_bit_cast(double, nk));
#pragma unroll
            for (int qq = 0; qq < kNnItems; qq++) {
                if ((pend >> qq) & 1u) {
                    const int32_t i = iq[qq];
                    const double sd = sqdist_strict(X + (int64_t)i * PF, 1, xs, 1, p);
                    const uint64_t key = __builtin_bit_cast(uint64_t, sd);
                    if (key_less(key, i, nk, ni)) {
                        const int pos = atomicAdd(&grp.count, 1);
                        keys[pos] = key;
                        idxs[pos] = i;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (grp.count > Np) select_keep(keys, idxs, S, grp, grp.count, Np);
    constexpr int E = SORTN / kNnBlock;
    uint64_t kr[E];
    int32_t ir[E];
#pragma unroll
    for (int qq = 0; qq < E; qq++) {
        const int e = tid * E + qq;
        kr[qq] = e < Np ? keys[e] : ~0ull;
        ir[qq] = e < Np ? idxs[e] : INT32_MAX;
    }
    bitonic_sort_regs<SORTN>(kr, ir, keys, idxs);
#pragma unroll
    for (int qq = 0; qq < E; qq++) {
        const int e = tid * E + qq;
        if (e < Np) pool[m * Np + e] = ir[qq];
    }
}

// G locations per workgroup, consecutive in cell order (so mostly of one
// cell), sharing the stream: the cells are visited in order of their smallest
// box distance over the G locations, a cell is streamed while any location can
// still have a pool member in it, and each row loaded serves every location
// whose own threshold admits the row's cell.  Per location the screen, the
// exact key, the buffer and the selections are those of nn_grid_kernel, so the
// pools are the same; G locations share each row's trip from L2 / MALL.
template <int G, int CAP, int SORTN, int PF>
__global__ __launch_bounds__(kNnBlock) void nn_grid_group_kernel(const double *__restrict__ X, int64_t N,
                                                                 const double *__restrict__ XX, int64_t M, int Np,
                                                                 int32_t *__restrict__ pool, NnGrid gr)
{
    static_assert(CAP >= SORTN + kNnChunk && CAP >= kGridCmax, "room for one chunk above the kept set");
    static_assert(G * kNnItems <= 32, "pending bits of every location and item in one word");
    constexpr int p = PF;
    constexpr float kU = 5.9604645e-8f;  // 2^-24
    constexpr double kMargin = 1.0 - 1.0 / (1 << 20);
    __shared__ uint64_t keys[G][CAP];
    __shared__ int32_t idxs[G][CAP];
    __shared__ double xs[G][PF];
    __shared__ NnGroup grp[G];
    __shared__ NnShared S;
    __shared__ int32_t pre[kGridCmax + 1];   // rows in the cells of rank < r
    __shared__ int16_t cellr[kGridCmax];     // cell of rank r (smallest group distance first)
    __shared__ float mindr[G][kGridCmax];    // <= squared distance from location g to the box of that cell

    const int tid = threadIdx.x, C = gr.C;
    // the XCD of this workgroup (blockIdx.x mod 8) takes the groups
    // [x q, (x + 1) q) of G consecutive locations in cell order
    const int64_t ngroups = (M + G - 1) / G, q = (ngroups + 7) / 8;
    const int64_t gi = (int64_t)(blockIdx.x & 7) * q + (blockIdx.x >> 3);
    if (gi >= ngroups) return;  // the whole workgroup, before any barrier
    const int64_t s0 = gi * G;
    const int ng = (int)(M - s0 < G ? M - s0 : G);
    int64_t mloc[G];
#pragma unroll
    for (int g = 0; g < G; g++) mloc[g] = g < ng ? gr.lperm[s0 + g] : 0;
    for (int t = tid; t < G * PF; t += kNnBlock) {
        const int g = t / PF, k = t - g * PF;
        xs[g][k] = g < ng ? XX[mloc[g] * p + k] : 0.0;
    }
    if (tid < G) {
        grp[tid].count = 0;
        grp[tid].full[0] = grp[tid].full[1] = 0;
        grp[tid].thr_k = ~0ull;
        grp[tid].thr_i = INT32_MAX;
    }
    __syncthreads();
    constexpr float kSlope = 1.0f - 2.0f * PF * kU;
    constexpr float kConst = 40.0f * PF * kU;
    // the screen's bound B from the design's bounding box and each location
    float bd = 0.0f;
#pragma unroll
    for (int k = 0; k < PF; k++) {
        const double lo = gr.part[((size_t)kGridParts * p + k) * 2], hi = gr.part[((size_t)kGridParts * p + k) * 2 + 1];
        const double mk = fmax(fabs(lo), fabs(hi));
        float f = (float)mk;
        if ((double)f < mk) f = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u);
        bd = fmaxf(bd, f);
    }
    float xf[G][PF], cB[G];
#pragma unroll
    for (int g = 0; g < G; g++) {
        float lmax = 0.0f;
#pragma unroll
        for (int k = 0; k < PF; k++) {
            xf[g][k] = (float)xs[g][k];
            lmax = fmaxf(lmax, fabsf(xf[g][k]));
        }
        const float bB = fmaxf(bd, lmax);
        cB[g] = kConst * bB * bB;
    }

    // ---- cells in order of their smallest squared box distance over the group
    auto box_sd = [&](int c, int g) {
        double sd = 0.0;
#pragma unroll
        for (int k = 0; k < PF; k++) {
            const double lo = gr.box[((size_t)c * p + k) * 2], hi = gr.box[((size_t)c * p + k) * 2 + 1];
            const double gap = fmax(fmax(lo - xs[g][k], xs[g][k] - hi), 0.0);
            sd = fma(gap, gap, sd);
        }
        return sd;
    };
    for (int c = tid; c < C; c += kNnBlock) {
        double sdm = INFINITY;
        bool nan = false;
#pragma unroll
        for (int g = 0; g < G; g++) {
            if (g >= ng) break;
            const double sd = box_sd(c, g);
            nan |= !(sd >= 0.0);
            sdm = fmin(sdm, sd);
        }
        keys[0][c] = __builtin_bit_cast(uint64_t, nan ? NAN : sdm);  // a NaN location's cells go last
        idxs[0][c] = c;
    }
    __syncthreads();
    bitonic_sort_n(keys[0], idxs[0], C);
    int32_t csum[4], tot = 0;
#pragma unroll
    for (int qq = 0; qq < 4; qq++) {
        const int r = 4 * tid + qq;
        csum[qq] = 0;
        if (r < C) {
            const int c = idxs[0][r];
            cellr[r] = (int16_t)c;
#pragma unroll
            for (int g = 0; g < G; g++) {
                const double md = g < ng ? box_sd(c, g) : INFINITY;
                float f = (float)md;  // rounded down to a float below md
                if (!(md >= 0.0)) f = INFINITY;
                else if ((double)f > md) f = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) - 1u);
                mindr[g][r] = f;
            }
            csum[qq] = gr.off[c + 1] - gr.off[c];
        }
        tot += csum[qq];
    }
    S.hist[tid] = (uint32_t)tot;
    __syncthreads();
    for (int o = 1; o < kNnBlock; o <<= 1) {
        const uint32_t add = tid >= o ? S.hist[tid - o] : 0u;
        __syncthreads();
        S.hist[tid] += add;
        __syncthreads();
    }
    int32_t run = (int32_t)S.hist[tid] - tot;
#pragma unroll
    for (int qq = 0; qq < 4; qq++) {
        const int r = 4 * tid + qq;
        if (r < C) pre[r] = run;
        run += csum[qq];
    }
    if (tid == 0) pre[C] = (int32_t)N;
    __syncthreads();

    // ---- the rows, cell by cell
    int rc = 0;  // rank of the cell that holds row vb
    for (int64_t vb = 0; vb < N; vb += kNnChunk) {
        const int par = (int)((vb / kNnChunk) & 1);
        uint64_t tk[G];
        int32_t ti[G];
        double td[G];
        float tf[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            tk[g] = grp[g].thr_k;
            ti[g] = grp[g].thr_i;
            td[g] = (tk[g] == ~0ull || g >= ng) ? INFINITY : __builtin_bit_cast(double, tk[g]);
            const float f = (float)td[g];
            tf[g] = (double)f < td[g] ? __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u) : f;
        }
        // every remaining cell is at least as far from each location as its
        // distance to the cell holding row vb (the order is by the group's
        // smallest distance, so this holds for the group minimum only): stop
        // when no location can use that cell or, as the group minimum only
        // grows, any later one
        rc = rank_from(pre, rc, vb);
        {
            float gmin = INFINITY;
            double tmax = 0.0;
#pragma unroll
            for (int g = 0; g < G; g++) {
                if (g >= ng) break;
                gmin = fminf(gmin, mindr[g][rc]);
                tmax = fmax(tmax, td[g]);
            }
            if ((double)gmin * kMargin > tmax) break;
        }
        int r = rc;
        uint32_t pend = 0;
        constexpr int kB = PF <= kNnBatchPmax ? 4 : 1;
#pragma unroll
        for (int it0 = 0; it0 < kNnItems; it0 += kB) {
            uint32_t usem[kB];  // bit g: location g reads this item's row
            int64_t rowb[kB];
#pragma unroll
            for (int b = 0; b < kB; b++) {
                const int64_t v = vb + (it0 + b) * kNnBlock + tid;
                const int64_t vc = v < N ? v : N - 1;
                r = rank_from(pre, r, vc);
                usem[b] = 0;
#pragma unroll
                for (int g = 0; g < G; g++)
                    if (g < ng && v < N && (double)mindr[g][r] * kMargin <= td[g]) usem[b] |= 1u << g;
                rowb[b] = gr.off[cellr[r]] + (vc - pre[r]);
            }
            float xb[kB][PF];
#pragma unroll
            for (int b = 0; b < kB; b++) {
                const int64_t row = usem[b] ? rowb[b] : 0;
#pragma unroll
                for (int k = 0; k < PF; k++) xb[b][k] = gr.x32[row * PF + k];
            }
#pragma unroll
            for (int b = 0; b < kB; b++) {
                if (!usem[b]) continue;
                const int it = it0 + b;
                const int64_t row = rowb[b];
                int32_t i = -1;
#pragma unroll
                for (int g = 0; g < G; g++) {
                    if (!((usem[b] >> g) & 1u)) continue;
                    float d32 = 0.0f;
#pragma unroll
                    for (int k = 0; k < PF; k++) {
                        const float t = xb[b][k] - xf[g][k];
                        d32 = fmaf(t, t, d32);
                    }
                    if (d32 * kSlope - cB[g] < tf[g]) {
                        if (i < 0) i = gr.perm[row];
                        const double sd = sqdist_strict(X + (int64_t)i * PF, 1, xs[g], 1, p);
                        const uint64_t key = __builtin_bit_cast(uint64_t, sd);
                        if (key_less(key, i, tk[g], ti[g])) {
                            const int pos = atomicAdd(&grp[g].count, 1);
                            if (pos < CAP) {
                                keys[g][pos] = key;
                                idxs[g][pos] = i;
                            } else {
                                pend |= 1u << (g * kNnItems + it);
                                grp[g].full[par] = 1;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        // a full buffer: as in nn_pool_kernel, location by location
#pragma unroll 1
        for (int g = 0; g < G; g++) {
            if (grp[g].full[par]) {
                select_keep(keys[g], idxs[g], S, grp[g], CAP, Np);
                const uint64_t nk = grp[g].thr_k;
                const int32_t ni = grp[g].thr_i;
#pragma unroll
                for (int it = 0; it < kNnItems; it++) {
                    if ((pend >> (g * kNnItems + it)) & 1u) {
                        const int64_t v = vb + it * kNnBlock + tid;
                        const int rr = rank_from(pre, rc, v);
                        const int32_t i = gr.perm[gr.off[cellr[rr]] + (v - pre[rr])];
                        const double sd = sqdist_strict(X + (int64_t)i * PF, 1, xs[g], 1, p);
                        const uint64_t key = __builtin_bit_cast(uint64_t, sd);
                        if (key_less(key, i, nk, ni)) {
                            const int pos = atomicAdd(&grp[g].count, 1);
                            keys[g][pos] = key;
                            idxs[g][pos] = i;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
#pragma unroll 1
    for (int g = 0; g < ng; g++) {
        if (grp[g].count > Np) select_keep(keys[g], idxs[g], S, grp[g], grp[g].count, Np);
        constexpr int E = SORTN / kNnBlock;
        uint64_t kr[E];
        int32_t ir[E];
#pragma unroll
        for (int qq = 0; qq < E; qq++) {
            const int e = tid * E + qq;
            kr[qq] = e < Np ? keys[g][e] : ~0ull;
            ir[qq] = e < Np ? idxs[g][e] : INT32_MAX;
        }
        bitonic_sort_regs<SORTN>(kr, ir, keys[g], idxs[g]);
#pragma unroll
        for (int qq = 0; qq < E; qq++) {
            const int e = tid * E + qq;
            if (e < Np) pool[mloc[g] * Np + e] = ir[qq];
        }
        __syncthreads();
    }
}

// Grouped grid pools for p <= kGridGroupPmax (G = 2 at every pool size, G = 4
// where four buffers of CAP keys fit in LDS).
constexpr int kGridGroupPmax = 8;

template <int G, int CAP, int SORTN>
static hipError_t launch_grid_group(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                                    int32_t *pool, const NnGrid &g, hipStream_t st)
{
    const int64_t groups = (M + G - 1) / G;
    const dim3 grid((unsigned)(8 * ((groups + 7) / 8)));
    switch (p) {
#define LAGP_NGG_CASE(P)                                                                                      \
    case P:                                                                                                   \
        hipLaunchKernelGGL((nn_grid_group_kernel<G, CAP, SORTN, P>), grid, dim3(kNnBlock), 0, st, X, N, XX, M, \
                           Np, pool, g);                                                                      \
        break;
        LAGP_NGG_CASE(1)
        LAGP_NGG_CASE(2)
        LAGP_NGG_CASE(3)
        LAGP_NGG_CASE(4)
        LAGP_NGG_CASE(5)
        LAGP_NGG_CASE(6)
        LAGP_NGG_CASE(7)
        LAGP_NGG_CASE(8)
#undef LAGP_NGG_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int CAP, int SORTN>
static hipError_t launch_grid_cap(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                                  int32_t *pool, const NnGrid &g, hipStream_t st, int group)
{
    if (group == 2 && p <= kGridGroupPmax) return launch_grid_group<2, CAP, SORTN>(X, N, p, XX, M, Np, pool, g, st);
    if constexpr (CAP <= 2048) {
        if (group == 4 && p <= kGridGroupPmax)
            return launch_grid_group<4, CAP, SORTN>(X, N, p, XX, M, Np, pool, g, st);
    }
    switch (p) {
#define LAGP_NG_CASE(P)                                                                                       \
    case P:                                                                                                   \
        hipLaunchKernelGGL((nn_grid_kernel<CAP, SORTN, P>), dim3((unsigned)(8 * ((M + 7) / 8))), dim3(kNnBlock), 0, \
                           st, X, N, XX, M, Np, pool, g);                                                     \
        break;
        LAGP_NG_CASE(1)
        LAGP_NG_CASE(2)
        LAGP_NG_CASE(3)
        LAGP_NG_CASE(4)
        LAGP_NG_CASE(5)
        LAGP_NG_CASE(6)
        LAGP_NG_CASE(7)
        LAGP_NG_CASE(8)
        LAGP_NG_CASE(9)
        LAGP_NG_CASE(10)
        LAGP_NG_CASE(11)
        LAGP_NG_CASE(12)
        LAGP_NG_CASE(13)
        LAGP_NG_CASE(14)
        LAGP_NG_CASE(15)
        LAGP_NG_CASE(16)
#undef LAGP_NG_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int nn_grid_groups(int p, int Np)
{
    if (p > kGridGroupPmax) return 1;
    return Np <= 1024 ? 3 : 2;  // G = 1, 2, 4 (four buffers of 3072 keys would not fit in LDS)
}

hipError_t launch_nn_grid(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np, int32_t *pool,
                          void *ws, hipStream_t st, int group)
{
    if (M == 0) return hipSuccess;
    if (p < 1 || p > kMaxP || !ws) return hipErrorInvalidValue;
    const NnGrid g = grid_layout(ws, N, p, M);
    const int64_t nb = (N + 255) / 256, mb = (M + 255) / 256;
    const unsigned rows_grid = (unsigned)(nb < 4096 ? nb : 4096), locs_grid = (unsigned)(mb < 4096 ? mb : 4096);
    const unsigned parts = (unsigned)(nb < kGridParts ? nb : kGridParts);
    hipLaunchKernelGGL(grid_minmax, dim3(parts), dim3(256), 0, st, X, N, p, g);
    hipLaunchKernelGGL(grid_final, dim3(1), dim3(256), 0, st, p, (int)parts, g);
    hipLaunchKernelGGL(grid_count, dim3(rows_grid), dim3(256), 0, st, X, N, p, g, g.cid, g.cnt);
    hipLaunchKernelGGL(grid_count, dim3(locs_grid), dim3(256), 0, st, XX, M, p, g, g.lcid, g.lcnt);
    hipLaunchKernelGGL(grid_scan, dim3(1), dim3(256), 0, st, N, g.C, g.cnt, g.off, g.cur);
    hipLaunchKernelGGL(grid_scan, dim3(1), dim3(256), 0, st, M, g.C, g.lcnt, g.loff, g.lcur);
    hipLaunchKernelGGL(grid_scatter, dim3(rows_grid), dim3(256), 0, st, X, N, p, g);
    hipLaunchKernelGGL(grid_order, dim3(locs_grid), dim3(256), 0, st, M, g);
    hipLaunchKernelGGL(grid_box, dim3((unsigned)g.C), dim3(256), 0, st, X, p, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (group != 1 && group != 2 && group != 4) return hipErrorInvalidValue;
    if (Np <= 512) return launch_grid_cap<2048, 512>(X, N, p, XX, M, Np, pool, g, st, group);
    if (Np <= 1024) return launch_grid_cap<2048, 1024>(X, N, p, XX, M, Np, pool, g, st, group);
    if (Np <= kNnMaxNp) return launch_grid_cap<3072, 2048>(X, N, p, XX, M, Np, pool, g, st, group);
    return hipErrorInvalidValue;
}

// Scratch of lagp_nn_pool_static: the bucketed design and the cell tables of
// launch_nn_grid.  Each GPU holds its own copy until the process ends; host
// code reaches it only through the address nn_static_scratch resolves.
static __device__ __align__(256) unsigned char scratch[kNnStaticScratch];

hipError_t nn_static_scratch(void **ptr)
{
    static std::mutex mu;
    static void *addr[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!a) return hipErrorInvalidSymbol;
        addr[dev] = a;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

int nn_pool_cap(int Np)
{
    if (Np <= 512) return 2048;
    if (Np <= 1024) return 2048;
    if (Np <= kNnMaxNp) return 3072;
    return 0;
}

template <int CAP, int SORTN>
static hipError_t launch_g(int G, const double *X, const float *X32, int64_t N, int p, const double *XX,
                           int64_t M, int Np, int32_t *pool, hipStream_t st)
{
    if (G == 1) return launch_cap<1, CAP, SORTN>(X, X32, N, p, XX, M, Np, pool, st);
    if constexpr (CAP <= 2048) {  // four buffers of 3072 keys would not fit in LDS
        if (G == 4) return launch_cap<4, CAP, SORTN>(X, X32, N, p, XX, M, Np, pool, st);
    }
    return launch_cap<2, CAP, SORTN>(X, X32, N, p, XX, M, Np, pool, st);
}

__global__ void nn_to_f32(const double *__restrict__ X, float *__restrict__ X32, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        X32[i] = (float)X[i];
}

int nn_pool_groupings(int Np)
{
    return Np <= 1024 ? 3 : 2;
}

hipError_t launch_nn_pool(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                          int32_t *pool, hipStream_t st, int grouping, float *x32)
{
    if (M == 0) return hipSuccess;
    if (p < 1 || p > kMaxP) return hipErrorInvalidValue;
    if (x32) {
        const int64_t count = N * p;
        const unsigned grid = (unsigned)((count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096);
        hipLaunchKernelGGL(nn_to_f32, dim3(grid), dim3(256), 0, st, X, x32, count);
    }
    const float *X32 = x32;
    // locations per workgroup: 1, 2 or 4.  One is the default: measured on
    // MI355X, sharing the pass over X costs more in serialised selections and
    // residency than it saves in L2 traffic (plans time all of them).
    const int G = grouping < 0 ? 1 : 1 << (grouping < nn_pool_groupings(Np) ? grouping : 0);
    if (Np <= 512) return launch_g<2048, 512>(G, X, X32, N, p, XX, M, Np, pool, st);
    if (Np <= 1024) return launch_g<2048, 1024>(G, X, X32, N, p, XX, M, Np, pool, st);
    if (Np <= kNnMaxNp) return launch_g<3072, 2048>(G > 2 ? 2 : G, X, X32, N, p, XX, M, Np, pool, st);
    return hipErrorInvalidValue;
}

}  // namespace lagp
