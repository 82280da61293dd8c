// Batched ALC scores of many candidates against one design, given K_j^{-1}:
// the computation of the paper's per-step GPU kernel (Fig. 3, with the sign
// of eq. piedef), as one launch over all candidates.
//
// For a candidate c with kernel vector q_c = K(X_j, c), c_x = K(c, x),
// h = K(X_j, x) and w = K_j^{-1} h:
//     s_c     = kappa - q_c^T K_j^{-1} q_c   (the Schur complement m^{-1}, eq. piedef)
//     cov_c   = c_x - q_c^T w
//     delta_c = cov_c^2 / s_c               (v_j(x) - v_{j+1}(x), eq. dxy)
// The quadratic forms of a tile of candidates are one dense product
// U = K_j^{-1} Q^T on the matrix cores followed by column sums of U o Q^T.
//
// MFMA mapping (16x16x4, float64 or float32).  A = a 16 x 4 block of
// K_j^{-1} (rows a, columns b), B = a 4 x 16 block of Q^T (rows b, one column
// per candidate).  Lane l owns candidate l % 16 and k-slot o = l / 16; the
// summation index b that slot o takes at k-step kk is perm(kk, o), chosen so
// that the rows of U a lane holds in its accumulator are exactly the b of its
// own B entries.  Each lane therefore finishes its part of q_c^T U_c with the
// kernel values it has already computed, and the four slots of a candidate
// are summed with two lane exchanges.  K_j^{-1} sits in LDS in A-fragment
// order (lane l of a fragment reads entry l: no bank conflicts).  K_j^{-1}
// is symmetric, and it is read by columns wherever that makes neighbouring
// lanes read neighbouring addresses.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>
#include <mutex>

namespace lagp {

namespace {

// Threads per workgroup: 256 (four waves), or 512 where the LDS of K_j^{-1}
// holds one workgroup per CU (float64, J >= 112), so that two waves per SIMD
// share it.  Each wave scores 16 candidates per tile.
template <typename T, int J>
constexpr int sc_block()
{
    return sizeof(T) == 8 && J >= 112 ? 512 : 256;
}

template <typename T>
struct ScMma;
template <>
struct ScMma<double> {
    typedef v4d acc;
    // row of the 16 x 16 result in accumulator element r of k-slot o's lanes
    static __device__ __forceinline__ int row(int o, int r) { return o + 4 * r; }
    static __device__ __forceinline__ acc run(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct ScMma<float> {
    typedef v4f acc;
    static __device__ __forceinline__ int row(int o, int r) { return 4 * o + r; }
    static __device__ __forceinline__ acc run(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Summation index of k-slot o at k-step kk: k-steps 4 rt .. 4 rt + 3 cover the
// 16 indices of row tile rt in the order the accumulator rows come.
template <typename T>
__host__ __device__ constexpr int perm(int kk, int o)
{
    return 16 * (kk >> 2) + (sizeof(T) == 8 ? o + 4 * (kk & 3) : 4 * o + (kk & 3));
}

struct ScArgs {
    const double *Xj;    // [j x p]
    int j, p;
    const double *Kinv;  // [j x j]
    const double *Xc;    // [Nc x p]
    int64_t Nc;
    const double *x;     // [p]
    const double *h;     // [j]
    double d, g;
    double *delta;       // [Nc]
};

// Squared distance of two points, summed over the coordinates in T.
template <typename T>
__device__ __forceinline__ T sqdist_t(const double *a, const double *b, int p)
{
    T s = 0;
#pragma unroll
    for (int k = 0; k < kMaxP; k++)
        if (k < p) {
            const T t = (T)a[k] - (T)b[k];
            s = fma(t, t, s);
        }
    return s;
}

template <typename T>
__device__ __forceinline__ T corr_t(T r2, T nid);
template <>
__device__ __forceinline__ double corr_t<double>(double r2, double nid)
{
    return exp(r2 * nid);
}
template <>
__device__ __forceinline__ float corr_t<float>(float r2, float nid)
{
    return expf(r2 * nid);
}

// Dynamic LDS: design rows [J][p] and the location (float64), then w [J] and
// K^{-1} fragments [J/16][J/4][64] in T.
template <typename T>
__host__ __device__ constexpr size_t sc_lds(int J, int p)
{
    return 8 * ((size_t)J * p + kMaxP) + sizeof(T) * ((size_t)J + (size_t)J * J);
}

template <typename T, int J>
__global__ __launch_bounds__((sc_block<T, J>())) void alc_scores_kernel(ScArgs a)
{
    constexpr int TB = sc_block<T, J>(), TILE = TB / 4;  // 16 candidates per wave
    constexpr int KK = J / 4, RT = J / 16;
    typedef typename ScMma<T>::acc acc_t;
    extern __shared__ double sc_dyn[];
    const int j = a.j, p = a.p;
    double *xj = sc_dyn;
    double *xs = xj + J * p;
    T *w = (T *)(xs + kMaxP);
    T *frag = w + J;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int t = tid; t < J * p; t += TB) xj[t] = t < j * p ? a.Xj[t] : 0.0;
    if (tid < p) xs[tid] = a.x[tid];
    // the loads below are unrolled so that many are in flight; indices outside
    // the j x j input are clamped to entry 0 and their values discarded
    if (tid < J) {  // w = K^{-1} h, row t read as column t (J <= block)
        const int t = tid;
        double s = 0.0;
#pragma unroll 8
        for (int b = 0; b < J; b++) {
            const bool in = t < j && b < j;
            const double kv = a.Kinv[in ? (int64_t)b * j + t : 0], hv = a.h[in ? b : 0];
            s = in ? fma(kv, hv, s) : s;
        }
        w[t] = (T)s;
    }
    static_assert(J <= TB, "one row of w per thread");
#pragma unroll 8
    for (int i = 0; i < (J * J + TB - 1) / TB; i++) {
        const int t = tid + i * TB;
        if (t >= J * J) break;  // the last round only: J * J is a multiple of 64
        const int l = t & 63, blk = t >> 6;  // blk = rt * KK + kk
        const int rt = blk / KK, kk = blk - rt * KK;
        const int row = 16 * rt + (l & 15), col = perm<T>(kk, l >> 4);
        const bool in = row < j && col < j;
        const double kv = a.Kinv[in ? (int64_t)col * j + row : 0];
        frag[t] = in ? (T)kv : (T)0;
    }
    __syncthreads();

    const T kappa = (T)(1.0 + a.g), nid = (T)(-1.0 / a.d);
    const int c16 = lane & 15, o = lane >> 4;
    const int64_t ntiles = (a.Nc + TILE - 1) / TILE;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t cand = tile * TILE + wv * 16 + c16;
        const bool valid = cand < a.Nc;
        double xc[kMaxP];
#pragma unroll
        for (int k = 0; k < kMaxP; k++) xc[k] = valid && k < p ? a.Xc[cand * p + k] : 0.0;
        const T cx = corr_t<T>(sqdist_t<T>(xc, xs, p), nid);
        // the kernel values this lane feeds to the matrix cores, and its part of q_c . w
        // (computed for every slot and selected afterwards: no branches, so the
        // independent exp chains interleave; padding rows of xj are zeros)
        T qv[KK];
        T cp = 0;
#pragma unroll
        for (int kk = 0; kk < KK; kk++) {
            const int b = perm<T>(kk, o);
            const T kv = corr_t<T>(sqdist_t<T>(xc, xj + b * p, p), nid);
            qv[kk] = valid && b < j ? kv : (T)0;
        }
#pragma unroll
        for (int kk = 0; kk < KK; kk++) cp = fma(qv[kk], w[perm<T>(kk, o)], cp);
        // row tiles of U in groups of RI, so that RI independent accumulations
        // keep the matrix core busy
        constexpr int RI = RT < 4 ? RT : 4;
        T qp = 0;
#pragma unroll
        for (int rt0 = 0; rt0 < RT; rt0 += RI) {
            acc_t acc[RI];
#pragma unroll
            for (int i = 0; i < RI; i++) acc[i] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < KK; kk++)
#pragma unroll
                for (int i = 0; i < RI; i++)
                    if (rt0 + i < RT)
                        acc[i] = ScMma<T>::run(frag[((rt0 + i) * KK + kk) * 64 + lane], qv[kk], acc[i]);
            // accumulator element r of tile rt: row perm(4 rt + r, o) of U for this candidate
#pragma unroll
            for (int i = 0; i < RI; i++)
                if (rt0 + i < RT)
#pragma unroll
                    for (int r = 0; r < 4; r++) qp = fma(acc[i][r], qv[4 * (rt0 + i) + r], qp);
        }
        const T q = row_sum4(qp), cv = row_sum4(cp);
        const T s = kappa - q, cov = cx - cv;
        if (o == 0 && valid) a.delta[cand] = s > (T)0 ? (double)(cov * cov / s) : -INFINITY;
    }
}

// Designs beyond kScoresJmax, whose K_j^{-1} (up to 2 MB in float64) cannot
// be staged in LDS: it is read straight from the caller's array (from L2 after
// the first tiles: every workgroup walks it in the same order).  A workgroup
// scores 16 candidates at a time.  Their kernel values Q (J x 16) sit in LDS;
// wave w forms the row blocks I = w, w + 4, ... of U = K_j^{-1} Q^T on the
// matrix cores (A: a 16 x 4 block of K_j^{-1} from global memory, B: a 4 x 16
// block of Q^T from LDS) and folds each block into the two sums every score
// needs, q_c^T U_c = q_c^T K_j^{-1} q_c and h^T U_c = h^T K_j^{-1} q_c (so no
// w = K_j^{-1} h is formed); the four waves' partial sums meet in LDS.
template <typename T>
__host__ __device__ constexpr size_t sb_lds(int J, int p)
{
    return 8 * ((size_t)J * p + kMaxP) + sizeof(T) * ((size_t)J + (size_t)J * 16 + 16 + 2 * 4 * 16);
}

constexpr int kSbBlock = 256;

template <typename T>
__global__ __launch_bounds__(kSbBlock) void alc_scores_big_kernel(ScArgs a)
{
    constexpr int TB = kSbBlock, NW = TB / kWave;
    typedef typename ScMma<T>::acc acc_t;
    extern __shared__ double sb_dyn[];
    const int j = a.j, p = a.p, J = (j + 15) & ~15, KK = J / 4, RT = J / 16;
    double *xj = sb_dyn;           // [J][p], zeros past j
    double *xs = xj + J * p;       // [kMaxP]
    T *hs = (T *)(xs + kMaxP);     // [J] h, zeros past j
    T *Q = hs + J;                 // [J][16] kernel values of the tile's candidates
    T *cxs = Q + J * 16;           // [16] K(c, x)
    T *part = cxs + 16;            // [2][NW][16] the waves' partial sums

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int t = tid; t < J * p; t += TB) xj[t] = t < j * p ? a.Xj[t] : 0.0;
    if (tid < p) xs[tid] = a.x[tid];
    for (int t = tid; t < J; t += TB) hs[t] = t < j ? (T)a.h[t] : (T)0;
    __syncthreads();

    const T kappa = (T)(1.0 + a.g), nid = (T)(-1.0 / a.d);
    const int c16 = tid & 15;
    const int64_t ntiles = (a.Nc + 15) / 16;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // kernel values: thread t takes candidate t % 16 and rows t / 16 + 16 i
        const int64_t cand = tile * 16 + c16;
        const bool valid = cand < a.Nc;
        double xc[kMaxP];
#pragma unroll
        for (int k = 0; k < kMaxP; k++) xc[k] = valid && k < p ? a.Xc[cand * p + k] : 0.0;
        for (int b = tid >> 4; b < J; b += TB / 16) {
            const T kv = corr_t<T>(sqdist_t<T>(xc, xj + b * p, p), nid);
            Q[b * 16 + c16] = valid && b < j ? kv : (T)0;
        }
        if (tid < 16) cxs[tid] = corr_t<T>(sqdist_t<T>(xc, xs, p), nid);
        __syncthreads();

        // row blocks of U, two at a time so that two accumulations are in flight
        T qp = 0, hp = 0;
        const int ko = lane >> 4, ci = lane & 15;
        for (int I0 = wv; I0 < RT; I0 += 2 * NW) {
            const int I1 = I0 + NW;
            const bool two = I1 < RT;
            acc_t acc0 = acc_t{0, 0, 0, 0}, acc1 = acc_t{0, 0, 0, 0};
            const int r0 = 16 * I0 + ci, r1 = 16 * I1 + ci;
#pragma unroll 8
            for (int kk = 0; kk < KK; kk++) {
                const int col = 4 * kk + ko;  // K_j^{-1} is symmetric: read column `row` as row `col`
                const bool in0 = r0 < j && col < j, in1 = two && r1 < j && col < j;
                const double k0 = a.Kinv[in0 ? (int64_t)col * j + r0 : 0];
                const double k1 = a.Kinv[in1 ? (int64_t)col * j + r1 : 0];
                const T bq = Q[col * 16 + ci];
                acc0 = ScMma<T>::run(in0 ? (T)k0 : (T)0, bq, acc0);
                acc1 = ScMma<T>::run(in1 ? (T)k1 : (T)0, bq, acc1);
            }
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int row0 = 16 * I0 + ScMma<T>::row(ko, r);
                qp = fma(acc0[r], Q[row0 * 16 + ci], qp);
                hp = fma(acc0[r], hs[row0], hp);
                if (two) {
                    const int row1 = 16 * I1 + ScMma<T>::row(ko, r);
                    qp = fma(acc1[r], Q[row1 * 16 + ci], qp);
                    hp = fma(acc1[r], hs[row1], hp);
                }
            }
        }
        qp = row_sum4(qp);
        hp = row_sum4(hp);
        if (lane < 16) {
            part[wv * 16 + lane] = qp;
            part[(NW + wv) * 16 + lane] = hp;
        }
        __syncthreads();
        if (tid < 16) {
            T q = 0, hw = 0;
#pragma unroll
            for (int v = 0; v < NW; v++) {
                q += part[v * 16 + tid];
                hw += part[(NW + v) * 16 + tid];
            }
            const T s = kappa - q, cov = cxs[tid] - hw;
            if (valid) a.delta[cand] = s > (T)0 ? (double)(cov * cov / s) : -INFINITY;
        }
        __syncthreads();  // Q and part are rewritten by the next tile
    }
}

template <typename T, int J>
const void *kernel_of()
{
    return (const void *)&alc_scores_kernel<T, J>;
}

// The kernel instance for a design of j points (J = j rounded up to 16).
template <typename T>
const void *scores_kernel(int J)
{
    switch (J) {
    case 16: return kernel_of<T, 16>();
    case 32: return kernel_of<T, 32>();
    case 48: return kernel_of<T, 48>();
    case 64: return kernel_of<T, 64>();
    case 80: return kernel_of<T, 80>();
    case 96: return kernel_of<T, 96>();
    case 112: return kernel_of<T, 112>();
    default: return kernel_of<T, 128>();
    }
}

// Once per device: every instance may use LDS beyond the 64 KB default.
hipError_t scores_setup()
{
    static std::mutex mu;
    static bool ready[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (ready[dev]) return hipSuccess;
    const int big = (int)sb_lds<double>(kScoresJbig, kMaxP);
    if ((e = hipFuncSetAttribute((const void *)&alc_scores_big_kernel<double>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)&alc_scores_big_kernel<float>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
        return e;
    for (int J = 16; J <= kScoresJmax; J += 16) {
        const int lim = (int)sc_lds<double>(J, kMaxP);
        if ((e = hipFuncSetAttribute(scores_kernel<double>(J), hipFuncAttributeMaxDynamicSharedMemorySize, lim)) !=
            hipSuccess)
            return e;
        if ((e = hipFuncSetAttribute(scores_kernel<float>(J), hipFuncAttributeMaxDynamicSharedMemorySize, lim)) !=
            hipSuccess)
            return e;
    }
    ready[dev] = true;
    return hipSuccess;
}

template <typename T, int J>
hipError_t launch_j(const ScArgs &a, hipStream_t st)
{
    constexpr int TB = sc_block<T, J>();
    const size_t lds = sc_lds<T>(J, a.p);
    int nb = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel_of<T, J>(), TB, lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t ntiles = (a.Nc + TB / 4 - 1) / (TB / 4);
    const int64_t resident = (int64_t)cus * (nb > 0 ? nb : 1);
    const dim3 grid((unsigned)(ntiles < resident ? ntiles : resident));
    hipLaunchKernelGGL((alc_scores_kernel<T, J>), grid, dim3(TB), lds, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_big(const ScArgs &a, hipStream_t st)
{
    const int J = (a.j + 15) & ~15;
    const size_t lds = sb_lds<T>(J, a.p);
    const void *k = (const void *)&alc_scores_big_kernel<T>;
    int nb = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kSbBlock, lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t ntiles = (a.Nc + 15) / 16;
    const int64_t resident = (int64_t)cus * (nb > 0 ? nb : 1);
    const dim3 grid((unsigned)(ntiles < resident ? ntiles : resident));
    hipLaunchKernelGGL((alc_scores_big_kernel<T>), grid, dim3(kSbBlock), lds, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const ScArgs &a, hipStream_t st)
{
    const int J = (a.j + 15) & ~15;
    if (J > kScoresJmax) return launch_big<T>(a, st);
    switch (J) {
#define LAGP_SC_CASE(JJ)              \
    case JJ:                          \
        return launch_j<T, JJ>(a, st);
        LAGP_SC_CASE(16)
        LAGP_SC_CASE(32)
        LAGP_SC_CASE(48)
        LAGP_SC_CASE(64)
        LAGP_SC_CASE(80)
        LAGP_SC_CASE(96)
        LAGP_SC_CASE(112)
        LAGP_SC_CASE(128)
#undef LAGP_SC_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_alc_scores(const double *Xj, int j, int p, const double *Kinv, const double *Xc, int64_t Nc,
                             const double *x, const double *h, double d, double g, bool mixed, double *delta,
                             hipStream_t st)
{
    if (Nc == 0) return hipSuccess;
    if (j < 1 || j > kScoresJbig || p < 1 || p > kMaxP) return hipErrorInvalidValue;
    hipError_t e = scores_setup();
    if (e != hipSuccess) return e;
    const ScArgs a{Xj, j, p, Kinv, Xc, Nc, x, h, d, g, delta};
    return mixed ? launch_t<float>(a, st) : launch_t<double>(a, st);
}

}  // namespace lagp
