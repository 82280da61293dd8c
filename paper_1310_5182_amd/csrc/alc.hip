// Greedy ALC local designs on gfx950 (Fig. 1 steps 2a, 2b and 5).
//
// One workgroup per predictive location x.  With R_j = L_j^{-1} the inverse
// of the lower Cholesky factor of K_j (so K_j^{-1} = R_j^T R_j), the score of
// candidate c (eq. dxy) is
//     Delta_c = (K(c,x) - z_c . z_h)^2 / (kappa - z_c . z_c),
//     z_c = R_j K(X_j, c),  z_h = R_j K(X_j, x),
// i.e. conditional covariance squared over conditional variance.  Adding the
// chosen point x* with l = R_j K(X_j, x*) and s* = kappa - l.l (the Schur
// complement m^{-1} of eq. piedef) borders the factor:
//     R_{j+1} = [[R_j, 0], [-l^T R_j / sqrt(s*), 1 / sqrt(s*)]],
// whose new last row is sqrt(s*) times the last row [g^T, m] of the
// partitioned inverse K_{j+1}^{-1} of eq. piedef.
//
// Work split.  Each wave owns CBW blocks of 16 candidates.  The candidate
// kernel matrix Q = K(candidates, X_j) stays in registers for the whole
// design, laid out as the B operand of the 16x16x4 MFMA (lane l of block cb
// holds Q[16 cb + l % 16][4 kg + l / 16] in register kg); every step appends
// one column.  R_j sits in LDS in A-operand fragment order, so Z^T = R_j Q^T
// is a chain of MFMAs over the non-zero (lower-triangular) tiles of R_j, and
// the epilogue folds z.z and z.z_h straight out of the accumulators.
//
// One greedy step: (1) every wave scores its candidates on the matrix cores
// and reduces its argmax; (2) each wave re-scores in float64 its own members
// of the near-best band (mixed) or the winner (float64), keeping its best z
// vector in LDS; (3) all waves border R_j with the winning z and append z_h,
// R Y and the new Q column.  Three workgroup barriers per step.
//
// Precision.  LAGP_FP64 runs the MFMA in float64.  LAGP_MIXED keeps Q and a
// float32 copy of R_j for float32 MFMA scoring; the float64 master R_j, the
// re-score of every candidate within kBandTau of the float32 best, the Schur
// complement of the chosen point, the update and the prediction stay in
// float64.  A step whose float32 scores look untrustworthy (band overflow,
// re-score disagreement above kTrustErr, a tiny float32 conditional variance,
// or a candidate outside the band that could still beat the best, see below)
// is re-scored entirely in float64 and counted in guard[m].
//
// Float32 scores lose most where s = kappa - z.z is small (cancellation), so
// the band members' re-scores also measure the absolute float32 errors of s
// and of cov = K(c,x) - z.z_h; with delta = 8 times the larger of the two
// (plus 2^-22 kappa), a candidate outside the band whose score could reach
// the float64 best, (|cov| + delta)^2 / (s - delta) >= best (or s <= delta),
// sends the step to float64.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>

namespace lagp {

template <typename T>
struct Mma;
// Accumulator element r of lane l holds row row(l, r), column l % 16, of the
// 16x16 result; the float32 and float64 16x16x4 instructions differ here.
template <>
struct Mma<float> {
    typedef v4f acc;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ __forceinline__ acc run(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mma<double> {
    typedef v4d acc;
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
    static __device__ __forceinline__ acc run(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

constexpr int kWaveBandCap = 6;        // band members a step may re-score before falling back
constexpr float kBandTau = 1.0f / 64;  // float32 scores within this of the best are re-scored
constexpr double kTrustErr = 1.0 / 256;
constexpr float kSmallS = 1.0f / 131072;
constexpr int kPmax = 8;

// Element (i, l) of an R-sized matrix stored in 16x4 A-fragment tiles.
template <int KG>
__device__ __forceinline__ int ridx(int i, int l)
{
    return ((i >> 4) * KG + (l >> 2)) * 64 + (i & 15) + 16 * (l & 3);
}

// Float64 z = R_j K(X_j, c) for candidate `slot` by one wave (lane i owns
// z_i).  The j-loop is unrolled by eight so the LDS loads overlap.
template <int SLOTS, int KG>
__device__ __forceinline__ double wave_z64(const double *cx, const int32_t *selslot, const double *RM,
                                           int slot, int j, int p, double d, int lane)
{
    double kl = 0.0;
    if (lane < j) kl = corr64(sqdist_strict(cx + selslot[lane], SLOTS, cx + slot, SLOTS, p), d);
    double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
    int l = 0;
    for (; l + 8 <= j; l += 8) {
        double r[8];
#pragma unroll
        for (int u = 0; u < 8; u++) r[u] = RM[ridx<KG>(lane, l + u)];
        z0 = fma(r[0], readlane(kl, l), z0);
        z1 = fma(r[1], readlane(kl, l + 1), z1);
        z2 = fma(r[2], readlane(kl, l + 2), z2);
        z3 = fma(r[3], readlane(kl, l + 3), z3);
        z0 = fma(r[4], readlane(kl, l + 4), z0);
        z1 = fma(r[5], readlane(kl, l + 5), z1);
        z2 = fma(r[6], readlane(kl, l + 6), z2);
        z3 = fma(r[7], readlane(kl, l + 7), z3);
    }
    for (; l < j; l++) z0 = fma(RM[ridx<KG>(lane, l)], readlane(kl, l), z0);
    return (z0 + z1) + (z2 + z3);
}

template <typename T, int NW, int CBW, int KG, int G>
__global__ __launch_bounds__(NW *kWave) void alc_kernel(AlcArgs a)
{
    using Acc = typename Mma<T>::acc;
    constexpr int kThreads = NW * kWave;
    constexpr int SLOTS = NW * CBW * 16;
    constexpr int WSLOTS = CBW * 16;  // candidates per wave
    constexpr int NMAX = 4 * KG;
    constexpr int NIB = (NMAX + 15) / 16;
    constexpr int ROWS = NIB * 16;
    constexpr int RT = NIB * KG * 64;
    constexpr bool MIXED = sizeof(T) == 4;
    static_assert(ROWS == 64, "one lane per row of R in the wave-level float64 routines");
    static_assert(CBW % G == 0 && WSLOTS % kWave == 0, "candidate blocks tile the wave");

    __shared__ double RM[RT];               // float64 R_j, A-fragment tiles
    __shared__ float RA32[MIXED ? RT : 1];  // float32 copy of R_j (mixed)
    __shared__ double cx[kPmax * SLOTS];    // candidate coordinates, [k][slot]
    __shared__ double cxv[SLOTS];           // K(candidate, x)
    __shared__ double cY[SLOTS];            // response of each slot
    __shared__ double alc_out[NMAX];        // score of the point added at each step
    __shared__ float alc_out32[MIXED ? NMAX : 1];  // its float32 score (NaN: step decided in float64)
    __shared__ int32_t cid[SLOTS];          // design index of each slot
    __shared__ uint8_t cflag[SLOTS];        // 0 candidate, 1 in design, 2 empty
    __shared__ T fz_s[MIXED ? SLOTS : 1], fz_c[MIXED ? SLOTS : 1];  // z.z, z.z_h over completed row blocks
    __shared__ double zh[ROWS], tY[ROWS];   // R_j K(X_j, x) and R_j Y_j
    __shared__ float zh32[MIXED ? ROWS : 1];
    __shared__ double zbest[NW][ROWS];      // each wave's best re-scored z
    __shared__ double xs[kPmax];
    __shared__ int32_t selslot[NMAX];
    __shared__ T red_s[NW];
    __shared__ int32_t red_i[NW], red_k[NW];
    __shared__ double rec_v[NW], rec_s[NW], rec_e[NW], rec_d[NW];
    __shared__ float fs32[MIXED ? SLOTS : 1], fc32[MIXED ? SLOTS : 1];  // float32 s and cov of each slot
    __shared__ float rec_v32[NW];
    __shared__ int32_t rec_i[NW], rec_k[NW], rec_n[NW];
    __shared__ int ctl_status, ctl_susp, ctl_wide;

    const T *RA;
    const T *zhT;
    if constexpr (MIXED) {
        RA = RA32;
        zhT = zh32;
    } else {
        RA = RM;
        zhT = zh;
    }

    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane0 = tid & 63;
    int64_t m = blockIdx.x;
    if (a.list) {  // a location list built on the device: blocks past its end have nothing to do
        if ((int)blockIdx.x >= *a.list_count) return;
        m = a.list[blockIdx.x];
    }
    // per-location sizes and lengthscale (checked by the list builder), or the uniform ones
    const int p = a.p, n0 = a.n0;
    const int Np = __builtin_amdgcn_readfirstlane(a.Np_per ? a.Np_per[m] : a.Np);
    const int n = __builtin_amdgcn_readfirstlane(a.n_per ? a.n_per[m] : a.n);
    const double d = uniform(a.d_per ? a.d_per[m] : a.d), kappa = 1.0 + a.g;
    const int64_t orow = a.sel_off ? a.sel_off[m] : m * (int64_t)a.n;
    const int64_t prow = m * (int64_t)(a.pool_stride ? a.pool_stride : a.Np);
    const float ninv_d32 = (float)(-1.0 / d);
    const int wbase = w * WSLOTS;

    // ---- stage the location, its pool and zeroed factors in LDS
    if (tid == 0) {
        ctl_status = kLocOk;
        ctl_susp = 0;
        ctl_wide = 0;
    }
    if (tid < p) xs[tid] = a.XX[m * p + tid];
    __syncthreads();
    for (int s = tid; s < SLOTS; s += kThreads) {
        bool valid = s < Np;
        int32_t di = valid ? a.pool[prow + s] : INT32_MAX;
        if (valid && (di < 0 || di >= a.N)) {  // never read outside X
            ctl_status = kLocBadPool;
            valid = false;
            di = INT32_MAX;
        }
        cid[s] = di;
        cflag[s] = valid ? 0 : 2;
        cY[s] = valid ? a.Y[di] : 0.0;
        if constexpr (MIXED) {
            fz_s[s] = (T)0;
            fz_c[s] = (T)0;
        }
        for (int k = 0; k < p; k++) cx[k * SLOTS + s] = valid ? a.X[(int64_t)di * p + k] : 0.0;
    }
    for (int i = tid; i < RT; i += kThreads) {
        RM[i] = 0.0;
        if constexpr (MIXED) RA32[i] = 0.0f;
    }
    for (int i = tid; i < ROWS; i += kThreads) {
        zh[i] = 0.0;
        tY[i] = 0.0;
        if constexpr (MIXED) zh32[i] = 0.0f;
    }
    __syncthreads();
    if (tid == 0)
        for (int k = 0; k < p; k++)
            if (!isfinite(xs[k]) && ctl_status == kLocOk) ctl_status = kLocNonfinite;
    for (int s = tid; s < SLOTS; s += kThreads)
        cxv[s] = s < Np ? corr64(sqdist_strict(cx + s, SLOTS, xs, 1, p), d) : 0.0;
    __syncthreads();

    int status = ctl_status;
    int guard_steps = 0;
    int j = 0;
    double psi_run = 0.0;  // psi_j = |R_j Y_j|^2 so far (lane 0 of wave 0), for a.normalize

    T Q[CBW][KG];
#pragma unroll
    for (int cb = 0; cb < CBW; cb++)
#pragma unroll
        for (int kg = 0; kg < KG; kg++) Q[cb][kg] = (T)0;
    T sc[MIXED ? CBW : 1];  // float32 score of candidate lane % 16 of each block (mixed)

    for (; status == kLocOk && j < n; j++) {
        // Per-lane addresses are cheap to rebuild and costly to keep live across
        // the whole design (they would be spilled), so the lane id is made opaque
        // to the optimiser once per step.
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        // ===== (1) score every candidate: Z^T = R_j Q^T on the matrix cores
        T bs = (T)0;
        int win_hint = j;  // the float64 path's winner; slot j for the NN start
        if (j >= n0) {
            T best_s = (T)-1;
            int32_t best_i = INT32_MAX, best_k = -1;
            bool susp = false;
            // Rows of R_j never change once added, so z_c restricted to a completed
            // 16-row block is the same at every later step: its sums z.z and z.z_h
            // are kept per slot (fz_s, fz_c) and only the block holding the newest
            // row is recomputed.  The first scored step computes every block.
            // (The float64 kernel, whose register budget is taken by Q, recomputes
            // every block instead.)
            constexpr bool FROZEN = MIXED;
            const int ib_hi = (j - 1) >> 4;
            const int ib_lo = (FROZEN && j != n0) ? ib_hi : 0;
            const bool closes = FROZEN && (j & 15) == 0;  // this step completes block ib_hi
            auto block = [&](int ib, int cg, T (&sp)[G], T (&cp)[G]) {
                Acc acc[G];
#pragma unroll
                for (int q = 0; q < G; q++) acc[q] = Acc{0, 0, 0, 0};
#pragma unroll
                for (int kg = 0; kg < KG; kg++) {
                    if (kg * 4 < j && kg <= ib * 4 + 3) {
                        const T av = RA[(ib * KG + kg) * 64 + lane];
#pragma unroll
                        for (int q = 0; q < G; q++) acc[q] = Mma<T>::run(av, Q[cg + q][kg], acc[q]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const T zr = zhT[ib * 16 + Mma<T>::row(lane, r)];
#pragma unroll
                    for (int q = 0; q < G; q++) {
                        const T z = acc[q][r];
                        sp[q] += z * z;
                        cp[q] += z * zr;
                    }
                }
            };
#pragma unroll
            for (int cg = 0; cg < CBW; cg += G) {
                T sp[G], cp[G];
#pragma unroll
                for (int q = 0; q < G; q++) sp[q] = cp[q] = (T)0;
                T s_[G], c_[G];
                if constexpr (FROZEN) {
                    T dp[G], dc[G];
#pragma unroll
                    for (int q = 0; q < G; q++) dp[q] = dc[q] = (T)0;
#pragma unroll 1
                    for (int ib = ib_lo; ib < ib_hi; ib++) block(ib, cg, dp, dc);
                    block(ib_hi, cg, sp, cp);
#pragma unroll
                    for (int q = 0; q < G; q++) {
                        const int slot = wbase + (cg + q) * 16 + (lane & 15);
                        T fs = fz_s[slot], fc = fz_c[slot];
                        if (ib_lo < ib_hi) {
                            fs += row_sum4(dp[q]);
                            fc += row_sum4(dc[q]);
                        }
                        s_[q] = fs + row_sum4(sp[q]);
                        c_[q] = fc + row_sum4(cp[q]);
                        if ((ib_lo < ib_hi || closes) && lane < 16) {
                            fz_s[slot] = closes ? s_[q] : fs;
                            fz_c[slot] = closes ? c_[q] : fc;
                        }
                    }
                } else {
#pragma unroll 1
                    for (int ib = 0; ib <= ib_hi; ib++) block(ib, cg, sp, cp);
#pragma unroll
                    for (int q = 0; q < G; q++) {
                        s_[q] = row_sum4(sp[q]);
                        c_[q] = row_sum4(cp[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < G; q++) {
                    const int slot = wbase + (cg + q) * 16 + (lane & 15);
                    const bool live = cflag[slot] == 0;
                    const T sv = (T)kappa - s_[q];
                    const T cv = (T)cxv[slot] - c_[q];
                    T score;
                    if constexpr (MIXED)
                        score = (live && sv > 0.0f) ? cv * cv * __builtin_amdgcn_rcpf(sv) : -1.0f;
                    else
                        score = (live && sv > 0.0) ? cv * cv / sv : -1.0;
                    if constexpr (MIXED) {
                        if (live && !(sv > kSmallS * (float)kappa)) susp = true;
                        sc[cg + q] = score;
                        if (lane < 16) {
                            fs32[slot] = sv;
                            fc32[slot] = cv;
                        }
                    }
                    const int32_t di = score >= (T)0 ? cid[slot] : INT32_MAX;
                    if (beats(score, di, best_s, best_i)) {
                        best_s = score;
                        best_i = di;
                        best_k = slot;
                    }
                }
            }
            wave_argmax(best_s, best_i, best_k);
            if (lane == 0) {
                red_s[w] = best_s;
                red_i[w] = best_i;
                red_k[w] = best_k;
            }
            if constexpr (MIXED)
                if (susp) ctl_susp = 1;
            __syncthreads();
            if constexpr (MIXED) {
                // lane q holds wave q's best; one wave-wide argmax combines them
                bs = lane < NW ? red_s[lane] : (T)-1;
                int32_t bi = lane < NW ? red_i[lane] : INT32_MAX;
                win_hint = lane < NW ? red_k[lane] : -1;
                wave_argmax(bs, bi, win_hint);
                // lane 0's copy, so that control flow is uniform even on invalid ties
                bs = uniform(bs);
                win_hint = __builtin_amdgcn_readfirstlane(win_hint);
            } else {
                // few waves: a short serial pass keeps register pressure low
                bs = red_s[0];
                int32_t bi = red_i[0];
                win_hint = red_k[0];
                for (int q = 1; q < NW; q++)
                    if (beats(red_s[q], red_i[q], bs, bi)) {
                        bs = red_s[q];
                        bi = red_i[q];
                        win_hint = red_k[q];
                    }
            }
            if (!(bs >= (T)0)) {  // no candidate with a positive conditional variance
                status = kLocStepFail;
                break;
            }
        }

        // ===== (2) float64 re-score: each wave its own band members
        bool fallback = false;
        if constexpr (MIXED) fallback = j >= n0 && ctl_susp != 0;
        double bv = -1.0, bsv = 0.0, err = 0.0, eabs = 0.0;
        float bv32 = -1.0f;  // float32 score of this wave's float64 best (-1: none)
        int32_t bi64 = INT32_MAX;
        int bk = -1, cnt = 0;
        auto consider = [&](int slot, double v32) {
            const double z = wave_z64<SLOTS, KG>(cx, selslot, RM, slot, j, p, d, lane);
            const double s = kappa - wave_sum(z * z);
            const double cov = cxv[slot] - wave_sum(z * zh[lane]);
            const double v = s > 0.0 ? cov * cov / s : -1.0;
            const int32_t di = v >= 0.0 ? cid[slot] : INT32_MAX;
            if (v32 >= 0.0) {
                err = v > 0.0 ? fmax(err, fabs(v32 - v) / v) : INFINITY;
                if constexpr (MIXED)
                    eabs = fmax(eabs, fmax(fabs((double)fs32[slot] - s), fabs((double)fc32[slot] - cov)));
            }
            if (beats(v, di, bv, bi64)) {
                bv = v;
                bi64 = di;
                bk = slot;
                bsv = s;
                bv32 = (float)v32;
                zbest[w][lane] = z;
            }
        };
        if (j < n0 || !MIXED) {
            if (win_hint >= wbase && win_hint < wbase + WSLOTS) consider(win_hint, -1.0);
        } else if (!fallback) {
            if constexpr (MIXED) {
                const float thr = (float)bs * (1.0f - kBandTau);
#pragma unroll
                for (int cb = 0; cb < CBW; cb++) {
                    unsigned long long mask = __ballot(lane < 16 && sc[cb] >= thr);
                    while (mask) {
                        const int b = __builtin_ctzll(mask);
                        mask &= mask - 1;
                        if (++cnt > kWaveBandCap) break;
                        const float v32 = __builtin_bit_cast(
                            float, __builtin_amdgcn_readlane(__builtin_bit_cast(unsigned, sc[cb]), b));
                        consider(wbase + cb * 16 + b, (double)v32);
                    }
                }
            }
        }
        if (lane == 0) {
            rec_v[w] = bv;
            rec_s[w] = bsv;
            rec_e[w] = err;
            rec_d[w] = eabs;
            rec_v32[w] = bv32;
            rec_i[w] = bi64;
            rec_k[w] = bk;
            rec_n[w] = cnt;
        }
        __syncthreads();
        double v;
        int vw, total = 0;
        if constexpr (MIXED) {
            // lane q holds wave q's record: argmax of the float64 scores, max error, member count
            v = lane < NW ? rec_v[lane] : -1.0;
            int32_t vi = lane < NW ? rec_i[lane] : INT32_MAX;
            vw = lane < NW ? lane : -1;
            wave_argmax(v, vi, vw);
            v = uniform(v);
            vw = __builtin_amdgcn_readfirstlane(vw);
            err = wave_max(lane < NW ? rec_e[lane] : 0.0);
            eabs = wave_max(lane < NW ? rec_d[lane] : 0.0);
            total = (int)wave_sum(lane < NW ? (float)rec_n[lane] : 0.0f);
        } else {
            // few waves: a short serial pass keeps register pressure low
            v = rec_v[0];
            int32_t vi = rec_i[0];
            vw = 0;
            for (int q = 1; q < NW; q++)
                if (beats(rec_v[q], rec_i[q], v, vi)) {
                    v = rec_v[q];
                    vi = rec_i[q];
                    vw = q;
                }
        }
        if constexpr (MIXED) {
            if (j >= n0 && !fallback && (!(v > 0.0) || err > kTrustErr || total > kWaveBandCap)) fallback = true;
            if (j >= n0 && !fallback) {
                // every candidate outside the band: could its score reach the best?
                const double delta = 8.0 * eabs + 0x1p-22 * kappa;
                const float thr = (float)bs * (1.0f - kBandTau);
                bool wide = false;
                for (int t = lane; t < WSLOTS; t += kWave) {
                    const int slot = wbase + t;
                    if (cflag[slot] != 0) continue;
                    const float s32 = fs32[slot], c32 = fc32[slot];
                    const float sc32 = s32 > 0.0f ? c32 * c32 * __builtin_amdgcn_rcpf(s32) : -1.0f;
                    if (sc32 >= thr) continue;  // a band member: re-scored in float64
                    const double sd = (double)s32 - delta, cu = fabs((double)c32) + delta;
                    if (!(sd > 0.0) || cu * cu / sd >= v * (1.0 - 0x1p-20)) wide = true;
                }
                if (__ballot(wide) && lane == 0) ctl_wide = 1;
                __syncthreads();
                if (ctl_wide) fallback = true;
            }
        }
        if (fallback) {
            // ===== the whole step in float64: each wave re-scores all its live candidates
            __syncthreads();
            bv = -1.0;
            bi64 = INT32_MAX;
            bk = -1;
            bv32 = -1.0f;
            for (int s = wbase; s < wbase + WSLOTS; s++)
                if (cflag[s] == 0) consider(s, -1.0);
            if (lane == 0) {
                rec_v[w] = bv;
                rec_s[w] = bsv;
                rec_i[w] = bi64;
                rec_k[w] = bk;
                rec_v32[w] = bv32;
            }
            __syncthreads();
            v = lane < NW ? rec_v[lane] : -1.0;
            int32_t vi = lane < NW ? rec_i[lane] : INT32_MAX;
            vw = lane < NW ? lane : -1;
            wave_argmax(v, vi, vw);
            v = uniform(v);
            vw = __builtin_amdgcn_readfirstlane(vw);
            guard_steps++;
        }

        // ===== (3) float64 update with l = zbest[vw] and s* = rec_s[vw]
        if (vw < 0) {
            status = j < n0 ? kLocInitNotPd : kLocStepFail;
            break;
        }
        const int win = rec_k[vw];
        const double sstar = rec_s[vw];
        if (win < 0 || !(sstar > 0.0) || !isfinite(sstar)) {
            status = j < n0 ? kLocInitNotPd : kLocStepFail;
            break;
        }
        const double lam = sqrt(sstar);
        const double *ell = zbest[vw];
        // new row of R: r_l = -(sum_{i=l}^{j-1} l_i R(i, l)) / lam, r_j = 1 / lam
        constexpr int COLS = (ROWS + NW - 1) / NW;
#pragma unroll
        for (int c = 0; c < COLS; c++) {
            const int l = w + c * NW;
            if (l <= j) {
                const double prod = lane < j ? ell[lane] * RM[ridx<KG>(lane, l)] : 0.0;
                const double sum = wave_sum(prod);
                if (lane == 0) {
                    const double r = l < j ? -sum / lam : 1.0 / lam;
                    RM[ridx<KG>(j, l)] = r;
                    if constexpr (MIXED) RA32[ridx<KG>(j, l)] = (float)r;
                }
            }
        }
        if (w == 0) {
            const double zz = wave_sum(ell[lane] * zh[lane]);
            const double zt = wave_sum(ell[lane] * tY[lane]);
            if (lane == 0) {
                zh[j] = (cxv[win] - zz) / lam;
                tY[j] = (cY[win] - zt) / lam;
                if constexpr (MIXED) zh32[j] = (float)zh[j];
                cflag[win] = 1;
                selslot[j] = win;
                // the score as chosen, or normalised by psi_j / (j - 2) (j >= n0 >= 3)
                const double nf = a.normalize && j >= n0 ? psi_run / (j - 2) : 1.0;
                alc_out[j] = j >= n0 ? v * nf : NAN;
                if constexpr (MIXED)
                    alc_out32[j] = (j >= n0 && rec_v32[vw] >= 0.0f) ? rec_v32[vw] * (float)nf : NAN;
                psi_run += tY[j] * tY[j];
                ctl_susp = 0;
                ctl_wide = 0;
            }
        }
        // new column j of Q, K(candidate, x*): one candidate per lane, then moved
        // into its B-operand place (lanes of group j % 4, register j / 4)
        {
            const int kgj = j >> 2;
            const bool mine = (lane >> 4) == (j & 3);
#pragma unroll
            for (int t = 0; t < CBW / 4; t++) {
                const int slot = wbase + t * kWave + lane;
                T vt = (T)0;
                if (slot < Np) {
                    const double r2 = sqdist_strict(cx + slot, SLOTS, cx + win, SLOTS, p);
                    if constexpr (MIXED)
                        vt = __expf((float)r2 * ninv_d32);  // float32 kernel vector entry
                    else
                        vt = corr64(r2, d);
                }
#pragma unroll
                for (int c4 = 0; c4 < 4; c4++) {
                    const T moved = __shfl(vt, c4 * 16 + (lane & 15), kWave);
#pragma unroll
                    for (int q = 0; q < KG; q++)
                        if (q == kgj && mine) Q[t * 4 + c4][q] = moved;
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();

    const int lane = lane0;
    // ===== outputs: the design in the order added, its scores, the prediction
    for (int jj = tid; jj < j; jj += kThreads) {
        a.sel[orow + jj] = cid[selslot[jj]];
        if (a.alc) a.alc[orow + jj] = alc_out[jj];
        if (a.alc32) a.alc32[orow + jj] = MIXED ? (double)alc_out32[jj] : NAN;
    }
    // padded rows (no offsets, n below the row length): fill the tail
    if (!a.sel_off)
        for (int jj = n + tid; jj < a.n; jj += kThreads) {
            a.sel[orow + jj] = -1;
            if (a.alc) a.alc[orow + jj] = NAN;
            if (a.alc32) a.alc32[orow + jj] = NAN;
        }
    // local prediction (eqs. predgp, preds2): mu = z_h.(R Y), psi = |R Y|^2
    if (w == 0) {
        const double zi = (status == kLocOk && lane < n) ? zh[lane] : 0.0;
        const double ti = (status == kLocOk && lane < n) ? tY[lane] : 0.0;
        const double mu = wave_sum(zi * ti);
        const double psi = wave_sum(ti * ti);
        const double zz = wave_sum(zi * zi);
        if (lane == 0) {
            const bool ok = status == kLocOk;
            const double vv = kappa - zz;
            const double s2 = psi * vv / n;
            if (a.mean) a.mean[m] = ok ? mu : NAN;
            if (a.s2) a.s2[m] = ok ? s2 : NAN;
            if (a.var) a.var[m] = (ok && n > 2) ? s2 * n / (n - 2) : NAN;
            if (a.status) a.status[m] = status;
            if (a.guard) a.guard[m] = guard_steps;
        }
        if (status != kLocOk)
            for (int jj = j + lane; jj < n; jj += kWave) {
                a.sel[orow + jj] = -1;
                if (a.alc) a.alc[orow + jj] = NAN;
                if (a.alc32) a.alc32[orow + jj] = NAN;
            }
    }
}

template <typename T, int NW, int CBW, int KG, int G>
static hipError_t launch_t(const AlcArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((alc_kernel<T, NW, CBW, KG, G>), dim3((unsigned)a.M), dim3(NW * kWave), 0, st, a);
    return hipGetLastError();
}

// Mixed precision over a device-built location list (grid a.M, the list's
// upper bound): pools of up to 512 (big = false) or 1024 candidates, n <= 64.
hipError_t launch_alc_mixed_list(const AlcArgs &a, bool big, hipStream_t st)
{
    if (a.M == 0) return hipSuccess;
    if (a.p > kPmax || !a.list || !a.list_count) return hipErrorInvalidValue;
    static_assert(kMixNmax == 64 && kMixNpMax == 1024, "the list schedules below");
    if (big) return launch_t<float, 8, 8, 16, 4>(a, st);
    return launch_t<float, 8, 4, 16, 4>(a, st);
}

static bool mfma_supported(int precision, int p, int Np, int n)
{
    if (p > kPmax || Np > 1024) return false;
    return precision == 0 ? n <= 52 : n <= 64;
}

// precision 0: float64, incremental columns where a schedule fits, else the
// MFMA kernel; 1: mixed (MFMA, float32 scores); 2: float64 scores re-formed
// every step on the matrix cores.
bool alc_supported(int precision, int p, int Np, int n)
{
    if (precision == 0 && alc_inc_supported(p, Np, n)) return true;
    return mfma_supported(precision == 1 ? 1 : 0, p, Np, n);
}

hipError_t launch_alc(const AlcArgs &a, int precision, hipStream_t st)
{
    if (a.M == 0) return hipSuccess;
    if (precision == 0 && alc_inc_supported(a.p, a.Np, a.n)) return launch_alc_inc(a, st);
    if (precision == 1 && !mixed_trusted(a.n, a.g) && alc_inc_supported(a.p, a.Np, a.n)) {
        // float32 scores cannot be trusted at this conditioning: float64, every step in guard
        AlcArgs b = a;
        b.f64_guard = 1;
        return launch_alc_inc(b, st);
    }
    if (precision == 2) precision = 0;
    if (!mfma_supported(precision, a.p, a.Np, a.n)) return hipErrorNotSupported;
    if (precision == 0) {
        if (a.Np <= 512) return launch_t<double, 4, 8, 13, 1>(a, st);
        return launch_t<double, 8, 8, 13, 1>(a, st);
    }
    if (a.Np <= 512) return launch_t<float, 8, 4, 16, 4>(a, st);
    if (a.n <= 52) return launch_t<float, 8, 8, 13, 4>(a, st);
    return launch_t<float, 8, 8, 16, 4>(a, st);
}

}  // namespace lagp
