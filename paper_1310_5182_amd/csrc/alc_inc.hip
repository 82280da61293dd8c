// Greedy ALC local designs by incremental Cholesky columns (Fig. 1 steps 2a,
// 2b and 5), float64.
//
// With L_j the lower Cholesky factor of K_j, the score of candidate c
// (eq. dxy) is Delta_c = (K(c,x) - z_c.z_h)^2 / (kappa - z_c.z_c) where
// z_c = L_j^{-1} K(X_j, c) and z_h = L_j^{-1} K(X_j, x).  Adding x* borders
// the factor with the row [l^T, lambda], l = z_{x*}, lambda^2 = s* (the Schur
// complement m^{-1} of eq. piedef), so every candidate's z_c grows by exactly
// one entry per step:
//     w_c = (K(c, x*) - z_c . l) / lambda,   z_c <- [z_c, w_c],
//     kappa - z_c.z_c  -=  w_c^2,            K(c,x) - z_c.z_h  -=  w_c w_h,
// with w_h the new entry of z_h.  A step therefore costs one dot product of
// length j per candidate (O(N' j)) instead of the O(N' j^2) of re-forming
// every quadratic form, and needs no inverse at all; the arithmetic is that
// of a row-by-row forward substitution, the same as a fresh factorisation.
//
// Work split.  One workgroup per location; lane t owns the pool positions
// t + s * TB (s < S).  Their z rows sit in registers (first ZR entries) and,
// past ZR, in LDS columns.  A step: each wave reduces the argmax of its
// candidates, every wave combines the per-wave winners, the winning lane
// publishes its z row (l) in LDS, and after one barrier every lane extends its
// own rows.  Two barriers per scored step, one per forced (initial) step.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>

namespace lagp {

namespace {

constexpr int kIncNmax = 128;  // largest n: z_h and R Y live in two lanes' worth of one wave
constexpr int kIncPmax = 8;

template <int TB, int S, int ZR>
__global__ __launch_bounds__(TB) void alc_inc_kernel(AlcArgs a, int zl_cols)
{
    constexpr int NW = TB / kWave;
    constexpr int CAP = TB * S;
    constexpr int NCH = ZR / 8;
    static_assert(ZR % 8 == 0 && NW <= kWave, "schedule shape");

    extern __shared__ double dyn[];
    double *cx = dyn;                            // candidate coordinates, [k][pos]
    double *cY = cx + a.p * CAP;                 // response of each pool position
    double *zl = cY + CAP;                       // z entries past ZR, [entry - ZR][pos]
    int32_t *cid = (int32_t *)(zl + (size_t)zl_cols * CAP);  // design index, INT32_MAX if none

    __shared__ double ell[2][kIncNmax];  // z row of the point being added (by step parity)
    __shared__ double pub_s[2];          // its conditional variance s*
    __shared__ double zhs[kIncNmax], tYs[kIncNmax], alc_out[kIncNmax];
    __shared__ int32_t selpos[kIncNmax];
    __shared__ double xs[kIncPmax];
    __shared__ double red_s[NW];
    __shared__ int32_t red_i[NW], red_k[NW];
    __shared__ int ctl_status;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t m = blockIdx.x;
    const int p = a.p, Np = a.Np, n = a.n, n0 = a.n0;
    const double d = a.d, kappa = 1.0 + a.g;

    // ---- stage the location and its pool in LDS
    if (tid == 0) ctl_status = kLocOk;
    if (tid < p) xs[tid] = a.XX[m * p + tid];
    __syncthreads();
    for (int pos = tid; pos < CAP; pos += TB) {
        bool valid = pos < Np;
        int32_t di = valid ? a.pool[m * Np + pos] : INT32_MAX;
        if (valid && (di < 0 || di >= a.N)) {  // never read outside X
            ctl_status = kLocBadPool;
            valid = false;
        }
        cid[pos] = valid ? di : INT32_MAX;
        cY[pos] = valid ? a.Y[di] : 0.0;
        for (int k = 0; k < p; k++) cx[k * CAP + pos] = valid ? a.X[(int64_t)di * p + k] : 0.0;
    }
    __syncthreads();
    int status = ctl_status;
    for (int k = 0; k < p; k++)
        if (status == kLocOk && !isfinite(xs[k])) status = kLocNonfinite;

    // ---- per-slot state: z row, conditional variance, conditional covariance
    double z[S][ZR];
    double sv[S], cv[S];
    int32_t di[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int pos = tid + s * TB;
        di[s] = cid[pos];
        const bool live = di[s] != INT32_MAX;
        cv[s] = live ? corr64(sqdist_strict(cx + pos, CAP, xs, 1, p), d) : 0.0;
        sv[s] = live ? kappa : -1.0;  // a negative variance marks "not a candidate"
#pragma unroll
        for (int q = 0; q < ZR; q++) z[s][q] = 0.0;
    }

    int j = 0;
    for (; status == kLocOk && j < n; j++) {
        const int par = j & 1;
        // ===== (1) the point to add: forced pool order for the initial design,
        // else the argmax of Delta (ties to the smaller design index)
        int wpos = j;
        double vbest = NAN;
        if (j >= n0) {
            double bs = -1.0;
            int32_t bi = INT32_MAX;
            int bk = -1;
#pragma unroll
            for (int s = 0; s < S; s++) {
                if (sv[s] > 0.0) {
                    const double sc = cv[s] * cv[s] / sv[s];
                    if (beats(sc, di[s], bs, bi)) {
                        bs = sc;
                        bi = di[s];
                        bk = tid + s * TB;
                    }
                }
            }
            wave_argmax(bs, bi, bk);
            if (lane == 0) {
                red_s[w] = bs;
                red_i[w] = bi;
                red_k[w] = bk;
            }
            __syncthreads();
            double v = lane < NW ? red_s[lane] : -1.0;
            int32_t vi = lane < NW ? red_i[lane] : INT32_MAX;
            int vk = lane < NW ? red_k[lane] : -1;
            wave_argmax(v, vi, vk);
            vbest = uniform(v);
            wpos = __builtin_amdgcn_readfirstlane(vk);
            if (!(vbest >= 0.0) || wpos < 0) {  // no candidate with positive variance left
                status = kLocStepFail;
                break;
            }
        }
        // ===== (2) the owner publishes l = z_{x*} and s*, and retires the slot
        const int ws = wpos / TB;
        if (tid == wpos - ws * TB) {
#pragma unroll
            for (int s = 0; s < S; s++) {
                if (s == ws) {
#pragma unroll
                    for (int c = 0; c < NCH; c++)
                        if (c * 8 < j)
#pragma unroll
                            for (int u = 0; u < 8; u++) ell[par][c * 8 + u] = z[s][c * 8 + u];
                    pub_s[par] = sv[s];
                    sv[s] = -1.0;
                }
            }
            for (int q = ZR; q < j; q++) ell[par][q] = zl[(q - ZR) * CAP + wpos];
        }
        __syncthreads();
        const double sstar = pub_s[par];
        if (!(sstar > 0.0) || !isfinite(sstar)) {
            status = j < n0 ? kLocInitNotPd : kLocStepFail;
            break;
        }
        const double lam = sqrt(sstar);
        const double *el = ell[par];

        // ===== (3) z_h and L^{-1} Y gain their entry j (every wave, same bits)
        double dz = 0.0, dt = 0.0;
        if (lane < j) {
            dz = el[lane] * zhs[lane];
            dt = el[lane] * tYs[lane];
        }
        if (lane + kWave < j) {
            dz = fma(el[lane + kWave], zhs[lane + kWave], dz);
            dt = fma(el[lane + kWave], tYs[lane + kWave], dt);
        }
        dz = wave_sum(dz);
        dt = wave_sum(dt);
        const double kxs = corr64(sqdist_strict(cx + wpos, CAP, xs, 1, p), d);
        const double wh = (kxs - dz) / lam;
        if (tid == 0) {
            zhs[j] = wh;
            tYs[j] = (cY[wpos] - dt) / lam;
            selpos[j] = wpos;
            alc_out[j] = vbest;
        }
        if (j + 1 == n) continue;  // the design is complete: no more scoring

        // ===== (4) every candidate's z row gains w_c = (K(c, x*) - z_c . l) / lambda
        double acc[S];
#pragma unroll
        for (int s = 0; s < S; s++) acc[s] = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; c++) {
            if (c * 8 < j) {
                double e[8];
#pragma unroll
                for (int u = 0; u < 8; u++) e[u] = el[c * 8 + u];
#pragma unroll
                for (int u = 0; u < 8; u++)
#pragma unroll
                    for (int s = 0; s < S; s++) acc[s] = fma(z[s][c * 8 + u], e[u], acc[s]);
            }
        }
        for (int q = ZR; q < j; q++) {
            const double e = el[q];
#pragma unroll
            for (int s = 0; s < S; s++) acc[s] = fma(zl[(q - ZR) * CAP + tid + s * TB], e, acc[s]);
        }
        const int jc = j >> 3, ju = j & 7;
#pragma unroll
        for (int s = 0; s < S; s++) {
            const int pos = tid + s * TB;
            const double kc = corr64(sqdist_strict(cx + pos, CAP, cx + wpos, CAP, p), d);
            const double wc = (kc - acc[s]) / lam;
            if (j < ZR) {
#pragma unroll
                for (int c = 0; c < NCH; c++)
                    if (c == jc)
#pragma unroll
                        for (int u = 0; u < 8; u++)
                            if (u == ju) z[s][c * 8 + u] = wc;
            } else {
                zl[(j - ZR) * CAP + pos] = wc;
            }
            sv[s] = fma(-wc, wc, sv[s]);
            cv[s] = fma(-wc, wh, cv[s]);
        }
    }
    __syncthreads();

    // ===== outputs: the design in the order added, its scores, the prediction
    for (int jj = tid; jj < j; jj += TB) {
        a.sel[m * n + jj] = cid[selpos[jj]];
        if (a.alc) a.alc[m * n + jj] = alc_out[jj];
    }
    // local prediction (eqs. predgp, preds2): mu = z_h.(L^{-1} Y), psi = |L^{-1} Y|^2
    if (w == 0) {
        const bool ok = status == kLocOk;
        double mu = 0.0, psi = 0.0, zz = 0.0;
        for (int i = lane; ok && i < n; i += kWave) {
            mu = fma(zhs[i], tYs[i], mu);
            psi = fma(tYs[i], tYs[i], psi);
            zz = fma(zhs[i], zhs[i], zz);
        }
        mu = wave_sum(mu);
        psi = wave_sum(psi);
        zz = wave_sum(zz);
        if (lane == 0) {
            const double s2 = psi * (kappa - zz) / n;
            if (a.mean) a.mean[m] = ok ? mu : NAN;
            if (a.s2) a.s2[m] = ok ? s2 : NAN;
            if (a.var) a.var[m] = (ok && n > 2) ? s2 * n / (n - 2) : NAN;
            if (a.status) a.status[m] = status;
            if (a.guard) a.guard[m] = 0;
        }
        if (!ok)
            for (int jj = j + lane; jj < n; jj += kWave) {
                a.sel[m * n + jj] = -1;
                if (a.alc) a.alc[m * n + jj] = NAN;
            }
    }
}

constexpr size_t kLdsLimit = 160 * 1024;
constexpr size_t kStaticReserve = 8 * 1024;  // the kernel's static LDS, rounded up

template <int TB, int S, int ZR>
size_t inc_dyn_lds(int p, int n)
{
    const int zl_cols = n - 1 > ZR ? n - 1 - ZR : 0;
    return (size_t)TB * S * (8 * (size_t)p + 8 + 4 + 8 * (size_t)zl_cols);
}

template <int TB, int S, int ZR>
hipError_t inc_launch(const AlcArgs &a, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)alc_inc_kernel<TB, S, ZR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kLdsLimit - kStaticReserve));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int zl_cols = a.n - 1 > ZR ? a.n - 1 - ZR : 0;
    const size_t lds = inc_dyn_lds<TB, S, ZR>(a.p, a.n);
    hipLaunchKernelGGL((alc_inc_kernel<TB, S, ZR>), dim3((unsigned)a.M), dim3(TB), lds, st, a, zl_cols);
    return hipGetLastError();
}

// Schedules: (threads, slots per lane, register entries per z row).
enum IncSched { kIncNone = -1, kInc256x2, kInc512x2 };

IncSched inc_pick(int p, int Np, int n)
{
    if (p > kIncPmax || n > kIncNmax) return kIncNone;
    if (Np <= 512 && inc_dyn_lds<256, 2, 40>(p, n) <= kLdsLimit - kStaticReserve) return kInc256x2;
    if (Np <= 1024 && inc_dyn_lds<512, 2, 40>(p, n) <= kLdsLimit - kStaticReserve) return kInc512x2;
    return kIncNone;
}

}  // namespace

bool alc_inc_supported(int p, int Np, int n)
{
    return inc_pick(p, Np, n) != kIncNone;
}

hipError_t launch_alc_inc(const AlcArgs &a, hipStream_t st)
{
    if (a.M == 0) return hipSuccess;
    switch (inc_pick(a.p, a.Np, a.n)) {
    case kInc256x2:
        return inc_launch<256, 2, 40>(a, st);
    case kInc512x2:
        return inc_launch<512, 2, 40>(a, st);
    default:
        return hipErrorNotSupported;
    }
}

}  // namespace lagp
