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
// The new entries of z_h and of t = L^{-1} Y need no dot products either:
// w_h = cov*/lambda and t_j = r*/lambda, where cov* and r* = y* - z_{x*}.t
// are the chosen candidate's carried conditional covariance and residual.
// The prediction (eqs. predgp, preds2) accumulates mu = z_h.t, psi = t.t and
// z_h.z_h entry by entry.
//
// Work split.  One workgroup per location at a time; lane t owns the pool
// positions t + s * TB (s < S).  Entry q of their z rows sits in registers
// (q < ZR), in LDS columns (q < ZR + zl_cols) or in a per-workgroup global
// workspace column (beyond), laid out [entry][position] so that every access
// is a coalesced, lane-private one.  A step: each wave reduces the argmax of
// its candidates and its best lane publishes that candidate's step scalars in
// LDS (double-buffered by step parity); after a barrier every wave combines
// the per-wave winners, the winning lane writes its z row to LDS and, after a
// second barrier, every lane extends its own rows.  (A row leaves its lane one
// LDS instruction per two entries; writing only the winner's saves the LDS
// pipe the rows of the other waves' proposals.)
//
// Locations come either one per workgroup (uniform n and N', grid = M) or
// from a queue that persistent workgroups drain with an atomic counter
// (per-location n and N'; the queue is ordered by schedule and, within a
// schedule, by decreasing cost so that the longest designs start first).
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>
#include <mutex>

namespace lagp {

namespace {

constexpr int kIncNmax = 128;  // z_h and L^{-1} Y live in two lanes' worth of one wave
constexpr int kIncPmax = 8;
constexpr int kIncBcastDefault = 0x3f;  // DPP row broadcast of the chosen row on every schedule

struct IncArgs {
    AlcArgs a;                // a.n / a.Np: uniform values, or the upper bounds
    const int32_t *n_per;     // [M] or NULL
    const int32_t *Np_per;    // [M] or NULL
    const int64_t *sel_off;   // [M + 1] or NULL: row m of sel / alc at m * a.n
    const double *d_per;      // [M] lengthscale of each location, or NULL: a.d
    int pool_stride;          // row stride of the pool (N'_max)
    const int32_t *queue;     // location list, NULL: location = blockIdx.x
    const int32_t *qinfo;     // [2]: first queue entry and count of this schedule
    int32_t *counter;         // next queue entry of this schedule
    double *gz;               // global z columns, gcols * CAP doubles per workgroup
    int gcols;
    int zl_cols;
    int zrow;                 // LDS row length of the chosen point's z row (a.n rounded up to 8)
};

// acc + z_0 l_0 + ... + z_7 l_7 in that order, fused multiply-adds, where l_u
// is lane OFF + u of the caller's 16-lane row: DPP row_newbcast delivers it as
// an operand, so the broadcast costs no instruction.  The s_nop gives the two
// wait states a DPP read needs after a VALU write of its source.
template <int OFF>
__device__ __forceinline__ double fma8_rowbcast(double acc, double l, double z0, double z1, double z2, double z3,
                                                double z4, double z5, double z6, double z7)
{
    asm volatile(
        "s_nop 1\n\t"
        "v_fmac_f64_dpp %0, %1, %2 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %3 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %4 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %5 row_newbcast:%13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %6 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %7 row_newbcast:%15 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %8 row_newbcast:%16 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, %1, %9 row_newbcast:%17 row_mask:0xf bank_mask:0xf"
        : "+v"(acc)
        : "v"(l), "v"(z0), "v"(z1), "v"(z2), "v"(z3), "v"(z4), "v"(z5), "v"(z6), "v"(z7), "n"(OFF),
          "n"(OFF + 1), "n"(OFF + 2), "n"(OFF + 3), "n"(OFF + 4), "n"(OFF + 5), "n"(OFF + 6), "n"(OFF + 7));
    return acc;
}

// Register part of the dot products z_c . l: chunk C holds entries 8C .. 8C+7,
// whose l values sit in lanes 8(C & 1) .. of row group C / 2.  Whole chunks
// below j: entries from j on are zero on both sides.
template <int C, int S, int ZR, int NR>
__device__ __forceinline__ void dot_rowbcast(double (&acc)[S], const double (&lr)[NR], const double (&z)[S][ZR],
                                             int j)
{
    if constexpr (C * 8 < ZR) {
        if (C * 8 < j) {
#pragma unroll
            for (int s = 0; s < S; s++)
                acc[s] = fma8_rowbcast<(C & 1) * 8>(acc[s], lr[C >> 1], z[s][C * 8], z[s][C * 8 + 1],
                                                    z[s][C * 8 + 2], z[s][C * 8 + 3], z[s][C * 8 + 4],
                                                    z[s][C * 8 + 5], z[s][C * 8 + 6], z[s][C * 8 + 7]);
        }
        dot_rowbcast<C + 1>(acc, lr, z, j);
    }
}

// |c - x*|^2 = |c|^2 + |x*|^2 - 2 c . x* for the S pool positions tid + s TB
// of a lane, from centred coordinates in LDS ([k][pos], K >= p of them read,
// rows k >= p weighed by x*_k = 0): a slot's loads are all issued before its
// first product uses one, so that their LDS round trips overlap.
template <int TB, int S, int CAP, int K>
__device__ __forceinline__ void sqdist_slots(const double *cx, const double *cq, int tid, int p,
                                             const double (&xw)[kIncPmax], double qw, double (&r2)[S])
{
#pragma unroll
    for (int s = 0; s < S; s++) {
        double c[K];
#pragma unroll
        for (int k = 0; k < K; k++) c[k] = cx[(k < p ? k : 0) * CAP + tid + s * TB];
        const double q = cq[tid + s * TB];
        __builtin_amdgcn_sched_barrier(0);
        double dt = 0.0;
#pragma unroll
        for (int k = 0; k < K; k++) dt = fma(c[k], xw[k], dt);
        r2[s] = fma(-2.0, dt, q + qw);
    }
}

// RL: the chosen row l reaches the lanes through DPP row broadcasts from a
// per-lane copy (no instruction of its own) instead of uniform-address LDS
// reads (LDS return bandwidth).
template <int TB, int S, int ZR, bool RL>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(2))) void alc_inc_kernel(IncArgs x)
{
    constexpr int NW = TB / kWave;
    constexpr int CAP = TB * S;
    constexpr int NCH = ZR / 8;
    static_assert(ZR % 8 == 0 && NW <= kWave && ZR <= kWave, "schedule shape");
    const AlcArgs &a = x.a;

    // Dynamic LDS: centred candidate coordinates [k][pos], their squared
    // norms, z entries ZR.. [entry - ZR][pos], and the chosen point's z row
    // [parity][entry].
    extern __shared__ double dyn[];
    double *cx = dyn;
    double *cq = cx + a.p * CAP;
    double *zl = cq + CAP;
    double *zb = zl + (size_t)x.zl_cols * CAP;
    const int zrow = x.zrow;

    // each wave's best: s, then 1 / lambda, w_h and t_j should it be chosen
    // (lambda = sqrt(s)), worked out before the barrier by its own lane
    __shared__ double pub[2][NW][4];
    __shared__ double red_s[2][NW];
    __shared__ int32_t red_i[2][NW], red_k[2][NW];
    __shared__ double alc_out[kIncNmax];
    __shared__ int32_t seldi[kIncNmax];
    __shared__ double xs[kIncPmax], sk[kIncPmax];  // x, and the coordinate scales 1 / sqrt(d_k)
    __shared__ int ctl_status, ctl_loc;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int p = a.p, n0 = a.n0;
    const double kappa = 1.0 + a.g;
    const int G0 = ZR + x.zl_cols;  // first entry kept in global memory
    double *gz = x.gz ? x.gz + (size_t)blockIdx.x * x.gcols * CAP : nullptr;

    for (int iter = 0;; iter++) {
        // ---- next location
        int64_t m;
        if (x.queue) {
            if (tid == 0) ctl_loc = atomicAdd(x.counter, 1);
            __syncthreads();
            const int q = __builtin_amdgcn_readfirstlane(ctl_loc);
            if (q >= x.qinfo[1]) break;
            m = __builtin_amdgcn_readfirstlane(x.queue[x.qinfo[0] + q]);
        } else {
            if (iter > 0) break;
            m = blockIdx.x;
        }
        // per-location scalars: wave-uniform, so that the step loop and its
        // bounds stay in scalar registers and scalar branches
        const int n = __builtin_amdgcn_readfirstlane(x.n_per ? x.n_per[m] : a.n);
        const int Np = __builtin_amdgcn_readfirstlane(x.Np_per ? x.Np_per[m] : a.Np);
        const int64_t orow = x.sel_off ? x.sel_off[m] : m * a.n;
        // separable kernel: coordinates scaled by 1 / sqrt(d_k), so that
        // exp(-sum_k (c_k - x_k)^2 / d_k) = exp(-|c' - x'|^2), lengthscale 1
        const double nid = a.dsep ? -1.0 : uniform(-1.0 / (x.d_per ? x.d_per[m] : a.d));  // checked > 0 by the queue

        // ---- stage the location; every lane loads its own pool positions
        if (tid == 0) {
            int st = kLocOk;
            if (a.dsep)
                for (int k = 0; k < p; k++)
                    if (!(a.dsep[k] > 0.0) || !isfinite(a.dsep[k])) st = kLocBadShape;
            ctl_status = st;
        }
        if (tid < p) {
            xs[tid] = a.XX[m * p + tid];
            sk[tid] = a.dsep ? 1.0 / sqrt(a.dsep[tid]) : 1.0;
        }
        __syncthreads();
        double z[S][ZR];
        double sv[S], cv[S], ty[S];  // conditional variance, covariance with x, residual of y
        int32_t di[S];
#pragma unroll
        for (int s = 0; s < S; s++) {
            const int pos = tid + s * TB;
            bool valid = pos < Np;
            int32_t id = valid ? a.pool[m * x.pool_stride + pos] : INT32_MAX;
            if (valid && (id < 0 || id >= a.N)) {  // never read outside X
                ctl_status = kLocBadPool;
                valid = false;
            }
            di[s] = valid ? id : INT32_MAX;
            double q = 0.0;
            for (int k = 0; k < p; k++) {
                const double c = valid ? (a.X[(int64_t)id * p + k] - xs[k]) * sk[k] : 0.0;  // sk = 1: exact
                cx[k * CAP + pos] = c;
                q = fma(c, c, q);
            }
            cq[pos] = q;
            cv[s] = valid ? exp(q * nid) : 0.0;  // K(c, x)
            sv[s] = valid ? kappa : -1.0;         // a negative variance marks "not a candidate"
            ty[s] = valid ? a.Y[id] : 0.0;
#pragma unroll
            for (int e = 0; e < ZR; e++) z[s][e] = 0.0;
        }
        __syncthreads();
        int status = __builtin_amdgcn_readfirstlane(ctl_status);
        for (int k = 0; k < p; k++)
            if (status == kLocOk && !isfinite(uniform(xs[k]))) status = kLocNonfinite;
        double ap0 = 0.0, ap1 = 0.0, ap2 = 0.0;  // z_h.t, t.t, z_h.z_h so far (wave 0)

        // the register entries of slot s's z row, [0, min(j, ZR)), into dst (one lane)
        auto put_row = [&](int s, int j, double *dst) {
#pragma unroll
            for (int c = 0; c < NCH; c++)
                if (c * 8 < j)
#pragma unroll
                    for (int u = 0; u < 8; u++) dst[c * 8 + u] = z[s][c * 8 + u];
            // (entries from ZR on are read where they are kept, at the chosen
            // position)
        };

        // the step scalars of slot s, should it be chosen: s, 1 / lambda,
        // w_h = cov / lambda, t_j = r / lambda with lambda = sqrt(s).  1 / lambda
        // is the hardware reciprocal square root refined by two Newton steps
        // (h -> 1 / (2 lambda) and g -> lambda together), within an ulp or so;
        // a NaN for s <= 0, which the chooser rejects by s itself.
        auto publish = [&](int s, double *dst) {
            const double sq = sv[s];
            const double r0 = __builtin_amdgcn_rsq(sq);
            double g = sq * r0, h = 0.5 * r0;
            double e = fma(-g, h, 0.5);
            g = fma(g, e, g);
            h = fma(h, e, h);
            e = fma(-g, h, 0.5);
            h = fma(h, e, h);
            const double il = 2.0 * h;
            dst[0] = sq;
            dst[1] = il;
            dst[2] = cv[s] * il;
            dst[3] = ty[s] * il;
        };

        int j = 0;
        for (; status == kLocOk && j < n; j++) {
            const int par = j & 1;
            double *zbp = zb + (size_t)par * zrow;
            // ===== (1) every wave proposes its best candidate (forced pool order
            // for the initial design) and that candidate's step scalars; one barrier
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
                wave_argmax_ballot(bs, bi, bk);
                if (lane == 0) {
                    red_s[par][w] = bs;
                    red_i[par][w] = bi;
                    red_k[par][w] = bk;
                }
                if (bk >= 0 && tid == bk % TB) {
                    const int sb = bk / TB;
#pragma unroll
                    for (int s = 0; s < S; s++)
                        if (s == sb) publish(s, pub[par][w]);
                }
            } else if (tid == j) {  // pool position j: slot 0 of thread j
                publish(0, pub[par][w]);
                red_i[par][w] = di[0];
            }
            __syncthreads();
            // ===== (2) the winner: argmax of Delta, ties to the smaller design index
            int wpos = j;
            int32_t wdi = -1;  // the chosen point's design index (from n0 on)
            double vbest = NAN;
            if (j >= n0) {
                double v = lane < NW ? red_s[par][lane] : -1.0;
                int32_t vi = lane < NW ? red_i[par][lane] : INT32_MAX;
                int vk = lane < NW ? red_k[par][lane] : -1;
                // NW <= 16 proposals: three exchange stages within each group of
                // eight lanes (a fourth across the two eights of a row) leave
                // lane 0 with the argmax (ties: smaller index)
                static_assert(NW <= 16, "one row of sixteen lanes");
                argmax_stage<0>(v, vi, vk);
                argmax_stage<1>(v, vi, vk);
                argmax_stage<2>(v, vi, vk);
                if constexpr (NW > 8) argmax_stage<3>(v, vi, vk);
                vbest = readlane(v, 0);
                wpos = __builtin_amdgcn_readlane(vk, 0);
                wdi = __builtin_amdgcn_readlane(vi, 0);
                if (!(vbest >= 0.0) || wpos < 0) {  // no candidate with positive variance left
                    status = kLocStepFail;
                    break;
                }
            }
            const int wt = wpos % TB, ws = wpos / TB;
            const int vw = wt >> 6;  // the winner's wave
            // the chosen point's centred coordinates, squared norm and Schur
            // complement in one LDS access: lane k < p loads coordinate k, lane
            // kIncPmax the squared norm and lane kIncPmax + 1 the complement s*;
            // the values go to scalar registers lane by lane (rather than one
            // round trip per value)
            const double vch = *(lane < p ? cx + lane * CAP + wpos
                                          : lane == kIncPmax + 1 ? &pub[par][vw][0] : cq + wpos);
            const double sstar = readlane(vch, kIncPmax + 1);
            if (!(sstar > 0.0) || !isfinite(sstar)) {
                status = j < n0 ? kLocInitNotPd : kLocStepFail;
                break;
            }
            // only the chosen point's z row goes through LDS (each row is written
            // by one lane, one LDS instruction per two entries): a second barrier
            // instead of every wave writing its proposal's row
            if (tid == wt) {
#pragma unroll
                for (int s = 0; s < S; s++)
                    if (s == ws) {
                        if (j + 1 < n) put_row(s, j, zbp);
                        sv[s] = -1.0;  // retire the chosen slot
                    }
            }
            // the chosen point's coordinates (zero from p on) and squared norm,
            // wave-uniform, from the access above
            double xw[kIncPmax];
#pragma unroll
            for (int k = 0; k < kIncPmax; k++) xw[k] = k < p ? readlane(vch, k) : 0.0;
            const double qw = readlane(vch, kIncPmax);
            // K(c, x*) of every slot from centred coordinates, |c - x*|^2 =
            // |c'|^2 + |x*'|^2 - 2 c'.x*', also before the barrier: the distances
            // and exps need only x*, so they hide the winner's row write
            double kcs[S];
            if (j + 1 < n) {
                double r2[S];
                if (p > 4)
                    sqdist_slots<TB, S, CAP, 8>(cx, cq, tid, p, xw, qw, r2);
                else if (p > 2)
                    sqdist_slots<TB, S, CAP, 4>(cx, cq, tid, p, xw, qw, r2);
                else
                    sqdist_slots<TB, S, CAP, 2>(cx, cq, tid, p, xw, qw, r2);
#pragma unroll
                for (int s = 0; s < S; s++) kcs[s] = exp(r2[s] * nid);
                __syncthreads();
            }
            // step scalars, wave-uniform (scalar registers): lanes 1, 2, 3 load
            // 1 / lambda, w_h and t_j in one LDS access
            double ilam, wh, tn;
            {
                const double v = pub[par][vw][lane < 4 ? lane : 0];
                ilam = readlane(v, 1);
                wh = readlane(v, 2);
                tn = readlane(v, 3);
            }
            const double *el = zbp;

            // ===== (3) z_h and t = L^{-1} Y gain their entry j
            if (tid == 0) {
                seldi[j] = j >= n0 ? wdi : red_i[par][vw];
                // ap1 still holds psi_j = t.t over the first j entries (wave 0):
                // the normalised score psi_j Delta / (j - 2) when asked (j >= n0 >= 3)
                alc_out[j] = a.normalize && j >= n0 ? vbest * ap1 / (j - 2) : vbest;
            }
            if (w == 0) {
                ap0 = fma(wh, tn, ap0);
                ap1 = fma(tn, tn, ap1);
                ap2 = fma(wh, wh, ap2);
            }
            if (j + 1 == n) continue;  // the design is complete: no more scoring

            // ===== (4) every candidate's z row gains w_c = (K(c, x*) - z_c . l) / lambda
            double acc[S];
#pragma unroll
            for (int s = 0; s < S; s++) acc[s] = 0.0;
            if constexpr (RL) {
                // lane i of every 16-lane row holds entries 16 k + i of l (zero
                // from j on), broadcast across the row inside the FMAs
                double lr[(ZR + 15) / 16];
#pragma unroll
                for (int k = 0; k < (ZR + 15) / 16; k++) {
                    const int e = 16 * k + (lane & 15);
                    lr[k] = e < j && e < ZR ? el[e] : 0.0;
                }
                dot_rowbcast<0>(acc, lr, z, j);
            } else {
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
            }
            const int jl = j < G0 ? j : G0;
#pragma unroll 4
            for (int q = ZR; q < jl; q++) {
                const double e = zl[(q - ZR) * CAP + wpos];
#pragma unroll
                for (int s = 0; s < S; s++) acc[s] = fma(zl[(q - ZR) * CAP + tid + s * TB], e, acc[s]);
            }
#pragma unroll 4
            for (int q = G0; q < j; q++) {
                const double e = gz[(size_t)(q - G0) * CAP + wpos];
                const double *col = gz + (size_t)(q - G0) * CAP + tid;
#pragma unroll
                for (int s = 0; s < S; s++) acc[s] = fma(col[s * TB], e, acc[s]);
            }
            // the entry index, as a scalar: the write below is a scalar branch, not
            // a select over every register column
            const int jc = __builtin_amdgcn_readfirstlane(j >> 3), ju = __builtin_amdgcn_readfirstlane(j & 7);
            double wcs[S];
#pragma unroll
            for (int s = 0; s < S; s++) {
                const int pos = tid + s * TB;
                const double wc = (kcs[s] - acc[s]) * ilam;
                wcs[s] = wc;
                if (j >= ZR) {
                    if (j < G0)
                        zl[(j - ZR) * CAP + pos] = wc;
                    else
                        gz[(size_t)(j - G0) * CAP + pos] = wc;
                }
                sv[s] = fma(-wc, wc, sv[s]);
                cv[s] = fma(-wc, wh, cv[s]);
                ty[s] = fma(-wc, tn, ty[s]);
            }
            // register column j of every slot, behind one scalar branch tree
            if (j < ZR) {
#pragma unroll
                for (int c = 0; c < NCH; c++)
                    if (c == jc)
#pragma unroll
                        for (int u = 0; u < 8; u++)
                            if (u == ju) {
                                asm volatile("");  // keeps this a scalar branch, not a select per column
#pragma unroll
                                for (int s = 0; s < S; s++) z[s][c * 8 + u] = wcs[s];
                            }
            }
        }
        __syncthreads();

        // ===== outputs: the design in the order added, its scores, the prediction
        for (int jj = tid; jj < j; jj += TB) {
            a.sel[orow + jj] = seldi[jj];
            if (a.alc) a.alc[orow + jj] = alc_out[jj];
            if (a.alc32) a.alc32[orow + jj] = NAN;  // no float32 scores on this path
        }
        // local prediction (eqs. predgp, preds2): mu = z_h.t, psi = t.t
        if (w == 0) {
            const bool ok = status == kLocOk;
            if (lane == 0) {
                const double mu = ap0, psi = ap1, zz = ap2;
                const double s2 = psi * (kappa - zz) / n;
                if (a.mean) a.mean[m] = ok ? mu : NAN;
                if (a.s2) a.s2[m] = ok ? s2 : NAN;
                if (a.var) a.var[m] = (ok && n > 2) ? s2 * n / (n - 2) : NAN;
                if (a.status) a.status[m] = status;
                // standing in for the mixed kernel: every step was decided in float64
                if (a.guard) a.guard[m] = a.f64_guard ? (j > n0 ? j - n0 : 0) : 0;
            }
            if (!ok)
                for (int jj = j + lane; jj < n; jj += kWave) {
                    a.sel[orow + jj] = -1;
                    if (a.alc) a.alc[orow + jj] = NAN;
                    if (a.alc32) a.alc32[orow + jj] = NAN;
                }
        }
        // padded rows (no offsets, n below the row length): fill the tail
        if (!x.sel_off)
            for (int jj = n + tid; jj < a.n; jj += TB) {
                a.sel[orow + jj] = -1;
                if (a.alc) a.alc[orow + jj] = NAN;
                if (a.alc32) a.alc32[orow + jj] = NAN;
            }
        __syncthreads();  // LDS is restaged for the next location
    }
}

// ---------------------------------------------------------------- schedules
constexpr size_t kLdsLimit = 160 * 1024;
constexpr size_t kStaticReserve = 4 * 1024;  // the kernel's static LDS, rounded up
constexpr size_t kDynLds = kLdsLimit - kStaticReserve;

struct Sched {
    int tb, s, zr;
    constexpr int cap() const { return tb * s; }
    // the chosen row's register entries are copied in whole chunks of 8, so a
    // row slot holds n_max rounded up to a multiple of 8
    static int zrow(int n_max) { return (n_max + 7) & ~7; }
    // dynamic LDS bytes: p coordinates and a norm per position, zl LDS
    // columns, and the double-buffered row of the chosen point
    size_t lds(int p, int zl, int n_max) const
    {
        return (size_t)cap() * 8 * ((size_t)p + 1 + (size_t)zl) + (size_t)2 * zrow(n_max) * 8;
    }
    // LDS columns that fit, capped at the n_max - 1 - ZR that are needed; -1
    // if not even the coordinates fit
    int zl_fit(int p, int n_max) const
    {
        const size_t base = lds(p, 0, n_max);
        if (base > kDynLds) return -1;
        const int need = n_max - 1 > zr ? n_max - 1 - zr : 0;
        const int fit = (int)((kDynLds - base) / (8 * (size_t)cap()));
        return need < fit ? need : fit;
    }
};

// Schedule b: TB threads per location, S pool positions per lane (so pools of
// up to TB S), ZR factor entries per position in registers.  3-5 put the pools
// of 0-2 on twice the waves with half the positions per lane (a SIMD then
// interleaves four waves, or two of eight for 512 threads, over a step's
// dependent phases, at the price of fewer registers per lane and a longer
// winner exchange).  Each pool-size class has a default (below) and a plan may
// time the others that hold its pools.
constexpr int kNumSched = 6;
constexpr Sched kSched[kNumSched] = {{256, 2, 40},  {512, 2, 40},  {512, 4, 16},
                                     {1024, 1, 40}, {1024, 2, 16}, {512, 1, 40}};

static_assert(kNumSched == kIncSchedules, "schedule count");

// Pool-size classes: class c holds pools of up to kClassCap[c] positions and
// runs on one schedule, the default below unless a plan chose another (the
// defaults are the plans' choices at the configurations measured: for pools of
// 1025 to 2048, 1024 x 2 / 16 over 512 x 4 / 16).
constexpr int kClassCap[kIncClasses] = {256, 512, 1024, 2048};
constexpr int kDefaultMap[kIncClasses] = {0, 0, 1, 4};

__host__ __device__ inline int class_of(int Np)
{
    return Np <= kClassCap[0] ? 0 : Np <= kClassCap[1] ? 1 : Np <= kClassCap[2] ? 2 : Np <= kClassCap[3] ? 3 : -1;
}

template <int B, bool RL>
constexpr auto kernel_of()
{
    return &alc_inc_kernel<kSched[B].tb, kSched[B].s, kSched[B].zr, RL>;
}

const void *kernel_ptr(int b, bool rl)
{
    switch (b) {
    case 0:
        return rl ? (const void *)kernel_of<0, true>() : (const void *)kernel_of<0, false>();
    case 1:
        return rl ? (const void *)kernel_of<1, true>() : (const void *)kernel_of<1, false>();
    case 2:
        return rl ? (const void *)kernel_of<2, true>() : (const void *)kernel_of<2, false>();
    case 3:
        return rl ? (const void *)kernel_of<3, true>() : (const void *)kernel_of<3, false>();
    case 4:
        return rl ? (const void *)kernel_of<4, true>() : (const void *)kernel_of<4, false>();
    default:
        return rl ? (const void *)kernel_of<5, true>() : (const void *)kernel_of<5, false>();
    }
}

bool rl_of(int bcast, int b)
{
    return ((bcast < 0 ? kIncBcastDefault : bcast) >> b) & 1;
}

__host__ __device__ inline int sched_for(int Np)
{
    const int c = class_of(Np);
    return c < 0 ? -1 : kDefaultMap[c];
}

// CUs of the current device; the schedules' LDS limit set once per device.
struct DevInfo {
    int cus = 0;
    bool ready = false;
};

hipError_t dev_info(DevInfo &out)
{
    static std::mutex mu;
    static DevInfo cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    DevInfo &c = cache[dev];
    if (!c.ready) {
        e = hipDeviceGetAttribute(&c.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        for (int b = 0; b < kNumSched; b++)
            for (int rl = 0; rl < 2; rl++) {
                e = hipFuncSetAttribute(kernel_ptr(b, rl), hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kDynLds);
                if (e != hipSuccess) return e;
            }
        c.ready = true;
    }
    out = c;
    return hipSuccess;
}

// Persistent grid of schedule b: every CU filled to the residency that its
// registers and this launch's LDS allow.
hipError_t persistent_grid(int b, size_t lds, int cus, int64_t *grid)
{
    int nb = 0;  // both broadcast variants use the same registers bound
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel_ptr(b, true), kSched[b].tb, lds);
    if (e != hipSuccess) return e;
    *grid = (int64_t)cus * (nb > 0 ? nb : 1);
    return hipSuccess;
}

template <int B>
void launch_b(bool rl, const IncArgs &x, dim3 grid, size_t lds, hipStream_t st)
{
    if (rl)
        hipLaunchKernelGGL((kernel_of<B, true>()), grid, dim3(kSched[B].tb), lds, st, x);
    else
        hipLaunchKernelGGL((kernel_of<B, false>()), grid, dim3(kSched[B].tb), lds, st, x);
}

hipError_t launch_sched(int b, bool rl, const IncArgs &x, dim3 grid, size_t lds, hipStream_t st)
{
    switch (b) {
    case 0:
        launch_b<0>(rl, x, grid, lds, st);
        break;
    case 1:
        launch_b<1>(rl, x, grid, lds, st);
        break;
    case 2:
        launch_b<2>(rl, x, grid, lds, st);
        break;
    case 3:
        launch_b<3>(rl, x, grid, lds, st);
        break;
    case 4:
        launch_b<4>(rl, x, grid, lds, st);
        break;
    default:
        launch_b<5>(rl, x, grid, lds, st);
        break;
    }
    return hipGetLastError();
}

// ------------------------------------------------- queue of uneven locations
constexpr int kBins = 64;  // cost classes per schedule
constexpr int kKeys = kNumSched * kBins;
constexpr size_t kHdrBytes = 4096;  // key counts, counters, queue slices

struct PlanWs {
    int32_t *hist;     // [kKeys] counts, then running insert offsets
    int32_t *counter;  // [kNumSched]
    int32_t *qinfo;    // [kNumSched][2]: first entry, count
    int32_t *mcount;   // [2] lengths of the mixed-precision lists
    int32_t *key;      // [M]
    int32_t *queue;    // [M]
    int32_t *mlist[2]; // [M] each: locations for the mixed kernel, pools <= 512 / <= 1024
    int mixed;         // route the locations the mixed kernel covers to mlist
    int smap[kIncClasses];  // schedule of each pool-size class
};

__global__ void plan_zero(PlanWs w)
{
    const int t = threadIdx.x;
    for (int i = t; i < kKeys; i += blockDim.x) w.hist[i] = 0;
    if (t < kNumSched) {
        w.counter[t] = 0;
        w.qinfo[2 * t] = 0;
        w.qinfo[2 * t + 1] = 0;
    }
    if (t < 2) w.mcount[t] = 0;
}

// Classify every location: its schedule (that of its pool-size class) and a
// cost class (four per octave of N' n^2, the order of its update work), or a
// shape error written in place.
__global__ void plan_classify(IncArgs x, PlanWs w, int64_t M)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const AlcArgs &a = x.a;
    const int n = x.n_per ? x.n_per[m] : a.n;
    const int Np = x.Np_per ? x.Np_per[m] : a.Np;
    const int64_t orow = x.sel_off ? x.sel_off[m] : m * a.n;
    const int64_t rowlen = x.sel_off ? x.sel_off[m + 1] - x.sel_off[m] : a.n;
    const double dm = x.d_per ? x.d_per[m] : a.d;
    const bool ok = n >= a.n0 && n <= a.n && Np >= n && Np <= x.pool_stride && rowlen >= n && dm > 0.0 &&
                    isfinite(dm);
    const int c = ok ? class_of(Np) : -1;
    const int b = c < 0 ? -1 : w.smap[c];
    if (b < 0) {
        w.key[m] = -1;
        if (a.mean) a.mean[m] = NAN;
        if (a.s2) a.s2[m] = NAN;
        if (a.var) a.var[m] = NAN;
        if (a.status) a.status[m] = kLocBadShape;
        if (a.guard) a.guard[m] = 0;
        for (int64_t jj = 0; jj < rowlen && jj < a.n; jj++) {
            a.sel[orow + jj] = -1;
            if (a.alc) a.alc[orow + jj] = NAN;
        }
        return;
    }
    if (w.mixed && n <= kMixNmax && Np <= kMixNpMax && mixed_trusted(n, a.g)) {  // the mixed kernel takes it
        const int l = Np <= kMixNpMax / 2 ? 0 : 1;
        w.mlist[l][atomicAdd(&w.mcount[l], 1)] = (int32_t)m;
        w.key[m] = -1;
        return;
    }
    const double cost = (double)Np * n * n;
    int bin = (int)(4.0 * log2(cost)) - 40;
    bin = bin < 0 ? 0 : bin > kBins - 1 ? kBins - 1 : bin;
    const int key = b * kBins + (kBins - 1 - bin);  // larger cost first within a schedule
    w.key[m] = key;
    atomicAdd(&w.hist[key], 1);
}

// Exclusive scan of the key counts, and each schedule's slice of the queue.
__global__ void plan_scan(PlanWs w)
{
    if (threadIdx.x != 0) return;
    int run = 0;
    for (int b = 0; b < kNumSched; b++) {
        w.qinfo[2 * b] = run;
        for (int i = 0; i < kBins; i++) {
            const int c = w.hist[b * kBins + i];
            w.hist[b * kBins + i] = run;
            run += c;
        }
        w.qinfo[2 * b + 1] = run - w.qinfo[2 * b];
    }
}

__global__ void plan_scatter(PlanWs w, int64_t M)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int key = w.key[m];
    if (key < 0) return;
    w.queue[atomicAdd(&w.hist[key], 1)] = (int32_t)m;
}

size_t align256(size_t v)
{
    return (v + 255) & ~(size_t)255;
}

// Global z columns per workgroup of schedule b for these bounds; -1 if the
// schedule cannot hold the coordinates at all.
int gcols_for(int b, int p, int n_max)
{
    const int zl = kSched[b].zl_fit(p, n_max);
    if (zl < 0) return -1;
    const int need = n_max - 1 - kSched[b].zr - zl;
    return need > 0 ? need : 0;
}

}  // namespace

// ---------------------------------------------------------------- host API
int alc_inc_schedule(int Np)
{
    return sched_for(Np);
}

int alc_inc_class(int Np)
{
    return class_of(Np);
}

int alc_inc_default_sched(int c)
{
    return c >= 0 && c < kIncClasses ? kDefaultMap[c] : -1;
}

bool alc_inc_admissible(int s, int c, int p, int n_max, bool on_chip)
{
    if (s < 0 || s >= kNumSched || c < 0 || c >= kIncClasses) return false;
    if (kSched[s].cap() < kClassCap[c]) return false;
    const int gc = gcols_for(s, p, n_max);
    return on_chip ? gc == 0 : gc >= 0;
}

void alc_inc_sched_name(int s, char *buf, size_t len)
{
    if (s < 0 || s >= kNumSched)
        snprintf(buf, len, "none");
    else
        snprintf(buf, len, "%dx%d/%d", kSched[s].tb, kSched[s].s, kSched[s].zr);
}

bool alc_inc_supported(int p, int Np, int n)
{
    if (p > kIncPmax || n > kIncNmax) return false;
    const int b = sched_for(Np);
    return b >= 0 && gcols_for(b, p, n) == 0;
}

hipError_t launch_alc_inc(const AlcArgs &a, hipStream_t st, int bcast, const int *smap)
{
    if (a.M == 0) return hipSuccess;
    if (!alc_inc_supported(a.p, a.Np, a.n)) return hipErrorNotSupported;
    DevInfo info;
    hipError_t e = dev_info(info);
    if (e != hipSuccess) return e;
    int b = sched_for(a.Np);
    if (smap) {  // the plan's schedule for this pool size, if it keeps every column on chip
        const int c = class_of(a.Np);
        if (alc_inc_admissible(smap[c], c, a.p, a.n, true)) b = smap[c];
    }
    IncArgs x{};
    x.a = a;
    x.pool_stride = a.Np;
    x.zl_cols = kSched[b].zl_fit(a.p, a.n);
    x.zrow = Sched::zrow(a.n);
    return launch_sched(b, rl_of(bcast, b), x, dim3((unsigned)a.M), kSched[b].lds(a.p, x.zl_cols, a.n), st);
}

bool alc_uneven_supported(int p, int Np_max, int n_max)
{
    if (p > kIncPmax || n_max > kIncNmax) return false;
    const int top = class_of(Np_max);
    if (top < 0) return false;
    for (int c = 0; c <= top; c++)
        if (!alc_inc_admissible(kDefaultMap[c], c, p, n_max, false)) return false;
    return true;
}

// The schedules a launch over classes 0 .. top may use: with a map, the
// mapped ones (a bit per schedule); without, every schedule admissible for
// one of those classes (the workspace holds the global columns of all of them,
// so that a plan may choose among them after the workspace is sized).
static unsigned sched_set(int top, int p, int n_max, const int *smap)
{
    unsigned set = 0;
    for (int c = 0; c <= top; c++) {
        if (smap) {
            set |= 1u << smap[c];
            continue;
        }
        for (int b = 0; b < kNumSched; b++)
            if (alc_inc_admissible(b, c, p, n_max, false)) set |= 1u << b;
    }
    return set;
}

hipError_t alc_uneven_workspace(int p, int64_t M, int Np_max, int n_max, size_t *bytes)
{
    DevInfo info;
    hipError_t e = dev_info(info);
    if (e != hipSuccess) return e;
    // header, keys, queue, the two mixed-precision lists, then the global
    // columns of every schedule a plan could map these classes to
    size_t total = kHdrBytes + 4 * align256((size_t)M * 4);
    const int top = class_of(Np_max);
    if (top < 0) return hipErrorInvalidValue;
    const unsigned set = sched_set(top, p, n_max, nullptr);
    for (int b = 0; b < kNumSched; b++) {
        if (!(set >> b & 1)) continue;
        const int gc = gcols_for(b, p, n_max);
        int64_t grid = 0;
        e = persistent_grid(b, kSched[b].lds(p, kSched[b].zl_fit(p, n_max), n_max), info.cus, &grid);
        if (e != hipSuccess) return e;
        total += align256((size_t)grid * kSched[b].cap() * gc * 8);
    }
    *bytes = total;
    return hipSuccess;
}

hipError_t launch_alc_uneven(const AlcArgs &a, const int32_t *n_per, const int32_t *Np_per,
                             const int64_t *sel_off, const double *d_per, void *ws, size_t ws_bytes,
                             hipStream_t st, int bcast, bool mixed, const int *smap)
{
    if (a.M == 0) return hipSuccess;
    const int top = class_of(a.Np);
    if (top < 0) return hipErrorInvalidValue;
    int map[kIncClasses];
    for (int c = 0; c < kIncClasses; c++) {
        map[c] = smap ? smap[c] : kDefaultMap[c];
        if (c <= top && !alc_inc_admissible(map[c], c, a.p, a.n, false)) return hipErrorInvalidValue;
    }
    DevInfo info;
    hipError_t e = dev_info(info);
    if (e != hipSuccess) return e;
    size_t need = 0;
    e = alc_uneven_workspace(a.p, a.M, a.Np, a.n, &need);
    if (e != hipSuccess) return e;
    if (ws_bytes < need) return hipErrorInvalidValue;

    char *base = (char *)ws;
    PlanWs w;
    w.hist = (int32_t *)base;
    w.counter = w.hist + kKeys;
    w.qinfo = w.counter + kNumSched;
    w.mcount = w.qinfo + 2 * kNumSched;
    size_t off = kHdrBytes;
    w.key = (int32_t *)(base + off);
    off += align256((size_t)a.M * 4);
    w.queue = (int32_t *)(base + off);
    off += align256((size_t)a.M * 4);
    for (int l = 0; l < 2; l++) {
        w.mlist[l] = (int32_t *)(base + off);
        off += align256((size_t)a.M * 4);
    }
    w.mixed = mixed && a.p <= kIncPmax;
    for (int c = 0; c < kIncClasses; c++) w.smap[c] = map[c];

    IncArgs x{};
    x.a = a;
    x.a.f64_guard = w.mixed;  // the float64 kernel stands in for the mixed one
    x.n_per = n_per;
    x.Np_per = Np_per;
    x.sel_off = sel_off;
    x.d_per = d_per;
    x.pool_stride = a.Np;
    x.queue = w.queue;

    const unsigned lgrid = (unsigned)((a.M + 255) / 256);
    hipLaunchKernelGGL(plan_zero, dim3(1), dim3(256), 0, st, w);
    hipLaunchKernelGGL(plan_classify, dim3(lgrid), dim3(256), 0, st, x, w, a.M);
    hipLaunchKernelGGL(plan_scan, dim3(1), dim3(64), 0, st, w);
    hipLaunchKernelGGL(plan_scatter, dim3(lgrid), dim3(256), 0, st, w, a.M);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (w.mixed) {
        // the locations the mixed kernel covers, one workgroup each
        for (int l = 0; l < 2; l++) {
            AlcArgs am = a;
            am.n_per = n_per;
            am.Np_per = Np_per;
            am.sel_off = sel_off;
            am.d_per = d_per;
            am.pool_stride = a.Np;
            am.list = w.mlist[l];
            am.list_count = w.mcount + l;
            if ((e = launch_alc_mixed_list(am, l == 1, st)) != hipSuccess) return e;
        }
    }

    // every admissible schedule owns a slice of the workspace (as sized by
    // alc_uneven_workspace); the mapped ones run, each draining its queue
    const unsigned all = sched_set(top, a.p, a.n, nullptr), used = sched_set(top, a.p, a.n, map);
    for (int b = 0; b < kNumSched; b++) {
        if (!(all >> b & 1)) continue;
        const int gc = gcols_for(b, a.p, a.n);
        x.zl_cols = kSched[b].zl_fit(a.p, a.n);
        x.zrow = Sched::zrow(a.n);
        const size_t lds = kSched[b].lds(a.p, x.zl_cols, a.n);
        int64_t grid64 = 0;
        if ((e = persistent_grid(b, lds, info.cus, &grid64)) != hipSuccess) return e;
        const unsigned grid = (unsigned)(grid64 < a.M ? grid64 : a.M);
        x.qinfo = w.qinfo + 2 * b;
        x.counter = w.counter + b;
        x.gcols = gc;
        x.gz = gc > 0 ? (double *)(base + off) : nullptr;
        off += align256((size_t)grid64 * kSched[b].cap() * gc * 8);
        if (!(used >> b & 1)) continue;
        e = launch_sched(b, rl_of(bcast, b), x, dim3(grid), lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lagp
