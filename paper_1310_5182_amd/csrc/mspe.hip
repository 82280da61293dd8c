// Local designs by the MSPE criterion (Sec. 2.2, eqs. mspe and newv), float64.
//
// At step j (design X_j of j points) the candidate x' chosen minimises
//   J(x') = (j + 1) psi_j / (j (j - 1)) v_{j+1}(x) + (d mu_j / d d)^2 / G_{j+1},
// eq. mspe with V_j of eq. newv and theta = d, the lengthscale the design is
// built at.  G_{j+1} is read as the expected information about d in j + 1
// responses of N(0, tau^2 K_{j+1}) with tau^2 unknown:
//   G_{j+1} = (tr(W^2) - tr(W)^2 / (j + 1)) / 2,  W = K_{j+1}^{-1} Kd_{j+1},
// Kd = dK/dd = K(D) * D / d^2 (the nugget does not depend on d).
//
// Square-root form.  With L_j the Cholesky factor of K_j and R = L_j^{-1}
// (K_j^{-1} = R^T R), and for a candidate c with k_c = K(X_j, c),
// kd_c = Kd(X_j, c):
//   z_c = R k_c,  zd_c = R kd_c,  M_j = R Kd_j R^T (symmetric),
//   g_c = zd_c - M_j z_c,  E_c = z_c^T M_j z_c,  e_c = -E_c - 2 g_c . z_c,
// the partitioned inverse of eq. piedef applied to K_{j+1} and Kd_{j+1} gives
//   tr W_{j+1}   = tr M_j + e_c / s_c,
//   tr W_{j+1}^2 = |M_j|_F^2 + 2 |g_c|^2 / s_c + e_c^2 / s_c^2,
// with s_c = kappa - z_c . z_c and cov_c = K(c, x) - z_c . z_h as for ALC
// (v_{j+1} = v_j - cov_c^2 / s_c), and d mu_j / dd = zd_h . t - z_h^T M_j t
// with t = R Y_j.  Adding x* (l = z_{x*}, lambda^2 = s*) borders R as for ALC
// and M as M_{j+1} = [[M_j, m], [m^T, mu]] with m = g_{x*} / lambda and
// mu = e_{x*} / s*, so that every candidate's vectors change by
//   w  = (K(c, x*) - l . z_c) / lambda,                   z_c <- [z_c, w],
//   wd = (Kd(c, x*) - l . g_c - (M_j l) . z_c) / lambda,
//   g_c <- [g_c - m w, wd - m . z_c - mu w],  E_c += 2 w m . z_c + mu w^2,
// and |g_c|^2 and g_c . z_c are summed afresh while g_c is rewritten.  A step
// costs a few length-j passes per candidate (O(N' j)); the factor columns of
// z and g live in a per-workgroup global workspace, [entry][position].
//
// One workgroup per location at a time (persistent workgroups stride over the
// locations); lane t owns pool positions t + s TB.  Per step: every wave
// proposes its smallest criterion (ties: smaller design index) and the
// proposing lane publishes that candidate's scalars and coordinates; after a
// barrier wave 0 borders M and works out the shared vectors (l, M_j l, m) and
// the prediction's running terms; after a second barrier every lane updates
// its candidates.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>
#include <mutex>

namespace lagp {

namespace {

constexpr int kMsTB = 256;
constexpr int kMsNW = kMsTB / kWave;
constexpr int kMsS = kMspeNpMax / kMsTB;  // pool positions per lane
constexpr int kMsLd = kMspeNmax + 1;      // row stride of M in LDS
constexpr int kMsPub = 10;                // published scalars per proposal (then p coordinates)

struct MsArgs {
    AlcArgs a;      // a.alc: criterion of each chosen point
    double *ws;     // per workgroup: z columns, then g columns, n * cap doubles each
    int cap;        // positions per column (pool size rounded up to the lanes)
};

__global__ __launch_bounds__(kMsTB) void mspe_kernel(MsArgs x)
{
    const AlcArgs &a = x.a;
    __shared__ double Mm[kMspeNmax * kMsLd];  // M_j, symmetric (row stride kMsLd)
    __shared__ double vl[kMspeNmax], vy[kMspeNmax], vm[kMspeNmax];  // l, M_j l, m of the step
    __shared__ double zh[kMspeNmax], zdh[kMspeNmax], tt[kMspeNmax], pt[kMspeNmax];  // z_h, zd_h, t, M t
    __shared__ double pub[kMsNW][kMsPub + kMspePmax];
    __shared__ double red_s[kMsNW];
    __shared__ int32_t red_i[kMsNW], red_k[kMsNW];
    __shared__ double crit_out[kMspeNmax];
    __shared__ int32_t seldi[kMspeNmax];
    __shared__ double xs[kMspePmax];
    // per-step scalars from wave 0: 1 / lambda, w_h, t_j, mu, |m|^2, coef, dm, T1, T2, v
    __shared__ double sh[10];
    __shared__ int ctl_status;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int p = a.p, n0 = a.n0, n = a.n, Np = a.Np, cap = x.cap;
    const double kappa = 1.0 + a.g, d = a.d, nid = -1.0 / d, id2 = 1.0 / (d * d);
    double *gzc = x.ws + (size_t)blockIdx.x * 2 * n * cap;  // z columns
    double *ggc = gzc + (size_t)n * cap;                    // g columns

    for (int64_t m = blockIdx.x; m < a.M; m += gridDim.x) {
        if (tid == 0) ctl_status = kLocOk;
        if (tid < p) xs[tid] = a.XX[m * p + tid];
        __syncthreads();
        // ---- stage: coordinates centred on x, K(c, x), responses; empty vectors
        double cc[kMsS][kMspePmax];
        double cq[kMsS], sv[kMsS], cv[kMsS], ty[kMsS], ee[kMsS], hh[kMsS], gz[kMsS];
        int32_t di[kMsS];
#pragma unroll
        for (int s = 0; s < kMsS; s++) {
            const int pos = tid + s * kMsTB;
            bool valid = pos < Np;
            const int32_t id = valid ? a.pool[m * Np + pos] : INT32_MAX;
            if (valid && (id < 0 || id >= a.N)) {  // never read outside X
                ctl_status = kLocBadPool;
                valid = false;
            }
            di[s] = valid ? id : INT32_MAX;
            double q = 0.0;
#pragma unroll
            for (int k = 0; k < kMspePmax; k++) {
                cc[s][k] = (valid && k < p) ? a.X[(int64_t)id * p + k] - xs[k] : 0.0;
                q = fma(cc[s][k], cc[s][k], q);
            }
            cq[s] = q;
            cv[s] = valid ? exp(q * nid) : 0.0;  // K(c, x)
            sv[s] = valid ? kappa : -1.0;         // a negative variance marks "not a candidate"
            ty[s] = valid ? a.Y[id] : 0.0;
            ee[s] = hh[s] = gz[s] = 0.0;          // E_c, |g_c|^2, g_c . z_c
        }
        for (int i = tid; i < kMspeNmax * kMsLd; i += kMsTB) Mm[i] = 0.0;
        if (tid < kMspeNmax) zh[tid] = zdh[tid] = tt[tid] = pt[tid] = 0.0;
        if (tid == 0) {
            // 1 / lambda, w_h, t_j, mu, |m|^2 (set per step); coef, dm, T1, T2, v
            for (int q = 0; q < 10; q++) sh[q] = 0.0;
            sh[9] = kappa;
        }
        __syncthreads();
        int status = __builtin_amdgcn_readfirstlane(ctl_status);
        for (int k = 0; k < p; k++)
            if (status == kLocOk && !isfinite(uniform(xs[k]))) status = kLocNonfinite;

        // the scalars of slot s, should it be chosen, into dst
        auto publish = [&](int s, double *dst) {
            dst[0] = sv[s];
            dst[1] = cv[s];
            dst[2] = ty[s];
            dst[3] = ee[s];
            dst[4] = gz[s];
            dst[5] = cq[s];
            for (int k = 0; k < p; k++) dst[kMsPub + k] = cc[s][k];
        };

        int j = 0;
        double psi = 0.0;  // t . t (wave 0)
        for (; status == kLocOk && j < n; j++) {
            // ===== (1) every wave proposes its smallest criterion; one barrier
            if (j >= n0) {
                const double coef = uniform(sh[5]), dm = uniform(sh[6]), T1 = uniform(sh[7]), T2 = uniform(sh[8]);
                const double vj = uniform(sh[9]);
                double bs = -INFINITY;  // minus the criterion
                int32_t bi = INT32_MAX;
                int bk = -1;
#pragma unroll
                for (int s = 0; s < kMsS; s++) {
                    if (sv[s] > 0.0) {
                        const double is = 1.0 / sv[s];
                        const double e = -ee[s] - 2.0 * gz[s];
                        const double tw = T1 + e * is;
                        const double tw2 = T2 + 2.0 * hh[s] * is + e * e * is * is;
                        const double G = 0.5 * (tw2 - tw * tw / (j + 1));
                        const double v1 = vj - cv[s] * cv[s] * is;
                        const double crit = coef * v1 + dm * dm / G;
                        const double sc = (G > 0.0 && isfinite(crit)) ? -crit : -INFINITY;
                        const int32_t id = sc > -INFINITY ? di[s] : INT32_MAX;
                        if (beats(sc, id, bs, bi)) {
                            bs = sc;
                            bi = id;
                            bk = tid + s * kMsTB;
                        }
                    }
                }
                wave_argmax_ballot(bs, bi, bk);
                if (lane == 0) {
                    red_s[w] = bs;
                    red_i[w] = bi;
                    red_k[w] = bk;
                }
                if (bk >= 0 && tid == bk % kMsTB) {
                    const int sb = bk / kMsTB;
#pragma unroll
                    for (int s = 0; s < kMsS; s++)
                        if (s == sb) publish(s, pub[w]);
                }
            } else if (tid == j) {  // the NN start: pool position j, slot 0 of thread j
                publish(0, pub[w]);
                red_i[w] = di[0];
                red_k[w] = j;
            }
            __syncthreads();
            // ===== (2) the winner (smallest criterion, ties to the smaller design index)
            int vw = j / kWave, wpos = j;
            double best = NAN;
            if (j >= n0) {
                double bs = red_s[0];
                int32_t bi = red_i[0];
                vw = 0;
                for (int q = 1; q < kMsNW; q++)
                    if (beats(red_s[q], red_i[q], bs, bi)) {
                        bs = red_s[q];
                        bi = red_i[q];
                        vw = q;
                    }
                if (!(bs > -INFINITY)) {  // no candidate with a finite criterion left
                    status = kLocStepFail;
                    break;
                }
                best = -bs;
                wpos = red_k[vw];
            }
            const double sstar = uniform(pub[vw][0]);
            if (!(sstar > 0.0) || !isfinite(sstar)) {
                status = j < n0 ? kLocInitNotPd : kLocStepFail;
                break;
            }
            if (wpos % kMsTB == tid)  // retire the chosen slot
#pragma unroll
                for (int s = 0; s < kMsS; s++)
                    if (s == wpos / kMsTB) sv[s] = -1.0;
            const double lam = sqrt(sstar), il = 1.0 / lam;
            const double wh = uniform(pub[vw][1]) * il, tj = uniform(pub[vw][2]) * il;
            if (tid == 0) {
                seldi[j] = red_i[vw];
                crit_out[j] = best;
            }
            // ===== (3) wave 0: the shared vectors and scalars of the new design
            if (w == 0) {
                const bool in = lane < j;
                const double l = in ? gzc[(size_t)lane * cap + wpos] : 0.0;   // z_{x*}
                const double gs = in ? ggc[(size_t)lane * cap + wpos] : 0.0;  // g_{x*}
                double yl = 0.0;  // (M_j l)_lane, before M is bordered
                for (int b = 0; b < j; b++) yl = fma(Mm[lane * kMsLd + b], readlane(l, b), yl);
                if (!in) yl = 0.0;
                const double e = -uniform(pub[vw][3]) - 2.0 * uniform(pub[vw][4]);  // e_{x*}
                const double mu = e / sstar, mv = gs * il;
                const double m2 = wave_sum(mv * mv);
                const double qx = uniform(pub[vw][5]);  // |x* - x|^2
                const double kdx = exp(qx * nid) * qx * id2;  // Kd(x*, x)
                // this lane's entries of z_h, zd_h, t and M t, grown by entry j
                double zl = zh[lane], zdl = zdh[lane], tl = tt[lane], pl = pt[lane];
                const double wdh = (kdx - wave_sum(l * zdl)) * il;
                const double mt = wave_sum(mv * tl);
                if (in) pl = fma(mv, tj, pl);
                if (lane == j) {
                    zl = wh;
                    zdl = wdh;
                    tl = tj;
                    pl = fma(mu, tj, mt);
                }
                zh[lane] = zl;
                zdh[lane] = zdl;
                tt[lane] = tl;
                pt[lane] = pl;
                vl[lane] = l;
                vy[lane] = yl;
                vm[lane] = mv;
                if (in) {
                    Mm[lane * kMsLd + j] = mv;
                    Mm[j * kMsLd + lane] = mv;
                }
                if (lane == j) Mm[j * kMsLd + j] = mu;
                psi = fma(tj, tj, psi);
                // d mu_{j+1} / dd = zd_h . t - z_h . (M t) over the grown vectors
                const double dmn = wave_sum(zdl * tl) - wave_sum(zl * pl);
                if (lane == 0) {
                    sh[0] = il;
                    sh[1] = wh;
                    sh[2] = tj;
                    sh[3] = mu;
                    sh[4] = m2;
                    sh[5] = (j + 2) * psi / ((double)(j + 1) * j);  // coef of the next step
                    sh[6] = dmn;
                    sh[7] += mu;                      // tr M_{j+1}
                    sh[8] += 2.0 * m2 + mu * mu;      // |M_{j+1}|_F^2
                    sh[9] = fma(-wh, wh, sh[9]);      // v_{j+1}
                }
            }
            // the chosen point's coordinates (centred) and squared norm
            double xw[kMspePmax];
#pragma unroll
            for (int k = 0; k < kMspePmax; k++) xw[k] = k < p ? uniform(pub[vw][kMsPub + k]) : 0.0;
            const double qw = uniform(pub[vw][5]);
            if (j + 1 == n) break;  // the design is complete
            __syncthreads();
            const double mu = uniform(sh[3]);

            // ===== (4) every candidate: new entries of z and g, g rewritten
#pragma unroll
            for (int s = 0; s < kMsS; s++) {
                if (!(sv[s] > 0.0)) continue;
                const int pos = tid + s * kMsTB;
                double L1 = 0.0, LY = 0.0, A = 0.0, Lg = 0.0;
                for (int e = 0; e < j; e++) {
                    const double z = gzc[(size_t)e * cap + pos], gg = ggc[(size_t)e * cap + pos];
                    const double le = vl[e];
                    L1 = fma(le, z, L1);
                    LY = fma(vy[e], z, LY);
                    A = fma(vm[e], z, A);
                    Lg = fma(le, gg, Lg);
                }
                double dt = 0.0;
#pragma unroll
                for (int k = 0; k < kMspePmax; k++) dt = fma(cc[s][k], xw[k], dt);
                const double r2 = fma(-2.0, dt, cq[s] + qw);  // |c - x*|^2
                const double kc = exp(r2 * nid), kdc = kc * r2 * id2;
                const double wv = (kc - L1) * il;
                const double wd = (kdc - Lg - LY) * il;
                double H = 0.0, GZ = 0.0;
                for (int e = 0; e < j; e++) {
                    const size_t o = (size_t)e * cap + pos;
                    const double gg = fma(-vm[e], wv, ggc[o]);
                    ggc[o] = gg;
                    H = fma(gg, gg, H);
                    GZ = fma(gg, gzc[o], GZ);
                }
                const double gn = wd - A - mu * wv;
                gzc[(size_t)j * cap + pos] = wv;
                ggc[(size_t)j * cap + pos] = gn;
                hh[s] = fma(gn, gn, H);
                gz[s] = fma(gn, wv, GZ);
                ee[s] = fma(mu * wv, wv, fma(2.0 * wv, A, ee[s]));
                sv[s] = fma(-wv, wv, sv[s]);
                cv[s] = fma(-wv, wh, cv[s]);
                ty[s] = fma(-wv, tj, ty[s]);
            }
            __syncthreads();
        }
        __syncthreads();

        // ===== outputs: the design, the criterion of each choice, the prediction
        const int jd = status == kLocOk ? n : j;
        for (int jj = tid; jj < jd; jj += kMsTB) {
            a.sel[m * n + jj] = seldi[jj];
            if (a.alc) a.alc[m * n + jj] = jj >= n0 ? crit_out[jj] : NAN;
        }
        for (int jj = jd + tid; jj < n; jj += kMsTB) {
            a.sel[m * n + jj] = -1;
            if (a.alc) a.alc[m * n + jj] = NAN;
        }
        if (w == 0) {
            const bool ok = status == kLocOk;
            const double zi = lane < n ? zh[lane] : 0.0, ti = lane < n ? tt[lane] : 0.0;
            const double mu = wave_sum(zi * ti), ps = wave_sum(ti * ti), zz = wave_sum(zi * zi);
            if (lane == 0) {
                const double s2 = ps * (kappa - zz) / n;
                if (a.mean) a.mean[m] = ok ? mu : NAN;
                if (a.s2) a.s2[m] = ok ? s2 : NAN;
                if (a.var) a.var[m] = (ok && n > 2) ? s2 * n / (n - 2) : NAN;
                if (a.status) a.status[m] = status;
            }
        }
        __syncthreads();  // LDS is restaged for the next location
    }
}

}  // namespace

int mspe_cap(int Np)
{
    return (Np + kMsTB - 1) / kMsTB * kMsTB;
}

static hipError_t mspe_grid(int64_t M, int64_t *grid)
{
    static std::mutex mu;
    static int cache[64][2];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    int cus = 0, nb = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!cache[dev][0]) {
            e = hipDeviceGetAttribute(&cache[dev][0], hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&cache[dev][1], mspe_kernel, kMsTB, 0);
            if (e != hipSuccess) return e;
        }
        cus = cache[dev][0];
        nb = cache[dev][1];
    }
    const int64_t g = (int64_t)cus * (nb > 0 ? nb : 1);
    *grid = g < M ? g : M;
    return hipSuccess;
}

hipError_t mspe_workspace(int64_t M, int Np, int n, size_t *bytes)
{
    int64_t grid = 0;
    hipError_t e = mspe_grid(M, &grid);
    if (e != hipSuccess) return e;
    *bytes = (size_t)(grid > 0 ? grid : 1) * 2 * n * mspe_cap(Np) * sizeof(double);
    return hipSuccess;
}

hipError_t launch_mspe(const AlcArgs &a, void *ws, size_t ws_bytes, hipStream_t st)
{
    if (a.M == 0) return hipSuccess;
    if (a.p > kMspePmax || a.n > kMspeNmax || a.Np > kMspeNpMax || a.n0 < 2) return hipErrorNotSupported;
    int64_t grid = 0;
    hipError_t e = mspe_grid(a.M, &grid);
    if (e != hipSuccess) return e;
    const size_t need = (size_t)grid * 2 * a.n * mspe_cap(a.Np) * sizeof(double);
    if (!ws || ws_bytes < need) return hipErrorInvalidValue;
    MsArgs x{a, (double *)ws, mspe_cap(a.Np)};
    hipLaunchKernelGGL(mspe_kernel, dim3((unsigned)grid), dim3(kMsTB), 0, st, x);
    return hipGetLastError();
}

}  // namespace lagp
