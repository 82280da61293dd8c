// Local likelihood, its derivatives, the local MLE of the lengthscale and
// prediction on a fixed local design (Sec. 2.1 eq. gpk; Fig. 1 steps 3, 5).
//
// One wave per location; lane r owns row r of every n x n matrix (n <= 64).
// The matrices live in LDS with an odd row stride; the wave is its own
// synchronisation domain, so the only ordering needed between lanes is a
// wave-scope fence.  Everything is float64.
//
// Negative log of eq. gpk with K = exp(-D2/d) + g I, A = K^{-1},
// alpha = A Y, psi = Y^T alpha:
//   nll = -lgamma(n/2) + (n/2) log(2 pi) + (1/2) log|K| + (n/2) log(psi/2)
// and with Kd = dK/dd = exp(-D2/d) D2/d^2, Kdd = exp(-D2/d)(D2^2/d^4 - 2 D2/d^3):
//   dnll/dd   = (1/2) tr(A Kd) - (n/2) alpha^T Kd alpha / psi
//   dnll/dg   = (1/2) tr(A)    - (n/2) alpha^T alpha / psi
//   d2nll/dd2 = (1/2) (tr(A Kdd) - tr(A Kd A Kd))
//               - (n/2) ((alpha^T Kdd alpha - 2 (Kd alpha)^T A (Kd alpha)) / psi
//                        + (alpha^T Kd alpha)^2 / psi^2)
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>

namespace lagp {

constexpr int kGpWaves = 1;  // waves (locations) per workgroup
constexpr int kGpNmax = 64;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct GpEval {
    double nll, dd, dg, d2;
    bool ok;
};

// Per-wave LDS workspace.
struct GpWave {
    double *M1;  // K, then its Cholesky factor L (lower), then A = K^{-1}
    double *M2;  // L^{-1}, then scratch
    double *xs;  // design rows [n][p]
    double *ys;  // responses [n]
    int S;       // row stride
    int n, p, lane;

    __device__ double r2(int a, int b) const
    {
        return sqdist_strict(xs + a * p, 1, xs + b * p, 1, p);
    }

    // Cholesky of M1 in place (lower triangle); false if a pivot is not positive.
    __device__ bool cholesky()
    {
        const int i = lane;
        for (int k = 0; k < n; k++) {
            const double akk = M1[k * S + k];
            if (!(akk > 0.0)) return false;
            const double lkk = sqrt(akk);
            double lik = 0.0;
            if (i > k && i < n) {
                lik = M1[i * S + k] / lkk;
                M1[i * S + k] = lik;
            }
            wave_sync();
            if (i == k) M1[k * S + k] = lkk;
            if (i > k && i < n) {
                int c = k + 1;
                for (; c + 4 <= i + 1; c += 4) {
                    const double a0 = M1[i * S + c], a1 = M1[i * S + c + 1];
                    const double a2 = M1[i * S + c + 2], a3 = M1[i * S + c + 3];
                    const double l0 = M1[c * S + k], l1 = M1[(c + 1) * S + k];
                    const double l2 = M1[(c + 2) * S + k], l3 = M1[(c + 3) * S + k];
                    M1[i * S + c] = a0 - lik * l0;
                    M1[i * S + c + 1] = a1 - lik * l1;
                    M1[i * S + c + 2] = a2 - lik * l2;
                    M1[i * S + c + 3] = a3 - lik * l3;
                }
                for (; c <= i; c++) M1[i * S + c] -= lik * M1[c * S + k];
            }
            wave_sync();
        }
        return true;
    }

    // Solve L w = b (b held one entry per lane), returns w in the lane.
    __device__ double forward(double b) const
    {
        double w = 0.0;
        for (int t = 0; t < n; t++) {
            const double wt = readlane(b, t) / M1[t * S + t];
            if (lane == t) w = wt;
            if (lane > t && lane < n) b -= M1[lane * S + t] * wt;
        }
        return w;
    }

    // Solve L^T x = w.
    __device__ double backward(double w) const
    {
        double x = 0.0;
        for (int t = n - 1; t >= 0; t--) {
            const double xt = readlane(w, t) / M1[t * S + t];
            if (lane == t) x = xt;
            if (lane < t) w -= M1[t * S + lane] * xt;
        }
        return x;
    }

    // M2 = L^{-1} (lower), row by row: lane j computes entry (i, j), j < i.
    __device__ void invert_l()
    {
        const int j = lane;
        for (int i = 0; i < n; i++) {
            const double lii = M1[i * S + i];
            double s = 0.0;
            if (j < i) {
#pragma unroll 4
                for (int t = j; t < i; t++) s += M1[i * S + t] * M2[t * S + j];
                M2[i * S + j] = -s / lii;
            } else if (j == i) {
                M2[i * S + i] = 1.0 / lii;
            } else if (j < n) {
                M2[i * S + j] = 0.0;
            }
            wave_sync();
        }
    }

    // M1 = A = L^{-T} L^{-1}: lane a accumulates row a, A_ab = sum_{t >= a, b} Li_ta Li_tb,
    // reading row t of L^{-1} as broadcasts.
    __device__ void form_inverse()
    {
        const int a = lane;
        double row[kGpNmax];
#pragma unroll
        for (int b = 0; b < kGpNmax; b++) row[b] = 0.0;
        for (int t = 0; t < n; t++) {
            const double lta = (a < n && a <= t) ? M2[t * S + a] : 0.0;
#pragma unroll
            for (int b = 0; b < kGpNmax; b++)
                if (b <= t) row[b] += lta * M2[t * S + b];
        }
        wave_sync();
        if (a < n)
#pragma unroll
            for (int b = 0; b < kGpNmax; b++)
                if (b < n) M1[a * S + b] = row[b];
        wave_sync();
    }

    // order 0: value; 1: + first derivatives; 2: + d2nll/dd2.
    __device__ GpEval eval(double d, double g, int order)
    {
        GpEval e{NAN, NAN, NAN, NAN, false};
        const int a = lane;
        for (int b = 0; b < n; b++)
            if (a < n) M1[a * S + b] = exp(-r2(a, b) / d) + (a == b ? g : 0.0);
        wave_sync();
        if (!cholesky()) return e;
        const double ya = a < n ? ys[a] : 0.0;
        const double w = forward(ya);
        const double alpha = backward(w);
        const double psi = wave_sum(ya * alpha);
        const double logdet = 2.0 * wave_sum(a < n ? log(M1[a * S + a]) : 0.0);
        e.nll = -lgamma(0.5 * n) + 0.5 * n * log(2.0 * M_PI) + 0.5 * logdet + 0.5 * n * log(0.5 * psi);
        e.ok = isfinite(e.nll);
        if (order == 0 || !e.ok) return e;

        invert_l();
        form_inverse();  // M1 = A
        // row a of Kd and Kdd on the fly; traces and quadratic forms
        double tr_akd = 0.0, tr_akdd = 0.0, kda = 0.0, kdda = 0.0;
        const double d2i = 1.0 / (d * d);
        for (int b = 0; b < n; b++) {
            const double alb = readlane(alpha, b);
            if (a < n) {
                const double q = r2(a, b);
                const double c = exp(-q / d);
                const double kd = c * q * d2i;
                const double kdd = c * (q * q * d2i * d2i - 2.0 * q * d2i / d);
                const double ab = M1[a * S + b];
                tr_akd += ab * kd;
                tr_akdd += ab * kdd;
                kda += kd * alb;
                kdda += kdd * alb;
            }
        }
        const double trA = wave_sum(a < n ? M1[a * S + a] : 0.0);
        const double aa = wave_sum(alpha * alpha);
        const double aKda = wave_sum(alpha * kda);
        e.dd = 0.5 * wave_sum(tr_akd) - 0.5 * n * aKda / psi;
        e.dg = 0.5 * trA - 0.5 * n * aa / psi;
        if (order < 2) return e;

        // (Kd alpha)^T A (Kd alpha): v = Kd alpha is `kda` in the lanes
        double av = 0.0;
        for (int b = 0; b < n; b++) {
            const double vb = readlane(kda, b);
            if (a < n) av += M1[a * S + b] * vb;
        }
        const double vAv = wave_sum(kda * av);
        const double aKdda = wave_sum(alpha * kdda);
        // tr(A Kd A Kd) = sum_ab B_ab B_ba with B = A Kd: M2 <- Kd, row a of B in
        // registers (row c of Kd read as broadcasts), B back into M2, then columns
        if (a < n)
            for (int b = 0; b < n; b++) {
                const double q = r2(a, b);
                M2[a * S + b] = exp(-q / d) * q * d2i;
            }
        wave_sync();
        double brow[kGpNmax];
#pragma unroll
        for (int b = 0; b < kGpNmax; b++) brow[b] = 0.0;
        for (int c = 0; c < n; c++) {
            const double aac = a < n ? M1[a * S + c] : 0.0;
#pragma unroll
            for (int b = 0; b < kGpNmax; b++)
                if (b < n) brow[b] += aac * M2[c * S + b];
        }
        wave_sync();
        if (a < n)
#pragma unroll
            for (int b = 0; b < kGpNmax; b++)
                if (b < n) M2[a * S + b] = brow[b];
        wave_sync();
        double trbb = 0.0;
        if (a < n)
            for (int b = 0; b < n; b++) trbb += M2[a * S + b] * M2[b * S + a];
        const double trBB = wave_sum(trbb);
        e.d2 = 0.5 * (wave_sum(tr_akdd) - trBB) - 0.5 * n * ((aKdda - 2.0 * vAv) / psi + aKda * aKda / (psi * psi));
        return e;
    }
};


template <int MODE>
__global__ __launch_bounds__(kGpWaves *kWave) void local_gp_kernel(GpArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * kGpWaves + (threadIdx.x >> 6);
    if (m >= a.M) return;
    const int n = a.n, p = a.p, S = n + 1;
    double *base = lds + (size_t)(threadIdx.x >> 6) * (2 * n * S + n * p + n);
    GpWave W{base, base + n * S, base + 2 * n * S, base + 2 * n * S + n * p, S, n, p, lane};

    // stage the design rows and responses
    int bad = 0;
    if (lane < n) {
        const int32_t di = a.sel[m * n + lane];
        if (di < 0 || di >= a.N) {
            bad = 1;
        } else {
            for (int k = 0; k < p; k++) W.xs[lane * p + k] = a.X[(int64_t)di * p + k];
            W.ys[lane] = a.Y[di];
        }
    }
    wave_sync();
    const bool bad_sel = __ballot(bad) != 0;
    const double g = a.g_arr ? a.g_arr[m] : a.g_scalar;
    const double d_in = a.d_arr ? a.d_arr[m] : a.d_scalar;

    if constexpr (MODE == kGpNll || MODE == kGpBackward) {
        const int order = MODE == kGpNll ? (a.d2 ? 2 : ((a.dd || a.dg) ? 1 : 0)) : 1;
        GpEval e{NAN, NAN, NAN, NAN, false};
        if (!bad_sel && d_in > 0.0 && g > 0.0) e = W.eval(d_in, g, order);
        if (lane == 0) {
            if constexpr (MODE == kGpNll) {
                if (a.nll) a.nll[m] = e.nll;
                if (a.dd) a.dd[m] = e.dd;
                if (a.dg) a.dg[m] = e.dg;
                if (a.d2) a.d2[m] = e.d2;
            } else {
                const double go = a.grad_out ? a.grad_out[m] : 1.0;
                if (a.dd) a.dd[m] = go * e.dd;
                if (a.dg) a.dg[m] = go * e.dg;
            }
            if (a.status) a.status[m] = bad_sel ? 4 : (e.ok ? 0 : 1);
        }
    } else if constexpr (MODE == kGpMle) {
        // projected Newton on [dmin, dmax] with backtracking (the reading of
        // Fig. 1 step 3 used throughout; same rule as the CPU reference)
        double d = fmin(fmax(d_in, a.dmin), a.dmax);
        int st = bad_sel ? 4 : 2, it = 0;
        GpEval f{NAN, NAN, NAN, NAN, false};
        if (!bad_sel) {
            f = W.eval(d, g, 2);
            if (!f.ok) st = 1;
        }
        if (st == 2) {
            for (it = 0; it < a.maxit; it++) {
                const double gr = f.dd, h = f.d2;
                if (fabs(gr) <= 1e-10 || (d <= a.dmin && gr > 0.0) || (d >= a.dmax && gr < 0.0)) {
                    st = 0;
                    break;
                }
                double step = h > 0.0 ? -gr / h : (gr > 0.0 ? -0.1 * d : 0.1 * d);
                double dn = d;
                bool ok = false;
                GpEval ft{NAN, NAN, NAN, NAN, false};
                for (int half = 0; half < 40; half++) {
                    dn = fmin(fmax(d + step, a.dmin), a.dmax);
                    ft = W.eval(dn, g, 2);
                    if (ft.ok && ft.nll <= f.nll + 1e-4 * gr * (dn - d)) {
                        ok = true;
                        break;
                    }
                    step *= 0.5;
                }
                if (!ok) {
                    st = 3;
                    break;
                }
                const double moved = fabs(dn - d);
                d = dn;
                f = ft;
                if (moved <= 1e-10 * d) {
                    st = 0;
                    it++;
                    break;
                }
            }
        }
        if (lane == 0) {
            if (a.d_hat) a.d_hat[m] = d;
            if (a.nll) a.nll[m] = f.nll;
            if (a.iters) a.iters[m] = it;
            if (a.status) a.status[m] = st;
        }
    } else {
        // prediction at XX[m] on the fixed design (eqs. predgp, preds2)
        const double *x = a.XX + m * p;
        const double kappa = 1.0 + g;
        double mu = NAN, s2 = NAN;
        int st = bad_sel ? 4 : 0;
        if (!bad_sel) {
            const int r = lane;
            for (int b = 0; b < n; b++)
                if (r < n) W.M1[r * S + b] = exp(-W.r2(r, b) / d_in) + (r == b ? g : 0.0);
            wave_sync();
            if (!W.cholesky()) {
                st = 1;
            } else {
                const double ya = r < n ? W.ys[r] : 0.0;
                const double h = r < n ? corr64(sqdist_strict(W.xs + r * p, 1, x, 1, p), d_in) : 0.0;
                const double alpha = W.backward(W.forward(ya));
                const double zh = W.forward(h);
                const double psi = wave_sum(ya * alpha);
                mu = wave_sum(h * alpha);
                s2 = psi * (kappa - wave_sum(zh * zh)) / n;
            }
        }
        if (lane == 0) {
            if (a.mean) a.mean[m] = mu;
            if (a.s2) a.s2[m] = s2;
            if (a.var) a.var[m] = n > 2 ? s2 * n / (n - 2) : NAN;
            if (a.status) a.status[m] = st;
        }
    }
}

size_t local_gp_lds(int n, int p)
{
    return (size_t)kGpWaves * (2 * n * (n + 1) + n * p + n) * sizeof(double);
}

bool local_gp_supported(int n, int p)
{
    return n >= 1 && n <= kGpNmax && p <= kMaxP && local_gp_lds(n, p) <= 160 * 1024;
}

hipError_t launch_local_gp(const GpArgs &a, int mode, hipStream_t st)
{
    if (a.M == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.M + kGpWaves - 1) / kGpWaves)), block(kGpWaves * kWave);
    const size_t lds = local_gp_lds(a.n, a.p);
    if (lds > 64 * 1024) {  // above the default dynamic-LDS limit
        hipError_t e = hipSuccess;
        switch (mode) {
        case kGpNll:
            e = hipFuncSetAttribute((const void *)local_gp_kernel<kGpNll>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            break;
        case kGpBackward:
            e = hipFuncSetAttribute((const void *)local_gp_kernel<kGpBackward>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            break;
        case kGpMle:
            e = hipFuncSetAttribute((const void *)local_gp_kernel<kGpMle>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            break;
        default:
            e = hipFuncSetAttribute((const void *)local_gp_kernel<kGpPredict>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        }
        if (e != hipSuccess) return e;
    }
    switch (mode) {
    case kGpNll:
        hipLaunchKernelGGL(local_gp_kernel<kGpNll>, grid, block, lds, st, a);
        break;
    case kGpBackward:
        hipLaunchKernelGGL(local_gp_kernel<kGpBackward>, grid, block, lds, st, a);
        break;
    case kGpMle:
        hipLaunchKernelGGL(local_gp_kernel<kGpMle>, grid, block, lds, st, a);
        break;
    default:
        hipLaunchKernelGGL(local_gp_kernel<kGpPredict>, grid, block, lds, st, a);
    }
    return hipGetLastError();
}

}  // namespace lagp
