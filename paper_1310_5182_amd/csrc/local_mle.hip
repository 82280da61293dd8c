// Local likelihood, its derivatives, the local MLE of the lengthscale and
// prediction on a fixed local design (Sec. 2.1 eq. gpk; Fig. 1 steps 3, 5).
//
// One 256-thread workgroup per location; every n x n step is spread over the
// whole workgroup (thread t owns the elements (a, b) with a = t/16 mod 16 and
// b = t mod 16 in steps of 16).  K^{-1} comes from the symmetric sweep
// (Gauss-Jordan on the positive-definite K, pivots in order): with v the
// current row k and p = v_k, every element takes A_ab - v_a v_b / p, row and
// column k become v / p and the pivot -1/p; after all n pivots the matrix is
// -K^{-1}.  It stays symmetric, so each thread keeps its (up to 16) elements
// in registers and only row k travels through LDS: one barrier per pivot.
// The pivots are the Schur complements, so log|K| is the sum of their logs.
// Everything is float64.
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
// tr(A Kd) and tr(A Kdd) are element sums (A and Kd symmetric), and
// tr(A Kd A Kd) = sum_ab (A Kd)_ab (Kd A)_ab, both products formed on the
// matrix cores.
#include "lagp_device.hpp"
#include "lagp_internal.hpp"

#include <math.h>

namespace lagp {

constexpr int kGpThreads = 256;
constexpr int kGpWaves = kGpThreads / kWave;
constexpr int kGpNmax = 64;
constexpr int kGpSlots = 4;  // rotating reduction slots (one barrier per reduction)
constexpr int kGpRed = 8;    // values per reduction

struct GpEval {
    double nll, dd, dg, d2;
    bool ok;
};

// Per-location LDS workspace and the workgroup's view of it.
struct GpBlock {
    double *M1;    // K, then A = K^{-1} (row stride S)
    double *M2;    // squared distances, then Kd
    double *xs;    // design rows [n][p]
    double *ys;    // responses [n]
    double *colk;  // sweep: pivot row (even pivots), then alpha
    double *rowk;  // sweep: pivot row (odd pivots), then Kd alpha
    double *piv;   // sweep pivots
    double (*red)[kGpWaves][kGpRed];
    int S, n, p, tid, lane, w, slot;
    double nll0;  // -lgamma(n/2) + (n/2) log(2 pi), the same at every evaluation

    __device__ double r2(int a, int b) const
    {
        return sqdist_strict(xs + a * p, 1, xs + b * p, 1, p);
    }

    // Block sums of K values (one per thread each); every thread gets them,
    // summed in the same order.  Contains the barrier that publishes them.
    template <int K>
    __device__ void bsum(double (&v)[K])
    {
        static_assert(K <= kGpRed, "reduction width");
        double (*r)[kGpRed] = red[slot];
        slot = (slot + 1) % kGpSlots;
#pragma unroll
        for (int q = 0; q < K; q++) {
            const double s = wave_sum(v[q]);
            if (lane == 0) r[w][q] = s;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < K; q++) {
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < kGpWaves; u++) s += r[u][q];
            v[q] = s;
        }
    }

    // M1 = K -> K^{-1} by the symmetric sweep, elements in registers; M1 must
    // hold K on entry (read once).  False if a pivot is not positive.
    __device__ bool invert()
    {
        const int ta = tid >> 4 & 15, tb = tid & 15;
        double e[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int a = ta + 16 * i, b = tb + 16 * j;
                e[i][j] = (a < n && b < n) ? M1[a * S + b] : 0.0;
            }
        for (int k = 0; k < n; k++) {
            double *v = (k & 1) ? rowk : colk;  // double-buffered pivot row
            const int k0 = k >> 4, kr = k & 15;  // slot and thread row/column of pivot k
            if (ta == kr) {
#pragma unroll
                for (int i = 0; i < 4; i++)
                    if (i == k0)  // uniform
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            if (tb + 16 * j < n) v[tb + 16 * j] = e[i][j];
            }
            __syncthreads();
            const double pk = v[k];
            if (!(pk > 0.0)) return false;  // uniform: every thread reads the same pivot
            const double ip = 1.0 / pk;
            if (tid == 0) piv[k] = pk;
            double va[4], vb[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                va[i] = ta + 16 * i < n ? v[ta + 16 * i] : 0.0;
                vb[i] = tb + 16 * i < n ? v[tb + 16 * i] : 0.0;
            }
            // every element takes A_ab - v_a v_b / p; row and column k are then
            // overwritten (v / p, and -1/p on the diagonal) by the threads that
            // hold them, behind a scalar branch on the slot and a lane mask
            double sa[4];
#pragma unroll
            for (int i = 0; i < 4; i++) sa[i] = va[i] * ip;
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) e[i][j] = fma(-sa[i], vb[j], e[i][j]);
#pragma unroll
            for (int i = 0; i < 4; i++)
                if (i == k0) {  // uniform
                    if (ta == kr)
#pragma unroll
                        for (int j = 0; j < 4; j++) e[i][j] = vb[j] * ip;
                    if (tb == kr)
#pragma unroll
                        for (int r = 0; r < 4; r++) e[r][i] = sa[r];
                    if (ta == kr && tb == kr) e[i][i] = -ip;
                }
        }
        // A = K^{-1} = minus the swept matrix
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int a = ta + 16 * i, b = tb + 16 * j;
                if (a < n && b < n) M1[a * S + b] = -e[i][j];
            }
        __syncthreads();
        return true;
    }

    // order 0: value; 1: + first derivatives; 2: + d2nll/dd2.
    __device__ GpEval eval(double d, double g, int order)
    {
        GpEval e{NAN, NAN, NAN, NAN, false};
        const int ta = tid >> 4 & 15, tb = tid & 15;
        const double nid = -1.0 / d;
        // K into M1; the squared distances are kept in M2 for the derivative pass
        for (int a = ta; a < n; a += 16)
            for (int b = tb; b < n; b += 16) {
                const double q = r2(a, b);
                M2[a * S + b] = q;
                M1[a * S + b] = exp(q * nid) + (a == b ? g : 0.0);
            }
        __syncthreads();
        if (!invert()) return e;
        // alpha = A Y (in colk), psi, log|K|
        double al = 0.0;
        if (tid < n) {
            for (int b = 0; b < n; b++) al = fma(M1[tid * S + b], ys[b], al);
            colk[tid] = al;
        }
        double s0[2] = {tid < n ? ys[tid] * al : 0.0, tid < n ? log(piv[tid]) : 0.0};
        bsum(s0);
        const double psi = s0[0], logdet = s0[1];
        e.nll = nll0 + 0.5 * logdet + 0.5 * n * log(0.5 * psi);
        e.ok = isfinite(e.nll);
        if (order == 0 || !e.ok) return e;

        // Kd into M2 (over the squared distances); traces and quadratic forms in
        // one pass over the elements
        const double d2i = 1.0 / (d * d), d3i = d2i / d;
        double s1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // tr(A Kd), tr(A Kdd), aKda, aKdda, tr A, a.a
        for (int a = ta; a < n; a += 16) {
            const double aa_ = colk[a];
            for (int b = tb; b < n; b += 16) {
                const double q = M2[a * S + b];  // this thread's own element, from the K pass
                const double c = exp(q * nid);
                const double kd = c * q * d2i;
                const double kdd = c * (q * q * d2i * d2i - 2.0 * q * d3i);
                M2[a * S + b] = kd;
                const double ab = M1[a * S + b];
                s1[0] = fma(ab, kd, s1[0]);
                s1[1] = fma(ab, kdd, s1[1]);
                const double ab_ = aa_ * colk[b];
                s1[2] = fma(ab_, kd, s1[2]);
                s1[3] = fma(ab_, kdd, s1[3]);
                if (a == b) s1[4] += ab;
            }
        }
        if (tid < n) s1[5] = colk[tid] * colk[tid];
        bsum(s1);
        const double aKda = s1[2];
        e.dd = 0.5 * s1[0] - 0.5 * n * aKda / psi;
        e.dg = 0.5 * s1[4] - 0.5 * n * s1[5] / psi;
        if (order < 2) return e;

        // v = Kd alpha (in rowk)
        if (tid < n) {
            double v = 0.0;
            for (int b = 0; b < n; b++) v = fma(M2[tid * S + b], colk[b], v);
            rowk[tid] = v;
        }
        __syncthreads();
        // v^T A v
        double s2[2] = {0.0, 0.0};
        if (tid < n) {
            double av = 0.0;
            for (int b = 0; b < n; b++) av = fma(M1[tid * S + b], rowk[b], av);
            s2[0] = rowk[tid] * av;
        }
        // tr(B B) with B = A Kd: since A and Kd are symmetric, B^T = Kd A, so
        // tr(B B) = sum_ab B_ab (Kd A)_ab, and tile (J, I) of that sum equals
        // tile (I, J).  Each wave takes tiles I <= J (16 x 16, zero beyond n) in
        // turn, forms both products on the 16x16x4 float64 MFMA and sums their
        // elementwise product in registers.
        const int T = (n + 15) >> 4;
        const int r16 = lane & 15, k4 = lane >> 4;
        for (int t = w; t < T * (T + 1) / 2; t += kGpWaves) {  // wave-uniform
            int I = 0, J = t;
            while (J >= T - I) J -= T - I++;
            J += I;
            const int a = 16 * I + r16, b = 16 * J + r16;
            // indices past the design are clamped into it for the (unconditional)
            // loads and their values replaced by zero
            const int ah = a < n ? a : n - 1, bh = b < n ? b : n - 1;
            v4d pb = {0.0, 0.0, 0.0, 0.0}, pc = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < 4 * T; kk++) {
                const int c = 4 * kk + k4, ch = c < n ? c : n - 1;
                const bool ac = a < n && c < n, bc = b < n && c < n;
                // A-operand lanes hold row a, column c; B-operand lanes row c, column b
                const double a1 = M1[ah * S + ch], b2 = M2[ch * S + bh], a2 = M2[ah * S + ch], b1 = M1[ch * S + bh];
                pb = __builtin_amdgcn_mfma_f64_16x16x4f64(ac ? a1 : 0.0, bc ? b2 : 0.0, pb, 0, 0, 0);
                pc = __builtin_amdgcn_mfma_f64_16x16x4f64(ac ? a2 : 0.0, bc ? b1 : 0.0, pc, 0, 0, 0);
            }
            const double wt = I == J ? 1.0 : 2.0;
#pragma unroll
            for (int r = 0; r < 4; r++) s2[1] = fma(wt * pb[r], pc[r], s2[1]);
        }
        bsum(s2);
        e.d2 = 0.5 * (s1[1] - s2[1]) - 0.5 * n * ((s1[3] - 2.0 * s2[0]) / psi + aKda * aKda / (psi * psi));
        return e;
    }
};

template <int MODE>
__global__ __launch_bounds__(kGpThreads) void local_gp_kernel(GpArgs a)
{
    extern __shared__ double lds[];
    __shared__ double red[kGpSlots][kGpWaves][kGpRed];
    __shared__ int ctl_bad;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t m = blockIdx.x;
    const int n = a.n, p = a.p, S = n + 1;
    double *base = lds;
    GpBlock W{base,           base + n * S,         base + 2 * n * S,
              base + 2 * n * S + n * p,             base + 2 * n * S + n * p + n,
              base + 2 * n * S + n * p + 2 * n,     base + 2 * n * S + n * p + 3 * n,
              red,            S, n, p, tid, lane, w, 0, -lgamma(0.5 * n) + 0.5 * n * log(2.0 * M_PI)};

    // stage the design rows and responses
    if (tid == 0) ctl_bad = 0;
    __syncthreads();
    if (tid < n) {
        const int32_t di = a.sel[m * n + tid];
        if (di < 0 || di >= a.N) {
            ctl_bad = 1;
        } else {
            for (int k = 0; k < p; k++) W.xs[tid * p + k] = a.X[(int64_t)di * p + k];
            W.ys[tid] = a.Y[di];
        }
    }
    __syncthreads();
    const bool bad_sel = ctl_bad != 0;
    const double g = a.g_arr ? a.g_arr[m] : a.g_scalar;
    const double d_in = a.d_arr ? a.d_arr[m] : a.d_scalar;

    if constexpr (MODE == kGpNll || MODE == kGpBackward) {
        const int order = MODE == kGpNll ? (a.d2 ? 2 : ((a.dd || a.dg) ? 1 : 0)) : 1;
        GpEval e{NAN, NAN, NAN, NAN, false};
        if (!bad_sel && d_in > 0.0 && g > 0.0) e = W.eval(d_in, g, order);
        if (tid == 0) {
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
        if (tid == 0) {
            if (a.d_hat) a.d_hat[m] = d;
            if (a.nll) a.nll[m] = f.nll;
            if (a.iters) a.iters[m] = it;
            if (a.status) a.status[m] = st;
        }
    } else {
        // prediction at XX[m] on the fixed design (eqs. predgp, preds2):
        // mu = h^T A Y, s2 = psi (kappa - h^T A h) / n
        const double *x = a.XX + m * p;
        const double kappa = 1.0 + g;
        double mu = NAN, s2 = NAN;
        int st = bad_sel ? 4 : 0;
        if (!bad_sel) {
            const int ta = tid >> 4 & 15, tb = tid & 15;
            for (int r = ta; r < n; r += 16)
                for (int b = tb; b < n; b += 16) {
                    const double k = exp(-W.r2(r, b) / d_in) + (r == b ? g : 0.0);
                    W.M1[r * S + b] = k;
                    W.M2[r * S + b] = k;  // K itself, kept for the refinement below
                }
            __syncthreads();
            if (!W.invert()) {
                st = 1;
            } else {
                // h in rowk; alpha = A Y (colk) and u = A h (piv) row by row.  The
                // sweep's inverse carries an error of order cond(K) eps, so both
                // solves get one step of iterative refinement against K:
                // alpha += A (Y - K alpha), u += A (h - K u), the residuals kept in
                // the unused last column of M2 and M1 (row stride n + 1).
                if (tid < n) W.rowk[tid] = corr64(sqdist_strict(W.xs + tid * p, 1, x, 1, p), d_in);
                __syncthreads();
                if (tid < n) {
                    double ay = 0.0, ah = 0.0;
                    for (int b = 0; b < n; b++) {
                        ay = fma(W.M1[tid * S + b], W.ys[b], ay);
                        ah = fma(W.M1[tid * S + b], W.rowk[b], ah);
                    }
                    W.colk[tid] = ay;
                    W.piv[tid] = ah;
                }
                __syncthreads();
                if (tid < n) {
                    double ky = 0.0, kh = 0.0;
                    for (int b = 0; b < n; b++) {
                        ky = fma(W.M2[tid * S + b], W.colk[b], ky);
                        kh = fma(W.M2[tid * S + b], W.piv[b], kh);
                    }
                    W.M2[tid * S + n] = W.ys[tid] - ky;
                    W.M1[tid * S + n] = W.rowk[tid] - kh;
                }
                __syncthreads();
                double s[3] = {0.0, 0.0, 0.0};  // h.A.Y, Y.A.Y, h.A.h
                if (tid < n) {
                    double cy = 0.0, ch = 0.0;
                    for (int b = 0; b < n; b++) {
                        cy = fma(W.M1[tid * S + b], W.M2[b * S + n], cy);
                        ch = fma(W.M1[tid * S + b], W.M1[b * S + n], ch);
                    }
                    const double ay = W.colk[tid] + cy, ah = W.piv[tid] + ch;
                    s[0] = W.rowk[tid] * ay;
                    s[1] = W.ys[tid] * ay;
                    s[2] = W.rowk[tid] * ah;
                }
                W.bsum(s);
                mu = s[0];
                s2 = s[1] * (kappa - s[2]) / n;
            }
        }
        if (tid == 0) {
            if (a.mean) a.mean[m] = mu;
            if (a.s2) a.s2[m] = s2;
            if (a.var) a.var[m] = n > 2 ? s2 * n / (n - 2) : NAN;
            if (a.status) a.status[m] = st;
        }
    }
}

size_t local_gp_lds(int n, int p)
{
    return (size_t)(2 * n * (n + 1) + n * p + 4 * n) * sizeof(double);
}

bool local_gp_supported(int n, int p)
{
    return n >= 1 && n <= kGpNmax && p <= kMaxP && local_gp_lds(n, p) <= 160 * 1024;
}

hipError_t launch_local_gp(const GpArgs &a, int mode, hipStream_t st)
{
    if (a.M == 0) return hipSuccess;
    const dim3 grid((unsigned)a.M), block(kGpThreads);
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
