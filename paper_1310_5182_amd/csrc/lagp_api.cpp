// C ABI of the local approximate GP library (declarations in lagp_alc.h).
// Host side only: argument validation, dispatch to the kernel launchers.
#include "lagp_alc.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "lagp_internal.hpp"

namespace {

thread_local char g_err[512] = "";

lagp_status fail(lagp_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

lagp_status ok()
{
    g_err[0] = '\0';
    return LAGP_OK;
}

}  // namespace

int lagp::set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

namespace {

lagp_status hip_fail(hipError_t e, const char *what)
{
    return fail(LAGP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

lagp_status check_common(const double *X, int64_t N, int32_t p, const double *XX, int64_t M, int32_t Np)
{
    if (M < 0) return fail(LAGP_EINVAL, "M = %lld < 0", (long long)M);
    if (p < 1) return fail(LAGP_EINVAL, "p = %d < 1", p);
    if (p > lagp::kMaxP) return fail(LAGP_EUNSUPPORTED, "p = %d > %d", p, lagp::kMaxP);
    if (N < 1 || N >= (int64_t)1 << 31) return fail(LAGP_EINVAL, "N = %lld outside [1, 2^31)", (long long)N);
    if (Np < 1 || Np > N) return fail(LAGP_EINVAL, "Np = %d outside [1, N = %lld]", Np, (long long)N);
    if (M > 0 && (!X || !XX)) return fail(LAGP_EINVAL, "X and XX must be non-NULL");
    if (M > (int64_t)0x7fffffff) return fail(LAGP_EUNSUPPORTED, "M = %lld exceeds one launch", (long long)M);
    return LAGP_OK;
}

lagp_status check_alc(const double *Y, int32_t Np, int32_t n0, int32_t n, double d, double g,
                      int32_t precision, const int32_t *sel, int64_t M)
{
    if (precision != LAGP_FP64 && precision != LAGP_MIXED && precision != LAGP_FP64_REFORM)
        return fail(LAGP_EINVAL, "precision = %d is not LAGP_FP64, LAGP_MIXED or LAGP_FP64_REFORM", precision);
    if (!(n0 >= 1 && n0 <= n && n <= Np))
        return fail(LAGP_EINVAL, "need 1 <= n0 <= n <= Np (n0 = %d, n = %d, Np = %d)", n0, n, Np);
    if (!(d > 0.0) || !isfinite(d)) return fail(LAGP_EINVAL, "lengthscale d must be finite and > 0");
    if (!(g > 0.0) || !isfinite(g)) return fail(LAGP_EINVAL, "nugget g must be finite and > 0");
    if (M > 0 && (!Y || !sel)) return fail(LAGP_EINVAL, "Y and sel must be non-NULL");
    return LAGP_OK;
}

}  // namespace

extern "C" {

lagp_status lagp_nn_pool(const double *X, int64_t N, int32_t p, const double *XX, int64_t M,
                         int32_t Np, int32_t *pool, void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np);
    if (s != LAGP_OK) return s;
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (lagp::nn_pool_cap(Np) == 0) return fail(LAGP_EUNSUPPORTED, "Np = %d too large for the pool kernel", Np);
    if (M == 0) return ok();
    hipError_t e = lagp::launch_nn_pool(X, N, p, XX, M, Np, pool, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "nn_pool launch");
    return ok();
}

lagp_status lagp_nn_pool_workspace(int64_t N, int32_t p, int64_t M, size_t *bytes)
{
    if (!bytes) return fail(LAGP_EINVAL, "bytes must be non-NULL");
    if (M < 0) return fail(LAGP_EINVAL, "M = %lld < 0", (long long)M);
    if (p < 1) return fail(LAGP_EINVAL, "p = %d < 1", p);
    if (p > lagp::kMaxP) return fail(LAGP_EUNSUPPORTED, "p = %d > %d", p, lagp::kMaxP);
    if (N < 1 || N >= (int64_t)1 << 31) return fail(LAGP_EINVAL, "N = %lld outside [1, 2^31)", (long long)N);
    *bytes = lagp::nn_pool_workspace(N, p, M);
    return ok();
}

lagp_status lagp_nn_pool_ws(const double *X, int64_t N, int32_t p, const double *XX, int64_t M,
                            int32_t Np, int32_t *pool, void *workspace, size_t workspace_bytes,
                            void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np);
    if (s != LAGP_OK) return s;
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (lagp::nn_pool_cap(Np) == 0) return fail(LAGP_EUNSUPPORTED, "Np = %d too large for the pool kernel", Np);
    if (M == 0) return ok();
    if (!workspace || ((uintptr_t)workspace & 15) || workspace_bytes < lagp::nn_pool_workspace(N, p, M))
        return fail(LAGP_EWORKSPACE, "workspace must be 16-byte aligned and hold %zu bytes",
                    lagp::nn_pool_workspace(N, p, M));
    hipError_t e = lagp::launch_nn_grid(X, N, p, XX, M, Np, pool, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "nn_pool launch");
    return ok();
}

lagp_status lagp_nn_pool_grouped(const double *X, int64_t N, int32_t p, const double *XX, int64_t M, int32_t Np,
                                 int32_t group, int32_t *pool, void *workspace, size_t workspace_bytes, void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np);
    if (s != LAGP_OK) return s;
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (group != 1 && group != 2 && group != 4) return fail(LAGP_EINVAL, "group = %d is not 1, 2 or 4", group);
    if (lagp::nn_pool_cap(Np) == 0) return fail(LAGP_EUNSUPPORTED, "Np = %d too large for the pool kernel", Np);
    if (group > 1 && (1 << (lagp::nn_grid_groups(p, Np) - 1)) < group)
        return fail(LAGP_EUNSUPPORTED, "no grouping of %d locations for p = %d, Np = %d", group, p, Np);
    if (M == 0) return ok();
    if (!workspace || ((uintptr_t)workspace & 15) || workspace_bytes < lagp::nn_pool_workspace(N, p, M))
        return fail(LAGP_EWORKSPACE, "workspace must be 16-byte aligned and hold %zu bytes",
                    lagp::nn_pool_workspace(N, p, M));
    hipError_t e = lagp::launch_nn_grid(X, N, p, XX, M, Np, pool, workspace, (hipStream_t)stream, group);
    if (e != hipSuccess) return hip_fail(e, "nn_pool launch");
    return ok();
}

lagp_status lagp_nn_pool_static(const double *X, int64_t N, int32_t p, const double *XX, int64_t M,
                                int32_t Np, int32_t *pool, void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np);
    if (s != LAGP_OK) return s;
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (lagp::nn_pool_cap(Np) == 0) return fail(LAGP_EUNSUPPORTED, "Np = %d too large for the pool kernel", Np);
    const size_t need = lagp::nn_pool_workspace(N, p, M);
    if (need > lagp::kNnStaticScratch)
        return fail(LAGP_EWORKSPACE, "N = %lld, p = %d, M = %lld need %zu bytes of scratch; the static scratch holds %zu",
                    (long long)N, p, (long long)M, need, lagp::kNnStaticScratch);
    if (M == 0) return ok();
    void *ws = nullptr;
    hipError_t e = lagp::nn_static_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, "static scratch address");
    e = lagp::launch_nn_grid(X, N, p, XX, M, Np, pool, ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "nn_pool launch");
    return ok();
}

lagp_status lagp_alc_scores(const double *Xj, int32_t j, int32_t p, const double *Kinv, const double *Xc,
                            int64_t Nc, const double *x, const double *h, double d, double g,
                            int32_t precision, double *delta, void *stream)
{
    if (precision != LAGP_FP64 && precision != LAGP_MIXED)
        return fail(LAGP_EINVAL, "precision = %d is not LAGP_FP64 or LAGP_MIXED", precision);
    if (j < 1) return fail(LAGP_EINVAL, "j = %d < 1", j);
    if (j > lagp::kScoresJbig) return fail(LAGP_EUNSUPPORTED, "j = %d > %d", j, lagp::kScoresJbig);
    if (p < 1) return fail(LAGP_EINVAL, "p = %d < 1", p);
    if (p > lagp::kMaxP) return fail(LAGP_EUNSUPPORTED, "p = %d > %d", p, lagp::kMaxP);
    if (Nc < 0) return fail(LAGP_EINVAL, "Nc = %lld < 0", (long long)Nc);
    if (!(d > 0.0) || !isfinite(d)) return fail(LAGP_EINVAL, "lengthscale d must be finite and > 0");
    if (!(g > 0.0) || !isfinite(g)) return fail(LAGP_EINVAL, "nugget g must be finite and > 0");
    if (Nc == 0) return ok();
    if (!Xj || !Kinv || !Xc || !x || !h || !delta)
        return fail(LAGP_EINVAL, "Xj, Kinv, Xc, x, h and delta must be non-NULL");
    hipError_t e = lagp::launch_alc_scores(Xj, j, p, Kinv, Xc, Nc, x, h, d, g, precision == LAGP_MIXED, delta,
                                           (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "alc_scores launch");
    return ok();
}

lagp_status lagp_alc_from_pool(const double *X, const double *Y, int64_t N, int32_t p,
                               const double *XX, int64_t M, const int32_t *pool, int32_t Np,
                               int32_t n0, int32_t n, double d, double g, int32_t precision,
                               double *mean, double *s2, double *var, int32_t *sel, double *alc,
                               double *alc32, int32_t *status, int32_t *guard, void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np);
    if (s != LAGP_OK) return s;
    s = check_alc(Y, Np, n0, n, d, g, precision, sel, M);
    if (s != LAGP_OK) return s;
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (!lagp::alc_supported(precision, p, Np, n))
        return fail(LAGP_EUNSUPPORTED, "no schedule for p = %d, Np = %d, n = %d, precision = %d", p, Np, n,
                    precision);
    if (M == 0) return ok();
    lagp::AlcArgs a{X, Y, N, p, XX, M, pool, Np, n0, n, d, g, mean, s2, var, sel, alc, alc32, status, guard};
    hipError_t e = lagp::launch_alc(a, precision, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "alc launch");
    return ok();
}

lagp_status lagp_mspe_workspace(int64_t M, int32_t Np, int32_t n, size_t *bytes)
{
    if (!bytes) return fail(LAGP_EINVAL, "bytes must be non-NULL");
    if (M < 0) return fail(LAGP_EINVAL, "M = %lld < 0", (long long)M);
    if (Np < 1 || n < 1) return fail(LAGP_EINVAL, "Np = %d and n = %d must be >= 1", Np, n);
    if (Np > lagp::kMspeNpMax || n > lagp::kMspeNmax)
        return fail(LAGP_EUNSUPPORTED, "MSPE designs need Np <= %d and n <= %d", lagp::kMspeNpMax, lagp::kMspeNmax);
    if (M == 0) {
        *bytes = 0;
        return ok();
    }
    hipError_t e = lagp::mspe_workspace(M, Np, n, bytes);
    if (e != hipSuccess) return hip_fail(e, "workspace query");
    return ok();
}

lagp_status lagp_mspe_from_pool(const double *X, const double *Y, int64_t N, int32_t p, const double *XX,
                                int64_t M, const int32_t *pool, int32_t Np, int32_t n0, int32_t n, double d,
                                double g, double *mean, double *s2, double *var, int32_t *sel, double *crit,
                                int32_t *status, void *workspace, size_t workspace_bytes, void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np);
    if (s != LAGP_OK) return s;
    s = check_alc(Y, Np, n0, n, d, g, LAGP_FP64, sel, M);
    if (s != LAGP_OK) return s;
    if (n0 < 2) return fail(LAGP_EINVAL, "MSPE designs need n0 >= 2 (eq. newv divides by j (j - 1))");
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (p > lagp::kMspePmax || Np > lagp::kMspeNpMax || n > lagp::kMspeNmax)
        return fail(LAGP_EUNSUPPORTED, "MSPE designs need p <= %d, Np <= %d and n <= %d", lagp::kMspePmax,
                    lagp::kMspeNpMax, lagp::kMspeNmax);
    if (M == 0) return ok();
    size_t need = 0;
    hipError_t e = lagp::mspe_workspace(M, Np, n, &need);
    if (e != hipSuccess) return hip_fail(e, "workspace query");
    if (!workspace || ((uintptr_t)workspace & 255) || workspace_bytes < need)
        return fail(LAGP_EWORKSPACE, "workspace must be 256-byte aligned and hold %zu bytes (%zu given)", need,
                    workspace_bytes);
    lagp::AlcArgs a{X, Y, N, p, XX, M, pool, Np, n0, n, d, g, mean, s2, var, sel, crit, nullptr, status, nullptr};
    e = lagp::launch_mspe(a, workspace, workspace_bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mspe launch");
    return ok();
}

}  // extern "C"

namespace {

size_t align256(size_t v)
{
    return (v + 255) & ~(size_t)255;
}

// Workspace parts of a problem: [queues / spilled columns][grid of the design][pools].
struct WsLayout {
    size_t alc = 0, nn = 0, pool = 0;
    size_t total() const { return align256(alc) + align256(nn) + align256(pool); }
};

// Checks every argument of lagp_alc_predict / lagp_alc_workspace that the host
// can see and works out the path and its workspace.  `out` may be NULL (the
// workspace query).
lagp_status resolve(const lagp_problem *pr, const lagp_outputs *out, lagp::PathArgs *P, WsLayout *L)
{
    if (!pr) return fail(LAGP_EINVAL, "problem must be non-NULL");
    if (pr->struct_size != sizeof(lagp_problem))
        return fail(LAGP_EINVAL, "lagp_problem.struct_size = %u, this library's is %zu (ABI version %d)",
                    pr->struct_size, sizeof(lagp_problem), LAGP_ABI_VERSION);
    if (out && out->struct_size != sizeof(lagp_outputs))
        return fail(LAGP_EINVAL, "lagp_outputs.struct_size = %u, this library's is %zu (ABI version %d)",
                    out->struct_size, sizeof(lagp_outputs), LAGP_ABI_VERSION);
    if (pr->flags & ~(LAGP_NORMALIZE_ALC | LAGP_NN_BRUTE))
        return fail(LAGP_EINVAL, "unknown flags 0x%x", pr->flags & ~(LAGP_NORMALIZE_ALC | LAGP_NN_BRUTE));
    if (pr->reserved != 0 || (out && out->reserved != 0)) return fail(LAGP_EINVAL, "reserved fields must be 0");
    lagp_status s = check_common(pr->X, pr->N, pr->p, pr->XX, pr->M, pr->Np);
    if (s != LAGP_OK) return s;
    const int prec = pr->precision;
    const bool uniform = !pr->n_per && !pr->Np_per && !pr->d_per && !(out && out->sel_off);
    s = check_alc(pr->Y, pr->Np, pr->n0, pr->n, pr->d, pr->g, prec, out ? out->sel : nullptr, out ? pr->M : 0);
    if (s != LAGP_OK) return s;
    if ((pr->flags & LAGP_NORMALIZE_ALC) && pr->n0 < 3)
        return fail(LAGP_EINVAL, "LAGP_NORMALIZE_ALC divides by j - 2: needs n0 >= 3 (n0 = %d)", pr->n0);
    if (lagp::nn_pool_cap(pr->Np) == 0)
        return fail(LAGP_EUNSUPPORTED, "Np = %d too large for the pool kernel", pr->Np);
    if (pr->d_sep) {
        if (prec != LAGP_FP64) return fail(LAGP_EUNSUPPORTED, "the separable kernel (d_sep) needs LAGP_FP64");
        if (pr->d_per) return fail(LAGP_EINVAL, "d_sep and d_per exclude each other");
    }
    // which ALC launch: the uniform kernels, or the cost-ordered queues
    bool queued;
    if (prec == LAGP_FP64_REFORM) {
        if (!uniform) return fail(LAGP_EUNSUPPORTED, "LAGP_FP64_REFORM needs uniform n, N' and d");
        if (!lagp::alc_supported(prec, pr->p, pr->Np, pr->n))
            return fail(LAGP_EUNSUPPORTED, "no schedule for p = %d, Np = %d, n = %d, precision = %d", pr->p,
                        pr->Np, pr->n, prec);
        queued = false;
    } else {
        // the separable kernel lives in the incremental kernel, uniform or queued
        queued = !uniform || (pr->d_sep ? !lagp::alc_inc_supported(pr->p, pr->Np, pr->n)
                                        : !lagp::alc_supported(prec, pr->p, pr->Np, pr->n));
        if (queued && !lagp::alc_uneven_supported(pr->p, pr->Np, pr->n))
            return fail(LAGP_EUNSUPPORTED, "no schedule for p = %d, Np = %d, n = %d", pr->p, pr->Np, pr->n);
    }
    WsLayout l;
    if (queued) {
        hipError_t e = lagp::alc_uneven_workspace(pr->p, pr->M, pr->Np, pr->n, &l.alc);
        if (e != hipSuccess) return hip_fail(e, "workspace query");
    }
    if (!(pr->flags & LAGP_NN_BRUTE)) l.nn = lagp::nn_pool_workspace(pr->N, pr->p, pr->M);
    l.pool = (size_t)pr->M * (size_t)pr->Np * 4;
    *L = l;
    if (P) {
        lagp::PathArgs q;
        lagp::AlcArgs &a = q.a;
        a = lagp::AlcArgs{pr->X, pr->Y, pr->N, pr->p, pr->XX, pr->M, nullptr, pr->Np, pr->n0, pr->n, pr->d, pr->g,
                          nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        if (out) {
            a.mean = out->mean;
            a.s2 = out->s2;
            a.var = out->var;
            a.sel = out->sel;
            a.alc = out->alc;
            a.alc32 = out->alc32;
            a.status = out->status;
            a.guard = out->guard;
            a.pool = q.pool = out->pool;
            a.sel_off = out->sel_off;
        }
        a.n_per = pr->n_per;
        a.Np_per = pr->Np_per;
        a.d_per = pr->d_per;
        a.dsep = pr->d_sep;
        a.normalize = (pr->flags & LAGP_NORMALIZE_ALC) != 0;
        q.precision = prec;
        q.nn_brute = (pr->flags & LAGP_NN_BRUTE) != 0;
        q.uniform = !queued;
        *P = q;
    }
    return LAGP_OK;
}

// Points the path at its parts of the workspace.
lagp_status carve(lagp::PathArgs *P, const WsLayout &l, void *ws, size_t ws_bytes)
{
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < l.total())
        return fail(LAGP_EWORKSPACE, "workspace must be 256-byte aligned and hold %zu bytes (%zu given)", l.total(),
                    ws_bytes);
    char *b = (char *)ws;
    P->alc_ws = l.alc ? b : nullptr;
    P->alc_ws_bytes = l.alc;
    P->nn_ws = l.nn ? b + align256(l.alc) : nullptr;
    if (!P->pool) P->a.pool = P->pool = (int32_t *)(b + align256(l.alc) + align256(l.nn));
    return LAGP_OK;
}

}  // namespace

lagp_status lagp::prepare_path(const lagp_problem *prob, const lagp_outputs *out, void *ws, size_t ws_bytes,
                               PathArgs *P)
{
    if (!out) return fail(LAGP_EINVAL, "outputs must be non-NULL");
    WsLayout l;
    lagp_status s = resolve(prob, out, P, &l);
    if (s != LAGP_OK) return s;
    return carve(P, l, ws, ws_bytes);
}

extern "C" {

lagp_status lagp_alc_workspace(const lagp_problem *prob, size_t *bytes)
{
    if (!bytes) return fail(LAGP_EINVAL, "bytes must be non-NULL");
    WsLayout l;
    lagp_status s = resolve(prob, nullptr, nullptr, &l);
    if (s != LAGP_OK) return s;
    *bytes = l.total();
    return ok();
}

lagp_status lagp_alc_predict(const lagp_problem *prob, const lagp_outputs *out, void *workspace,
                             size_t workspace_bytes, void *stream)
{
    if (!out) return fail(LAGP_EINVAL, "outputs must be non-NULL");
    lagp::PathArgs P;
    WsLayout l;
    lagp_status s = resolve(prob, out, &P, &l);
    if (s != LAGP_OK) return s;
    if (prob->M == 0) return ok();
    if ((s = carve(&P, l, workspace, workspace_bytes)) != LAGP_OK) return s;
    hipError_t e = lagp::run_path(P, -1, -1, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "alc_predict launch");
    return ok();
}

int32_t lagp_abi_version(void)
{
    return LAGP_ABI_VERSION;
}

lagp_status lagp_alc_uneven_workspace(int32_t p, int64_t M, int32_t Np_max, int32_t n_max, size_t *bytes)
{
    if (!bytes) return fail(LAGP_EINVAL, "bytes must be non-NULL");
    if (M < 0 || p < 1 || Np_max < 1 || n_max < 1)
        return fail(LAGP_EINVAL, "need M >= 0, p >= 1, Np_max >= 1, n_max >= 1");
    if (!lagp::alc_uneven_supported(p, Np_max, n_max))
        return fail(LAGP_EUNSUPPORTED, "no schedule for p = %d, Np_max = %d, n_max = %d", p, Np_max, n_max);
    hipError_t e = lagp::alc_uneven_workspace(p, M, Np_max, n_max, bytes);
    if (e != hipSuccess) return hip_fail(e, "workspace query");
    return ok();
}

lagp_status lagp_alc_uneven_from_pool(const double *X, const double *Y, int64_t N, int32_t p,
                                      const double *XX, int64_t M, const int32_t *pool, int32_t Np_max,
                                      int32_t n0, int32_t n_max, const int32_t *n_per,
                                      const int32_t *Np_per, const int64_t *sel_off, const double *d_per,
                                      double d, double g, int32_t precision, double *mean, double *s2,
                                      double *var, int32_t *sel, double *alc, int32_t *status,
                                      int32_t *guard, void *workspace, size_t workspace_bytes, void *stream)
{
    lagp_status s = check_common(X, N, p, XX, M, Np_max);
    if (s != LAGP_OK) return s;
    s = check_alc(Y, Np_max, n0, n_max, d, g, precision, sel, M);
    if (s != LAGP_OK) return s;
    if (M > 0 && !pool) return fail(LAGP_EINVAL, "pool must be non-NULL");
    if (precision != LAGP_FP64)
        return fail(LAGP_EUNSUPPORTED, "per-location designs are computed in float64 only (LAGP_FP64)");
    if (!lagp::alc_uneven_supported(p, Np_max, n_max))
        return fail(LAGP_EUNSUPPORTED, "no schedule for p = %d, Np_max = %d, n_max = %d", p, Np_max, n_max);
    if (M == 0) return ok();
    size_t need = 0;
    hipError_t e = lagp::alc_uneven_workspace(p, M, Np_max, n_max, &need);
    if (e != hipSuccess) return hip_fail(e, "workspace query");
    if (!workspace || workspace_bytes < need)
        return fail(LAGP_EWORKSPACE, "workspace of %zu bytes given, %zu needed", workspace_bytes, need);
    lagp::AlcArgs a{X, Y, N, p, XX, M, pool, Np_max, n0, n_max, d, g, mean, s2, var, sel, alc, nullptr, status,
                    guard};
    e = lagp::launch_alc_uneven(a, n_per, Np_per, sel_off, d_per, workspace, workspace_bytes,
                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "uneven alc launch");
    return ok();
}

static lagp_status check_local(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                               int64_t M, int32_t n)
{
    if (M < 0) return fail(LAGP_EINVAL, "M = %lld < 0", (long long)M);
    if (p < 1) return fail(LAGP_EINVAL, "p = %d < 1", p);
    if (N < 1 || N >= (int64_t)1 << 31) return fail(LAGP_EINVAL, "N = %lld outside [1, 2^31)", (long long)N);
    if (n < 1 || n > N) return fail(LAGP_EINVAL, "n = %d outside [1, N]", n);
    if (M > 0 && (!X || !Y || !sel)) return fail(LAGP_EINVAL, "X, Y and sel must be non-NULL");
    if (!lagp::local_gp_supported(n, p)) return fail(LAGP_EUNSUPPORTED, "local design of n = %d, p = %d", n, p);
    if (M > (int64_t)0x7fffffff) return fail(LAGP_EUNSUPPORTED, "M = %lld exceeds one launch", (long long)M);
    return LAGP_OK;
}

lagp_status lagp_local_nll(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                           int64_t M, int32_t n, const double *d, const double *g, double *nll,
                           double *dnll_dd, double *dnll_dg, double *d2nll_dd2, int32_t *status, void *stream)
{
    lagp_status s = check_local(X, Y, N, p, sel, M, n);
    if (s != LAGP_OK) return s;
    if (M > 0 && (!d || !g)) return fail(LAGP_EINVAL, "d and g must be non-NULL");
    if (M == 0) return ok();
    lagp::GpArgs a{};
    a.X = X; a.Y = Y; a.N = N; a.p = p; a.sel = sel; a.M = M; a.n = n;
    a.d_arr = d; a.g_arr = g; a.nll = nll; a.dd = dnll_dd; a.dg = dnll_dg; a.d2 = d2nll_dd2; a.status = status;
    hipError_t e = lagp::launch_local_gp(a, lagp::kGpNll, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "local_nll launch");
    return ok();
}

lagp_status lagp_local_nll_backward(const double *X, const double *Y, int64_t N, int32_t p,
                                    const int32_t *sel, int64_t M, int32_t n, const double *d,
                                    const double *g, const double *grad_out, double *grad_d, double *grad_g,
                                    void *stream)
{
    lagp_status s = check_local(X, Y, N, p, sel, M, n);
    if (s != LAGP_OK) return s;
    if (M > 0 && (!d || !g)) return fail(LAGP_EINVAL, "d and g must be non-NULL");
    if (M == 0) return ok();
    lagp::GpArgs a{};
    a.X = X; a.Y = Y; a.N = N; a.p = p; a.sel = sel; a.M = M; a.n = n;
    a.d_arr = d; a.g_arr = g; a.grad_out = grad_out; a.dd = grad_d; a.dg = grad_g;
    hipError_t e = lagp::launch_local_gp(a, lagp::kGpBackward, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "local_nll_backward launch");
    return ok();
}

lagp_status lagp_local_mle_d(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                             int64_t M, int32_t n, const double *d0, double g, double dmin, double dmax,
                             int32_t maxit, double *d_hat, double *nll, int32_t *iters, int32_t *status,
                             void *stream)
{
    lagp_status s = check_local(X, Y, N, p, sel, M, n);
    if (s != LAGP_OK) return s;
    if (M > 0 && (!d0 || !d_hat)) return fail(LAGP_EINVAL, "d0 and d_hat must be non-NULL");
    if (!(g > 0.0) || !isfinite(g)) return fail(LAGP_EINVAL, "nugget g must be finite and > 0");
    if (!(dmin > 0.0) || !(dmax >= dmin) || !isfinite(dmax))
        return fail(LAGP_EINVAL, "need 0 < dmin <= dmax < inf");
    if (maxit < 0) return fail(LAGP_EINVAL, "maxit = %d < 0", maxit);
    if (M == 0) return ok();
    lagp::GpArgs a{};
    a.X = X; a.Y = Y; a.N = N; a.p = p; a.sel = sel; a.M = M; a.n = n;
    a.d_arr = d0; a.g_scalar = g; a.dmin = dmin; a.dmax = dmax; a.maxit = maxit;
    a.d_hat = d_hat; a.nll = nll; a.iters = iters; a.status = status;
    hipError_t e = lagp::launch_local_gp(a, lagp::kGpMle, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "local_mle_d launch");
    return ok();
}

lagp_status lagp_local_predict(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                               int64_t M, int32_t n, const double *XX, const double *d, double g, double *mean,
                               double *s2, double *var, int32_t *status, void *stream)
{
    lagp_status s = check_local(X, Y, N, p, sel, M, n);
    if (s != LAGP_OK) return s;
    if (M > 0 && (!XX || !d)) return fail(LAGP_EINVAL, "XX and d must be non-NULL");
    if (!(g > 0.0) || !isfinite(g)) return fail(LAGP_EINVAL, "nugget g must be finite and > 0");
    if (M == 0) return ok();
    lagp::GpArgs a{};
    a.X = X; a.Y = Y; a.N = N; a.p = p; a.sel = sel; a.M = M; a.n = n;
    a.d_arr = d; a.g_scalar = g; a.XX = XX; a.mean = mean; a.s2 = s2; a.var = var; a.status = status;
    hipError_t e = lagp::launch_local_gp(a, lagp::kGpPredict, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "local_predict launch");
    return ok();
}

const char *lagp_status_string(lagp_status s)
{
    switch (s) {
    case LAGP_OK:
        return "LAGP_OK";
    case LAGP_EINVAL:
        return "LAGP_EINVAL";
    case LAGP_EWORKSPACE:
        return "LAGP_EWORKSPACE";
    case LAGP_EHIP:
        return "LAGP_EHIP";
    case LAGP_EUNSUPPORTED:
        return "LAGP_EUNSUPPORTED";
    default:
        return "unknown lagp_status";
    }
}

const char *lagp_last_error(void)
{
    return g_err;
}

const char *lagp_version(void)
{
    return "lagp-alc 0.1 (gfx950)";
}

}  // extern "C"
