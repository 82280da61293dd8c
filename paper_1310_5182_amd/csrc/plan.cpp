// Graph-captured, autotuned runs of the whole path (lagp_plan_* of lagp_alc.h).
//
// A plan binds one problem's buffers, picks the fastest variant of each
// tunable launch by timing it on those very inputs (the NN variant: locations
// per workgroup over the whole design, the stream of a float32 copy of it, or
// the grid-pruned stream; for every pool-size schedule of the ALC kernel, how
// the chosen factor row is broadcast), and captures the chosen launches - NN pools,
// queue planning, persistent ALC workgroups - into one HIP graph.  Replaying
// the graph costs one launch call; every node is a kernel (no memset nodes).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "lagp_alc.h"
#include "lagp_internal.hpp"

struct lagp_plan_s {
    lagp::AlcArgs a;
    const int32_t *n_per, *Np_per;
    const int64_t *sel_off;
    const double *d_per;
    int32_t *pool;
    void *ws;         // the ALC kernels' part of the workspace
    size_t ws_bytes;
    void *nnws;       // then the NN kernels' workspace
    int grouping = -1;  // NN variant: 2^grouping locations per workgroup, kNnF32 or kNnGrid

    int bcast = -1;     // ALC broadcast mask
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string info;
};

namespace lagp {

// Enqueue the whole path with the given variants.
// NN variants beyond the location groupings 0 .. nn_pool_groupings(Np) - 1
constexpr int kNnF32 = 100, kNnGrid = 101;

static const char *nn_name(int v, char *buf, size_t n)
{
    if (v == kNnGrid)
        snprintf(buf, n, "grid");
    else if (v == kNnF32)
        snprintf(buf, n, "g=1 x32");
    else
        snprintf(buf, n, "g=%d", 1 << v);
    return buf;
}

static hipError_t run_path(const lagp_plan_s &P, int nnv, int bcast, hipStream_t st)
{
    hipError_t e = nnv == kNnGrid ? launch_nn_grid(P.a.X, P.a.N, P.a.p, P.a.XX, P.a.M, P.a.Np, P.pool, P.nnws, st)
                   : nnv == kNnF32
                       ? launch_nn_pool(P.a.X, P.a.N, P.a.p, P.a.XX, P.a.M, P.a.Np, P.pool, st, 0, (float *)P.nnws)
                       : launch_nn_pool(P.a.X, P.a.N, P.a.p, P.a.XX, P.a.M, P.a.Np, P.pool, st, nnv, nullptr);
    if (e != hipSuccess) return e;
    // uniform n, N' and d with every factor column on chip: one workgroup per
    // location, no queue to classify and order
    if (!P.n_per && !P.Np_per && !P.sel_off && !P.d_per && alc_inc_supported(P.a.p, P.a.Np, P.a.n))
        return launch_alc_inc(P.a, st, bcast);
    return launch_alc_uneven(P.a, P.n_per, P.Np_per, P.sel_off, P.d_per, P.ws, P.ws_bytes, st, bcast);
}

// Milliseconds of one run (the best of `reps`, after one untimed run).
static hipError_t time_path(const lagp_plan_s &P, int nnv, int bcast, hipStream_t st, int reps, float *ms)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    float best = 1e30f;
    e = run_path(P, nnv, bcast, st);
    for (int r = 0; e == hipSuccess && r < reps; r++) {
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        if ((e = run_path(P, nnv, bcast, st)) != hipSuccess) break;
        if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float t = 0.0f;
        if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
        if (t < best) best = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return e;
}

// Coordinate search: the NN variant first, then each schedule's broadcast bit.
// The timing runs use at most the first kTuneLocations locations (their
// outputs are overwritten later), so that tuning stays short for large M.
constexpr int64_t kTuneLocations = 65536;

static hipError_t tune(lagp_plan_s &Pfull, hipStream_t st)
{
    lagp_plan_s P = Pfull;
    if (P.a.M > kTuneLocations) P.a.M = kTuneLocations;
    char line[160], nm[32];
    float best = 0.0f;
    int v_best = kNnGrid, mask = 0x7;
    hipError_t e = time_path(P, kNnGrid, mask, st, 2, &best);
    if (e != hipSuccess) return e;
    snprintf(line, sizeof line, "nn grid alc mask=%x: %.3f ms", mask, best);
    P.info += line;
    int variants[8], nv = 0;
    for (int g = 0; g < nn_pool_groupings(P.a.Np); g++) variants[nv++] = g;
    variants[nv++] = kNnF32;
    for (int q = 0; q < nv; q++) {
        float t = 0.0f;
        if ((e = time_path(P, variants[q], mask, st, 2, &t)) != hipSuccess) return e;
        snprintf(line, sizeof line, "; nn %s: %.3f ms", nn_name(variants[q], nm, sizeof nm), t);
        P.info += line;
        if (t < best) {
            best = t;
            v_best = variants[q];
        }
    }
    const int top = alc_inc_schedule(P.a.Np);
    for (int b = 0; b <= top; b++) {
        const int m2 = mask ^ (1 << b);
        float t = 0.0f;
        if ((e = time_path(P, v_best, m2, st, 2, &t)) != hipSuccess) return e;
        snprintf(line, sizeof line, "; alc mask=%x: %.3f ms", m2, t);
        P.info += line;
        if (t < best) {
            best = t;
            mask = m2;
        }
    }
    Pfull.grouping = v_best;
    Pfull.bcast = mask;
    snprintf(line, sizeof line, "; chosen nn %s alc mask=%x (%.3f ms on %lld locations)",
             nn_name(v_best, nm, sizeof nm), mask, best, (long long)P.a.M);
    Pfull.info = P.info + line;
    return hipSuccess;
}

}  // namespace lagp

namespace {
lagp_status plan_fail(lagp_status code, const char *msg, hipError_t e = hipSuccess)
{
    if (e != hipSuccess) return lagp::set_error(code, "%s: %s", msg, hipGetErrorString(e));
    return lagp::set_error(code, "%s", msg);
}
}  // namespace

extern "C" {

lagp_status lagp_plan_workspace(int64_t N, int32_t p, int64_t M, int32_t Np_max, int32_t n_max, size_t *bytes)
{
    size_t nn = 0;
    lagp_status s = lagp_nn_pool_workspace(N, p, M, &nn);
    if (s != LAGP_OK) return s;
    s = lagp_alc_uneven_workspace(p, M, Np_max, n_max, bytes);
    if (s != LAGP_OK) return s;
    *bytes = ((*bytes + 255) & ~(size_t)255) + nn;
    return LAGP_OK;
}

lagp_status lagp_plan_create(const double *X, const double *Y, int64_t N, int32_t p, const double *XX,
                             int64_t M, int32_t n0, int32_t n_max, int32_t Np_max, const int32_t *n_per,
                             const int32_t *Np_per, const int64_t *sel_off, const double *d_per, double d,
                             double g, int32_t *pool, double *mean, double *s2, double *var, int32_t *sel,
                             double *alc, int32_t *status, int32_t *guard, void *workspace,
                             size_t workspace_bytes, int32_t flags, void *stream, lagp_plan *out)
{
    if (!out) return plan_fail(LAGP_EINVAL, "out must be non-NULL");
    *out = nullptr;
    if (M < 1) return plan_fail(LAGP_EINVAL, "a plan needs M >= 1");
    // every argument check of the two calls it strings together, before any launch
    lagp_status s = lagp_alc_uneven_from_pool(X, Y, N, p, XX, 0, pool, Np_max, n0, n_max, n_per, Np_per,
                                              sel_off, d_per, d, g, LAGP_FP64, mean, s2, var, sel, alc, status,
                                              guard, workspace, workspace_bytes, stream);
    if (s != LAGP_OK) return s;  // its message stays in lagp_last_error()
    if (!pool) return plan_fail(LAGP_EINVAL, "pool must be non-NULL");
    if (lagp::nn_pool_cap(Np_max) == 0) return plan_fail(LAGP_EUNSUPPORTED, "Np_max too large for the pool kernel");
    size_t need = 0, need_alc = 0;
    hipError_t e = lagp::alc_uneven_workspace(p, M, Np_max, n_max, &need_alc);
    if (e != hipSuccess) return plan_fail(LAGP_EHIP, "workspace query", e);
    need_alc = (need_alc + 255) & ~(size_t)255;
    need = need_alc + lagp::nn_pool_workspace(N, p, M);
    if (!workspace || ((uintptr_t)workspace & 15) || workspace_bytes < need)
        return lagp::set_error(LAGP_EWORKSPACE, "workspace must be 16-byte aligned and hold %zu bytes", need);
    if (!X || !Y || !XX || !sel) return plan_fail(LAGP_EINVAL, "X, Y, XX and sel must be non-NULL");

    lagp_plan_s *P = new lagp_plan_s();
    P->a = lagp::AlcArgs{X, Y, N, p, XX, M, pool, Np_max, n0, n_max, d, g, mean, s2, var, sel, alc, nullptr,
                         status, guard};
    P->n_per = n_per;
    P->Np_per = Np_per;
    P->sel_off = sel_off;
    P->d_per = d_per;
    P->pool = pool;
    P->ws = workspace;
    P->ws_bytes = need_alc;
    P->nnws = (char *)workspace + need_alc;
    hipStream_t st = (hipStream_t)stream;
    P->grouping = lagp::kNnGrid;  // the default NN variant
    if (flags & LAGP_PLAN_NO_TUNE) {
        P->info = "defaults (not tuned: nn grid)";
    } else if ((e = lagp::tune(*P, st)) != hipSuccess) {
        delete P;
        return plan_fail(LAGP_EHIP, "autotuning run", e);
    }
    // capture on a private stream, so that the caller's stream may be the null stream
    hipStream_t cs = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
        delete P;
        return plan_fail(LAGP_EHIP, "capture stream", e);
    }
    if ((e = hipStreamSynchronize(st)) == hipSuccess &&
        (e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) == hipSuccess) {
        hipError_t run = lagp::run_path(*P, P->grouping, P->bcast, cs);
        e = hipStreamEndCapture(cs, &P->graph);
        if (run != hipSuccess) e = run;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(P->exec, st);  // the outputs hold one run's results
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (P->exec) (void)hipGraphExecDestroy(P->exec);
        if (P->graph) (void)hipGraphDestroy(P->graph);
        delete P;
        return plan_fail(LAGP_EHIP, "graph capture", e);
    }
    *out = P;
    return lagp::set_error(LAGP_OK, "");
}

lagp_status lagp_plan_launch(lagp_plan plan, void *stream)
{
    if (!plan || !plan->exec) return plan_fail(LAGP_EINVAL, "not a plan");
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return plan_fail(LAGP_EHIP, "graph launch", e);
    return LAGP_OK;
}

lagp_status lagp_plan_describe(lagp_plan plan, char *buf, size_t len)
{
    if (!plan || !buf || len == 0) return plan_fail(LAGP_EINVAL, "plan and buf must be non-NULL");
    snprintf(buf, len, "%s", plan->info.c_str());
    return LAGP_OK;
}

lagp_status lagp_plan_destroy(lagp_plan plan)
{
    if (!plan) return LAGP_OK;
    hipError_t e1 = plan->exec ? hipGraphExecDestroy(plan->exec) : hipSuccess;
    hipError_t e2 = plan->graph ? hipGraphDestroy(plan->graph) : hipSuccess;
    delete plan;
    if (e1 != hipSuccess) return plan_fail(LAGP_EHIP, "graph exec destroy", e1);
    if (e2 != hipSuccess) return plan_fail(LAGP_EHIP, "graph destroy", e2);
    return LAGP_OK;
}

}  // extern "C"
