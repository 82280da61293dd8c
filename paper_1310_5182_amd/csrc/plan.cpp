// Graph-captured, autotuned runs of the whole path (lagp_plan_* of lagp_alc.h).
//
// A plan binds one problem of lagp_alc_predict to its buffers, picks the
// fastest variant of each tunable launch by timing it on those very inputs (the
// NN variant: locations per workgroup over the whole design, the stream of a
// float32 copy of it, or the grid-pruned stream; for every pool-size class of
// the float64 ALC kernel that the problem's locations fall into, the schedule
// that serves it - threads per location, positions per lane, factor entries in
// registers, down to one wave per location - and, for every schedule that
// runs, how the chosen factor row is broadcast), and captures the chosen
// launches - NN pools, queue planning, persistent ALC workgroups - into one
// HIP graph.  Replaying the graph costs one launch call; every node is a
// kernel (no memset nodes).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "lagp_alc.h"
#include "lagp_internal.hpp"

struct lagp_plan_s {
    lagp::PathArgs P;
    int nnv = -1;       // NN variant: 2^nnv locations per workgroup, kNnF32 or kNnGrid
    int bcast = -1;     // ALC broadcast mask
    int smap[lagp::kIncClasses] = {-1, -1, -1, -1};  // schedule of each pool-size class (-1: default)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string info;
};

static_assert(lagp::kIncSchedules == LAGP_PLAN_SCHEDULES, "the schedules of LAGP_PLAN_SCHEDULE");

namespace lagp {

// NN variants beyond the location groupings 0 .. nn_pool_groupings(Np) - 1:
// the float32 stream, and the grid-pruned pools with 1, 2 or 4 locations per
// workgroup
constexpr int kNnF32 = 100, kNnGrid = 101, kNnGrid2 = 102, kNnGrid4 = 103;

static const char *nn_name(int v, char *buf, size_t n)
{
    if (v == kNnGrid)
        snprintf(buf, n, "grid");
    else if (v == kNnGrid2 || v == kNnGrid4)
        snprintf(buf, n, "grid g=%d", v == kNnGrid2 ? 2 : 4);
    else if (v == kNnF32)
        snprintf(buf, n, "g=1 x32");
    else if (v < 0)
        snprintf(buf, n, "default");
    else
        snprintf(buf, n, "g=%d", 1 << v);
    return buf;
}

// The whole path with the given NN variant (-1: the grid, or the default
// location grouping under LAGP_NN_BRUTE), broadcast mask of the float64
// incremental kernel (-1: its default) and schedule per pool-size class (NULL:
// the defaults).
hipError_t run_path(const PathArgs &P, int nnv, int bcast, hipStream_t st, const int *smap)
{
    const AlcArgs &a = P.a;
    if (nnv < 0 && !P.nn_brute) nnv = kNnGrid;
    hipError_t e = nnv == kNnGrid    ? launch_nn_grid(a.X, a.N, a.p, a.XX, a.M, a.Np, P.pool, P.nn_ws, st)
                   : nnv == kNnGrid2 ? launch_nn_grid(a.X, a.N, a.p, a.XX, a.M, a.Np, P.pool, P.nn_ws, st, 2)
                   : nnv == kNnGrid4 ? launch_nn_grid(a.X, a.N, a.p, a.XX, a.M, a.Np, P.pool, P.nn_ws, st, 4)
                   : nnv == kNnF32 ? launch_nn_pool(a.X, a.N, a.p, a.XX, a.M, a.Np, P.pool, st, 0, (float *)P.nn_ws)
                                   : launch_nn_pool(a.X, a.N, a.p, a.XX, a.M, a.Np, P.pool, st, nnv, nullptr);
    if (e != hipSuccess) return e;
    if (P.uniform) {
        // uniform n, N' and d with every factor column on chip: one workgroup per
        // location, no queue to classify and order
        if (P.precision == 0 && alc_inc_supported(a.p, a.Np, a.n)) return launch_alc_inc(a, st, bcast, smap);
        return launch_alc(a, P.precision, st);
    }
    return launch_alc_uneven(a, a.n_per, a.Np_per, a.sel_off, a.d_per, P.alc_ws, P.alc_ws_bytes, st, bcast,
                             P.precision == 1, smap);
}

// Milliseconds of one run (the best of `reps`, after one untimed run).
static hipError_t time_path(const PathArgs &P, int nnv, int bcast, const int *smap, hipStream_t st, int reps,
                            float *ms)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    float best = 1e30f;
    e = run_path(P, nnv, bcast, st, smap);
    for (int r = 0; e == hipSuccess && r < reps; r++) {
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        if ((e = run_path(P, nnv, bcast, st, smap)) != hipSuccess) break;
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

// Coordinate search: the NN variant first, then the schedule of each pool-size
// class the locations fall into (among the schedules that can serve it), then
// the broadcast bit of each schedule that runs.  A change is kept only if it
// is at least 1 % faster.  The timing runs use at most the first
// kTuneLocations locations (their outputs are overwritten later), so that
// tuning stays short for large M.
constexpr int64_t kTuneLocations = 65536;

// The pool-size classes that the locations of P use (a flag per class), and
// the highest class of its bound N'; -1 if the incremental kernel does not run.
static hipError_t classes_of(const PathArgs &P, bool (&present)[kIncClasses], int *top)
{
    for (int c = 0; c < kIncClasses; c++) present[c] = false;
    *top = -1;
    const bool inc = P.precision != 2 && (!P.uniform || (P.precision == 0 && alc_inc_supported(P.a.p, P.a.Np, P.a.n)));
    const int t = alc_inc_class(P.a.Np);
    if (!inc || t < 0) return hipSuccess;
    if (P.a.Np_per) {
        std::vector<int32_t> np((size_t)P.a.M);
        hipError_t e = hipMemcpy(np.data(), P.a.Np_per, np.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        for (int32_t v : np) {
            const int c = alc_inc_class(v);
            if (c >= 0 && c <= t) present[c] = true;
        }
    } else {
        present[t] = true;
    }
    *top = t;
    return hipSuccess;
}

static hipError_t tune(lagp_plan_s &plan, hipStream_t st, int forced)
{
    PathArgs P = plan.P;
    if (P.a.M > kTuneLocations) P.a.M = kTuneLocations;
    char line[200], nm[32];
    std::string info;
    int variants[8], nv = 0;
    if (!P.nn_brute) {
        variants[nv++] = kNnGrid;
        const int gg = nn_grid_groups(P.a.p, P.a.Np);
        if (gg >= 2) variants[nv++] = kNnGrid2;
        if (gg >= 3) variants[nv++] = kNnGrid4;
    }
    for (int g = 0; g < nn_pool_groupings(P.a.Np); g++) variants[nv++] = g;
    if (!P.nn_brute) variants[nv++] = kNnF32;
    // the incremental kernel's pool-size classes that this problem's locations use
    bool present[kIncClasses];
    int top = -1, map[kIncClasses];
    hipError_t e = classes_of(P, present, &top);
    if (e != hipSuccess) return e;
    for (int c = 0; c < kIncClasses; c++) {
        map[c] = c <= top ? alc_inc_default_sched(c) : -1;
        if (c <= top && forced >= 0 && alc_inc_admissible(forced, c, P.a.p, P.a.n, P.uniform)) map[c] = forced;
    }
    const int *mp = top >= 0 ? map : nullptr;
    int mask = -1, v_best = variants[0];
    float best = 0.0f;
    e = time_path(P, v_best, mask, mp, st, 2, &best);
    if (e != hipSuccess) return e;
    snprintf(line, sizeof line, "nn %s: %.3f ms", nn_name(v_best, nm, sizeof nm), best);
    info += line;
    for (int q = 1; q < nv; q++) {
        float t = 0.0f;
        if ((e = time_path(P, variants[q], mask, mp, st, 2, &t)) != hipSuccess) return e;
        snprintf(line, sizeof line, "; nn %s: %.3f ms", nn_name(variants[q], nm, sizeof nm), t);
        info += line;
        if (t < best) {
            best = t;
            v_best = variants[q];
        }
    }
    mask = 0;
    for (int b = 0; b < kIncSchedules; b++) mask |= 1 << b;  // DPP broadcast everywhere to start with
    if (mp) {
        for (int c = 0; c <= top && forced < 0; c++) {
            if (!present[c]) continue;
            for (int s = 0; s < kIncSchedules; s++) {
                if (s == map[c] || !alc_inc_admissible(s, c, P.a.p, P.a.n, P.uniform)) continue;
                int trial[kIncClasses];
                for (int q = 0; q < kIncClasses; q++) trial[q] = map[q];
                trial[c] = s;
                float t = 0.0f;
                if ((e = time_path(P, v_best, mask, trial, st, 2, &t)) != hipSuccess) return e;
                alc_inc_sched_name(s, nm, sizeof nm);
                snprintf(line, sizeof line, "; class %d on %s: %.3f ms", c, nm, t);
                info += line;
                if (t < 0.99f * best) {
                    best = t;
                    map[c] = s;
                }
            }
        }
        unsigned used = 0;
        for (int c = 0; c <= top; c++)
            if (present[c]) used |= 1u << map[c];
        for (int b = 0; b < kIncSchedules; b++) {
            if (!(used >> b & 1)) continue;
            const int m2 = mask ^ (1 << b);
            float t = 0.0f;
            if ((e = time_path(P, v_best, m2, mp, st, 2, &t)) != hipSuccess) return e;
            snprintf(line, sizeof line, "; alc mask=%x: %.3f ms", m2, t);
            info += line;
            if (t < 0.99f * best) {
                best = t;
                mask = m2;
            }
        }
    }
    plan.nnv = v_best;
    plan.bcast = mask;
    for (int c = 0; c < kIncClasses; c++) plan.smap[c] = map[c];
    snprintf(line, sizeof line, "; chosen nn %s alc mask=%x", nn_name(v_best, nm, sizeof nm), mask);
    info += line;
    for (int c = 0; mp && c <= top; c++) {
        if (!present[c]) continue;
        alc_inc_sched_name(map[c], nm, sizeof nm);
        snprintf(line, sizeof line, " class%d=%s", c, nm);
        info += line;
    }
    snprintf(line, sizeof line, " (%.3f ms on %lld locations)", best, (long long)P.a.M);
    plan.info = info + line;
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

lagp_status lagp_plan_create(const lagp_problem *prob, const lagp_outputs *out, void *workspace,
                             size_t workspace_bytes, int32_t plan_flags, void *stream, lagp_plan *plan)
{
    if (!plan) return plan_fail(LAGP_EINVAL, "plan must be non-NULL");
    *plan = nullptr;
    if (plan_flags & ~(LAGP_PLAN_NO_TUNE | (0xf << 8))) return plan_fail(LAGP_EINVAL, "unknown plan flags");
    const int forced = ((plan_flags >> 8) & 0xf) - 1;  // LAGP_PLAN_SCHEDULE(s), or -1
    if (forced >= lagp::kIncSchedules) return plan_fail(LAGP_EINVAL, "LAGP_PLAN_SCHEDULE(s) needs s < LAGP_PLAN_SCHEDULES");
    lagp::PathArgs path;
    lagp_status s = lagp::prepare_path(prob, out, workspace, workspace_bytes, &path);
    if (s != LAGP_OK) return s;  // its message stays in lagp_last_error()
    if (path.a.M < 1) return plan_fail(LAGP_EINVAL, "a plan needs M >= 1");

    lagp_plan_s *P = new lagp_plan_s();
    P->P = path;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (plan_flags & LAGP_PLAN_NO_TUNE) {
        P->info = path.nn_brute ? "defaults (not tuned: nn default)" : "defaults (not tuned: nn grid)";
        bool present[lagp::kIncClasses];
        int top = -1;
        if (forced >= 0 && (e = lagp::classes_of(path, present, &top)) == hipSuccess) {
            for (int c = 0; c <= top; c++)
                P->smap[c] = lagp::alc_inc_admissible(forced, c, path.a.p, path.a.n, path.uniform)
                                 ? forced : lagp::alc_inc_default_sched(c);
            char nm[32];
            lagp::alc_inc_sched_name(forced, nm, sizeof nm);
            P->info += std::string("; schedule ") + nm + " where it serves";
        }
        if (e != hipSuccess) {
            delete P;
            return plan_fail(LAGP_EHIP, "pool sizes", e);
        }
    } else if ((e = lagp::tune(*P, st, forced)) != hipSuccess) {
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
        hipError_t run = lagp::run_path(P->P, P->nnv, P->bcast, cs, P->smap[0] >= 0 ? P->smap : nullptr);
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
    *plan = P;
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
