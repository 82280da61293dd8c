// Internal host-side interface between the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lagp {

// Records the calling thread's message for lagp_last_error() and returns code.
int set_error(int code, const char *fmt, ...);

constexpr int kMaxP = 16;  // largest input dimension any kernel accepts
constexpr int kScoresJmax = 128;  // largest design whose K_j^{-1} the batch-scores kernel stages in LDS
constexpr int kScoresJbig = 512;  // largest design of the batch scores (K_j^{-1} read from L2 beyond 128)

// Per-location status codes (the LAGP_LOC_* values of the public header).
constexpr int kLocOk = 0, kLocInitNotPd = 1, kLocStepFail = 2, kLocNonfinite = 3, kLocBadPool = 4,
              kLocBadShape = 5;

struct AlcArgs {
    const double *X;
    const double *Y;
    int64_t N;
    int p;
    const double *XX;
    int64_t M;
    const int32_t *pool;
    int Np;
    int n0;
    int n;
    double d;
    double g;
    double *mean;
    double *s2;
    double *var;
    int32_t *sel;
    double *alc;
    double *alc32;  // mixed: float32 score of each chosen point (nullable)
    int32_t *status;
    int32_t *guard;
    // Per-location designs (all NULL: a.n, a.Np and a.d everywhere, row m of
    // sel / alc / alc32 at m * a.n).  With them a.n and a.Np are upper bounds.
    const int32_t *n_per = nullptr;
    const int32_t *Np_per = nullptr;
    const int64_t *sel_off = nullptr;
    const double *d_per = nullptr;
    int pool_stride = 0;          // row stride of pool (0: a.Np)
    const int32_t *list = nullptr;       // mixed kernel: locations to run, list[b] for block b
    const int32_t *list_count = nullptr; // ... of which the first *list_count are valid
    int normalize = 0;   // scores reported as psi_j Delta / (j - 2) (Sec. 3.1, Fig. 3 step 9)
    int f64_guard = 0;   // float64 kernel standing in for LAGP_MIXED: guard counts every step
    const double *dsep = nullptr;  // [p] separable lengthscales (float64 incremental kernel only), or NULL
};

// Internal form of lagp_problem / lagp_outputs after validation, with the
// workspace carved up.
struct PathArgs {
    AlcArgs a;          // per-location fields set; a.pool = pool
    int32_t *pool = nullptr;  // the pools: the caller's, or in the workspace
    int precision = 0;
    bool nn_brute = false;
    bool uniform = true;  // no per-location n, N', d or row offsets
    void *alc_ws = nullptr;   // queues and spilled factor columns of per-location designs
    size_t alc_ws_bytes = 0;
    void *nn_ws = nullptr;    // grid of the design, and the float32 copy of the NN variants
};

// Whole path (pools, designs, predictions) with the given NN variant (see
// plan.cpp; -1: the default) and incremental-kernel broadcast mask / shape.
hipError_t run_path(const PathArgs &P, int nn_variant, int bcast, hipStream_t st, const int *smap = nullptr);

}  // namespace lagp

struct lagp_problem;
struct lagp_outputs;

namespace lagp {

// Validates a problem and its outputs (as lagp_alc_predict does) and carves the
// workspace; sets lagp_last_error on failure.
int prepare_path(const lagp_problem *prob, const lagp_outputs *out, void *ws, size_t ws_bytes, PathArgs *P);

// Largest LDS buffer the NN kernel needs for a pool of Np (0 if unsupported).
int nn_pool_cap(int Np);
// Number of location groupings (2^g locations per workgroup) for pools of Np;
// grouping < 0 picks the default.
int nn_pool_groupings(int Np);
// Workspace of the pool kernels that take one (nn_pool_workspace(N, p)
// bytes): x32 below uses its first N p floats for a float32 copy of X, which
// the stream then reads instead of X; launch_nn_grid uses all of it for the
// grid of the design (cells, their boxes, the rows cell by cell) and prunes.
size_t nn_pool_workspace(int64_t N, int p, int64_t M);
// Allocation-free grid-pruned pools: the same kernels on a file-scope
// device array of kNnStaticScratch bytes (one copy per GPU, resolved to its
// device address once per device).
constexpr size_t kNnStaticScratch = (size_t)128 << 20;
hipError_t nn_static_scratch(void **ptr);
// group: locations per workgroup sharing the stream of cells (1, 2 or 4; see
// nn_grid_groups for what a problem supports).
hipError_t launch_nn_grid(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np, int32_t *pool,
                          void *ws, hipStream_t st, int group = 1);
// Number of grid groupings (1, 2, 4 locations per workgroup) compiled for (p, Np).
int nn_grid_groups(int p, int Np);
hipError_t launch_nn_pool(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                          int32_t *pool, hipStream_t st, int grouping = -1, float *x32 = nullptr);

// Returns hipErrorNotSupported (without launching) when no compiled schedule
// covers (p, Np, n, precision).
bool alc_supported(int precision, int p, int Np, int n);
hipError_t launch_alc(const AlcArgs &a, int precision, hipStream_t st);

// Float64 greedy ALC by incremental Cholesky columns.  `bcast` selects, per
// schedule, how the chosen factor row reaches the lanes (bit b set: DPP row
// broadcasts from a per-lane copy, clear: uniform LDS reads); negative: the
// default.  `smap` (kIncClasses entries, or NULL for the defaults) names the
// schedule of each pool-size class.
constexpr int kIncSchedules = 6, kIncClasses = 4;  // LAGP_PLAN_SCHEDULES of the public header
int alc_inc_schedule(int Np);  // default schedule serving pools of Np (-1: none)
int alc_inc_class(int Np);     // pool-size class of Np (-1: none)
int alc_inc_default_sched(int c);  // the schedule of class c without a plan
// Whether schedule s can serve class c at (p, n_max): the class's pools fit
// it and its LDS holds the coordinates; `on_chip` also asks for every factor
// column in registers or LDS (the uniform launch).
bool alc_inc_admissible(int s, int c, int p, int n_max, bool on_chip);
void alc_inc_sched_name(int s, char *buf, size_t len);
bool alc_inc_supported(int p, int Np, int n);
hipError_t launch_alc_inc(const AlcArgs &a, hipStream_t st, int bcast = -1, const int *smap = nullptr);
// Per-location n, N' (a.n, a.Np are the upper bounds; pool rows of a.Np) and,
// when d_per is not NULL, lengthscale d.
bool alc_uneven_supported(int p, int Np_max, int n_max);
hipError_t alc_uneven_workspace(int p, int64_t M, int Np_max, int n_max, size_t *bytes);
// With `mixed`, locations with n_m <= 64, N'_m <= 1024 and
// mixed_trusted(n_m, g) run the mixed (float32 MFMA) kernel and the others run
// in float64 with every step counted in guard.
hipError_t launch_alc_uneven(const AlcArgs &a, const int32_t *n_per, const int32_t *Np_per,
                             const int64_t *sel_off, const double *d_per, void *ws, size_t ws_bytes,
                             hipStream_t st, int bcast = -1, bool mixed = false, const int *smap = nullptr);
// Mixed (float32 MFMA) kernel over the locations of a.list (per-location
// sizes from a's per-location fields); `big` selects the 1024-slot schedule.
hipError_t launch_alc_mixed_list(const AlcArgs &a, bool big, hipStream_t st);
constexpr int kMixNmax = 64, kMixNpMax = 1024;
// Float32 scores are used only where the nugget keeps every K_j well enough
// conditioned for them: the correlation part of K_j has eigenvalues in
// [0, j], so cond(K_j) <= (j + g) / g, and float32 scoring is trusted while
// that bound for the whole design times the float32 unit roundoff 2^-24 is at
// most 2^-4 (n / g up to about 10^6).  Other locations asking for mixed
// precision run in float64 with every step counted in guard.
__host__ __device__ inline bool mixed_trusted(int n, double g)
{
    return (n + g) / g * 0x1p-24 <= 0x1p-4;
}

// Local designs by the MSPE criterion (eq. mspe), float64, uniform n and N':
// workspace for M locations, and the launch (a.alc receives the criterion of
// each chosen point).
constexpr int kMspeNmax = 64, kMspeNpMax = 1024, kMspePmax = 8;
hipError_t mspe_workspace(int64_t M, int Np, int n, size_t *bytes);
hipError_t launch_mspe(const AlcArgs &a, void *ws, size_t ws_bytes, hipStream_t st);

// Local likelihood / MLE / fixed-design prediction, one wave per location.
struct GpArgs {
    const double *X, *Y;
    int64_t N;
    int p;
    const int32_t *sel;
    int64_t M;
    int n;
    // per-location parameters (arrays of M) or scalars
    const double *d_arr;
    double d_scalar;
    const double *g_arr;
    double g_scalar;
    // outputs / inputs by mode
    double *nll, *dd, *dg, *d2;
    const double *grad_out;
    double dmin, dmax;
    int maxit;
    double *d_hat;
    int32_t *iters, *status;
    const double *XX;
    double *mean, *s2, *var;
};

enum GpMode { kGpNll = 0, kGpBackward = 1, kGpMle = 2, kGpPredict = 3 };
bool local_gp_supported(int n, int p);
size_t local_gp_lds(int n, int p);
hipError_t launch_local_gp(const GpArgs &a, int mode, hipStream_t st);

// Batch scores of Nc candidates against one design of j points given K_j^{-1}
// and h (lagp_alc_scores); float32 arithmetic when `mixed`.
hipError_t launch_alc_scores(const double *Xj, int j, int p, const double *Kinv, const double *Xc, int64_t Nc,
                             const double *x, const double *h, double d, double g, bool mixed, double *delta,
                             hipStream_t st);

}  // namespace lagp
