/*
 * lagp_alc.h -- C ABI of the MI355X (gfx950) library for local approximate
 * Gaussian-process regression with greedy ALC local designs.
 *
 * Method: Gramacy, Niemi & Weiss, "Massively parallel approximate Gaussian
 * process regression" (arXiv:1310.5182).  For every predictive location x:
 *   1. the pool of the N' design points nearest to x (Sec. 2.2 NN sub-design,
 *      Sec. 3.1 search over N' nearest neighbours);
 *   2. a local design grown from the n0 nearest to n points, each step adding
 *      the candidate with the largest reduction in predictive variance at x,
 *      v_j(x) - v_{j+1}(x) (eq. dxy, Fig. 1 step 2), folded in with the
 *      partitioned-inverse update (eq. piedef);
 *   3. the local predictive mean, scale and variance (eqs. predgp, preds2,
 *      Student-t with n degrees of freedom, Sec. 2.1).
 * Correlation: K(x, x') = exp(-||x - x'||^2 / d) (Sec. 2.1); the nugget g is
 * added to the diagonal of the design covariance only, and K(x', x') = 1 + g
 * for candidates and for x (Fig. 3 step 5).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers on the current HIP device,
 *     caller-owned, row-major, float64 unless stated, int32 indices (0-based).
 *     The library never allocates or frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     and the call returns; the caller synchronises.
 *   - Arguments are validated on the host before any HIP call; on failure
 *     nothing is enqueued or written and LAGP_EINVAL is returned.  HIP
 *     launch failures return LAGP_EHIP.  lagp_last_error() gives a
 *     human-readable message for the calling thread's last failure.
 *   - Per-location numerical failures do not fail the call: they are
 *     reported in status[m] and that location's outputs are NaN.
 *   - Calls that overlap on one device must not share output buffers.
 */
#ifndef LAGP_ALC_H
#define LAGP_ALC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lagp_status;
#define LAGP_OK 0
#define LAGP_EINVAL (-1)        /* invalid argument                        */
#define LAGP_EWORKSPACE (-2)    /* workspace too small                     */
#define LAGP_EHIP (-3)          /* HIP runtime or launch error             */
#define LAGP_EUNSUPPORTED (-4)  /* sizes outside the compiled schedules    */

/* Arithmetic of the candidate scoring (Fig. 1 step 2b). */
#define LAGP_FP64 0   /* everything in float64; each candidate's factor row    */
                      /* grows by one entry per step (O(N' j) per step)        */
#define LAGP_MIXED 1  /* candidate kernel vectors and scores in float32 with   */
                      /* float32 accumulation; the inverse-factor update, the  */
                      /* Schur complement of the chosen point, a re-score of   */
                      /* the near-best candidates and the prediction in       */
                      /* float64                                               */
#define LAGP_FP64_REFORM 2  /* float64, every candidate's quadratic form       */
                            /* re-formed each step on the matrix cores (the   */
                            /* per-step route of Fig. 3, O(N' j^2) per step)  */

/* Per-location status codes written to status[m]. */
#define LAGP_LOC_OK 0
#define LAGP_LOC_INIT_NOT_PD 1  /* K_{n0} not numerically positive definite    */
#define LAGP_LOC_STEP_FAIL 2    /* Schur complement of a chosen point <= 0, or */
                                /* no candidate with a positive one             */
#define LAGP_LOC_NONFINITE 3    /* x not finite                                 */
#define LAGP_LOC_BAD_POOL 4     /* a pool entry outside [0, N): the location is */
                                /* skipped, no design row is read               */
#define LAGP_LOC_BAD_SHAPE 5    /* per-location n, N' or d outside the bounds   */
                                /* of lagp_alc_uneven_from_pool                 */

/*
 * lagp_nn_pool -- nearest-neighbour candidate pools (Sec. 2.2, Sec. 3.1).
 *
 *   X    [N x p]  design            XX  [M x p]  predictive locations
 *   pool [M x Np] out: for location m, the Np design indices with the
 *                 smallest squared distance sum_k (X[i,k] - XX[m,k])^2,
 *                 evaluated in float64 left to right with no fused
 *                 multiply-add, sorted ascending by (distance, index).
 * Requires 1 <= Np <= N, N < 2^31, p >= 1.  M = 0 is a no-op.
 */
lagp_status lagp_nn_pool(const double *X, int64_t N, int32_t p, const double *XX, int64_t M,
                         int32_t Np, int32_t *pool, void *stream);

/*
 * lagp_nn_pool_workspace -- bytes of device workspace that lagp_nn_pool_ws
 *   needs for N design rows and M locations (about N (4 p + 8) + 8 M bytes
 *   plus the cells: 1024 boxes and counters).
 * lagp_nn_pool_ws -- lagp_nn_pool with the design bucketed, once per call,
 *   into up to 1024 cells of a regular grid over its bounding box (a float32
 *   copy of the rows cell by cell, their indices, the exact float64 bounding
 *   box of each cell's rows, all in `workspace`; the locations are taken in
 *   cell order, each XCD of the GPU a contiguous run of them, so that the
 *   workgroups sharing an L2 read mostly the same cells).  Each location visits the
 *   cells in order of the distance from x to their boxes and stops at the
 *   first cell that is farther than its current N'-th nearest row: the pools
 *   are identical to lagp_nn_pool's (pools of locations with a non-finite
 *   coordinate are unspecified in both).  workspace: device memory of at
 *   least lagp_nn_pool_workspace(N, p) bytes, 16-byte aligned (else
 *   LAGP_EWORKSPACE); calls that overlap must not share it.
 */
lagp_status lagp_nn_pool_workspace(int64_t N, int32_t p, int64_t M, size_t *bytes);
lagp_status lagp_nn_pool_ws(const double *X, int64_t N, int32_t p, const double *XX, int64_t M,
                            int32_t Np, int32_t *pool, void *workspace, size_t workspace_bytes,
                            void *stream);

/*
 * lagp_nn_pool_grouped -- lagp_nn_pool_ws with `group` (1, 2 or 4) locations
 *   per workgroup, consecutive in the cell order, sharing one stream of the
 *   cells: the cells are visited in order of their smallest box distance over
 *   the group, and each row loaded serves every location whose own threshold
 *   admits its cell.  The pools are identical to lagp_nn_pool's; the grouping
 *   trades LDS (one key buffer per location) for fewer trips of each row from
 *   L2 and the last-level cache.  group 2 is compiled for p <= 8, group 4 for
 *   p <= 8 and Np <= 1024 (else LAGP_EUNSUPPORTED); workspace as for
 *   lagp_nn_pool_ws.
 */
lagp_status lagp_nn_pool_grouped(const double *X, int64_t N, int32_t p, const double *XX, int64_t M, int32_t Np,
                                 int32_t group, int32_t *pool, void *workspace, size_t workspace_bytes, void *stream);

/*
 * lagp_nn_pool_static -- lagp_nn_pool_ws without caller workspace, for
 *   callers that cannot allocate device memory (code under stream capture,
 *   serving loops that forbid allocation).  The grid-pruned pools are built
 *   in a static device array of LAGP_NN_STATIC_SCRATCH_BYTES (128 MiB) that
 *   the library holds on each GPU it runs on until the process ends; the call
 *   itself allocates nothing.  Same arguments and pools as lagp_nn_pool_ws;
 *   LAGP_EWORKSPACE if lagp_nn_pool_workspace(N, p, M) exceeds the static
 *   size (about N (12 p + 8) + 8 M bytes: at p = 8, e.g. N = M = 10^6).
 *   Every call on one GPU shares that GPU's array: calls that overlap on one
 *   GPU (different streams, threads) race and must be serialised by the
 *   caller.  The stream must belong to the current device.
 */
#define LAGP_NN_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
lagp_status lagp_nn_pool_static(const double *X, int64_t N, int32_t p, const double *XX, int64_t M,
                                int32_t Np, int32_t *pool, void *stream);

/*
 * lagp_alc_from_pool -- greedy ALC local designs and local predictions
 * (Fig. 1 steps 2a, 2b and 5) from given candidate pools.
 *
 *   X [N x p], Y [N]        design and responses (Y used raw: zero-mean GP)
 *   XX [M x p]              predictive locations
 *   pool [M x Np]           candidate pools as written by lagp_nn_pool; the
 *                           local design starts from pool[m][0 .. n0-1]
 *   n0, n                   start and final local design sizes
 *                           (1 <= n0 <= n <= Np)
 *   d, g                    lengthscale and nugget (finite, > 0)
 *   precision               LAGP_FP64 or LAGP_MIXED
 * Outputs (any may be NULL except sel):
 *   mean [M]                local predictive mean k^T K_n^{-1} Y_n (eq. predgp)
 *   s2   [M]                Student-t scale psi (1 + g - k^T K_n^{-1} k) / n
 *                           (eq. preds2 with N -> n)
 *   var  [M]                predictive variance s2 n / (n - 2); NaN if n <= 2
 *   sel  [M x n]            design indices of the local design in the order
 *                           added; row m starts with pool[m][0 .. n0-1]
 *   alc  [M x n]            float64 score v_j(x) - v_{j+1}(x) of the point
 *                           added at step j (unnormalised, eq. dxy); NaN for
 *                           j < n0
 *   alc32 [M x n]           LAGP_MIXED: the float32 score of that point as the
 *                           float32 scoring saw it, for the float32-vs-float64
 *                           error report; NaN for j < n0, for steps decided
 *                           entirely in float64, and everywhere for LAGP_FP64
 *   status [M]              LAGP_LOC_* code
 *   guard  [M]              LAGP_MIXED: number of steps whose float32 scores
 *                           were not trusted and were redone in float64; 0 for
 *                           LAGP_FP64
 * Exact score ties go to the smallest design index.
 * LAGP_MIXED uses float32 scores only where the nugget bounds the conditioning
 * enough for them: cond(K_j) <= (j + g) / g, and (n + g) / g * 2^-24 <= 2^-4
 * (n / g up to about 10^6, e.g. n = 50 with g >= 5e-5).  Otherwise the
 * designs are computed in float64 with all n - n0 steps counted in guard.
 * Supported sizes: p <= 8 and Np <= 1024; LAGP_MIXED needs n <= 64,
 * LAGP_FP64_REFORM n <= 52, and LAGP_FP64 every candidate's factor row on
 * chip (n <= 50 at p = 8, N' = 1024; larger n at smaller p or N').  Others
 * return LAGP_EUNSUPPORTED (lagp_alc_uneven_from_pool covers them in float64).
 */
lagp_status lagp_alc_from_pool(const double *X, const double *Y, int64_t N, int32_t p,
                               const double *XX, int64_t M, const int32_t *pool, int32_t Np,
                               int32_t n0, int32_t n, double d, double g, int32_t precision,
                               double *mean, double *s2, double *var, int32_t *sel, double *alc,
                               double *alc32, int32_t *status, int32_t *guard, void *stream);

/*
 * lagp_alc_scores -- the scores of a batch of candidates against one design,
 * given K_j^{-1}: the per-step computation of the paper's GPU kernel (Fig. 3
 * steps 2-6, with the sign of eq. piedef), over all candidates in one launch.
 *
 *   Xj [j x p]     design X_j             Kinv [j x j]  K_j^{-1}, K_j =
 *                                                       K(X_j, X_j) + g I
 *                                                       (symmetric: read by
 *                                                       rows or by columns)
 *   Xc [Nc x p]    candidates             x [p], h [j]  location and K(X_j, x)
 *   d, g           lengthscale and nugget (finite, > 0)
 *   precision      LAGP_FP64: float64 throughout; LAGP_MIXED: kernel values,
 *                  the products with K_j^{-1} and the scores in float32 with
 *                  float32 accumulation (K_j^{-1} and w = K_j^{-1} h are formed
 *                  or rounded from the float64 inputs)
 *   delta [Nc]     out: v_j(x) - v_{j+1}(x) for each candidate (eq. dxy),
 *                  computed as (K(c,x) - k_c^T K_j^{-1} h)^2 / s_c with
 *                  s_c = 1 + g - k_c^T K_j^{-1} k_c; -INFINITY where s_c <= 0
 * The quadratic forms k_c^T K_j^{-1} k_c of candidate tiles are products on
 * the matrix cores (16x16x4 MFMA); K_j^{-1} is staged in LDS up to j = 128
 * and read from global memory (L2) beyond.  Supported: 1 <= j <= 512,
 * p <= 16 (the design sizes of the paper's ALC-in-isolation sweep, Sec. 4);
 * Nc = 0 is a no-op.
 */
lagp_status lagp_alc_scores(const double *Xj, int32_t j, int32_t p, const double *Kinv, const double *Xc,
                            int64_t Nc, const double *x, const double *h, double d, double g,
                            int32_t precision, double *delta, void *stream);

/*
 * lagp_mspe_workspace -- bytes of device workspace lagp_mspe_from_pool needs
 *   for M locations with pools of Np and designs of n points (about
 *   16 n Np bytes per resident workgroup; 0 for M = 0).
 * lagp_mspe_from_pool -- local designs by the MSPE criterion (Sec. 2.2,
 *   eq. mspe with the variance term of eq. newv) instead of ALC, and the
 *   local predictions on them.  From the NN start of n0 pool points, step j
 *   adds the candidate minimising
 *     J(x') = (j + 1) psi_j / (j (j - 1)) v_{j+1}(x) + (d mu_j / dd)^2 / G_{j+1}
 *   with psi_j = Y_j^T K_j^{-1} Y_j, v_{j+1}(x) the predictive variance term
 *   kappa - k^T K^{-1} k on X_j + {x'}, d mu_j / dd the derivative of the
 *   predictive mean (eq. predgp) in the lengthscale, and G_{j+1} read as the
 *   expected information about d in j + 1 responses of N(0, tau^2 K_{j+1})
 *   with the scale tau^2 unknown: (tr(W^2) - tr(W)^2 / (j + 1)) / 2,
 *   W = K_{j+1}^{-1} dK_{j+1}/dd.  Exact ties go to the smaller design index.
 *   Arguments, pools, outputs and status codes as for lagp_alc_from_pool
 *   (float64 only); crit [M x n] receives J of each chosen point (NaN for
 *   j < n0).  workspace: at least lagp_mspe_workspace(M, Np, n) bytes,
 *   256-byte aligned (else LAGP_EWORKSPACE); calls that overlap must not
 *   share it.  Requires 2 <= n0 <= n <= Np <= N (EINVAL); supported p <= 8,
 *   Np <= 1024, n <= 64 (else LAGP_EUNSUPPORTED).  M = 0 is a no-op.
 */
lagp_status lagp_mspe_workspace(int64_t M, int32_t Np, int32_t n, size_t *bytes);
lagp_status lagp_mspe_from_pool(const double *X, const double *Y, int64_t N, int32_t p, const double *XX,
                                int64_t M, const int32_t *pool, int32_t Np, int32_t n0, int32_t n, double d,
                                double g, double *mean, double *s2, double *var, int32_t *sel, double *crit,
                                int32_t *status, void *workspace, size_t workspace_bytes, void *stream);

/*
 * ---------------------------------------------------------------------------
 * The whole hot path in one call: problem and outputs as structs.
 *
 * Every struct begins with struct_size, which the caller sets to
 * sizeof(struct) as compiled against this header: the library rejects any
 * other value with LAGP_EINVAL (an ABI guard: a caller built against another
 * layout of the structs fails loudly instead of passing shifted fields).
 * lagp_abi_version() returns LAGP_ABI_VERSION of the library.
 */
#define LAGP_ABI_VERSION 3

/* lagp_problem.flags */
#define LAGP_NORMALIZE_ALC 1u  /* report each selected point's score multiplied */
                               /* by psi_j / (j - 2), psi_j = Y_j^T K_j^{-1} Y_j */
                               /* of the design it was chosen for: the          */
                               /* normalisation by the global variance estimate  */
                               /* of Sec. 3.1 (Fig. 3 step 9).  The choices are  */
                               /* unchanged (the factor is positive and common   */
                               /* to all candidates of a step).  Needs n0 >= 3.  */
#define LAGP_NN_BRUTE 2u       /* pools by streaming the whole design for every */
                               /* location (lagp_nn_pool) instead of the grid of */
                               /* lagp_nn_pool_ws; the pools are identical       */

typedef struct lagp_problem {
    uint32_t struct_size;      /* = sizeof(lagp_problem)                          */
    uint32_t flags;            /* LAGP_NORMALIZE_ALC | LAGP_NN_BRUTE              */
    const double *X;           /* [N x p] design                                   */
    const double *Y;           /* [N] responses (used raw: zero-mean GP)           */
    const double *XX;          /* [M x p] predictive locations                     */
    int64_t N, M;              /* 1 <= N < 2^31; M >= 0 (M = 0: nothing to do)     */
    int32_t p;                 /* 1 <= p <= 8                                       */
    int32_t n0;                /* start size: the n0 nearest (Fig. 1 step 2a)      */
    int32_t n;                 /* final design size, or the largest n_per[m]       */
    int32_t Np;                /* candidate pool size N', or the largest Np_per[m] */
    const int32_t *n_per;      /* [M] per-location n, or NULL (n everywhere)       */
    const int32_t *Np_per;     /* [M] per-location N', or NULL (Np everywhere)     */
    const double *d_per;       /* [M] per-location lengthscale, or NULL (d)        */
    double d, g;               /* lengthscale and nugget, finite and > 0           */
    int32_t precision;         /* LAGP_FP64, LAGP_MIXED or LAGP_FP64_REFORM        */
    int32_t reserved;          /* 0                                                */
    const double *d_sep;       /* [p] lengthscales of the separable kernel, or    */
                               /* NULL (isotropic, d / d_per): K(x, x') =         */
                               /* exp(-sum_k (x_k - x'_k)^2 / d_sep[k]), the      */
                               /* vectorised lengthscale of Sec. 3.1; d is then   */
                               /* unused.  LAGP_FP64 only, not with d_per.  The   */
                               /* pools stay Euclidean.  A d_sep entry that is    */
                               /* not finite and > 0 gives every location         */
                               /* LAGP_LOC_BAD_SHAPE.                             */
} lagp_problem;

typedef struct lagp_outputs {
    uint32_t struct_size;      /* = sizeof(lagp_outputs)                          */
    uint32_t reserved;         /* 0                                                */
    double *mean, *s2, *var;   /* [M] each, nullable: eqs. predgp, preds2 (N -> n) */
    int32_t *sel;              /* design indices, required: row m at sel_off[m],  */
                               /* or at m * n padded with -1 past n_per[m]         */
    const int64_t *sel_off;    /* [M + 1] int64 row offsets of sel / alc / alc32,  */
                               /* or NULL                                          */
    double *alc;               /* nullable: score of each added point (eq. dxy),   */
                               /* NaN before n0 and in padding                     */
    double *alc32;             /* nullable: LAGP_MIXED float32 score of that point */
    int32_t *pool;             /* [M x Np] nullable: the candidate pools; NULL     */
                               /* keeps them in the workspace                      */
    int32_t *status;           /* [M] nullable: LAGP_LOC_* codes                   */
    int32_t *guard;            /* [M] nullable: steps of the location decided in   */
                               /* float64 under LAGP_MIXED (see below); 0 else     */
} lagp_outputs;

/*
 * lagp_alc_workspace -- bytes of device workspace that lagp_alc_predict and
 *   lagp_plan_create need for this problem on the current device: the grid of
 *   the design (unless LAGP_NN_BRUTE), the location queues and factor-row
 *   entries of per-location designs, and room for the M x Np pools (used
 *   only when outputs->pool is NULL).  Arguments are checked as by
 *   lagp_alc_predict.
 *
 * lagp_alc_predict -- for every location: the N' nearest design rows (Sec.
 *   2.2, Sec. 3.1), the greedy ALC design from the n0 nearest to n points
 *   (Fig. 1 steps 2a, 2b; eqs. dxy, piedef) and the local prediction (eqs.
 *   predgp, preds2; Fig. 1 step 5).  Uniform sizes (n_per, Np_per, d_per and
 *   sel_off all NULL) run one workgroup per location with the arithmetic of
 *   `precision`; otherwise locations are ordered by cost on the device and
 *   drained by persistent workgroups.  With per-location sizes, LAGP_MIXED
 *   scores the locations with n_m <= 64, N'_m <= 1024 and
 *   (n_m + g) / g * 2^-24 <= 2^-4 (the conditioning rule of
 *   lagp_alc_from_pool) in mixed precision and computes the others in
 *   float64, counting all of their n_m - n0 steps in guard[m];
 *   LAGP_FP64_REFORM needs uniform sizes.
 *   workspace: device memory of at least lagp_alc_workspace bytes, 256-byte
 *   aligned (else LAGP_EWORKSPACE); calls that overlap must not share it.
 *   Supported: p <= 8, N' <= 2048, n <= 128 (float64; LAGP_MIXED n <= 64 and
 *   N' <= 1024 for uniform sizes, LAGP_FP64_REFORM n <= 52 and N' <= 1024);
 *   others return LAGP_EUNSUPPORTED.  Requires 1 <= n0 <= n_m <= N'_m <= N.
 */
lagp_status lagp_alc_workspace(const lagp_problem *prob, size_t *bytes);
lagp_status lagp_alc_predict(const lagp_problem *prob, const lagp_outputs *out, void *workspace,
                             size_t workspace_bytes, void *stream);

/* LAGP_ABI_VERSION of the library. */
int32_t lagp_abi_version(void);

/*
 * lagp_alc_uneven_workspace -- bytes of device workspace that
 * lagp_alc_uneven_from_pool needs for these bounds on the current device.
 */
lagp_status lagp_alc_uneven_workspace(int32_t p, int64_t M, int32_t Np_max, int32_t n_max, size_t *bytes);

/*
 * lagp_alc_uneven_from_pool -- lagp_alc_from_pool with a design size n_m
 * and a pool size N'_m of its own for every location (float64).
 *
 *   pool [M x Np_max]       pools as written by lagp_nn_pool with Np_max;
 *                           location m uses its first N'_m entries, which are
 *                           exactly its N'_m nearest neighbours
 *   n_per [M], Np_per [M]   per-location n and N' (device int32; NULL means
 *                           n_max, respectively Np_max, everywhere); each
 *                           needs n0 <= n_m <= n_max and n_m <= N'_m <= Np_max,
 *                           else status[m] = LAGP_LOC_BAD_SHAPE
 *   sel_off [M + 1]         device int64 row offsets of sel and alc (row m is
 *                           [sel_off[m], sel_off[m] + n_m)); NULL: row m
 *                           starts at m * n_max and entries n_m .. n_max - 1
 *                           are set to -1 (alc NaN)
 *   d_per [M]               per-location lengthscale (device float64; NULL
 *                           means d everywhere), e.g. the d_hat of
 *                           lagp_local_mle_d for a second design stage with
 *                           each location's own estimate (Fig. 1 step 4);
 *                           each must be finite and > 0, else status[m] =
 *                           LAGP_LOC_BAD_SHAPE
 *   workspace               device memory of at least the size reported by
 *                           lagp_alc_uneven_workspace (else LAGP_EWORKSPACE);
 *                           holds the location queue and the factor-row
 *                           entries that do not fit on chip.  Calls that
 *                           overlap must not share it.
 * Locations are ordered on the device by pool size class and then by
 * decreasing cost N'_m n_m^2; persistent workgroups take them from that
 * queue.  Other arguments and outputs as for lagp_alc_from_pool.
 * Supported: precision LAGP_FP64, p <= 8, Np_max <= 2048, n_max <= 128.
 */
lagp_status lagp_alc_uneven_from_pool(const double *X, const double *Y, int64_t N, int32_t p,
                                      const double *XX, int64_t M, const int32_t *pool, int32_t Np_max,
                                      int32_t n0, int32_t n_max, const int32_t *n_per,
                                      const int32_t *Np_per, const int64_t *sel_off, const double *d_per,
                                      double d, double g, int32_t precision, double *mean, double *s2,
                                      double *var, int32_t *sel, double *alc, int32_t *status,
                                      int32_t *guard, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Plans: lagp_alc_predict for one problem, bound to its buffers, autotuned
 * and captured into one HIP graph.
 *
 * lagp_plan_create -- arguments as for lagp_alc_predict (the workspace of
 *   lagp_alc_workspace).  Unless plan_flags has LAGP_PLAN_NO_TUNE, the plan
 *   first times the variants of each tunable launch on these inputs, on at
 *   most their first 65,536 locations, and keeps the fastest: the NN variant
 *   (the grid-pruned pools, one, two or four locations per workgroup over the
 *   whole design, or one over a float32 copy of it), for each pool-size class
 *   of the float64 ALC kernel that the locations fall into (pools of up to
 *   256, 512, 1024, 2048) the schedule that serves it among those that can:
 *   threads per location (256, 512 or 1024), pool positions per lane and
 *   factor entries kept in registers, and for each schedule that runs how the
 *   chosen factor row reaches the lanes.  A change is kept if it is at least
 *   1 % faster.  LAGP_PLAN_SCHEDULE(s) in plan_flags instead runs schedule s
 *   (0 <= s < LAGP_PLAN_SCHEDULES) for every class it can serve, without
 *   timing schedules (diagnostics; the results are the same bits on every
 *   schedule).  The chosen launches are then captured into a graph.  Creation runs the
 *   path on `stream` (several times when tuning), synchronises it, and
 *   finally enqueues one graph launch, whose results the outputs hold once
 *   `stream` has been synchronised.  M >= 1.  Every buffer the structs point
 *   to must stay allocated until the plan is destroyed (the structs
 *   themselves are copied).
 * lagp_plan_launch -- enqueues one run (one graph launch) on `stream`.
 * lagp_plan_describe -- the timings and the chosen variants, as text.
 * lagp_plan_destroy -- frees the plan (NULL is a no-op).
 */
typedef struct lagp_plan_s *lagp_plan;
#define LAGP_PLAN_NO_TUNE 1
#define LAGP_PLAN_SCHEDULES 6
#define LAGP_PLAN_SCHEDULE(s) ((int32_t)((s) + 1) << 8)

lagp_status lagp_plan_create(const lagp_problem *prob, const lagp_outputs *out, void *workspace,
                             size_t workspace_bytes, int32_t plan_flags, void *stream, lagp_plan *plan);
lagp_status lagp_plan_launch(lagp_plan plan, void *stream);
lagp_status lagp_plan_describe(lagp_plan plan, char *buf, size_t len);
lagp_status lagp_plan_destroy(lagp_plan plan);

/*
 * Local likelihood on fixed local designs (Sec. 2.1 eq. gpk, Fig. 1 step 3).
 * For each location m the design is rows sel[m][0 .. n-1] of X (sel: M x n
 * int32, e.g. the `sel` output of lagp_alc_from_pool), with responses Y.
 * K = exp(-||x_a - x_b||^2 / d) + g I.  The negative log likelihood is
 *   nll = -lgamma(n/2) + (n/2) log(2 pi) + (1/2) log|K| + (n/2) log(psi/2),
 *   psi = Y^T K^{-1} Y.
 * Supported: 1 <= n <= 64, p <= 16.  All arithmetic in float64.
 * Per-location status (nullable): 0 ok, 1 K not positive definite or the
 * value not finite, 4 a design index outside [0, N).
 *
 * lagp_local_nll -- nll[M] and, for every non-NULL output, dnll_dd[M],
 *   dnll_dg[M], d2nll_dd2[M] at d[M], g[M] (device arrays, > 0).
 */
lagp_status lagp_local_nll(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                           int64_t M, int32_t n, const double *d, const double *g, double *nll,
                           double *dnll_dd, double *dnll_dg, double *d2nll_dd2, int32_t *status,
                           void *stream);

/*
 * lagp_local_nll_backward -- hand-written reverse pass of lagp_local_nll:
 *   grad_d[m] = grad_out[m] * dnll/dd,  grad_g[m] = grad_out[m] * dnll/dg
 * (grad_out NULL means ones; either gradient output may be NULL).
 */
lagp_status lagp_local_nll_backward(const double *X, const double *Y, int64_t N, int32_t p,
                                    const int32_t *sel, int64_t M, int32_t n, const double *d,
                                    const double *g, const double *grad_out, double *grad_d,
                                    double *grad_g, void *stream);

/*
 * lagp_local_mle_d -- maximum-likelihood lengthscale per location with the
 * nugget g fixed (Fig. 1 step 3): projected Newton on [dmin, dmax] from
 * d0[m] with analytic first and second derivatives, backtracking halvings
 * (at most 40) to sufficient decrease nll(d+s) <= nll(d) + 1e-4 nll'(d) s,
 * a gradient step of 0.1 d when nll'' <= 0; stops when |step| <= 1e-10 d,
 * |nll'| <= 1e-10, on a bound with nll' pointing out, or after maxit steps.
 * Outputs: d_hat[M], nll[M] (nullable), iters[M] (nullable), status[M]
 * (nullable: 0 converged, 1 not PD, 2 iteration limit, 3 line search failed,
 * 4 bad design index).
 */
lagp_status lagp_local_mle_d(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                             int64_t M, int32_t n, const double *d0, double g, double dmin, double dmax,
                             int32_t maxit, double *d_hat, double *nll, int32_t *iters, int32_t *status,
                             void *stream);

/*
 * lagp_local_predict -- predictive mean, scale and variance at XX[m] (M x p)
 * on the fixed design sel[m] with per-location lengthscale d[M] and nugget
 * g (eqs. predgp, preds2 with N -> n; Fig. 1 step 5).  status as above.
 */
lagp_status lagp_local_predict(const double *X, const double *Y, int64_t N, int32_t p, const int32_t *sel,
                               int64_t M, int32_t n, const double *XX, const double *d, double g,
                               double *mean, double *s2, double *var, int32_t *status, void *stream);

/* Name of a status code. */
const char *lagp_status_string(lagp_status s);

/* Message describing the calling thread's last failed call ("" if none). */
const char *lagp_last_error(void);

/* Library version string. */
const char *lagp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LAGP_ALC_H */
