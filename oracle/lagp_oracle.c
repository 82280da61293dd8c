/*
 * Plain FP64 CPU oracle for local approximate GP regression with greedy
 * ALC (active learning Cohn) local designs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the GPU library.
 *
 * Method (Gramacy, Niemi & Weiss, "Massively parallel approximate Gaussian
 * process regression", arXiv:1310.5182):
 *   - Sec. 2.1: isotropic Gaussian correlation K(x,x') = exp(-||x-x'||^2/d),
 *     nugget g on the diagonal of the design covariance only; predictive
 *     mean (eq. predgp) mu = k^T K^{-1} Y, scale (eq. preds2)
 *     s2 = psi [K(x,x) - k^T K^{-1} k] / n with psi = Y^T K^{-1} Y,
 *     variance V = s2 n / (n - 2).
 *   - Sec. 2.2 / Fig. 1: local design for each predictive location x:
 *     nearest-neighbour start X_{n0}(x), then for j = n0..n-1 add the
 *     candidate that maximises the reduction in predictive variance
 *     v_j(x) - v_{j+1}(x) (eqs. newv and dxy).
 *   - Sec. 3.1: candidates restricted to the N' nearest neighbours of x.
 *
 * Mode A (the plain definition) recomputes a Cholesky factor L_j of K_j at
 * every step.  For a candidate c with k_c = K(X_j, c), z_c = L_j^{-1} k_c and
 * z_h = L_j^{-1} K(X_j, x), the conditional (given D_j) variance of c is
 * s_c = kappa - z_c.z_c and its conditional covariance with x is
 * cov_c = K(c, x) - z_c.z_h; adding c reduces the variance at x by exactly
 * cov_c^2 / s_c (the textbook rank-one conditioning identity), which is the
 * quantity v_j(x) - v_{j+1}(x) of eq. dxy.
 *
 * Mode B (optional, for route noise) is the paper's own route: K_j^{-1}
 * carried by the partitioned-inverse update (eq. piedef) and the score
 * evaluated term by term as printed in eq. dxy.
 *
 * Readings of the paper taken here:
 *   - kappa = K(x',x') = 1 + g for candidates and for the predictive location
 *     (Fig. 3 step 5 uses 1 + eta); cross-covariances carry no nugget.
 *   - the score is the unnormalised reduction (Sec. 3.1, last paragraph:
 *     normalisation does not change the argmax).
 *   - candidates at step j are the pool minus X_j; X_{n0} is the first n0
 *     pool entries, the pool sorted by (squared distance, design index).
 *   - exact ties in the score go to the smallest design index.
 *   - a candidate whose computed conditional variance s_c is not positive is
 *     numerically a duplicate of the design and is never selected.
 *
 * Squared distances are summed left to right over coordinates; the file is
 * compiled with -ffp-contract=off so no multiply-add is fused.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORC_OK = 0,
    ORC_INIT_NOT_PD = 1,   /* K_{n0} not positive definite                 */
    ORC_STEP_FAIL = 2,     /* K_j not positive definite / no valid choice  */
    ORC_NONFINITE = 3,     /* non-finite input                             */
    ORC_BAD_FORCED = 4,    /* forced sequence not a valid pool sequence    */
    ORC_BAD_ARGS = 5,
};

/* ||a - b||^2, summed left to right (no contraction). */
static double sqdist(const double *a, const double *b, int p)
{
    double s = 0.0;
    for (int k = 0; k < p; k++) {
        double t = a[k] - b[k];
        s = s + t * t;
    }
    return s;
}

/* Isotropic Gaussian correlation, Sec. 2.1. */
static double kern(const double *a, const double *b, int p, double d)
{
    return exp(-sqdist(a, b, p) / d);
}

/* The separable version with one lengthscale per input (the vectorised
 * lengthscale Sec. 3.1 names as a simple modification of the candidate-vector
 * steps): exp(-sum_k (a_k - b_k)^2 / dsep_k), summed left to right.  dsep NULL:
 * the isotropic kernel with lengthscale d. */
static double kern2(const double *a, const double *b, int p, double d, const double *dsep)
{
    if (!dsep) return kern(a, b, p, d);
    double s = 0.0;
    for (int k = 0; k < p; k++) {
        double t = a[k] - b[k];
        s = s + t * t / dsep[k];
    }
    return exp(-s);
}

/* ------------------------------------------------------------------ */
/* Nearest-neighbour pool (Sec. 2.2 NN sub-design; Sec. 3.1 N' NNs).    */
/* ------------------------------------------------------------------ */

typedef struct {
    double key;
    int32_t idx;
} keyed;

static int cmp_keyed(const void *pa, const void *pb)
{
    const keyed *a = (const keyed *)pa, *b = (const keyed *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Pool of the Np nearest rows of X (N x p) to each row of XX (M x p),
 * sorted by (squared distance, index).  pool is M x Np. */
int orc_nn_pool(const double *X, int64_t N, int p, const double *XX, int64_t M,
                int Np, int32_t *pool, int nthreads)
{
    if (Np < 1 || Np > N || p < 1) return ORC_BAD_ARGS;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int bad = 0;
#pragma omp parallel
    {
        keyed *buf = (keyed *)malloc(sizeof(keyed) * (size_t)N);
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t m = 0; m < M; m++) {
                const double *x = XX + m * p;
                for (int64_t i = 0; i < N; i++) {
                    buf[i].key = sqdist(X + i * p, x, p);
                    buf[i].idx = (int32_t)i;
                }
                qsort(buf, (size_t)N, sizeof(keyed), cmp_keyed);
                for (int r = 0; r < Np; r++) pool[m * Np + r] = buf[r].idx;
            }
            free(buf);
        }
    }
    return bad ? ORC_BAD_ARGS : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Dense linear algebra (plain, unblocked).                             */
/* ------------------------------------------------------------------ */

/* Lower Cholesky factor of the j x j SPD matrix A (row-major) into L.
 * Returns 0 on success, 1 if a pivot is not positive. */
static int cholesky(const double *A, double *L, int j)
{
    memset(L, 0, sizeof(double) * (size_t)j * j);
    for (int r = 0; r < j; r++) {
        for (int c = 0; c <= r; c++) {
            double s = A[r * j + c];
            for (int k = 0; k < c; k++) s -= L[r * j + k] * L[c * j + k];
            if (r == c) {
                if (!(s > 0.0)) return 1;
                L[r * j + r] = sqrt(s);
            } else {
                L[r * j + c] = s / L[c * j + c];
            }
        }
    }
    return 0;
}

/* Solve L z = b (L lower triangular, j x j). */
static void forward_solve(const double *L, const double *b, double *z, int j)
{
    for (int r = 0; r < j; r++) {
        double s = b[r];
        for (int k = 0; k < r; k++) s -= L[r * j + k] * z[k];
        z[r] = s / L[r * j + r];
    }
}

/* Solve L^T z = b. */
static void backward_solve_t(const double *L, const double *b, double *z, int j)
{
    for (int r = j - 1; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < j; k++) s -= L[k * j + r] * z[k];
        z[r] = s / L[r * j + r];
    }
}

static double dot(const double *a, const double *b, int j)
{
    double s = 0.0;
    for (int k = 0; k < j; k++) s += a[k] * b[k];
    return s;
}

/* ------------------------------------------------------------------ */
/* GP prediction from a fixed design (eqs. predgp and preds2).          */
/* ------------------------------------------------------------------ */

/* Design rows D (n x p, row-major), responses Yd (n), location x.
 * out[0] = mean, out[1] = s2 (Student-t scale, df n), out[2] = V = s2 n/(n-2)
 * (NaN if n <= 2), out[3] = v = kappa - k^T K^{-1} k, out[4] = psi.
 * Returns 0, or 1 if K is not positive definite. */
static int gp_predict(const double *D, const double *Yd, int n, int p, const double *x,
                      double d, const double *dsep, double g, double *out)
{
    double kappa = 1.0 + g;
    double *K = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *L = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *h = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *alpha = (double *)malloc(sizeof(double) * (size_t)n);
    double *zh = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    for (int a = 0; a < n; a++) {
        for (int b = 0; b < n; b++) K[a * n + b] = kern2(D + a * p, D + b * p, p, d, dsep);
        K[a * n + a] += g;
        h[a] = kern2(D + a * p, x, p, d, dsep);
    }
    if (cholesky(K, L, n)) {
        rc = 1;
        for (int q = 0; q < 5; q++) out[q] = NAN;
    } else {
        forward_solve(L, Yd, w, n);
        backward_solve_t(L, w, alpha, n);
        forward_solve(L, h, zh, n);
        double mu = dot(h, alpha, n);
        double psi = dot(Yd, alpha, n);
        double v = kappa - dot(zh, zh, n);
        double s2 = psi * v / n;
        out[0] = mu;
        out[1] = s2;
        out[2] = n > 2 ? s2 * n / (n - 2) : NAN;
        out[3] = v;
        out[4] = psi;
    }
    free(K); free(L); free(h); free(w); free(alpha); free(zh);
    return rc;
}

int orc_gp_predict(const double *D, const double *Yd, int n, int p, const double *x,
                   double d, double g, double *out)
{
    return gp_predict(D, Yd, n, p, x, d, NULL, g, out);
}

/* orc_gp_predict with the separable kernel (dsep: p lengthscales). */
int orc_gp_predict_sep(const double *D, const double *Yd, int n, int p, const double *x,
                       const double *dsep, double g, double *out)
{
    return gp_predict(D, Yd, n, p, x, 1.0, dsep, g, out);
}

/* ------------------------------------------------------------------ */
/* Greedy ALC local design for one location (Fig. 1 steps 2a, 2b, 5).   */
/* ------------------------------------------------------------------ */

typedef struct {
    /* per step j = 0..n-1 (entries j < n0 describe the NN start) */
    int32_t *sel;     /* design index added at step j                        */
    double *dsel;     /* mode-A score of that choice (NaN for j < n0)        */
    double *dmax;     /* best mode-A score at step j (NaN for j < n0)        */
    int32_t *amax;    /* its design index (-1 for j < n0)                    */
    double *dsecond;  /* runner-up score (NaN if none)                       */
    double *nu;       /* route noise max|dA - dB| / dmax (NaN if mode B off) */
    double *vtraj;    /* v_j(x) before step j, and v_n at index n (n + 1)   */
    double *psitraj;  /* psi_j = Y_j^T K_j^{-1} Y_j before step j (0 at j=0) */
    double pred[5];   /* mean, s2, V, v, psi on the final design             */
    double pred_b[5]; /* the same from the mode-B inverse (NaN if mode B off) */
} orc_trace;

typedef struct {
    double *K, *L, *h, *zh, *kc, *zc, *Kinv, *Kinv2, *u, *gv, *Dn, *Yn, *yj, *ty;
    uint8_t *chosen;
} orc_work;

static int work_alloc(orc_work *w, int n, int Np, int p)
{
    size_t nn = (size_t)n * n;
    w->K = (double *)malloc(sizeof(double) * nn);
    w->L = (double *)malloc(sizeof(double) * nn);
    w->Kinv = (double *)malloc(sizeof(double) * nn);
    w->Kinv2 = (double *)malloc(sizeof(double) * nn);
    w->h = (double *)malloc(sizeof(double) * n);
    w->zh = (double *)malloc(sizeof(double) * n);
    w->kc = (double *)malloc(sizeof(double) * n);
    w->zc = (double *)malloc(sizeof(double) * n);
    w->u = (double *)malloc(sizeof(double) * n);
    w->gv = (double *)malloc(sizeof(double) * n);
    w->Dn = (double *)malloc(sizeof(double) * (size_t)n * p);
    w->Yn = (double *)malloc(sizeof(double) * n);
    w->yj = (double *)malloc(sizeof(double) * n);
    w->ty = (double *)malloc(sizeof(double) * n);
    w->chosen = (uint8_t *)malloc((size_t)Np);
    return w->K && w->L && w->Kinv && w->Kinv2 && w->h && w->zh && w->kc && w->zc && w->u &&
           w->gv && w->Dn && w->Yn && w->yj && w->ty && w->chosen;
}

static void work_free(orc_work *w)
{
    free(w->K); free(w->L); free(w->Kinv); free(w->Kinv2); free(w->h); free(w->zh);
    free(w->kc); free(w->zc); free(w->u); free(w->gv); free(w->Dn); free(w->Yn);
    free(w->yj); free(w->ty); free(w->chosen);
}

/* Mode B: grow K^{-1} (j x j, row-major, stride j) to (j+1) x (j+1) with the
 * partitioned inverse (eq. piedef): for the new point with k' = K(X_j, x')
 * and kappa, u = K^{-1} k', m^{-1} = kappa - k'.u, g = -m u and
 * K_{j+1}^{-1} = [[K^{-1} + g g^T m^{-1}, g], [g^T, m]]. */
static int piedef_grow(const double *Kinv, double *Kout, const double *kp, double kappa,
                       double *u, double *gv, int j)
{
    for (int a = 0; a < j; a++) u[a] = dot(Kinv + a * j, kp, j);
    double minv = kappa - dot(kp, u, j);
    if (!(minv > 0.0)) return 1;
    double m = 1.0 / minv;
    for (int a = 0; a < j; a++) gv[a] = -m * u[a];
    int J = j + 1;
    for (int a = 0; a < j; a++) {
        for (int b = 0; b < j; b++) Kout[a * J + b] = Kinv[a * j + b] + gv[a] * gv[b] * minv;
        Kout[a * J + j] = gv[a];
        Kout[j * J + a] = gv[a];
    }
    Kout[j * J + j] = m;
    return 0;
}

/* Mode B prediction on a fixed design (eqs. predgp, preds2): K_n^{-1} grown
 * row by row over the design in the given order by the partitioned inverse
 * (eq. piedef), then mu = h^T K^{-1} Y, psi = Y^T K^{-1} Y, v = kappa -
 * h^T K^{-1} h.  out as for orc_gp_predict.  Returns 0, or 1 if a Schur
 * complement is not positive. */
int orc_gp_predict_b(const double *D, const double *Yd, int n, int p, const double *x,
                     double d, double g, double *out)
{
    const double kappa = 1.0 + g;
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *B = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *kp = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *gv = (double *)malloc(sizeof(double) * (size_t)n);
    double *h = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    for (int j = 0; j < n && rc == 0; j++) {
        for (int a = 0; a < j; a++) kp[a] = kern(D + (size_t)a * p, D + (size_t)j * p, p, d);
        if (piedef_grow(A, B, kp, kappa, u, gv, j)) rc = 1;
        double *t = A; A = B; B = t;
    }
    if (rc) {
        for (int q = 0; q < 5; q++) out[q] = NAN;
    } else {
        double mu = 0.0, psi = 0.0, hwh = 0.0;
        for (int a = 0; a < n; a++) h[a] = kern(D + (size_t)a * p, x, p, d);
        for (int a = 0; a < n; a++) {
            double alpha_a = dot(A + (size_t)a * n, Yd, n);
            mu += h[a] * alpha_a;
            psi += Yd[a] * alpha_a;
            hwh += h[a] * dot(A + (size_t)a * n, h, n);
        }
        double v = kappa - hwh, s2 = psi * v / n;
        out[0] = mu;
        out[1] = s2;
        out[2] = n > 2 ? s2 * n / (n - 2) : NAN;
        out[3] = v;
        out[4] = psi;
    }
    free(A); free(B); free(kp); free(u); free(gv); free(h);
    return rc;
}

/* Mode B score, eq. dxy term by term:
 *   h^T G m^{-1} h + 2 h^T g K(x',x) + K(x',x)^2 m,  G = g g^T. */
static double dxy_score(const double *Kinv, const double *kc, const double *h, double kcx,
                        double kappa, double *u, double *gv, int j)
{
    for (int a = 0; a < j; a++) u[a] = dot(Kinv + a * j, kc, j);
    double minv = kappa - dot(kc, u, j);
    if (!(minv > 0.0)) return -INFINITY;
    double m = 1.0 / minv;
    for (int a = 0; a < j; a++) gv[a] = -m * u[a];
    double hg = dot(h, gv, j);
    return hg * hg * minv + 2.0 * hg * kcx + kcx * kcx * m;
}

/*
 * One location.  X (N x p), Y (N); x (p); pool (Np sorted design indices).
 * forced: NULL for the oracle's own greedy choices, else n design indices to
 * add in that order (the scores of every candidate are still evaluated).
 * Returns a status code; the trace is filled as far as it got.
 */
static int alc_one(const double *X, const double *Y, int p, const double *x,
                   const int32_t *pool, int Np, int n0, int n, double d, const double *dsep, double g,
                   const int32_t *forced, int mode_b, orc_trace *tr, orc_work *w)
{
    const double kappa = 1.0 + g;
    for (int k = 0; k < p; k++)
        if (!isfinite(x[k])) return ORC_NONFINITE;
    memset(w->chosen, 0, (size_t)Np);
    for (int q = 0; q < 5; q++) tr->pred[q] = tr->pred_b[q] = NAN;
    int32_t *slot_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n); /* pool slot of X_j rows */
    int rc = ORC_OK;

    for (int j = 0; j < n; j++) {
        tr->dsel[j] = tr->dmax[j] = tr->dsecond[j] = tr->nu[j] = tr->vtraj[j] = tr->psitraj[j] = NAN;
        tr->amax[j] = -1;
        tr->sel[j] = -1;
    }
    tr->vtraj[n] = NAN;

    /* mode B state */
    double *Kinv = w->Kinv, *Kinv2 = w->Kinv2;

    for (int j = 0; j < n; j++) {
        /* Design covariance K_j and its Cholesky factor (mode A). */
        if (j > 0) {
            for (int a = 0; a < j; a++) {
                const double *xa = X + (int64_t)pool[slot_of[a]] * p;
                for (int b = 0; b < j; b++)
                    w->K[a * j + b] = kern2(xa, X + (int64_t)pool[slot_of[b]] * p, p, d, dsep);
                w->K[a * j + a] += g;
                w->h[a] = kern2(xa, x, p, d, dsep);
                w->yj[a] = Y[pool[slot_of[a]]];
            }
            if (cholesky(w->K, w->L, j)) { rc = j <= n0 ? ORC_INIT_NOT_PD : ORC_STEP_FAIL; break; }
            forward_solve(w->L, w->h, w->zh, j);
            /* psi_j = Y_j^T K_j^{-1} Y_j = |L_j^{-1} Y_j|^2 (Sec. 2.1 eq. preds2) */
            forward_solve(w->L, w->yj, w->ty, j);
        }
        double vj = kappa - (j > 0 ? dot(w->zh, w->zh, j) : 0.0);
        tr->vtraj[j] = vj;
        tr->psitraj[j] = j > 0 ? dot(w->ty, w->ty, j) : 0.0;

        int take_slot = -1;
        if (j < n0) {
            /* NN start X_{n0}: pool entries in order (Fig. 1 step 2a). */
            if (forced) {
                for (int s = 0; s < Np; s++)
                    if (pool[s] == forced[j]) { take_slot = s; break; }
                if (take_slot < 0 || w->chosen[take_slot]) { rc = ORC_BAD_FORCED; break; }
            } else {
                take_slot = j;
            }
        } else {
            /* Score every remaining candidate (Fig. 1 step 2b). */
            double best = -INFINITY, second = -INFINITY, maxdiff = 0.0;
            int best_slot = -1;
            double forced_score = NAN;
            int forced_slot = -1;
            for (int s = 0; s < Np; s++) {
                if (w->chosen[s]) continue;
                const double *xc = X + (int64_t)pool[s] * p;
                for (int a = 0; a < j; a++)
                    w->kc[a] = kern2(X + (int64_t)pool[slot_of[a]] * p, xc, p, d, dsep);
                forward_solve(w->L, w->kc, w->zc, j);
                double sc = kappa - dot(w->zc, w->zc, j);
                double kcx = kern2(xc, x, p, d, dsep);
                double cov = kcx - dot(w->zc, w->zh, j);
                double delta = sc > 0.0 ? cov * cov / sc : -INFINITY;
                if (mode_b) {
                    double db = dxy_score(Kinv, w->kc, w->h, kcx, kappa, w->u, w->gv, j);
                    if (isfinite(delta) && isfinite(db)) {
                        double df = fabs(delta - db);
                        if (df > maxdiff) maxdiff = df;
                    }
                }
                if (forced && pool[s] == forced[j]) { forced_score = delta; forced_slot = s; }
                int better = delta > best ||
                             (delta == best && best_slot >= 0 && pool[s] < pool[best_slot]);
                if (better) {
                    if (best_slot >= 0 && best > second) second = best;
                    best = delta;
                    best_slot = s;
                } else if (delta > second) {
                    second = delta;
                }
            }
            if (best_slot < 0 || !(best > -INFINITY)) { rc = ORC_STEP_FAIL; break; }
            tr->dmax[j] = best;
            tr->amax[j] = pool[best_slot];
            tr->dsecond[j] = second > -INFINITY ? second : NAN;
            tr->nu[j] = mode_b ? maxdiff / best : NAN;
            if (forced) {
                if (forced_slot < 0) { rc = ORC_BAD_FORCED; break; }
                take_slot = forced_slot;
                tr->dsel[j] = forced_score;
            } else {
                take_slot = best_slot;
                tr->dsel[j] = best;
            }
        }

        /* Mode B bookkeeping: grow K^{-1} by the partitioned inverse. */
        if (mode_b) {
            const double *xn = X + (int64_t)pool[take_slot] * p;
            for (int a = 0; a < j; a++) w->kc[a] = kern2(X + (int64_t)pool[slot_of[a]] * p, xn, p, d, dsep);
            if (piedef_grow(Kinv, Kinv2, w->kc, kappa, w->u, w->gv, j)) mode_b = 0;
            double *t = Kinv; Kinv = Kinv2; Kinv2 = t;
        }

        /* D_{j+1} = D_j U (x_{j+1}, y_{j+1}). */
        w->chosen[take_slot] = 1;
        slot_of[j] = take_slot;
        tr->sel[j] = pool[take_slot];
    }

    if (rc == ORC_OK) {
        /* Local prediction on the final design (Fig. 1 step 5). */
        for (int a = 0; a < n; a++) {
            memcpy(w->Dn + (size_t)a * p, X + (int64_t)tr->sel[a] * p, sizeof(double) * p);
            w->Yn[a] = Y[tr->sel[a]];
        }
        if (gp_predict(w->Dn, w->Yn, n, p, x, d, dsep, g, tr->pred)) rc = ORC_STEP_FAIL;
        else tr->vtraj[n] = tr->pred[3];
        /* Mode B: the same prediction from K_n^{-1} as grown by eq. piedef
         * (eqs. predgp, preds2 with the explicit inverse): the output route noise. */
        if (rc == ORC_OK && mode_b) {
            double mu = 0.0, psi = 0.0, hwh = 0.0;
            for (int a = 0; a < n; a++) w->h[a] = kern2(w->Dn + (size_t)a * p, x, p, d, dsep);
            for (int a = 0; a < n; a++) {
                double alpha_a = dot(Kinv + (size_t)a * n, w->Yn, n);
                double wa = dot(Kinv + (size_t)a * n, w->h, n);
                mu += w->h[a] * alpha_a;
                psi += w->Yn[a] * alpha_a;
                hwh += w->h[a] * wa;
            }
            const double v = kappa - hwh, scale = psi * v / n;
            tr->pred_b[0] = mu;
            tr->pred_b[1] = scale;
            tr->pred_b[2] = n > 2 ? scale * n / (n - 2) : NAN;
            tr->pred_b[3] = v;
            tr->pred_b[4] = psi;
        }
    }
    free(slot_of);
    return rc;
}

/*
 * Batched driver over M locations (OpenMP over locations, Sec. 2.2 last
 * paragraph: every location is independent).
 *
 * pool: M x Np_stride design indices (row m holds Np_m valid entries).
 * n_per / Np_per: per-location sizes or NULL for the uniform n / Np.
 * forced: NULL, or M x n_stride sequences to evaluate instead of choosing.
 * Per-step outputs are M x n_stride (row m holds n_m entries); vtraj is
 * M x (n_stride + 1); pred is M x 5.  Any per-step output may be NULL.
 * psitraj (M x n_stride): psi_j = Y_j^T K_j^{-1} Y_j before step j, the
 * global variance estimate of the normalisation of Sec. 3.1 (Fig. 3 step 9).
 * dsep: NULL, or p lengthscales of the separable kernel (kern2), replacing d
 * (not with d_per).
 * pred_b (M x 5): with mode_b, pred recomputed from the K_n^{-1} that the
 * partitioned-inverse update (eq. piedef) built along the design, i.e. the
 * output of the paper's route; its gap to pred measures the output route
 * noise.  NaN without mode_b.
 */
int orc_alc(const double *X, const double *Y, int64_t N, int p, const double *XX, int64_t M,
            const int32_t *pool, int Np_stride, const int32_t *Np_per, int Np,
            const int32_t *n_per, int n, int n_stride, int n0, double d, const double *d_per,
            const double *dsep, double g,
            const int32_t *forced, int mode_b, int nthreads,
            int32_t *sel, double *dsel, double *dmax, int32_t *amax, double *dsecond,
            double *nu, double *vtraj, double *pred, int32_t *status, double *psitraj, double *pred_b)
{
    if (!(d > 0.0) || !(g > 0.0) || !isfinite(d) || !isfinite(g) || p < 1 || n0 < 1)
        return ORC_BAD_ARGS;
    if (dsep) {
        if (d_per) return ORC_BAD_ARGS;  /* one lengthscale per location, or one per input */
        for (int k = 0; k < p; k++)
            if (!(dsep[k] > 0.0) || !isfinite(dsep[k])) return ORC_BAD_ARGS;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        orc_work w;
        int ok = work_alloc(&w, n_stride, Np_stride, p);
        int32_t *t_sel = (int32_t *)malloc(sizeof(int32_t) * n_stride);
        int32_t *t_amax = (int32_t *)malloc(sizeof(int32_t) * n_stride);
        double *t_d = (double *)malloc(sizeof(double) * n_stride * 5);
        double *t_v = (double *)malloc(sizeof(double) * (n_stride + 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t m = 0; m < M; m++) {
            int nm = n_per ? n_per[m] : n;
            int Npm = Np_per ? Np_per[m] : Np;
            const double dm = d_per ? d_per[m] : d;  /* the location's own lengthscale */
            orc_trace tr = {t_sel, t_d, t_d + n_stride, t_amax, t_d + 2 * n_stride,
                            t_d + 3 * n_stride, t_v, t_d + 4 * n_stride, {0}, {0}};
            int rc;
            if (!ok || nm > n_stride || Npm > Np_stride || nm > Npm || n0 > nm || Npm > N || !(dm > 0.0) ||
                !isfinite(dm))
                rc = ORC_BAD_ARGS;
            else
                rc = alc_one(X, Y, p, XX + m * p, pool + m * (int64_t)Np_stride, Npm, n0, nm, dm, dsep, g,
                             forced ? forced + m * (int64_t)n_stride : NULL, mode_b, &tr, &w);
            if (rc == ORC_BAD_ARGS) {
                for (int j = 0; j < n_stride; j++) { t_sel[j] = -1; t_amax[j] = -1; }
                for (int j = 0; j < 5 * n_stride; j++) t_d[j] = NAN;
                for (int j = 0; j <= n_stride; j++) t_v[j] = NAN;
                for (int q = 0; q < 5; q++) tr.pred[q] = tr.pred_b[q] = NAN;
                nm = n_stride;
            }
            if (rc != ORC_OK)
                for (int q = 0; q < 5; q++) tr.pred[q] = tr.pred_b[q] = NAN;
            int64_t o = m * (int64_t)n_stride;
            for (int j = 0; j < nm; j++) {
                if (sel) sel[o + j] = t_sel[j];
                if (dsel) dsel[o + j] = t_d[j];
                if (dmax) dmax[o + j] = t_d[n_stride + j];
                if (amax) amax[o + j] = t_amax[j];
                if (dsecond) dsecond[o + j] = t_d[2 * n_stride + j];
                if (nu) nu[o + j] = t_d[3 * n_stride + j];
                if (psitraj) psitraj[o + j] = t_d[4 * n_stride + j];
            }
            if (vtraj)
                for (int j = 0; j <= nm; j++) vtraj[m * (int64_t)(n_stride + 1) + j] = t_v[j];
            if (pred)
                for (int q = 0; q < 5; q++) pred[m * 5 + q] = tr.pred[q];
            if (pred_b)
                for (int q = 0; q < 5; q++) pred_b[m * 5 + q] = tr.pred_b[q];
            if (status) status[m] = rc;
        }
        if (ok) work_free(&w);
        free(t_sel); free(t_amax); free(t_d); free(t_v);
    }
    return ORC_OK;
}

/* Threads OpenMP would use (for reporting). */
/* ------------------------------------------------------------------ */
/* Scores of a batch of candidates against one design (eq. dxy; the     */
/* quantity the paper's per-step GPU kernel evaluates, Fig. 3).         */
/* ------------------------------------------------------------------ */

/*
 * Design Xj (j x p), location x (p), candidates Xc (Nc x p).  For every
 * candidate c, delta[c] = v_j(x) - v_{j+1}(x) when c is added to the design:
 *   mode_b = 0: the plain definition through a Cholesky factor of K_j,
 *               cov_c^2 / s_c (as in alc_one);
 *   mode_b = 1: the paper's route, K_j^{-1} and the three terms of eq. dxy.
 * -INFINITY where the candidate's conditional variance s_c is not positive.
 * Optional outputs: Kinv (j x j) = K_j^{-1}, formed column by column from the
 * factor, and h (j) = K(X_j, x).  Returns 0, 1 if K_j is not PD, 5 on bad
 * arguments.
 */
int orc_alc_scores(const double *Xj, int j, int p, const double *Xc, int64_t Nc, const double *x,
                   double d, double g, int mode_b, double *Kinv, double *h, double *delta)
{
    if (j < 1 || p < 1 || Nc < 0 || !(d > 0.0) || !(g > 0.0)) return ORC_BAD_ARGS;
    const double kappa = 1.0 + g;
    size_t jj = (size_t)j * j;
    double *K = (double *)malloc(sizeof(double) * jj);
    double *L = (double *)malloc(sizeof(double) * jj);
    double *Ki = (double *)malloc(sizeof(double) * jj);
    double *hv = (double *)malloc(sizeof(double) * (size_t)j);
    double *zh = (double *)malloc(sizeof(double) * (size_t)j);
    double *e = (double *)malloc(sizeof(double) * (size_t)j);
    double *col = (double *)malloc(sizeof(double) * (size_t)j);
    int rc = ORC_OK;
    for (int a = 0; a < j; a++) {
        for (int b = 0; b < j; b++) K[a * j + b] = kern(Xj + (size_t)a * p, Xj + (size_t)b * p, p, d);
        K[a * j + a] += g;
        hv[a] = kern(Xj + (size_t)a * p, x, p, d);
    }
    if (cholesky(K, L, j)) {
        rc = ORC_INIT_NOT_PD;
        goto done;
    }
    /* K^{-1} e_b = L^{-T} L^{-1} e_b */
    for (int b = 0; b < j; b++) {
        for (int a = 0; a < j; a++) e[a] = a == b ? 1.0 : 0.0;
        forward_solve(L, e, zh, j);
        backward_solve_t(L, zh, col, j);
        for (int a = 0; a < j; a++) Ki[a * j + b] = col[a];
    }
    forward_solve(L, hv, zh, j);
    if (Kinv) memcpy(Kinv, Ki, sizeof(double) * jj);
    if (h) memcpy(h, hv, sizeof(double) * (size_t)j);
#pragma omp parallel
    {
        double *kc = (double *)malloc(sizeof(double) * (size_t)j);
        double *z = (double *)malloc(sizeof(double) * (size_t)j);
        double *u = (double *)malloc(sizeof(double) * (size_t)j);
        double *gv = (double *)malloc(sizeof(double) * (size_t)j);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < Nc; c++) {
            const double *xc = Xc + (size_t)c * p;
            for (int a = 0; a < j; a++) kc[a] = kern(Xj + (size_t)a * p, xc, p, d);
            const double kcx = kern(xc, x, p, d);
            if (mode_b) {
                delta[c] = dxy_score(Ki, kc, hv, kcx, kappa, u, gv, j);
            } else {
                forward_solve(L, kc, z, j);
                const double sc = kappa - dot(z, z, j);
                const double cov = kcx - dot(z, zh, j);
                delta[c] = sc > 0.0 ? cov * cov / sc : -INFINITY;
            }
        }
        free(kc);
        free(z);
        free(u);
        free(gv);
    }
done:
    free(K);
    free(L);
    free(Ki);
    free(hv);
    free(zh);
    free(e);
    free(col);
    return rc;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Local likelihood in the lengthscale d (eq. gpk; Fig. 1 step 3).      */
/* ------------------------------------------------------------------ */

/*
 * Negative log of eq. gpk for the design D (n x p) with responses Yd:
 *   nll = -lgamma(n/2) + (n/2) log(2 pi) + (1/2) log|K| + (n/2) log(psi/2),
 *   K = exp(-D2/d) + g I,  psi = Y^T K^{-1} Y.
 * With A = K^{-1}, alpha = A Y, Kd = dK/dd = exp(-D2/d) * D2 / d^2 and
 * Kdd = d2K/dd2 = exp(-D2/d) * (D2^2/d^4 - 2 D2/d^3):
 *   dnll/dd   = (1/2) tr(A Kd) - (n/2) (alpha^T Kd alpha) / psi
 *   dnll/dg   = (1/2) tr(A)    - (n/2) (alpha^T alpha) / psi
 *   d2nll/dd2 = (1/2) tr(A Kdd - A Kd A Kd)
 *               - (n/2) [ (alpha^T Kdd alpha - 2 alpha^T Kd A Kd alpha) / psi
 *                         + (alpha^T Kd alpha)^2 / psi^2 ]
 * out = {nll, dnll/dd, dnll/dg, d2nll/dd2}.  Returns 1 if K is not PD.
 */
int orc_nll(const double *D, const double *Yd, int n, int p, double d, double g, double *out)
{
    size_t nn = (size_t)n * n;
    double *K = (double *)malloc(sizeof(double) * nn);
    double *L = (double *)malloc(sizeof(double) * nn);
    double *A = (double *)malloc(sizeof(double) * nn);
    double *Kd = (double *)malloc(sizeof(double) * nn);
    double *Kdd = (double *)malloc(sizeof(double) * nn);
    double *B = (double *)malloc(sizeof(double) * nn);
    double *e = (double *)malloc(sizeof(double) * n);
    double *col = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *alpha = (double *)malloc(sizeof(double) * n);
    double *v = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            double r2 = sqdist(D + a * p, D + b * p, p);
            double c = exp(-r2 / d);
            K[a * n + b] = c + (a == b ? g : 0.0);
            Kd[a * n + b] = c * r2 / (d * d);
            Kdd[a * n + b] = c * (r2 * r2 / (d * d * d * d) - 2.0 * r2 / (d * d * d));
        }
    if (cholesky(K, L, n)) {
        rc = 1;
        for (int q = 0; q < 4; q++) out[q] = NAN;
    } else {
        /* A = K^{-1}, column by column */
        for (int c = 0; c < n; c++) {
            for (int r = 0; r < n; r++) e[r] = r == c ? 1.0 : 0.0;
            forward_solve(L, e, w, n);
            backward_solve_t(L, w, col, n);
            for (int r = 0; r < n; r++) A[r * n + c] = col[r];
        }
        forward_solve(L, Yd, w, n);
        backward_solve_t(L, w, alpha, n);
        double psi = dot(Yd, alpha, n);
        double logdet = 0.0;
        for (int r = 0; r < n; r++) logdet += 2.0 * log(L[r * n + r]);
        double nll = -lgamma(0.5 * n) + 0.5 * n * log(2.0 * M_PI) + 0.5 * logdet + 0.5 * n * log(0.5 * psi);
        /* B = A Kd */
        for (int r = 0; r < n; r++)
            for (int c = 0; c < n; c++) {
                double s = 0.0;
                for (int k = 0; k < n; k++) s += A[r * n + k] * Kd[k * n + c];
                B[r * n + c] = s;
            }
        double trAKd = 0.0, trAKdd = 0.0, trBB = 0.0, trA = 0.0;
        for (int r = 0; r < n; r++) {
            trAKd += B[r * n + r];
            trA += A[r * n + r];
            for (int c = 0; c < n; c++) {
                trAKdd += A[r * n + c] * Kdd[c * n + r];
                trBB += B[r * n + c] * B[c * n + r];
            }
        }
        /* v = Kd alpha */
        for (int r = 0; r < n; r++) v[r] = dot(Kd + r * n, alpha, n);
        double aKda = dot(alpha, v, n);
        double aa = dot(alpha, alpha, n);
        double aKdda = 0.0;
        for (int r = 0; r < n; r++) aKdda += alpha[r] * dot(Kdd + r * n, alpha, n);
        /* Kd A Kd quadratic form: v^T A v */
        double vAv = 0.0;
        for (int r = 0; r < n; r++) vAv += v[r] * dot(A + r * n, v, n);
        out[0] = nll;
        out[1] = 0.5 * trAKd - 0.5 * n * aKda / psi;
        out[2] = 0.5 * trA - 0.5 * n * aa / psi;
        out[3] = 0.5 * (trAKdd - trBB) - 0.5 * n * ((aKdda - 2.0 * vAv) / psi + aKda * aKda / (psi * psi));
    }
    free(K); free(L); free(A); free(Kd); free(Kdd); free(B);
    free(e); free(col); free(w); free(alpha); free(v);
    return rc;
}

/*
 * Maximum likelihood lengthscale on a fixed local design (Fig. 1 step 3),
 * g held fixed.  The paper only says "Newton-like" with analytic
 * derivatives; the reading taken is a projected Newton iteration on
 * [dmin, dmax]: step -f'/f'' when f'' > 0, else a gradient step of length
 * 0.1 d along -f'; backtracking halvings (at most 40) until the sufficient
 * decrease f(d+s) <= f(d) + 1e-4 f' s holds; stop when |step| <= 1e-10 d,
 * when |f'| <= 1e-10, when the iterate sits on a bound with f' pointing out
 * of the interval, or after maxit iterations.
 * out = {d_hat, nll(d_hat), iterations, status}; status 0 converged,
 * 1 not PD, 2 iteration limit, 3 line search failed.
 */
int orc_mle_d(const double *D, const double *Yd, int n, int p, double d0, double g, double dmin,
              double dmax, int maxit, double *out)
{
    double d = d0 < dmin ? dmin : (d0 > dmax ? dmax : d0);
    double f[4], ft[4];
    int status = 2, it = 0;
    if (orc_nll(D, Yd, n, p, d, g, f)) { out[0] = d; out[1] = NAN; out[2] = 0; out[3] = 1; return 1; }
    for (it = 0; it < maxit; it++) {
        double gr = f[1], h = f[3];
        if (fabs(gr) <= 1e-10 || (d <= dmin && gr > 0.0) || (d >= dmax && gr < 0.0)) { status = 0; break; }
        double step = h > 0.0 ? -gr / h : (gr > 0.0 ? -0.1 * d : 0.1 * d);
        double dn = 0.0;
        int ok = 0;
        for (int half = 0; half < 40; half++) {
            dn = d + step;
            if (dn < dmin) dn = dmin;
            if (dn > dmax) dn = dmax;
            if (orc_nll(D, Yd, n, p, dn, g, ft) == 0 && ft[0] <= f[0] + 1e-4 * gr * (dn - d)) { ok = 1; break; }
            step *= 0.5;
        }
        if (!ok) { status = 3; break; }
        double moved = fabs(dn - d);
        d = dn;
        for (int q = 0; q < 4; q++) f[q] = ft[q];
        if (moved <= 1e-10 * d) { status = 0; it++; break; }
    }
    out[0] = d;
    out[1] = f[0];
    out[2] = it;
    out[3] = status;
    return 0;
}

/* Batched over M designs of n rows (sel: M x n design indices into X). */
int orc_local_mle(const double *X, const double *Y, int p, const int32_t *sel, int64_t M, int n,
                  const double *d0, double g, double dmin, double dmax, int maxit, int nthreads,
                  double *out /* M x 4 */)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *Dn = (double *)malloc(sizeof(double) * (size_t)n * p);
        double *Yn = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t m = 0; m < M; m++) {
            for (int a = 0; a < n; a++) {
                memcpy(Dn + (size_t)a * p, X + (int64_t)sel[m * n + a] * p, sizeof(double) * p);
                Yn[a] = Y[sel[m * n + a]];
            }
            orc_mle_d(Dn, Yn, n, p, d0[m], g, dmin, dmax, maxit, out + m * 4);
        }
        free(Dn);
        free(Yn);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* MSPE criterion for the local design (Sec. 2.2, eqs. mspe and newv). */
/* ------------------------------------------------------------------ */

/*
 * The candidate x' minimising
 *   J(x', x) = V_j(x | x') + (d mu_j(x) / d theta)^2 / G_{j+1}(theta)
 * with theta the lengthscale d (the value the design is built at):
 *   V_j(x | x') = (j + 1) psi_j / (j (j - 1)) * v_{j+1}(x)          (eq. newv)
 *   v_{j+1}(x)  = kappa - k_{j+1}(x)^T K_{j+1}^{-1} k_{j+1}(x),  X_{j+1} = X_j + {x'}
 *   mu_j(x)     = k_j(x)^T K_j^{-1} Y_j                            (eq. predgp)
 *   d mu_j / dd = kdot_j(x)^T K_j^{-1} Y_j - k_j(x)^T K_j^{-1} Kdot_j K_j^{-1} Y_j
 *   G_{j+1}     = (1/2) [tr(W^2) - tr(W)^2 / (j + 1)],  W = K_{j+1}^{-1} Kdot_{j+1}
 * where Kdot = dK/dd = exp(-D/d) * D / d^2 (the nugget does not depend on d)
 * and G is the expected information about d in j + 1 responses of
 * N(0, tau^2 K_{j+1}) with the scale tau^2 unknown (the information of d
 * less what tau^2 absorbs); it does not depend on the unseen response
 * y_{j+1}, so the expectation over the future response is exact.
 *
 * Mode A (plain): for every candidate a fresh Cholesky inverse of K_{j+1}
 * and the products above written out.  Mode B (for route noise): K_{j+1}^{-1}
 * bordered from K_j^{-1} by the partitioned inverse (eq. piedef), so that
 *   v_{j+1} = v_j - cov^2 / s,
 *   tr W_{j+1}   = tr(K_j^{-1} Kdot_j) + e / s,
 *   tr W_{j+1}^2 = tr((K_j^{-1} Kdot_j)^2) + 2 a^T K_j^{-1} a / s + e^2 / s^2,
 * with u = K_j^{-1} k', s = kappa - k'.u, cov = K(x', x) - k_j(x).u,
 * e = u^T Kdot_j u - 2 kdot'.u and a = kdot' - Kdot_j u.
 * nu_j = max over candidates of |J_A - J_B| / |J_min|.
 */

/* Inverse of the SPD matrix A (n x n) through its Cholesky factor (L is
 * scratch); 1 if A is not positive definite. */
static int spd_inverse(const double *A, double *Ai, double *L, double *e, double *t, double *col, int n)
{
    if (cholesky(A, L, n)) return 1;
    for (int c = 0; c < n; c++) {
        for (int r = 0; r < n; r++) e[r] = r == c ? 1.0 : 0.0;
        forward_solve(L, e, t, n);
        backward_solve_t(L, t, col, n);
        for (int r = 0; r < n; r++) Ai[r * n + c] = col[r];
    }
    return 0;
}

typedef struct {
    double *K, *Kd, *Ki, *L, *A1, *Ki1, *Kd1, *W, *e, *t, *col, *h, *hd, *al, *wv, *tmp, *kc, *kdc, *u, *a,
        *ta, *k1;
    int32_t *slot;
    uint8_t *chosen;
} mspe_work;

static int mspe_alloc(mspe_work *w, int n, int Np)
{
    size_t n1 = (size_t)(n + 1);
    double **mats[] = {&w->K, &w->Kd, &w->Ki, &w->L, &w->A1, &w->Ki1, &w->Kd1, &w->W};
    for (int q = 0; q < 8; q++) *mats[q] = (double *)malloc(sizeof(double) * n1 * n1);
    double **vecs[] = {&w->e, &w->t, &w->col, &w->h, &w->hd, &w->al, &w->wv, &w->tmp, &w->kc, &w->kdc, &w->u,
                       &w->a, &w->ta, &w->k1};
    for (int q = 0; q < 14; q++) *vecs[q] = (double *)malloc(sizeof(double) * n1);
    w->slot = (int32_t *)malloc(sizeof(int32_t) * n1);
    w->chosen = (uint8_t *)malloc((size_t)Np);
    int ok = w->slot && w->chosen;
    for (int q = 0; q < 8; q++) ok = ok && *mats[q];
    for (int q = 0; q < 14; q++) ok = ok && *vecs[q];
    return ok;
}

static void mspe_free(mspe_work *w)
{
    double *all[] = {w->K, w->Kd, w->Ki, w->L, w->A1, w->Ki1, w->Kd1, w->W, w->e, w->t, w->col, w->h, w->hd,
                     w->al, w->wv, w->tmp, w->kc, w->kdc, w->u, w->a, w->ta, w->k1};
    for (int q = 0; q < 22; q++) free(all[q]);
    free(w->slot);
    free(w->chosen);
}

/* Correlation and its derivative in d for two rows. */
static void kern_dk(const double *a, const double *b, int p, double d, double *k, double *kd)
{
    const double r2 = sqdist(a, b, p);
    *k = exp(-r2 / d);
    *kd = *k * r2 / (d * d);
}

/* One location.  Per step j (entries j < n0 describe the NN start): sel, the
 * criterion of the choice (jsel), the smallest criterion (jmin) and its design
 * index (amin), the route noise (nu, mode B), d mu_j / dd (dmu) and G_{j+1}
 * of the choice (gsel).  pred as in orc_alc. */
static int mspe_one(const double *X, const double *Y, int p, const double *x, const int32_t *pool, int Np,
                    int n0, int n, double d, double g, const int32_t *forced, int mode_b, int32_t *sel,
                    double *jsel, double *jmin, int32_t *amin, double *nu, double *dmu, double *gsel,
                    double *pred, mspe_work *w)
{
    const double kappa = 1.0 + g;
    for (int k = 0; k < p; k++)
        if (!isfinite(x[k])) return ORC_NONFINITE;
    memset(w->chosen, 0, (size_t)Np);
    for (int q = 0; q < 5; q++) pred[q] = NAN;
    for (int j = 0; j < n; j++) {
        sel[j] = amin[j] = -1;
        jsel[j] = jmin[j] = nu[j] = dmu[j] = gsel[j] = NAN;
    }
    int rc = ORC_OK;
    for (int j = 0; j < n; j++) {
        int take = -1;
        if (j < n0) {
            if (forced) {
                for (int s = 0; s < Np; s++)
                    if (pool[s] == forced[j]) { take = s; break; }
                if (take < 0 || w->chosen[take]) { rc = ORC_BAD_FORCED; break; }
            } else {
                take = j;
            }
        } else {
            /* the current design: K_j, Kdot_j, K_j^{-1}, alpha, w = K^{-1} h, psi_j, v_j */
            for (int a = 0; a < j; a++) {
                const double *xa = X + (int64_t)pool[w->slot[a]] * p;
                for (int b = 0; b < j; b++) {
                    double kv, kdv;
                    kern_dk(xa, X + (int64_t)pool[w->slot[b]] * p, p, d, &kv, &kdv);
                    w->K[a * j + b] = kv + (a == b ? g : 0.0);
                    w->Kd[a * j + b] = kdv;
                }
                kern_dk(xa, x, p, d, &w->h[a], &w->hd[a]);
            }
            if (spd_inverse(w->K, w->Ki, w->L, w->e, w->t, w->col, j)) { rc = ORC_STEP_FAIL; break; }
            double psi = 0.0, hw = 0.0, hd_al = 0.0, w_kd_al = 0.0;
            for (int a = 0; a < j; a++) {
                w->al[a] = 0.0;
                w->wv[a] = 0.0;
                for (int b = 0; b < j; b++) {
                    w->al[a] += w->Ki[a * j + b] * Y[pool[w->slot[b]]];
                    w->wv[a] += w->Ki[a * j + b] * w->h[b];
                }
            }
            for (int a = 0; a < j; a++) {
                psi += Y[pool[w->slot[a]]] * w->al[a];
                hw += w->h[a] * w->wv[a];
                hd_al += w->hd[a] * w->al[a];
                double kda = 0.0;
                for (int b = 0; b < j; b++) kda += w->Kd[a * j + b] * w->al[b];
                w_kd_al += w->wv[a] * kda;
            }
            const double vj = kappa - hw;
            const double dm = hd_al - w_kd_al;  /* d mu_j / dd */
            const double coef = (j + 1) * psi / ((double)j * (j - 1));
            /* mode B constants: tr(K^{-1} Kdot) and tr((K^{-1} Kdot)^2) */
            double T1 = 0.0, T2 = 0.0;
            if (mode_b) {
                for (int a = 0; a < j; a++)
                    for (int b = 0; b < j; b++) {
                        double s = 0.0;
                        for (int c = 0; c < j; c++) s += w->Ki[a * j + c] * w->Kd[c * j + b];
                        w->W[a * j + b] = s;
                    }
                for (int a = 0; a < j; a++) {
                    T1 += w->W[a * j + a];
                    for (int b = 0; b < j; b++) T2 += w->W[a * j + b] * w->W[b * j + a];
                }
            }
            double best = INFINITY, maxdiff = 0.0, fj = NAN, fg = NAN, bg = NAN;
            int best_slot = -1, fslot = -1;
            const int J1 = j + 1;
            for (int s = 0; s < Np; s++) {
                if (w->chosen[s]) continue;
                const double *xc = X + (int64_t)pool[s] * p;
                for (int a = 0; a < j; a++) kern_dk(X + (int64_t)pool[w->slot[a]] * p, xc, p, d, &w->kc[a], &w->kdc[a]);
                double kcx, kdcx;
                kern_dk(xc, x, p, d, &kcx, &kdcx);
                /* mode A: K_{j+1} and Kdot_{j+1} written out, a fresh inverse */
                for (int a = 0; a < J1; a++)
                    for (int b = 0; b < J1; b++) {
                        double kv, kdv;
                        if (a < j && b < j) {
                            kv = w->K[a * j + b];
                            kdv = w->Kd[a * j + b];
                        } else if (a < j) {
                            kv = w->kc[a];
                            kdv = w->kdc[a];
                        } else if (b < j) {
                            kv = w->kc[b];
                            kdv = w->kdc[b];
                        } else {
                            kv = kappa;
                            kdv = 0.0;
                        }
                        w->A1[a * J1 + b] = kv;
                        w->Kd1[a * J1 + b] = kdv;
                    }
                double crit = INFINITY, G = NAN;
                if (!spd_inverse(w->A1, w->Ki1, w->L, w->e, w->t, w->col, J1)) {
                    for (int a = 0; a < j; a++) w->k1[a] = w->h[a];
                    w->k1[j] = kcx;
                    double q = 0.0;
                    for (int a = 0; a < J1; a++) {
                        double r = 0.0;
                        for (int b = 0; b < J1; b++) r += w->Ki1[a * J1 + b] * w->k1[b];
                        q += w->k1[a] * r;
                    }
                    const double v1 = kappa - q;
                    double tW = 0.0, tW2 = 0.0;
                    for (int a = 0; a < J1; a++)
                        for (int b = 0; b < J1; b++) {
                            double r = 0.0;
                            for (int c = 0; c < J1; c++) r += w->Ki1[a * J1 + c] * w->Kd1[c * J1 + b];
                            w->W[a * J1 + b] = r;
                        }
                    for (int a = 0; a < J1; a++) {
                        tW += w->W[a * J1 + a];
                        for (int b = 0; b < J1; b++) tW2 += w->W[a * J1 + b] * w->W[b * J1 + a];
                    }
                    G = 0.5 * (tW2 - tW * tW / J1);
                    if (G > 0.0) crit = coef * v1 + dm * dm / G;
                }
                if (mode_b) {
                    /* the same criterion through the partitioned inverse */
                    double sB = kappa, covB = kcx, e = 0.0, aKa = 0.0;
                    for (int a = 0; a < j; a++) {
                        w->u[a] = 0.0;
                        for (int b = 0; b < j; b++) w->u[a] += w->Ki[a * j + b] * w->kc[b];
                    }
                    for (int a = 0; a < j; a++) {
                        sB -= w->kc[a] * w->u[a];
                        covB -= w->h[a] * w->u[a];
                        double kdu = 0.0;
                        for (int b = 0; b < j; b++) kdu += w->Kd[a * j + b] * w->u[b];
                        e += w->u[a] * kdu - 2.0 * w->kdc[a] * w->u[a];
                        w->a[a] = w->kdc[a] - kdu;
                    }
                    for (int a = 0; a < j; a++) {
                        double r = 0.0;
                        for (int b = 0; b < j; b++) r += w->Ki[a * j + b] * w->a[b];
                        aKa += w->a[a] * r;
                    }
                    double critB = INFINITY;
                    if (sB > 0.0) {
                        const double v1 = vj - covB * covB / sB;
                        const double tW = T1 + e / sB, tW2 = T2 + 2.0 * aKa / sB + e * e / (sB * sB);
                        const double GB = 0.5 * (tW2 - tW * tW / J1);
                        if (GB > 0.0) critB = coef * v1 + dm * dm / GB;
                    }
                    if (isfinite(crit) && isfinite(critB)) {
                        const double df = fabs(crit - critB);
                        if (df > maxdiff) maxdiff = df;
                    }
                }
                if (forced && pool[s] == forced[j]) { fj = crit; fslot = s; fg = G; }
                if (crit < best || (crit == best && best_slot >= 0 && pool[s] < pool[best_slot])) {
                    best = crit;
                    best_slot = s;
                    bg = G;
                }
            }
            if (best_slot < 0 || !isfinite(best)) { rc = ORC_STEP_FAIL; break; }
            jmin[j] = best;
            amin[j] = pool[best_slot];
            nu[j] = mode_b ? maxdiff / fabs(best) : NAN;
            dmu[j] = dm;
            if (forced) {
                if (fslot < 0) { rc = ORC_BAD_FORCED; break; }
                take = fslot;
                jsel[j] = fj;
                gsel[j] = fg;
            } else {
                take = best_slot;
                jsel[j] = best;
                gsel[j] = bg;
            }
        }
        w->chosen[take] = 1;
        w->slot[j] = take;
        sel[j] = pool[take];
    }
    if (rc == ORC_OK) {
        double *Dn = w->Ki1, *Yn = w->k1;
        for (int a = 0; a < n; a++) {
            memcpy(Dn + (size_t)a * p, X + (int64_t)sel[a] * p, sizeof(double) * p);
            Yn[a] = Y[sel[a]];
        }
        if (orc_gp_predict(Dn, Yn, n, p, x, d, g, pred)) rc = ORC_STEP_FAIL;
    }
    return rc;
}

/* Batched MSPE designs (OpenMP over locations); outputs M x n (pred M x 5). */
int orc_mspe(const double *X, const double *Y, int64_t N, int p, const double *XX, int64_t M,
             const int32_t *pool, int Np, int n0, int n, double d, double g, const int32_t *forced, int mode_b,
             int nthreads, int32_t *sel, double *jsel, double *jmin, int32_t *amin, double *nu, double *dmu,
             double *gsel, double *pred, int32_t *status)
{
    if (!(d > 0.0) || !(g > 0.0) || !isfinite(d) || !isfinite(g) || p < 1 || n0 < 2 || n0 > n || n > Np ||
        Np > N)
        return ORC_BAD_ARGS;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        mspe_work w;
        int ok = mspe_alloc(&w, n, Np) && p <= n + 1;  /* Dn reuses an (n + 1)^2 buffer */
#pragma omp for schedule(dynamic, 1)
        for (int64_t m = 0; m < M; m++) {
            const int64_t o = m * (int64_t)n;
            int rc = ok ? mspe_one(X, Y, p, XX + m * p, pool + m * (int64_t)Np, Np, n0, n, d, g,
                                   forced ? forced + o : NULL, mode_b, sel + o, jsel + o, jmin + o, amin + o,
                                   nu + o, dmu + o, gsel + o, pred + m * 5, &w)
                        : ORC_BAD_ARGS;
            if (rc != ORC_OK)
                for (int q = 0; q < 5; q++) pred[m * 5 + q] = NAN;
            status[m] = rc;
        }
        mspe_free(&w);
    }
    return ORC_OK;
}
