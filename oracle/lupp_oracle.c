/* Plain CPU oracle for batched LU with partial pivoting and for the per-point
 * Newton constitutive update — TEST INFRASTRUCTURE ONLY (see lupp_oracle.h).
 *
 * Every routine is the textbook definition written out with plain loops, in
 * the order the paper describes it, so that it can be checked against the
 * paper by eye.  Build: gcc -O2 -ffp-contract=off (no fast-math).
 */
#include "lupp_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting (Section 2.2).                                   */
/* Right-looking Gaussian elimination: at step k the pivot is the candidate  */
/* of largest magnitude in column k (lowest row index on ties), rows k and p */
/* are exchanged across all columns, the multipliers l_ik = a_ik / a_kk are  */
/* stored below the diagonal, and the trailing submatrix (Schur complement)  */
/* receives a_ij <- a_ij - l_ik * u_kj.                                      */
/* ------------------------------------------------------------------------ */
/* a - l*u as one rounded multiply and one rounded subtract (strict mode), or
 * as one fused multiply-add (FMA mode). */
static inline double oracle_msub(double a, double l, double u, int use_fma)
{
    return use_fma ? fma(-l, u, a) : a - l * u;
}

/* Index of the first largest |col[i]| over lo <= i < hi (lowest row on ties). */
static int oracle_argmax_abs(const double *col, int lo, int hi)
{
    int p = lo;
    double best = fabs(col[lo]);
    for (int i = lo + 1; i < hi; ++i) {
        double v = fabs(col[i]);
        if (v > best) {
            best = v;
            p = i;
        }
    }
    return p;
}

/* ts <= 0 or ts >= n: textbook partial pivoting. Otherwise tile-local
 * pivoting (Section 3.2.2, the Tiled solvers; Section 4.2): the candidates at
 * step k are first the rows k .. (end of the diagonal tile of size ts holding
 * k); only if the best of them is below thresh in magnitude does the search
 * extend to every row k .. n-1 (counted in *oot). */
static int oracle_getrf_rule(int n, double *a, int lda, int32_t *ipiv, double *gap, int ts,
                             double thresh, int use_fma, int *oot)
{
    int info = 0;
    double g = 1.0;
    for (int k = 0; k < n; ++k) {
        const double *col = a + (int64_t)k * lda;
        int p;
        if (ts > 0 && ts < n) {
            int k1 = (k / ts + 1) * ts;
            if (k1 > n) k1 = n;
            p = oracle_argmax_abs(col, k, k1);
            if (fabs(col[p]) < thresh) {
                p = oracle_argmax_abs(col, k, n);
                if (oot != NULL) ++*oot;
            }
        } else {
            p = oracle_argmax_abs(col, k, n);
        }
        const double best = fabs(col[p]);
        if (gap != NULL && k + 1 < n) {
            double second = -1.0;
            for (int i = k; i < n; ++i) {
                if (i == p) continue;
                double v = fabs(a[i + (int64_t)k * lda]);
                if (v > second) second = v;
            }
            double gk = best > 0.0 ? (best - second) / best : 0.0;
            if (gk < g) g = gk;
        }
        ipiv[k] = p + 1;
        if (a[p + (int64_t)k * lda] == 0.0) {
            if (info == 0) info = k + 1;
            continue;
        }
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[k + (int64_t)j * lda];
                a[k + (int64_t)j * lda] = a[p + (int64_t)j * lda];
                a[p + (int64_t)j * lda] = t;
            }
        }
        for (int i = k + 1; i < n; ++i)
            a[i + (int64_t)k * lda] = a[i + (int64_t)k * lda] / a[k + (int64_t)k * lda];
        for (int j = k + 1; j < n; ++j)
            for (int i = k + 1; i < n; ++i)
                a[i + (int64_t)j * lda] = oracle_msub(a[i + (int64_t)j * lda], a[i + (int64_t)k * lda],
                                                      a[k + (int64_t)j * lda], use_fma);
    }
    if (gap != NULL) *gap = g;
    return info;
}

int oracle_getrf(int n, double *a, int lda, int32_t *ipiv, double *gap)
{
    return oracle_getrf_rule(n, a, lda, ipiv, gap, 0, 0.0, 0, NULL);
}

int oracle_getrf_tiled(int n, double *a, int lda, int32_t *ipiv, int ts, double thresh,
                       int *out_of_tile)
{
    if (out_of_tile != NULL) *out_of_tile = 0;
    return oracle_getrf_rule(n, a, lda, ipiv, NULL, ts, thresh, 0, out_of_tile);
}

/* Triangular solves (Section 2.2): apply the interchanges to b, then L y = P b
 * (unit lower, column by column, ascending), then U x = y (column by column,
 * descending: divide by the diagonal, then eliminate the column above it). */
static void oracle_getrs_mode(int n, const double *lu, int lda, const int32_t *ipiv, double *b,
                              int use_fma)
{
    for (int k = 0; k < n; ++k) {
        int p = ipiv[k] - 1;
        if (p != k) {
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i)
            b[i] = oracle_msub(b[i], lu[i + (int64_t)j * lda], b[j], use_fma);
    for (int j = n - 1; j >= 0; --j) {
        b[j] = b[j] / lu[j + (int64_t)j * lda];
        for (int i = 0; i < j; ++i)
            b[i] = oracle_msub(b[i], lu[i + (int64_t)j * lda], b[j], use_fma);
    }
}

void oracle_getrs(int n, const double *lu, int lda, const int32_t *ipiv, double *b)
{
    oracle_getrs_mode(n, lu, lda, ipiv, b, 0);
}

int oracle_gesv(int n, double *a, int lda, double *b, int32_t *ipiv, double *gap)
{
    int info = oracle_getrf(n, a, lda, ipiv, gap);
    if (info == 0) oracle_getrs(n, a, lda, ipiv, b);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Batch drivers: one system per task, static chunks over POSIX threads.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    void (*body)(void *ctx, int64_t lo, int64_t hi);
    void *ctx;
    int64_t lo, hi;
} oracle_task;

static void *oracle_task_run(void *p)
{
    oracle_task *t = (oracle_task *)p;
    t->body(t->ctx, t->lo, t->hi);
    return NULL;
}

static void oracle_parallel_for(int64_t count, int nthreads,
                                void (*body)(void *, int64_t, int64_t), void *ctx)
{
    if (nthreads <= 1 || count < 2) {
        body(ctx, 0, count);
        return;
    }
    if (nthreads > 256) nthreads = 256;
    if (nthreads > count) nthreads = (int)count;
    pthread_t th[256];
    oracle_task tk[256];
    int started[256];
    int64_t per = (count + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        tk[t].body = body;
        tk[t].ctx = ctx;
        tk[t].lo = t * per < count ? t * per : count;
        tk[t].hi = (t + 1) * per < count ? (t + 1) * per : count;
        started[t] = pthread_create(&th[t], NULL, oracle_task_run, &tk[t]) == 0;
        if (!started[t]) oracle_task_run(&tk[t]);
    }
    for (int t = 0; t < nthreads; ++t)
        if (started[t]) pthread_join(th[t], NULL);
}

typedef struct {
    int n, lda;
    int64_t strideA, strideB;
    double *a, *b, *gap;
    int32_t *ipiv, *info;
} batch_ctx;

static void batch_body(void *p, int64_t lo, int64_t hi)
{
    batch_ctx *c = (batch_ctx *)p;
    for (int64_t s = lo; s < hi; ++s) {
        double g;
        c->info[s] = oracle_gesv(c->n, c->a + s * c->strideA, c->lda, c->b + s * c->strideB,
                                 c->ipiv + s * c->n, c->gap ? &g : NULL);
        if (c->gap) c->gap[s] = g;
    }
}

typedef struct {
    int n, lda, ts, use_fma;
    double thresh;
    int64_t strideA, strideB;
    double *a, *b;
    int32_t *ipiv, *info, *oot;
} rule_ctx;

static void rule_body(void *p, int64_t lo, int64_t hi)
{
    rule_ctx *c = (rule_ctx *)p;
    for (int64_t s = lo; s < hi; ++s) {
        int oot = 0;
        double *a = c->a + s * c->strideA;
        int32_t *ipiv = c->ipiv + s * c->n;
        const int info =
            oracle_getrf_rule(c->n, a, c->lda, ipiv, NULL, c->ts, c->thresh, c->use_fma, &oot);
        if (info == 0) oracle_getrs_mode(c->n, a, c->lda, ipiv, c->b + s * c->strideB, c->use_fma);
        c->info[s] = info;
        if (c->oot) c->oot[s] = oot;
    }
}

void oracle_gesv_batch_mode(int n, int64_t batch, double *a, int lda, int64_t strideA,
                            double *b, int64_t strideB, int32_t *ipiv, int32_t *info, int ts,
                            double thresh, int use_fma, int32_t *out_of_tile, int nthreads)
{
    rule_ctx c = {n, lda, ts, use_fma, thresh, strideA, strideB, a, b, ipiv, info, out_of_tile};
    oracle_parallel_for(batch, nthreads, rule_body, &c);
}

void oracle_gesv_batch(int n, int64_t batch, double *a, int lda, int64_t strideA,
                       double *b, int64_t strideB, int32_t *ipiv, int32_t *info,
                       double *gap, int nthreads)
{
    batch_ctx c = {n, lda, strideA, strideB, a, b, gap, ipiv, info};
    oracle_parallel_for(batch, nthreads, batch_body, &c);
}

typedef struct {
    const int32_t *n;
    const int64_t *offA, *offB;
    double *a, *b;
    int32_t *ipiv, *info;
} ragged_ctx;

static void ragged_body(void *p, int64_t lo, int64_t hi)
{
    ragged_ctx *c = (ragged_ctx *)p;
    for (int64_t s = lo; s < hi; ++s)
        c->info[s] = oracle_gesv(c->n[s], c->a + c->offA[s], c->n[s], c->b + c->offB[s],
                                 c->ipiv + c->offB[s], NULL);
}

void oracle_gesv_ragged(int64_t batch, const int32_t *n, const int64_t *offA,
                        const int64_t *offB, double *a, double *b, int32_t *ipiv,
                        int32_t *info, int nthreads)
{
    ragged_ctx c = {n, offA, offB, a, b, ipiv, info};
    oracle_parallel_for(batch, nthreads, ragged_body, &c);
}

/* ------------------------------------------------------------------------ */
/* Constitutive laws, Kelvin-Mandel notation, backward Euler.                */
/*                                                                          */
/* eel = eel_t + d_eel, sig = lambda tr(eel) 1 + 2 mu eel, s = K sig with    */
/* K = I - 1/3 1 1^T.  Norton: xi = s; with Armstrong-Frederick:             */
/* alpha = alpha_t + d_alpha, X = 2/3 C alpha, xi = s - X.                   */
/* seq = sqrt(3/2 xi.xi), N = 3/2 xi / seq (N = 0 when seq = 0).             */
/* Residuals: F_e = d_eel + dp N - deps;  F_p = dp - dt A seq^m;             */
/*            F_a = d_alpha - dp N + D dp alpha.                            */
/* The Jacobian is the exact derivative of these residuals.                  */
/* ------------------------------------------------------------------------ */
/* Lame constants of the isotropic elastic stiffness. */
static void oracle_lame(const oracle_law *law, double *lam, double *mu)
{
    *lam = law->E * law->nu / ((1.0 + law->nu) * (1.0 - 2.0 * law->nu));
    *mu = law->E / (2.0 * (1.0 + law->nu));
}

void oracle_law_eval(const oracle_law *law, const double *deps, const double *state_t,
                     const double *y, double *F, double *J, double *sig)
{
    const int nunk = law->kind;
    const int af = (law->kind == 13);
    double lam, mu;
    oracle_lame(law, &lam, &mu);

    double eel[6], s[6], xi[6], alpha[6], N[6];
    for (int i = 0; i < 6; ++i) eel[i] = state_t[i] + y[i];
    double tr = eel[0] + eel[1] + eel[2];
    for (int i = 0; i < 6; ++i) sig[i] = 2.0 * mu * eel[i] + (i < 3 ? lam * tr : 0.0);
    double trs = sig[0] + sig[1] + sig[2];
    for (int i = 0; i < 6; ++i) s[i] = sig[i] - (i < 3 ? trs / 3.0 : 0.0);
    for (int i = 0; i < 6; ++i) {
        alpha[i] = af ? state_t[7 + i] + y[7 + i] : 0.0;
        xi[i] = s[i] - (af ? 2.0 / 3.0 * law->C * alpha[i] : 0.0);
    }
    double xx = 0.0;
    for (int i = 0; i < 6; ++i) xx += xi[i] * xi[i];
    double seq = sqrt(1.5 * xx);
    for (int i = 0; i < 6; ++i) N[i] = seq > 0.0 ? 1.5 * xi[i] / seq : 0.0;

    const double dp = y[6];
    for (int i = 0; i < 6; ++i) F[i] = y[i] + dp * N[i] - deps[i];
    F[6] = dp - law->dt * law->A * pow(seq, law->m);
    if (af)
        for (int i = 0; i < 6; ++i) F[7 + i] = y[7 + i] - dp * N[i] + law->D * dp * alpha[i];

    if (J == NULL) return;
    for (int c = 0; c < nunk * nunk; ++c) J[c] = 0.0;
#define JAC(r, c) J[(r) + (c) * nunk]
    /* dN/dxi = (3/2 I - N N^T) / seq, the deviatoric projector K, and
     * (dN/dxi) K which is dN/d(d_eel) divided by 2 mu. */
    double Hp[6][6], Km[6][6], HK[6][6], KN[6];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            Hp[a][b] = seq > 0.0 ? (1.5 * (a == b ? 1.0 : 0.0) - N[a] * N[b]) / seq : 0.0;
            Km[a][b] = (a == b ? 1.0 : 0.0) - (a < 3 && b < 3 ? 1.0 / 3.0 : 0.0);
        }
    for (int a = 0; a < 6; ++a) {
        KN[a] = 0.0;
        for (int b = 0; b < 6; ++b) KN[a] += Km[a][b] * N[b];
        for (int b = 0; b < 6; ++b) {
            HK[a][b] = 0.0;
            for (int c = 0; c < 6; ++c) HK[a][b] += Hp[a][c] * Km[c][b];
        }
    }
    /* d(dt A seq^m)/dseq */
    const double gdot = seq > 0.0 ? law->dt * law->A * law->m * pow(seq, law->m - 1.0) : 0.0;
    for (int a = 0; a < 6; ++a) {
        for (int b = 0; b < 6; ++b) JAC(a, b) = (a == b ? 1.0 : 0.0) + dp * 2.0 * mu * HK[a][b];
        JAC(a, 6) = N[a];
        JAC(6, a) = -gdot * 2.0 * mu * KN[a];
    }
    JAC(6, 6) = 1.0;
    if (af) {
        const double c23 = 2.0 / 3.0 * law->C;
        for (int a = 0; a < 6; ++a) {
            for (int b = 0; b < 6; ++b) {
                JAC(a, 7 + b) = -c23 * dp * Hp[a][b];
                JAC(7 + a, b) = -dp * 2.0 * mu * HK[a][b];
                JAC(7 + a, 7 + b) = (1.0 + law->D * dp) * (a == b ? 1.0 : 0.0) + c23 * dp * Hp[a][b];
            }
            JAC(6, 7 + a) = c23 * gdot * N[a];
            JAC(7 + a, 6) = -N[a] + law->D * alpha[a];
        }
    }
#undef JAC
}

/* Newton-Raphson for one point (Section 2.1, Algorithm 2): start from zero
 * increments; at each iterate evaluate F; stop on a non-finite residual, on
 * ||F||_inf < tol, or after maxit linear solves; otherwise factor J with
 * partial pivoting, solve J dx = -F and update x += dx. */
/* Consistent tangent operator at a converged point (Section 2.5: the
 * consistent linearisation of the implicit update; Section 4.3: one
 * multi-right-hand-side solve after convergence). With F(y; deps) = 0 at the
 * converged unknowns y and dF/d(deps) = -[I6; 0], the sensitivity is
 * dy/d(deps) = J^-1 [I6; 0]: factor the Jacobian J of the converged iterate
 * with partial pivoting and solve for the six unit right-hand sides. The
 * stress sig = D (eel_t + d_eel) then gives dsig/d(deps) = D X_e, X_e the
 * first six rows of the solution. Output row-major: tan[6*r + c] =
 * dsig_r / d(deps)_c. A singular J gives NaN entries. */
static void oracle_tangent(const oracle_law *law, double *J, double *tan)
{
    const int nunk = law->kind;
    double lam, mu;
    oracle_lame(law, &lam, &mu);
    int32_t piv[13];
    if (oracle_getrf(nunk, J, nunk, piv, NULL) != 0) {
        for (int i = 0; i < 36; ++i) tan[i] = NAN;
        return;
    }
    for (int c = 0; c < 6; ++c) {
        double x[13];
        for (int i = 0; i < nunk; ++i) x[i] = (i == c) ? 1.0 : 0.0;
        oracle_getrs(nunk, J, nunk, piv, x);
        const double tr = x[0] + x[1] + x[2];
        for (int r = 0; r < 6; ++r) tan[6 * r + c] = 2.0 * mu * x[r] + (r < 3 ? lam * tr : 0.0);
    }
}

static void oracle_newton_point(const oracle_law *law, const double *deps, double *state,
                                double *sig, int32_t *iters, int32_t *status, double *resid,
                                double *tan, double *yout, double tol, int maxit)
{
    const int nunk = law->kind;
    double y[13], F[13], J[169], dx[13];
    int32_t piv[13];
    memset(y, 0, sizeof(y));
    int st = 1, k = 0;
    double nrm = 0.0;
    for (k = 0;; ++k) {
        oracle_law_eval(law, deps, state, y, F, J, sig);
        int finite = 1;
        nrm = 0.0;
        for (int i = 0; i < nunk; ++i) {
            if (!isfinite(F[i])) finite = 0;
            else if (fabs(F[i]) > nrm) nrm = fabs(F[i]);
        }
        if (!finite) {
            st = 3;
            nrm = NAN;
            break;
        }
        if (nrm < tol) {
            st = 0;
            break;
        }
        if (k == maxit) {
            st = 1;
            break;
        }
        for (int i = 0; i < nunk; ++i) dx[i] = -F[i];
        if (oracle_gesv(nunk, J, nunk, dx, piv, NULL) != 0) {
            st = 2;
            break;
        }
        for (int i = 0; i < nunk; ++i) y[i] = y[i] + dx[i];
    }
    *iters = k;
    *status = st;
    *resid = nrm;
    /* J holds the (unfactored) Jacobian of the converged iterate */
    if (st == 0 && tan != NULL) oracle_tangent(law, J, tan);
    if (yout != NULL)
        for (int i = 0; i < nunk; ++i) yout[i] = y[i];
    if (st == 0)
        for (int i = 0; i < nunk; ++i) state[i] = state[i] + y[i];
}

typedef struct {
    const oracle_law *law;
    const double *deps;
    double *state, *sig, *resid, *tan, *yout;
    int32_t *iters, *status;
    double tol;
    int maxit;
} newton_ctx;

static void newton_body(void *p, int64_t lo, int64_t hi)
{
    newton_ctx *c = (newton_ctx *)p;
    const int nunk = c->law->kind;
    for (int64_t s = lo; s < hi; ++s)
        oracle_newton_point(c->law, c->deps + 6 * s, c->state + nunk * s, c->sig + 6 * s,
                            c->iters + s, c->status + s, c->resid + s,
                            c->tan ? c->tan + 36 * s : NULL, c->yout ? c->yout + nunk * s : NULL,
                            c->tol, c->maxit);
}

void oracle_constitutive_update(const oracle_law *law, int64_t count, const double *deps,
                                double *state, double *sig, int32_t *iters,
                                int32_t *status, double *resid, double *tangent, double *yout,
                                double tol, int maxit, int nthreads)
{
    newton_ctx c = {law, deps, state, sig, resid, tangent, yout, iters, status, tol, maxit};
    oracle_parallel_for(count, nthreads, newton_body, &c);
}
