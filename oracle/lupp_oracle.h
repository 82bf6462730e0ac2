/* Plain, slow, obviously-correct CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library. The HIP product path never includes, links or calls it, and it
 * shares no code with the HIP path.
 *
 * Arithmetic: IEEE binary64, round-to-nearest, built with -ffp-contract=off and
 * no fast-math, plain loops, no BLAS.
 *
 * Matrices are column-major: element (i, j) of a system is a[i + j*lda].
 */
#ifndef LUPP_ORACLE_H
#define LUPP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LU factorisation with partial pivoting of one n x n matrix, in place
 * (Section 2.2: Gaussian elimination column by column, PA = LU with row
 * interchanges choosing the largest-magnitude pivot).  On return the strict
 * lower triangle holds the unit-lower factor L (rows stored in the permuted
 * order, as LAPACK does), the upper triangle holds U, and ipiv[k] (1-based) is
 * the row exchanged with row k at step k.  Returns info: 0, or k+1 for the
 * first step k whose pivot is exactly zero (the factorisation still runs to
 * the end).  If gap != NULL it receives the minimum over steps of
 * (|best| - |second best|) / |best| among the pivot candidates (1.0 when a
 * step has a single candidate, 0.0 for exact ties or a zero pivot). */
int oracle_getrf(int n, double *a, int lda, int32_t *ipiv, double *gap);

/* Solve A x = b with the factors of oracle_getrf (Section 2.2: L y = P b,
 * then U x = y).  b is overwritten with x. */
void oracle_getrs(int n, const double *lu, int lda, const int32_t *ipiv, double *b);

/* getrf, then getrs when info == 0 (b is left unchanged when info > 0). */
int oracle_gesv(int n, double *a, int lda, double *b, int32_t *ipiv, double *gap);

/* A batch of independent systems, AoS: system s has its matrix at
 * a + s*strideA (leading dimension lda), its right-hand side at b + s*strideB
 * and its pivots at ipiv + s*n.  Runs on `nthreads` POSIX threads (<= 0: 1).
 * gap may be NULL. */
void oracle_gesv_batch(int n, int64_t batch, double *a, int lda, int64_t strideA,
                       double *b, int64_t strideB, int32_t *ipiv, int32_t *info,
                       double *gap, int nthreads);

/* Tile-local partial pivoting, the pivoting rule of the paper's Tiled
 * solvers (Section 3.2.2; Section 4.2): at step k the pivot is sought among
 * rows k .. (last row of the diagonal tile of size ts that holds k) and, only
 * if the best of them has magnitude below thresh, among all rows k .. n-1
 * (an out-of-tile pivot, counted in *out_of_tile). Ties go to the lowest row;
 * interchange, multipliers, update and solves are those of oracle_getrf /
 * oracle_getrs. ts <= 0 or ts >= n is textbook partial pivoting. */
int oracle_getrf_tiled(int n, double *a, int lda, int32_t *ipiv, int ts, double thresh,
                       int *out_of_tile);
/* Batched dgesv (AoS, as oracle_gesv_batch) under a chosen pivoting rule
 * (ts, thresh as oracle_getrf_tiled; ts = 0 textbook) and arithmetic mode:
 * use_fma = 0 is strict (every multiply-subtract a - l*u of the elimination
 * and of both substitutions rounds the product and then the difference),
 * use_fma = 1 computes each of them as one fused multiply-add fma(-l, u, a);
 * multipliers and diagonal divisions are true divisions in both modes.
 * out_of_tile[batch] or NULL. */
void oracle_gesv_batch_mode(int n, int64_t batch, double *a, int lda, int64_t strideA,
                            double *b, int64_t strideB, int32_t *ipiv, int32_t *info, int ts,
                            double thresh, int use_fma, int32_t *out_of_tile, int nthreads);

/* Ragged batch: system s has size n[s], matrix at a + offA[s] (lda = n[s]),
 * right-hand side and pivots at offset offB[s]. */
void oracle_gesv_ragged(int64_t batch, const int32_t *n, const int64_t *offA,
                        const int64_t *offB, double *a, double *b, int32_t *ipiv,
                        int32_t *info, int nthreads);

/* ---------------------------------------------------------------------------
 * Implicit constitutive update (Section 2.1 and Algorithm 2: per integration
 * point, Newton iterations J dx = -F, x += dx, until the residual is small).
 *
 * Kelvin-Mandel vectors v = (v11, v22, v33, sqrt2 v12, sqrt2 v13, sqrt2 v23).
 * kind 7 : Norton viscoplasticity, unknowns (d_eel[6], dp).
 * kind 13: Norton + Armstrong-Frederick kinematic hardening,
 *          unknowns (d_eel[6], dp, d_alpha[6]).
 */
typedef struct {
    int kind;      /* 7 or 13 */
    double E, nu;  /* Young's modulus, Poisson ratio */
    double A, m;   /* Norton: dp/dt = A * seq^m */
    double C, D;   /* Armstrong-Frederick: X = 2/3 C alpha, recall D */
    double dt;     /* time step */
} oracle_law;

/* Residual F (nunk) and Jacobian J (nunk x nunk, column-major, J[r + c*nunk] =
 * dF_r / dy_c) at unknowns y, for strain increment deps[6] and state at the
 * start of the step state_t (kind 7: eel[6], p; kind 13: eel[6], p, alpha[6]).
 * sig[6] receives the stress at y.  J may be NULL. */
void oracle_law_eval(const oracle_law *law, const double *deps, const double *state_t,
                     const double *y, double *F, double *J, double *sig);

/* Per-point Newton loop, AoS: deps[count][6], state[count][kind] (updated only
 * where status == 0), sig[count][6], iters/status[count], resid[count] = the
 * infinity norm of the residual that decided the stop (NAN if non-finite).
 * status: 0 converged, 1 maxit reached, 2 singular Jacobian, 3 non-finite
 * residual. tangent: NULL, or [count][36] receiving the consistent tangent
 * dsig/d(deps) (row-major 6x6, Kelvin) of every converged point (Section
 * 2.5; Section 4.3: a multi-right-hand-side solve with the factors of the
 * Jacobian at the converged iterate); other points' entries are untouched.
 * yout: NULL, or [count][kind] receiving the unknowns (increments) of the
 * returned iterate, whatever the status (a side output for comparisons at a
 * given iterate: with tol = 0 the loop stops after exactly maxit solves). */
void oracle_constitutive_update(const oracle_law *law, int64_t count, const double *deps,
                                double *state, double *sig, int32_t *iters,
                                int32_t *status, double *resid, double *tangent, double *yout,
                                double tol, int maxit, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
