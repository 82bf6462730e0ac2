/* lupp — batched LU with partial pivoting for millions of tiny (n <= 32)
 * double-precision systems, and a fused per-point Newton constitutive update,
 * on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The operations follow the paper "Accelerating the Solving of Many Tiny
 * General Linear Systems on GPUs: Application to Constitutive Laws":
 *   - PA = LU by Gaussian elimination with partial pivoting, then L y = P b and
 *     U x = y (Section 2.2);
 *   - host-launched batched solves over device arrays of independent systems
 *     (Section 3.1, the getrf/getrs/gesv roles);
 *   - a device-callable solve used inside a per-point Newton loop, the whole
 *     loop in one kernel (Section 2.1, equations 1-3; Section 3.3; Algorithm 2).
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers owned by the caller. The library never
 *     frees them and keeps no reference after the work it enqueued completes.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream): results are valid once that stream's work completes.
 *   - Return value: 0 on success; -k if the k-th argument is invalid (nothing
 *     is enqueued, nothing is printed); LUPP_E_UNSUPPORTED for a valid request
 *     no compiled kernel serves; LUPP_E_HIP_BASE - e for a HIP runtime error e.
 *     No C++ exception crosses the ABI.
 *   - Numerics (strict mode): IEEE binary64, no FMA contraction, true
 *     divisions. Results are bitwise identical to the textbook algorithm's
 *     whatever kernel variant, layout or batch composition serves a call.
 */
#ifndef LUPP_H
#define LUPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LUPP_E_UNSUPPORTED (-900)
#define LUPP_E_NOMEM (-901)
#define LUPP_E_TOO_LARGE (-902) /* beyond the allocation-free workspace */
#define LUPP_E_HIP_BASE (-1000)

/* Matrix layouts.
 * LUPP_AOS: system s, element (i, j) at A[s*strideA + i + j*lda] (column-major
 *           per system); b[s*strideB + i]; ipiv[s*n + k].
 * LUPP_SOA: interleaved: A[(i + j*lda)*ldbatch + s]; b[i*strideB + s];
 *           ipiv[k*ldbatch + s]. Consecutive systems are adjacent in memory,
 *           so lane s of a wave reads consecutive doubles. */
#define LUPP_AOS 0
#define LUPP_SOA 1

/* Flags. LUPP_KEEP_A: do not write the factors back (A is left unchanged).
 * LUPP_RAGGED_PER_SIZE (lupp_batched_solve_ragged only): instead of the
 * launches per size class, read the size histogram back to the host and
 * launch one kernel per size (the plain baseline; it synchronises the
 * stream).
 * LUPP_FMA (lupp_batched_solve only): fused multiply-add arithmetic, see
 * lupp_batched_solve. */
#define LUPP_KEEP_A 1u
#define LUPP_RAGGED_PER_SIZE 2u
#define LUPP_FMA 4u

/* Kernel variants (for lupp_force_variant and lupp_variant_info). */
#define LUPP_VARIANT_AUTO 0
#define LUPP_VARIANT_THREAD 1 /* one lane per system, registers only      */
#define LUPP_VARIANT_LANES 2  /* `lanes` lanes per system (segment of a wave64) */

typedef struct lupp_ctx lupp_ctx;

/* Create a context bound to HIP device `device` (its current state is not
 * changed). The context owns the per-size dispatch table and the library's
 * device workspace. One context may be used from one host thread at a time.
 * Returns 0 or an error; *ctx is NULL on error. */
int lupp_create(lupp_ctx **ctx, int device);

/* Release a context (waits for nothing: the caller synchronises its streams
 * first). NULL is accepted. */
void lupp_destroy(lupp_ctx *ctx);

/* The HIP device a context is bound to. */
int lupp_get_device(const lupp_ctx *ctx, int *device);

/* Batched dgesv (Section 2.2; Section 3.1): for each of `batch` independent
 * n x n systems, factor PA = LU with partial pivoting and, where the
 * factorisation has no zero pivot, overwrite b with x = A^-1 b.
 *   n       : 1..32.
 *   batch   : >= 0 (0 is a no-op).
 *   layout  : LUPP_AOS or LUPP_SOA.
 *   A       : matrices; on return the LAPACK-ordered factors L\U (unit lower L
 *             below the diagonal, U on and above), unless LUPP_KEEP_A.
 *   lda     : >= n.
 *   strideA : AoS: distance between systems, >= lda*n.
 *             SoA: ldbatch, the distance between consecutive elements of one
 *             system, >= batch.
 *   b       : right-hand sides, overwritten by the solutions where info == 0
 *             and left unchanged where info > 0.
 *   strideB : AoS: >= n; SoA: >= batch.
 *   ipiv    : int32 LAPACK interchange sequence: ipiv[k] = r (1-based) means
 *             rows k+1 and r were exchanged at step k; r >= k+1.
 *   info    : int32 per system: 0, or k+1 for the first step k whose pivot
 *             is exactly zero (the factorisation still completes).
 *   flags   : 0, LUPP_KEEP_A, LUPP_FMA, or both. LUPP_FMA: FMA arithmetic -
 *             every multiply-subtract of the elimination and of both
 *             substitutions is one fused multiply-add (divisions and pivoting
 *             as in strict mode); results are then bitwise those of the
 *             oracle's FMA mode rather than of the strict default. Not
 *             combined with tile-local pivoting (LUPP_E_UNSUPPORTED).
 * Inputs containing NaN or Inf produce unspecified factors and info.
 * Address range: the kernels address memory through 32-bit offsets from
 * per-workgroup bases. AoS takes any batch while 256 * strideA * 8 and
 * 256 * strideB * 8 stay below 2^31 bytes. SoA with the thread variant takes
 * any ldbatch; the lanes variant needs 3 * ldbatch * 8 + 128 < 2^31 bytes
 * (ldbatch below 89,478,485; 2-lane segments: twice that) - beyond it sizes
 * up to 13 switch to the thread variant and larger sizes return
 * LUPP_E_UNSUPPORTED. */
int lupp_batched_solve(lupp_ctx *ctx, int n, int64_t batch, int layout, double *A, int64_t lda,
                       int64_t strideA, double *b, int64_t strideB, int32_t *ipiv,
                       int32_t *info, unsigned flags, void *stream);

/* Validate the arguments of lupp_batched_solve (numbered as in that call,
 * ctx being argument 1) without enqueuing anything: 0 or -k. Host-only; it
 * needs no device. */
int lupp_check_solve_args(int n, int64_t batch, int layout, const double *A, int64_t lda,
                          int64_t strideA, const double *b, int64_t strideB, const int32_t *ipiv,
                          const int32_t *info, unsigned flags);

/* Mixed sizes in one launch (Section 4.1: size-aware dispatch): system s has
 * size n[s] in 1..32, its matrix column-major at A + offA[s] with lda = n[s],
 * its right-hand side at b + offB[s] and its pivots at ipiv + offB[s].
 * Systems must not overlap. n, offA, offB are device arrays of `batch`
 * (<= 2^31 - 1) entries. The library groups systems by size on the device
 * (histogram, plan, scatter; workspace owned by the context, grown with
 * hipMalloc when a larger batch arrives) and serves the sizes from one
 * kernel launch per size class queued back to back on `stream` (sizes
 * 24..32, 17..23, then 1..16: each kernel's register budget fits its sizes),
 * largest sizes first; no host synchronisation. Each size uses the lane count of the
 * context's ragged table (lupp_set_ragged_lanes). A system whose n is
 * outside 1..32 gets info = -1 and is not touched. flags: LUPP_KEEP_A,
 * LUPP_RAGGED_PER_SIZE.
 * Calls on one context share its workspace: a call on a different stream
 * than the previous one first waits (on the device) for the previous call's
 * kernels, so calls from one host thread may use any streams. A call made
 * while `stream` is being captured into a graph is not ordered that way:
 * replays of such a graph must not overlap other ragged calls on the same
 * context. */
int lupp_batched_solve_ragged(lupp_ctx *ctx, int64_t batch, const int32_t *n,
                              const int64_t *offA, const int64_t *offB, double *A, double *b,
                              int32_t *ipiv, int32_t *info, unsigned flags, void *stream);

/* Several uniform batches of different sizes in one call (Section 4.1:
 * size-aware dispatch): group g holds groups[g].batch systems of size
 * groups[g].n, AoS, system s at A + s*strideA (column-major, leading
 * dimension lda), right-hand side at b + s*strideB, pivots at ipiv + s*n and
 * info[s]. The groups are served by one launch per size class (sizes 17..32,
 * then 1..16), kMaxGroups = 32 groups per launch, largest sizes first, each
 * size with the lane count of the context's ragged table; every workgroup
 * takes one work item of one group, found in the launch's argument table.
 * No device workspace, no grouping kernels, no host synchronisation; the
 * groups array is read during the call only (host memory). Results are
 * bitwise those of lupp_batched_solve on each group (textbook pivoting,
 * strict arithmetic). Groups must not overlap.
 *   ngroups : >= 0 (0 is a no-op).
 *   groups  : host array of ngroups descriptors: n in 1..32, batch in
 *             0..2^31-1, and for batch > 0: non-NULL A, b, ipiv, info,
 *             lda >= n, strideA >= lda*n, strideB >= n; otherwise -3.
 *   flags   : 0 or LUPP_KEEP_A (-4 otherwise). */
typedef struct {
    int n;
    int64_t batch;
    double *A;
    int64_t lda, strideA;
    double *b;
    int64_t strideB;
    int32_t *ipiv;
    int32_t *info;
} lupp_group;
int lupp_batched_solve_grouped(lupp_ctx *ctx, int ngroups, const lupp_group *groups,
                               unsigned flags, void *stream);

/* Allocation-free form of lupp_batched_solve_ragged, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. It calls no hipMalloc, hipFree or
 * allocating library routine: the grouping workspace (size plan and sorted
 * system indices) is a fixed array of about 16 MiB in the library's device
 * code, which each GPU holds from the first context created on it until the
 * process ends. Arguments, results and flags as lupp_batched_solve_ragged,
 * except:
 *   - batch must not exceed LUPP_NOALLOC_MAX_BATCH (LUPP_E_TOO_LARGE);
 *   - LUPP_RAGGED_PER_SIZE is refused (-10): it synchronises with the host;
 *   - every call on a GPU shares that GPU's one workspace, whatever the
 *     context: calls that overlap on one GPU (other streams, other threads,
 *     replays of graphs holding such calls) race and give wrong results. The
 *     caller serialises them. A call clears what it needs, so the contents
 *     left by an earlier call do not matter. */
#define LUPP_NOALLOC_MAX_BATCH 4194304
int lupp_batched_solve_ragged_noalloc(lupp_ctx *ctx, int64_t batch, const int32_t *n,
                                      const int64_t *offA, const int64_t *offB, double *A,
                                      double *b, int32_t *ipiv, int32_t *info, unsigned flags,
                                      void *stream);

/* Lanes per system of the ragged path (Section 4.1: size-aware dispatch).
 * The ragged kernels hold, for every size n, the lane counts
 * lupp_ragged_lanes_supported(n, lanes) accepts: 1 (one thread per system,
 * n <= 5), 2 (n = 2..4), 4 (n = 3..8), 8 (n = 5..16) and 16 (n >= 9).
 * 32 lanes (measured slower than 16 for every n >= 17) and 64 (half of a
 * wave64 without a row for any n <= 32) are not built. A context starts from the table the autotuner
 * measured on gfx950. lupp_ragged_lanes_supported: 1 or 0 (host-only, no
 * device needed). lupp_set_ragged_lanes: 0, -2 for n outside 1..32, -3 for
 * an unsupported lane count. lupp_get_ragged_lanes: the lane count, or -2. */
int lupp_ragged_lanes_supported(int n, int lanes);
int lupp_set_ragged_lanes(lupp_ctx *ctx, int n, int lanes);
int lupp_get_ragged_lanes(const lupp_ctx *ctx, int n);

/* Autotune the ragged lane count of size n: time the ragged path
 * (the same call lupp_batched_solve_ragged makes) on `batch` systems of size
 * n for every supported lane count, keep the fastest in the context's ragged
 * table and report it (lanes, median ms). A is `batch` packed column-major
 * n x n matrices (device, read only), b `batch` packed right-hand sides.
 * Synchronous: allocates and frees its own device workspace (copies of A and
 * b, offsets, pivots, info) and waits for `stream`. reps >= 1 timed runs per
 * candidate after one warm-up. Returns 0, -2 (n), -3 (batch outside
 * 1..2^31-1), -4 / -5 (NULL A / b), -6 (reps), or an error code. */
int lupp_autotune_ragged(lupp_ctx *ctx, int n, int64_t batch, const double *A, const double *b,
                         int reps, int *lanes, float *ms, void *stream);

/* Pivoting rule of later lupp_batched_solve calls on this context.
 *   tile = 0 (the default): textbook partial pivoting (Section 2.2).
 *   tile >= 1: tile-local pivoting, the rule of the paper's Tiled solvers
 *   (Section 3.2.2; statistics in Section 4.2): at step k the pivot is sought
 *   first among rows k .. (end of the diagonal tile of size `tile` holding
 *   k), and among all rows k .. n-1 only when the best in-tile candidate has
 *   magnitude below `threshold` (the paper uses 1e-10). It admits more pivot
 *   growth than textbook pivoting. tile >= n is textbook pivoting.
 * Applies to every variant of lupp_batched_solve (not to the ragged path or
 * the Newton updates, which always pivot textbook-style). Returns -2 for
 * tile outside 0..32, -3 for a negative or NaN threshold. */
int lupp_set_pivoting(lupp_ctx *ctx, int tile, double threshold);
int lupp_get_pivoting(const lupp_ctx *ctx, int *tile, double *threshold);

/* Restrict later lupp_batched_solve calls on this context to one variant
 * (LUPP_VARIANT_AUTO restores the size-aware dispatch table). lanes is the
 * segment width for LUPP_VARIANT_LANES (2, 4, 8, 16 or 32), wpb the number of
 * wave64s per workgroup (1, 2 or 4; 0 = default). In the SoA layout the lanes
 * variant has a fixed workgroup of 16 systems (staged through LDS) and
 * ignores wpb. Returns LUPP_E_UNSUPPORTED
 * if a later call's n cannot be served by the forced variant. */
int lupp_force_variant(lupp_ctx *ctx, int variant, int lanes, int wpb);

/* Set / read the dispatch-table entry used for size n, layout and batches of
 * the size class of `batch` (below 32768 systems, or from 32768 on). The
 * table starts from the entries the autotuner measured on gfx950. */
int lupp_set_dispatch(lupp_ctx *ctx, int n, int layout, int64_t batch, int variant, int lanes,
                      int wpb);
int lupp_get_dispatch(lupp_ctx *ctx, int n, int layout, int64_t batch, int *variant, int *lanes,
                      int *wpb);

/* Autotune the dispatch entry for size n, layout and the size class of batch
 * (Section 4.1: launch
 * configuration chosen per problem by measurement): time every compiled
 * kernel variant and workgroup size on a device copy of the caller's batch
 * (A and b are only read), keep the fastest in the context's dispatch table,
 * and report it. Synchronous: allocates and frees its own device workspace
 * (the size of A, b, ipiv and info) and waits for `stream`. reps >= 1 timed
 * launches per candidate after one warm-up; the median is compared. */
int lupp_autotune(lupp_ctx *ctx, int n, int64_t batch, int layout, const double *A, int64_t lda,
                  int64_t strideA, const double *b, int64_t strideB, int reps, int *variant,
                  int *lanes, int *wpb, float *ms, void *stream);

/* Compile-time resources of one kernel variant: VGPRs, AGPRs and SGPRs per
 * lane, private (scratch) bytes per lane, and LDS bytes per workgroup.
 * variant: LUPP_VARIANT_THREAD or LUPP_VARIANT_LANES (with lanes) for the
 * batched solve of size n in `layout`; 100 + a law kind for the fused Newton
 * kernel of that law, keep_a != 0 then selecting its tangent-computing form.
 * Returns LUPP_E_UNSUPPORTED if the variant does not exist. */
typedef struct {
    int vgprs, agprs, sgprs, scratch_bytes, lds_bytes, max_threads;
} lupp_kernel_info;
int lupp_variant_info(int n, int layout, int variant, int lanes, int keep_a,
                      lupp_kernel_info *out);

/* ---------------------------------------------------------------------------
 * Implicit constitutive update with a fused Newton loop (Section 2.1;
 * Section 3.3; Algorithm 2): one kernel in which every integration point runs
 * its own Newton iterations, assembling the residual F and Jacobian J of the
 * law, solving J dx = -F with the device-callable LU, and updating x += dx,
 * until ||F||_inf < tol.
 *
 * Laws (Kelvin-Mandel vectors, backward Euler, unknowns x):
 *   LUPP_LAW_NORTON7      Norton viscoplasticity, x = (d_eel[6], dp);
 *   LUPP_LAW_NORTON_AF13  Norton + Armstrong-Frederick kinematic hardening,
 *                         x = (d_eel[6], dp, d_alpha[6]).
 * eel = eel_t + d_eel; sig = lambda tr(eel) 1 + 2 mu eel; xi = dev(sig) - 2/3 C
 * alpha; seq = sqrt(3/2 xi.xi); N = 3/2 xi / seq;
 * F_e = d_eel + dp N - deps; F_p = dp - dt A seq^m; F_a = d_alpha - dp N +
 * D dp alpha.  The start is x = 0. At each iterate: a non-finite residual
 * stops with status 3; ||F||_inf < tol stops with status 0; after maxit linear
 * solves status 1; a zero pivot status 2. The linear solves use the FMA mode
 * of lupp_batched_solve (LUPP_FMA) with textbook pivoting and one division
 * per elimination step (multipliers and back substitution by the pivot's
 * reciprocal), and the law multiplies by 1/seq and 1/3 where the formulas
 * divide.
 *
 * Consistent tangent (Section 2.5; Section 4.3: one multi-right-hand-side
 * solve after convergence), when pts->tangent is not NULL: with F(y; deps) =
 * 0 at the converged unknowns and dF/d(deps) = -[I6; 0], dy/d(deps) =
 * J^-1 [I6; 0]. The kernel factors the Jacobian of the converged iterate
 * once (partial pivoting, the same device-callable LU), solves for the six
 * unit right-hand sides, and returns dsig/d(deps) = D dy_e/d(deps), D the
 * elastic stiffness. A singular Jacobian there gives NaN entries.
 */
#define LUPP_MAXIT_LIMIT 10000 /* largest accepted maxit (bounds every kernel's run time) */
#define LUPP_LAW_NORTON7 7
#define LUPP_LAW_NORTON_AF13 13

typedef struct {
    int kind;      /* LUPP_LAW_NORTON7 or LUPP_LAW_NORTON_AF13 */
    double E, nu;  /* Young's modulus, Poisson ratio */
    double A, m;   /* Norton: dp/dt = A seq^m */
    double C, D;   /* Armstrong-Frederick modulus and recall (kind 13) */
    double dt;     /* time step */
} lupp_law;

typedef struct {
    int64_t count;        /* number of integration points */
    int64_t ld;           /* component stride (SoA), >= count */
    const double *deps;   /* [6][ld]   Kelvin total strain increment */
    double *state;        /* [kind][ld] eel(6), p, (alpha(6)); updated only where status == 0 */
    double *sig;          /* [6][ld]   stress at the returned iterate */
    int32_t *iters;       /* [count]   linear solves performed */
    int32_t *status;      /* [count]   0 converged, 1 maxit, 2 singular J, 3 non-finite */
    double *tangent;      /* NULL, or [36][ld]: consistent tangent dsig/d(deps) of every
                             converged point, entry (r, c) at component 6*r + c (Kelvin);
                             untouched for points with status != 0 */
} lupp_points;

int constitutive_update(lupp_ctx *ctx, const lupp_points *pts, const lupp_law *law, double tol,
                        int maxit, void *stream);

/* Mapping of the fused update for law `kind` on this context (Section 3.2:
 * single- versus multi-threaded device-callable solvers): lanes = 1 runs one
 * lane per point (the whole Jacobian in one lane's registers); 4 or 8 (kind
 * 7) and 8 or 16 (kind 13) run that many lanes per point, each building its
 * own Jacobian rows, with the lanes LU. Results are bitwise the same for
 * every mapping. 0 restores the measured default. Calls that request the
 * tangent always run one lane per point. Returns -k for the k-th argument. */
int lupp_set_newton_variant(lupp_ctx *ctx, int kind, int lanes);
int lupp_get_newton_variant(const lupp_ctx *ctx, int kind, int *lanes);

/* CPU-driven batched form of the same update (Algorithm 1; Section 2.5),
 * for comparison with the fused kernel: each Newton iteration is an assemble
 * launch over all points, one batched LU solve launch over all Jacobians
 * (interleaved layout) and an update launch, after which
 * the host reads one counter of points still iterating. Finished points are
 * carried through the remaining batched solves but do not change, so every
 * output (sig, state, iters, status, tangent) is bitwise the one
 * constitutive_update computes. Blocks the calling thread until done (it
 * synchronises `stream` once per iteration). The context keeps the device
 * workspace (about 8 (kind^2 + kind + 3) bytes per point) between calls.
 *   flags      : 0, or LUPP_BATCHED_GRAPH to capture one iteration in a HIP
 *                graph and replay it (one launch per iteration).
 *   iterations : NULL, or receives the number of host-driven iterations.
 * The batched solve is the library's thread solver in the arithmetic of the
 * fused kernel's Newton steps (textbook pivoting whatever the context's
 * setting). Returns as constitutive_update, or -6 for unknown flags. */
#define LUPP_BATCHED_GRAPH 1u
int constitutive_update_batched(lupp_ctx *ctx, const lupp_points *pts, const lupp_law *law,
                                double tol, int maxit, unsigned flags, void *stream,
                                int *iterations);

/* ---------------------------------------------------------------------------
 * Time-step sweeps captured in a HIP graph. An implicit constitutive update
 * runs at every step of the global solution (Section 2.5); a sweep records
 * `steps` successive constitutive_update launches on the same points (step t
 * reads the strain increments at pts->deps + t * deps_step and starts from
 * the state the previous step committed) as kernel nodes of one graph, and
 * each lupp_sweep_launch replays all of them with one launch on `stream`.
 *   deps_step : elements between the increments of successive steps, >= 6 * ld,
 *               or 0 to apply the same increments at every step.
 * The buffers named by pts are bound at creation and must stay valid until
 * lupp_sweep_destroy; sig/iters/status/tangent hold the last step's values
 * after a replay. Replays on one sweep must not overlap (they share the
 * buffers). Returns 0 or -k for the k-th argument (as constitutive_update,
 * -6 steps < 1, -7 deps_step, -8 out == NULL). */
typedef struct lupp_sweep lupp_sweep;
int lupp_sweep_create(lupp_ctx *ctx, const lupp_points *pts, const lupp_law *law, double tol,
                      int maxit, int steps, int64_t deps_step, lupp_sweep **out);
int lupp_sweep_launch(lupp_sweep *sweep, void *stream);
void lupp_sweep_destroy(lupp_sweep *sweep);

/* ---------------------------------------------------------------------------
 * Serving loop: continuous batching of solve and constitutive-update requests
 * under an HBM budget.
 *
 * A scheduler thread admits waiting requests in submission order while one
 * of max_inflight slots is free and the arena (a device allocation of
 * hbm_budget_bytes) holds their staging buffers; a request whose point set is
 * busy lets later requests pass. Everything admitted in one scheduling pass
 * runs together on one of `streams` HIP streams (successive passes overlap on
 * the GPU):
 *   LUPP_SERVE_MERGED (default): the solve requests of the pass with fewer
 *     than 32768 systems are the groups of one grouped solve (see
 *     lupp_batched_solve_grouped), larger ones are solved one call each with
 *     the size-aware dispatch table, and the update requests with the same
 *     law, tol, maxit and tangent choice share one fused-Newton launch over
 *     their point sets;
 *   LUPP_SERVE_PER_REQUEST: one pass and one launch per request (each solve
 *     with lupp_batched_solve's dispatch table).
 * A context with tile-local pivoting or a forced variant has its solves run
 * per request in either mode, with those settings.
 *
 * Request pointers may be host or device pointers (detected per pointer).
 * Device data is used in place: a device A is only read (the factors are
 * written to lu, if given), the right-hand sides are copied into a device x
 * (unless x == b) and solved there, device outputs are written directly.
 * Host inputs are copied into the arena and host outputs copied back from
 * it; so are outputs given as NULL (and then dropped). The arena holds only
 * these staging buffers. Pointers must stay valid until the ticket
 * completes. Host buffers should be pinned (hipHostMalloc) for the copies to
 * overlap; pageable ones work but copy synchronously.
 *
 * Integration-point state is device-resident: a point set is registered
 * once and every update request on it advances its state (committed per
 * point on convergence). Requests on the same set run in submission order.
 * Results of a request are bitwise identical whether it runs alone or among
 * others, in either mode: each system or point is computed independently and
 * identically. The server works on a context of its own holding a copy of
 * the creating context's settings (dispatch and ragged tables, pivoting,
 * Newton mapping) at creation.
 */
typedef struct lupp_server lupp_server;

#define LUPP_SERVE_MERGED 0
#define LUPP_SERVE_PER_REQUEST 1

typedef struct {
    int64_t hbm_budget_bytes; /* device arena; 0 = a quarter of the free memory */
    int max_inflight;         /* requests admitted at once, >= 1 */
    int streams;              /* HIP streams, 1..64 */
    int mode;                 /* LUPP_SERVE_MERGED or LUPP_SERVE_PER_REQUEST */
} lupp_server_config;

#define LUPP_REQ_SOLVE 1
#define LUPP_REQ_UPDATE 2

typedef struct {
    int kind; /* LUPP_REQ_SOLVE or LUPP_REQ_UPDATE */
    /* LUPP_REQ_SOLVE: `batch` (1..2^31-1) packed column-major systems of size
     * n (1..32) */
    int n;
    int64_t batch;
    const double *A; /* [batch][n*n] in */
    const double *b; /* [batch][n] in: right-hand sides */
    double *x;       /* [batch][n] out: solutions where info == 0, the right-hand
                        side where info > 0 (may alias b) */
    int32_t *ipiv;   /* [batch][n] out, or NULL */
    int32_t *info;   /* [batch] out, or NULL */
    double *lu;      /* [batch][n*n] out: the factors, or NULL to skip them */
    /* LUPP_REQ_UPDATE: one Newton update of every point of a point set */
    int64_t set_id;
    int64_t count;   /* must equal the set's point count */
    const lupp_law *law; /* law->kind must equal the set's kind */
    double tol;
    int maxit;
    const double *deps; /* [6][count] in */
    double *sig;        /* [6][count] out, or NULL */
    int32_t *iters;     /* [count] out, or NULL */
    int32_t *status;    /* [count] out, or NULL */
    double *tangent;    /* [36][count] out, or NULL: consistent tangent of the
                           converged points (see constitutive_update); entries of
                           points with status != 0 are unspecified */
} lupp_request;

typedef struct {
    int64_t submitted, completed, rejected, failed, queued;
    int inflight, peak_inflight;
    int64_t peak_bytes, budget_bytes;
    double p50_ms, p99_ms, mean_ms, max_ms; /* submit -> completion, completed requests */
    double elapsed_s;                        /* first submit -> last completion */
    int64_t passes;                          /* scheduling passes run */
    int64_t launches;                        /* solve / update calls they made */
} lupp_server_stats;

/* Create a server on ctx's device (it uses a context of its own internally).
 * Starts one scheduler thread. */
int lupp_server_create(lupp_ctx *ctx, const lupp_server_config *cfg, lupp_server **server);
/* Finish every queued and admitted request, then release everything. */
void lupp_server_destroy(lupp_server *server);
/* Register count points of law kind (7 or 13) with initial state [kind][count]
 * (host or device; NULL = virgin). Synchronous. */
int lupp_server_add_points(lupp_server *server, int kind, int64_t count, const double *state,
                           int64_t *set_id);
/* Copy a point set's state out ([kind][count]) after its queued requests. */
int lupp_server_read_points(lupp_server *server, int64_t set_id, double *state);
/* Queue a request: returns a ticket > 0, -2 for an invalid request, or
 * LUPP_E_NOMEM if its footprint exceeds the whole budget. */
int64_t lupp_server_submit(lupp_server *server, const lupp_request *req);
/* 1 if the ticket has completed, 0 if not, negative if unknown. */
int lupp_server_poll(lupp_server *server, int64_t ticket);
/* Block until the ticket completes; returns its status (0 or a lupp error)
 * and its latency; the ticket is then retired. */
int lupp_server_wait(lupp_server *server, int64_t ticket, double *latency_ms);
int lupp_server_get_stats(lupp_server *server, lupp_server_stats *stats);
int lupp_server_reset_stats(lupp_server *server);

/* Human-readable text for a return code (static storage). */
const char *lupp_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif
