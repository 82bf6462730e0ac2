/* The constitutive laws of the fused and batched Newton updates: residual,
 * exact Jacobian and stress (Section 2.1, equations 1-3), and the consistent
 * tangent after convergence (Section 2.5; Section 4.3).
 *
 * Laws (Kelvin-Mandel 6-vectors, backward Euler), unknowns y:
 *   Norton (7):      y = (d_eel[6], dp)
 *   Norton + AF(13): y = (d_eel[6], dp, d_alpha[6])
 *   eel = eel_t + d_eel, sig = lambda tr(eel) 1 + 2 mu eel,
 *   xi  = dev(sig) - 2/3 C alpha,  seq = sqrt(3/2 xi.xi),  N = 3/2 xi / seq,
 *   F_e = d_eel + dp N - deps,  F_p = dp - dt A seq^m,
 *   F_a = d_alpha - dp N + D dp alpha,
 * with the exact Jacobian of these residuals.
 */
#ifndef LUPP_LAW_H
#define LUPP_LAW_H

#include "internal.h"
#include "lupp_device.h"

namespace lupp {

/* Arithmetic of the Newton updates' linear solves (the Newton step and the
 * tangent): one fused multiply-add per multiply-subtract (the library's FMA
 * mode), and one division per elimination step - the multipliers and the
 * back substitution use the pivot's reciprocal - with textbook pivoting. The
 * fused kernels, the lanes-per-point kernels and the CPU-driven batched form
 * all use it, so they stay bitwise equal to each other; against the strict
 * oracle the updates agree within the Newton tolerance. (The 7-unknown
 * tangent keeps its factors for six right-hand sides and so divides.) */
constexpr bool kNewtonFMA = true;
constexpr bool kNewtonRecip = true;

/* 1/3 rounded once: the means of the law multiply by it */
constexpr double kThird = 1.0 / 3.0;

struct LawK {
    double lam, two_mu, dtA, m, c23, D;
    int mi; /* m when it is an integer in 1..64 (powers by multiplication), else 0 */
};

/* seq^(m-1) and seq^m for seq > 0. An integer exponent (the benchmark's
 * m = 5) takes repeated squaring: a handful of multiplies instead of two
 * pow calls (each a log/exp sequence of ~100 instructions), and within a
 * few ulps of pow, as pow itself is of the correctly rounded power. The loop
 * count is uniform across the wave. */
__device__ __forceinline__ void law_powers(const LawK &P, double seq, double &pm1, double &pm)
{
    if (P.mi > 0) {
        double r = 1.0, b = seq;
        for (int e = P.mi - 1; e != 0; e >>= 1) {
            if (e & 1) r = r * b;
            b = b * b;
        }
        pm1 = r;
        pm = r * seq;
    } else {
        pm1 = pow(seq, P.m - 1.0);
        pm = pow(seq, P.m);
    }
}

/* What the residual and every Jacobian row need at the unknowns y: stress,
 * flow direction N, back-strain alpha, the scalars of the Jacobian blocks,
 * and the residual F itself. */
template <int NU>
struct LawC {
    double sig[6], Nv[6], al[6], F[NU];
    double inv, dp, gd, dp2mu, cdp, nmean;
};

/* Stress at the unknowns y: sig = lambda tr(eel) 1 + 2 mu eel, eel = eel_t +
 * d_eel (the expression law_common uses, so the result is the same bits). */
template <int NU>
__device__ __forceinline__ void law_stress(const LawK &P, const double (&st)[NU],
                                           const double (&y)[NU], double (&sig)[6])
{
    double e[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = st[i] + y[i];
    const double tr = e[0] + e[1] + e[2];
#pragma unroll
    for (int i = 0; i < 6; ++i) sig[i] = P.two_mu * e[i] + (i < 3 ? P.lam * tr : 0.0);
}

template <int NU>
__device__ __forceinline__ void law_common(const LawK &P, const double (&de)[6],
                                           const double (&st)[NU], const double (&y)[NU],
                                           LawC<NU> &C)
{
    constexpr bool af = (NU == 13);
    double xi[6];
    law_stress<NU>(P, st, y, C.sig);
    const double mean = (C.sig[0] + C.sig[1] + C.sig[2]) * kThird;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        xi[i] = C.sig[i] - (i < 3 ? mean : 0.0);
        if constexpr (af) {
            C.al[i] = st[7 + i] + y[7 + i];
            xi[i] = xi[i] - P.c23 * C.al[i];
        } else {
            C.al[i] = 0.0;
        }
    }
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) q += xi[i] * xi[i];
    const double seq = sqrt(1.5 * q);
    const bool pl = seq > 0.0;
    C.inv = pl ? 1.0 / seq : 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) C.Nv[i] = pl ? 1.5 * xi[i] * C.inv : 0.0;

    const double dp = y[6];
    double sm1 = 0.0, sm = 0.0;
    if (pl) law_powers(P, seq, sm1, sm);
#pragma unroll
    for (int i = 0; i < 6; ++i) C.F[i] = y[i] + dp * C.Nv[i] - de[i];
    C.F[6] = dp - P.dtA * sm;
    if constexpr (af) {
#pragma unroll
        for (int i = 0; i < 6; ++i) C.F[7 + i] = y[7 + i] - dp * C.Nv[i] + P.D * dp * C.al[i];
    }
    C.dp = dp;
    C.nmean = (C.Nv[0] + C.Nv[1] + C.Nv[2]) * kThird;
    C.gd = P.dtA * P.m * sm1; /* d(dt A seq^m)/dseq */
    C.dp2mu = dp * P.two_mu;
    C.cdp = P.c23 * dp;
}

/* The Jacobian blocks. G = dN/dxi = (3/2 I - N N^T) / seq and GK = G K (K:
 * the deviatoric projector), so that dN/d(d_eel) = 2 mu GK and
 * dN/d(d_alpha) = -2/3 C G. Row a of G and GK needs only N_a: */
__device__ __forceinline__ void law_g_row(const double (&Nv)[6], double inv, int a, double Na,
                                          double (&G)[6], double (&GK)[6])
{
#pragma unroll
    for (int b = 0; b < 6; ++b) G[b] = ((a == b ? 1.5 : 0.0) - Na * Nv[b]) * inv;
    const double rowmean = (G[0] + G[1] + G[2]) * kThird;
#pragma unroll
    for (int b = 0; b < 6; ++b) GK[b] = G[b] - (b < 3 ? rowmean : 0.0);
}

/* v[i] for a lane-varying i by a compare/select chain. Each element passes
 * through an empty asm so that the compiler cannot turn the chain back into
 * a dynamically indexed (scratch-memory) array load. */
template <int M>
__device__ __forceinline__ double select_at(const double (&v)[M], int i)
{
    double r = v[0];
#pragma unroll
    for (int k = 1; k < M; ++k) {
        double x = v[k];
        asm volatile("" : "+v"(x));
        r = (i == k) ? x : r;
    }
    return r;
}

/* Row r (0 <= r < NU) of the Jacobian, row[c] = dF_r/dy_c; r may differ
 * between lanes. Every entry is the expression law_jacobian uses. */
template <int NU>
__device__ __forceinline__ void law_jac_row(const LawK &P, const LawC<NU> &C, int r,
                                            double (&row)[NU])
{
    constexpr bool af = (NU == 13);
    /* N_a and alpha_a of the row's component, by selects (no dynamic index) */
    const int a = r < 6 ? r : r - 7;
    const double Na = select_at<6>(C.Nv, a);
    const double ala = af ? select_at<6>(C.al, a) : 0.0;
    if (r == 6) {
#pragma unroll
        for (int b = 0; b < 6; ++b) row[b] = -C.gd * P.two_mu * (C.Nv[b] - (b < 3 ? C.nmean : 0.0));
        row[6] = 1.0;
        if constexpr (af) {
#pragma unroll
            for (int b = 0; b < 6; ++b) row[7 + b] = P.c23 * C.gd * C.Nv[b];
        }
        return;
    }
    double G[6], GK[6];
    law_g_row(C.Nv, C.inv, a, Na, G, GK);
    if (r < 6) {
#pragma unroll
        for (int b = 0; b < 6; ++b) row[b] = (a == b ? 1.0 : 0.0) + C.dp2mu * GK[b];
        row[6] = Na;
        if constexpr (af) {
#pragma unroll
            for (int b = 0; b < 6; ++b) row[7 + b] = -C.cdp * G[b];
        }
    } else if constexpr (af) {
#pragma unroll
        for (int b = 0; b < 6; ++b) row[b] = -C.dp2mu * GK[b];
        row[6] = -Na + P.D * ala;
#pragma unroll
        for (int b = 0; b < 6; ++b) row[7 + b] = (a == b ? 1.0 + P.D * C.dp : 0.0) + C.cdp * G[b];
    }
}

/* The whole Jacobian, J[c][r] = dF_r/dy_c (the solver's column-major form). */
template <int NU>
__device__ __forceinline__ void law_jacobian(const LawK &P, const LawC<NU> &C, double (&J)[NU][NU])
{
    constexpr bool af = (NU == 13);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double G[6], GK[6];
        law_g_row(C.Nv, C.inv, a, C.Nv[a], G, GK);
#pragma unroll
        for (int b = 0; b < 6; ++b) J[b][a] = (a == b ? 1.0 : 0.0) + C.dp2mu * GK[b];
        J[6][a] = C.Nv[a];
        if constexpr (af) {
#pragma unroll
            for (int b = 0; b < 6; ++b) {
                J[7 + b][a] = -C.cdp * G[b];                  /* dF_e / d(d_alpha) */
                J[b][7 + a] = -C.dp2mu * GK[b];               /* dF_a / d(d_eel)   */
                J[7 + b][7 + a] = (a == b ? 1.0 + P.D * C.dp : 0.0) + C.cdp * G[b];
            }
            J[6][7 + a] = -C.Nv[a] + P.D * C.al[a];           /* dF_a / d(dp)      */
        }
    }
#pragma unroll
    for (int b = 0; b < 6; ++b) J[b][6] = -C.gd * P.two_mu * (C.Nv[b] - (b < 3 ? C.nmean : 0.0));
    J[6][6] = 1.0;
    if constexpr (af) {
#pragma unroll
        for (int b = 0; b < 6; ++b) J[7 + b][6] = P.c23 * C.gd * C.Nv[b]; /* dF_p / d(d_alpha) */
    }
}

/* Residual, Jacobian and stress at the unknowns y. */
template <int NU>
__device__ __forceinline__ void law_assemble(const LawK &P, const double (&de)[6],
                                             const double (&st)[NU], const double (&y)[NU],
                                             double (&F)[NU], double (&J)[NU][NU], double (&sig)[6])
{
    LawC<NU> C;
    law_common<NU>(P, de, st, y, C);
    law_jacobian<NU>(P, C, J);
#pragma unroll
    for (int i = 0; i < NU; ++i) F[i] = C.F[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) sig[i] = C.sig[i];
}

/* Consistent tangent (Section 2.5; Section 4.3: one multi-right-hand-side
 * solve after convergence) at the converged unknowns y: with dF/d(deps) =
 * -[I6; 0], dy/d(deps) = J^-1 [I6; 0] for the Jacobian J of the converged
 * iterate, and dsig/d(deps) = D dy_e/d(deps). Column c of the result needs
 * J^-1 e_c: LU with partial pivoting, then the interchanges and the forward
 * and back substitutions applied to e_c. Column c is stored at tangent
 * components 6 r + c, r = 0..5. */
template <int NU>
__device__ __forceinline__ void tangent_store_col(const LawK &P, const lupp_points &pts, int64_t p0,
                                                  uint32_t nb, uint32_t vo, int c,
                                                  const double (&x)[NU], bool sing)
{
    const double lt = P.lam * (x[0] + x[1] + x[2]);
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const double t = P.two_mu * x[r] + (r < 3 ? lt : 0.0);
        const auto rt = make_rsrc(pts.tangent + (6 * r + c) * pts.ld + p0, nb);
        buf_store_f64(rt, vo, 0, sing ? __builtin_nan("") : t);
    }
}

/* 7 unknowns: J is factored once and the six unit vectors are solved with
 * the kept factors (all of it fits in registers next to the Newton loop). */
__device__ __forceinline__ void newton_tangent7(const LawK &P, const double (&de)[6],
                                                const double (&st)[7], const double (&y)[7],
                                                const lupp_points &pts, int64_t p0, uint32_t nb,
                                                uint32_t vo)
{
    double J[7][7], Fc[7], sc[6], z[7];
    int piv[7], perm[7];
    law_assemble<7>(P, de, st, y, Fc, J, sc);
#pragma unroll
    for (int i = 0; i < 7; ++i) z[i] = 0.0;
    const bool sing = thread_getrf_solve<7, true, kNewtonFMA>(J, z, piv) != 0;
    thread_ipiv_to_perm<7>(piv, perm);
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
        double x[7];
        thread_solve_unit<7, kNewtonFMA>(J, perm, c, x);
        tangent_store_col<7>(P, pts, p0, nb, vo, c, x, sing);
    }
}

/* 13 unknowns: the 13 x 13 factors and a solution vector do not fit in
 * registers together, so each column re-assembles J and runs the fused
 * factor-and-solve on e_c. Every column sees the same factorization and the
 * same operation sequence, so the result is bitwise that of the factor-once
 * form. Inlined: after the loop the caller holds nothing but the loop's
 * inputs (kept in LDS by the fused kernel), so it fits the loop's register
 * budget without scratch; a call boundary would force its array arguments
 * into scratch memory. */
static __device__ __forceinline__ void newton_tangent13(const LawK &P, const double (&de)[6],
                                                           const double (&st)[13],
                                                           const double (&y)[13],
                                                           const lupp_points &pts, int64_t p0,
                                                           uint32_t nb, uint32_t vo)
{
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
        double J[13][13], Fc[13], sc[6], x[13];
        int piv[13];
        law_assemble<13>(P, de, st, y, Fc, J, sc);
#pragma unroll
        for (int i = 0; i < 13; ++i) x[i] = (i == c) ? 1.0 : 0.0;
        const bool sing =
            thread_getrf_solve<13, false, kNewtonFMA, false, kNewtonRecip>(J, x, piv) != 0;
        tangent_store_col<13>(P, pts, p0, nb, vo, c, x, sing);
    }
}

static inline LawK law_constants(const lupp_law *law)
{
    LawK P;
    P.lam = law->E * law->nu / ((1.0 + law->nu) * (1.0 - 2.0 * law->nu));
    P.two_mu = law->E / (1.0 + law->nu);
    P.dtA = law->dt * law->A;
    P.m = law->m;
    P.mi = (law->m >= 1.0 && law->m <= 64.0 && law->m == (double)(int)law->m) ? (int)law->m : 0;
    P.c23 = law->kind == LUPP_LAW_NORTON_AF13 ? 2.0 / 3.0 * law->C : 0.0;
    P.D = law->kind == LUPP_LAW_NORTON_AF13 ? law->D : 0.0;
    return P;
}

}  // namespace lupp

#endif
