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

struct LawK {
    double lam, two_mu, dtA, m, c23, D;
};

/* Residual, Jacobian (J[c][r] = dF_r/dy_c, the solver's column-major form)
 * and stress at the unknowns y. */
template <int NU>
__device__ __forceinline__ void law_assemble(const LawK &P, const double (&de)[6],
                                             const double (&st)[NU], const double (&y)[NU],
                                             double (&F)[NU], double (&J)[NU][NU], double (&sig)[6])
{
    constexpr bool af = (NU == 13);
    double e[6], xi[6], al[6], Nv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = st[i] + y[i];
    const double tr = e[0] + e[1] + e[2];
#pragma unroll
    for (int i = 0; i < 6; ++i) sig[i] = P.two_mu * e[i] + (i < 3 ? P.lam * tr : 0.0);
    const double mean = (sig[0] + sig[1] + sig[2]) / 3.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        xi[i] = sig[i] - (i < 3 ? mean : 0.0);
        if constexpr (af) {
            al[i] = st[7 + i] + y[7 + i];
            xi[i] = xi[i] - P.c23 * al[i];
        } else {
            al[i] = 0.0;
        }
    }
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) q += xi[i] * xi[i];
    const double seq = sqrt(1.5 * q);
    const bool pl = seq > 0.0;
    const double inv = pl ? 1.0 / seq : 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) Nv[i] = pl ? 1.5 * xi[i] / seq : 0.0;

    const double dp = y[6];
    const double sm1 = pl ? pow(seq, P.m - 1.0) : 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) F[i] = y[i] + dp * Nv[i] - de[i];
    F[6] = dp - P.dtA * (pl ? pow(seq, P.m) : 0.0);
    if constexpr (af) {
#pragma unroll
        for (int i = 0; i < 6; ++i) F[7 + i] = y[7 + i] - dp * Nv[i] + P.D * dp * al[i];
    }

    /* G = dN/dxi = (3/2 I - N N^T) / seq;  GK = G K (K: deviatoric projector)
     * so that dN/d(d_eel) = 2 mu GK and dN/d(d_alpha) = -2/3 C G. */
    double G[6][6], GK[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 6; ++b) G[a][b] = ((a == b ? 1.5 : 0.0) - Nv[a] * Nv[b]) * inv;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        const double rowmean = (G[a][0] + G[a][1] + G[a][2]) / 3.0;
#pragma unroll
        for (int b = 0; b < 6; ++b) GK[a][b] = G[a][b] - (b < 3 ? rowmean : 0.0);
    }
    const double nmean = (Nv[0] + Nv[1] + Nv[2]) / 3.0;
    const double gd = P.dtA * P.m * sm1; /* d(dt A seq^m)/dseq */
    const double dp2mu = dp * P.two_mu;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
#pragma unroll
        for (int a = 0; a < 6; ++a) J[b][a] = (a == b ? 1.0 : 0.0) + dp2mu * GK[a][b];
        J[b][6] = -gd * P.two_mu * (Nv[b] - (b < 3 ? nmean : 0.0));
        J[6][b] = Nv[b];
    }
    J[6][6] = 1.0;
    if constexpr (af) {
        const double cdp = P.c23 * dp;
#pragma unroll
        for (int b = 0; b < 6; ++b) {
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                J[7 + b][a] = -cdp * G[a][b];                 /* dF_e / d(d_alpha) */
                J[b][7 + a] = -dp2mu * GK[a][b];              /* dF_a / d(d_eel)   */
                J[7 + b][7 + a] = (a == b ? 1.0 + P.D * dp : 0.0) + cdp * G[a][b];
            }
            J[7 + b][6] = P.c23 * gd * Nv[b];                 /* dF_p / d(d_alpha) */
            J[6][7 + b] = -Nv[b] + P.D * al[b];               /* dF_a / d(dp)      */
        }
    }
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
    const bool sing = thread_getrf_solve<7, true>(J, z, piv) != 0;
    thread_ipiv_to_perm<7>(piv, perm);
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
        double x[7];
        thread_solve_unit<7>(J, perm, c, x);
        tangent_store_col<7>(P, pts, p0, nb, vo, c, x, sing);
    }
}

/* 13 unknowns: the 13 x 13 factors and a solution vector do not fit in
 * registers together, so each column re-assembles J and runs the fused
 * factor-and-solve on e_c. Every column sees the same factorization and the
 * same operation sequence, so the result is bitwise that of the factor-once
 * form. Not inlined: it gets its own register budget instead of adding to
 * the Newton loop's. */
static __device__ __attribute__((noinline)) void newton_tangent13(const LawK &P, const double (&de)[6],
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
        const bool sing = thread_getrf_solve<13, false>(J, x, piv) != 0;
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
    P.c23 = law->kind == LUPP_LAW_NORTON_AF13 ? 2.0 / 3.0 * law->C : 0.0;
    P.D = law->kind == LUPP_LAW_NORTON_AF13 ? law->D : 0.0;
    return P;
}

}  // namespace lupp

#endif
