/*
 * Oracle: the one-dimensional finite-difference stencils of Sec. II.B.1,
 * applied to u[0] with stride s.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 * Kept in a file of their own so that the exact-derivative build of the CCZ4
 * right-hand side (orc_ccz4_jvp.cpp) can compile them with dual numbers.
 */
#include "oracle.h"

/* Sec. II.B.1: 4th-order centred first derivative
 *   (U_{i-2} - 8 U_{i-1} + 8 U_{i+1} - U_{i+2}) / (12 dx),
 * evaluated as differences of symmetric neighbours. */
double orc_d1(const double* u, long s, double h)
{
    return (8.0 * (u[s] - u[-s]) - (u[2 * s] - u[-2 * s])) / (12.0 * h);
}

/* Sec. II.B.1: 4th-order second derivative along one axis
 *   (-U_{i-2} + 16 U_{i-1} - 30 U_i + 16 U_{i+1} - U_{i+2}) / (12 dx^2),
 * evaluated as weighted second differences about U_i. */
double orc_d2(const double* u, long s, double h)
{
    double c = u[0];
    double a1 = (u[s] - c) + (u[-s] - c);
    double a2 = (u[2 * s] - c) + (u[-2 * s] - c);
    return (16.0 * a1 - a2) / (12.0 * h * h);
}

/* Sec. II.B.1: lop-sided 4th-order advection derivative used for beta d_x U.
 * beta < 0 uses points i-3..i+1, beta > 0 uses i-1..i+3; at beta == 0 the term
 * vanishes and the beta > 0 branch is taken (a fixed choice).  Weighted
 * differences about U_i. */
double orc_adv(const double* u, long s, double h, double beta)
{
    double c = u[0];
    if (beta >= 0.0) {
        return ((u[3 * s] - c) - 6.0 * (u[2 * s] - c) + 18.0 * (u[s] - c)
                - 3.0 * (u[-s] - c)) / (12.0 * h);
    }
    return (-(u[-3 * s] - c) + 6.0 * (u[-2 * s] - c) - 18.0 * (u[-s] - c)
            + 3.0 * (u[s] - c)) / (12.0 * h);
}

/* Sec. II.B.1: Kreiss-Oliger dissipation along one axis,
 *   sigma/(64 dx) (U_{i-3} - 6U_{i-2} + 15U_{i-1} - 20U_i + 15U_{i+1} - 6U_{i+2} + U_{i+3}),
 * as weighted symmetric second differences about U_i. */
double orc_ko(const double* u, long s, double h, double sigma)
{
    double c = u[0];
    double a1 = (u[s] - c) + (u[-s] - c);
    double a2 = (u[2 * s] - c) + (u[-2 * s] - c);
    double a3 = (u[3 * s] - c) + (u[-3 * s] - c);
    return sigma * (a3 - 6.0 * a2 + 15.0 * a1) / (64.0 * h);
}

/* Sec. II.B.1: cross derivative D_ab U = D_b(D_a U). */
double orc_dmix(const double* u, long sa, double ha, long sb, double hb)
{
    double dp1 = orc_d1(u + sb, sa, ha);
    double dm1 = orc_d1(u - sb, sa, ha);
    double dp2 = orc_d1(u + 2 * sb, sa, ha);
    double dm2 = orc_d1(u - 2 * sb, sa, ha);
    return (8.0 * (dp1 - dm1) - (dp2 - dm2)) / (12.0 * hb);
}
