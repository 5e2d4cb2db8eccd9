/*
 * Oracle: discrete adjoint of the periodic scalar-wave RK4 step and the
 * sphere-integral objective.  The paper has no adjoint; this is the exact
 * transpose of the discrete map built by orc_core.c, written in scatter form
 * (each output point sends its stencil weights back to the points it read).
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int wrapi(int a, int n)
{
    int m = a % n;
    return m < 0 ? m + n : m;
}

/* Transpose of the wave right-hand side (Sec. IV.A with KO on both fields).
 * lam holds adjoint values on interior points; lamU receives, on every point
 * of the ghosted box, sum_c lam(c) dR(c)/dU(point).  lamU is overwritten. */
void orc_wave_rhs_adjoint(const double* lam, double* lamU, int nx, int ny, int nz,
                          const double h[3], const orc_params* p)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    long st[3] = {1, NX, NX * NY};
    static const double kow[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};
    static const double d2w[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    memset(lamU, 0, sizeof(double) * 2 * vol);
    for (int k = ORC_G; k < nz + ORC_G; ++k)
        for (int j = ORC_G; j < ny + ORC_G; ++j)
            for (int i = ORC_G; i < nx + ORC_G; ++i) {
                long c = (k * NY + j) * NX + i;
                double lp = lam[c], lq = lam[vol + c];
                /* R_phi(c) = -Pi(c) + sum_d KO(phi)(c) */
                lamU[vol + c] -= lp;
                for (int d = 0; d < 3; ++d) {
                    double kc = p->sigma / (64.0 * h[d]);
                    for (int m = -3; m <= 3; ++m) {
                        lamU[c + m * st[d]] += lp * kc * kow[m + 3];
                        lamU[vol + c + m * st[d]] += lq * kc * kow[m + 3];
                    }
                    /* R_Pi(c) = -sum_d D_dd phi(c) + sum_d KO(Pi)(c) */
                    double dc = 1.0 / (12.0 * h[d] * h[d]);
                    for (int m = -2; m <= 2; ++m) lamU[c + m * st[d]] -= lq * dc * d2w[m + 2];
                }
            }
}

void orc_fill_periodic_adjoint(double* A, int nf, int nx, int ny, int nz)
{
    int NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    for (int f = 0; f < nf; ++f) {
        double* a = A + (long)f * NX * NY * NZ;
        for (int k = 0; k < NZ; ++k)
            for (int j = 0; j < NY; ++j)
                for (int i = 0; i < NX; ++i) {
                    int gi = i - ORC_G, gj = j - ORC_G, gk = k - ORC_G;
                    if (gi >= 0 && gi < nx && gj >= 0 && gj < ny && gk >= 0 && gk < nz)
                        continue;
                    int si = wrapi(gi, nx) + ORC_G, sj = wrapi(gj, ny) + ORC_G,
                        sk = wrapi(gk, nz) + ORC_G;
                    long g = ((long)k * NY + j) * NX + i;
                    a[((long)sk * NY + sj) * NX + si] += a[g];
                    a[g] = 0.0;
                }
    }
}

/* J = sum over interior points with |x| < rad of (U_field - shift) dx dy dz,
 * x_i = xlo + i h (interior index i). */
double orc_sphere_integral(const double* U, int field, int nx, int ny, int nz,
                           const double xlo[3], const double h[3], double rad,
                           double shift)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    double s = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double x = xlo[0] + i * h[0], y = xlo[1] + j * h[1], z = xlo[2] + k * h[2];
                if (x * x + y * y + z * z < rad * rad)
                    s += U[field * vol + ((long)(k + ORC_G) * NY + j + ORC_G) * NX + i + ORC_G] - shift;
            }
    return s * h[0] * h[1] * h[2];
}

/* Reverse sweep of nsteps RK4 steps (RK44 tableau).  The forward step is
 *   Us_s = U + b_s k_{s-1} (ghosts refilled), k_s = dt L(Us_s),
 *   U' = U + sum_s c_s k_s;
 * for the linear wave operator its transpose needs no forward states:
 *   lk4 = c4 lam,            m4 = fill^T(dt L^T lk4),
 *   lk3 = c3 lam + m4,       m3 = fill^T(dt L^T lk3),
 *   lk2 = c2 lam + m3 / 2,   m2 = fill^T(dt L^T lk2),
 *   lk1 = c1 lam + m2 / 2,   m1 = fill^T(dt L^T lk1),
 *   lam <- lam + m1 + m2 + m3 + m4. */
void orc_wave_adjoint_run(double* lam0, int nx, int ny, int nz, const double h[3],
                          const double xlo[3], double dt, int nsteps, double rad,
                          const orc_params* p)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ, n = 2 * vol;
    static const double cw[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    static const double bsub[4] = {0.0, 0.5, 0.5, 1.0};
    double* lam = lam0;
    double* lk = (double*)calloc(n, sizeof(double));
    double* m = (double*)calloc(n, sizeof(double));
    double* msum = (double*)calloc(n, sizeof(double));
    memset(lam, 0, sizeof(double) * n);
    double dV = h[0] * h[1] * h[2];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double x = xlo[0] + i * h[0], y = xlo[1] + j * h[1], z = xlo[2] + k * h[2];
                if (x * x + y * y + z * z < rad * rad)
                    lam[((long)(k + ORC_G) * NY + j + ORC_G) * NX + i + ORC_G] = dV;
            }
    for (int step = 0; step < nsteps; ++step) {
        memset(msum, 0, sizeof(double) * n);
        memset(m, 0, sizeof(double) * n);
        for (int s = 3; s >= 0; --s) {
            /* lk_s = c_s lam + b_{s+1} m_{s+1} */
            for (long q = 0; q < n; ++q) lk[q] = cw[s] * lam[q] + (s < 3 ? bsub[s + 1] * m[q] : 0.0);
            orc_wave_rhs_adjoint(lk, m, nx, ny, nz, h, p);
            for (long q = 0; q < n; ++q) m[q] *= dt;
            orc_fill_periodic_adjoint(m, 2, nx, ny, nz);
            for (long q = 0; q < n; ++q) msum[q] += m[q];
        }
        for (long q = 0; q < n; ++q) lam[q] += msum[q];
    }
    free(lk);
    free(m);
    free(msum);
}
