/*
 * Oracle core: stencils, periodic ghost fill, scalar wave right-hand side and
 * the explicit Runge-Kutta driver.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

int orc_nfields(int system)
{
    switch (system) {
    case ORC_WAVE: return 2;
    case ORC_MHD: return 8;
    case ORC_MHD_GLM: return 9;
    case ORC_CCZ4: return 25;
    }
    return -1;
}

static int wrapi(int a, int n)
{
    int m = a % n;
    return m < 0 ? m + n : m;
}

/* Periodic boundary: every ghost point takes the value of the interior point
 * congruent to it modulo the patch size (works for any n >= 1). */
void orc_fill_periodic(double* U, int nf, int nx, int ny, int nz)
{
    int NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    for (int f = 0; f < nf; ++f) {
        double* u = U + (long)f * NX * NY * NZ;
        for (int k = 0; k < NZ; ++k)
            for (int j = 0; j < NY; ++j)
                for (int i = 0; i < NX; ++i) {
                    int gi = i - ORC_G, gj = j - ORC_G, gk = k - ORC_G;
                    if (gi >= 0 && gi < nx && gj >= 0 && gj < ny && gk >= 0 && gk < nz)
                        continue;
                    int si = wrapi(gi, nx) + ORC_G, sj = wrapi(gj, ny) + ORC_G,
                        sk = wrapi(gk, nz) + ORC_G;
                    u[((long)k * NY + j) * NX + i] = u[((long)sk * NY + sj) * NX + si];
                }
    }
}

/* Sec. IV.A wave equation, first order in time:
 *   d_t phi = -Pi,   d_t Pi = -eta^{ij} d_i d_j phi   (eta^{ij} = delta^{ij}),
 * plus KO dissipation on both fields (semi-discrete form, Sec. II.A). */
void orc_wave_rhs(const double* U, double* R, int nx, int ny, int nz,
                  const double h[3], const orc_params* p)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    long st[3] = {1, NX, NX * NY};
    const double* phi = U;
    const double* Pi = U + vol;
    for (int k = ORC_G; k < nz + ORC_G; ++k)
        for (int j = ORC_G; j < ny + ORC_G; ++j)
            for (int i = ORC_G; i < nx + ORC_G; ++i) {
                long c = (k * NY + j) * NX + i;
                double lap = 0.0, kphi = 0.0, kpi = 0.0;
                for (int d = 0; d < 3; ++d) {
                    lap += orc_d2(phi + c, st[d], h[d]);
                    kphi += orc_ko(phi + c, st[d], h[d], p->sigma);
                    kpi += orc_ko(Pi + c, st[d], h[d], p->sigma);
                }
                R[c] = -Pi[c] + kphi;
                R[vol + c] = -lap + kpi;
            }
}

void orc_rhs(int system, const double* U, double* R, int nx, int ny, int nz,
             const double h[3], const orc_params* p)
{
    switch (system) {
    case ORC_WAVE: orc_wave_rhs(U, R, nx, ny, nz, h, p); break;
    case ORC_MHD: orc_mhd_rhs(U, R, nx, ny, nz, h, p); break;
    case ORC_MHD_GLM: orc_mhd_glm_rhs(U, R, nx, ny, nz, h, p); break;
    case ORC_CCZ4: orc_ccz4_rhs(U, R, nx, ny, nz, h, p); break;
    }
}

/* Butcher tableaux (eq. eRK):
 *   U^(i) = U^n + sum_{j<i} b_ij k_j,  k_j = dt L(U^(j)),  U^{n+1} = U^n + sum c_i k_i.
 * RK(4,4): Table RK44.  SSP-RK(3,3) as in App. D with the stage-3 state
 * U^n + k1/4 + k2/4 and weights (1, 1, 4)/6 (the reading that reproduces the
 * SSP dense output of App. C at theta = 1). */
static int rk_tableau(int scheme, double b[4][4], double c[4])
{
    memset(b, 0, sizeof(double) * 16);
    if (scheme == ORC_RK4) {
        b[1][0] = 0.5;
        b[2][1] = 0.5;
        b[3][2] = 1.0;
        c[0] = 1.0 / 6.0; c[1] = 2.0 / 6.0; c[2] = 2.0 / 6.0; c[3] = 1.0 / 6.0;
        return 4;
    }
    b[1][0] = 1.0;
    b[2][0] = 0.25; b[2][1] = 0.25;
    c[0] = 1.0 / 6.0; c[1] = 1.0 / 6.0; c[2] = 4.0 / 6.0; c[3] = 0.0;
    return 3;
}

void orc_rk_scalar(int scheme, double zr, double zi, double* outr, double* outi)
{
    double b[4][4], c[4];
    int s = rk_tableau(scheme, b, c);
    double kr[4], ki[4];
    for (int i = 0; i < s; ++i) {
        double ur = 1.0, ui = 0.0;
        for (int j = 0; j < i; ++j) { ur += b[i][j] * kr[j]; ui += b[i][j] * ki[j]; }
        kr[i] = zr * ur - zi * ui;
        ki[i] = zr * ui + zi * ur;
    }
    double ur = 1.0, ui = 0.0;
    for (int i = 0; i < s; ++i) { ur += c[i] * kr[i]; ui += c[i] * ki[i]; }
    *outr = ur; *outi = ui;
}

void orc_rk_run(int system, int scheme, double* U, int nx, int ny, int nz,
                const double h[3], double dt, int nsteps, const orc_params* p)
{
    int nf = orc_nfields(system);
    long vol = (long)(nx + 2 * ORC_G) * (ny + 2 * ORC_G) * (nz + 2 * ORC_G);
    long n = vol * nf;
    double b[4][4], c[4];
    int s = rk_tableau(scheme, b, c);
    double* k[4];
    for (int i = 0; i < s; ++i) k[i] = (double*)calloc(n, sizeof(double));
    double* Us = (double*)calloc(n, sizeof(double));
    double* R = (double*)calloc(n, sizeof(double));
    for (int step = 0; step < nsteps; ++step) {
        for (int i = 0; i < s; ++i) {
            for (long q = 0; q < n; ++q) {
                double v = U[q];
                for (int j = 0; j < i; ++j) v += b[i][j] * k[j][q];
                Us[q] = v;
            }
            orc_fill_periodic(Us, nf, nx, ny, nz);
            orc_rhs(system, Us, R, nx, ny, nz, h, p);
            for (long q = 0; q < n; ++q) k[i][q] = dt * R[q];
        }
        for (long q = 0; q < n; ++q) {
            double acc = 0.0;
            for (int i = 0; i < s; ++i) acc += c[i] * k[i][q];
            U[q] += acc;
        }
        orc_fill_periodic(U, nf, nx, ny, nz);
    }
    for (int i = 0; i < s; ++i) free(k[i]);
    free(Us);
    free(R);
}
