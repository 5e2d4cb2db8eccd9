/*
 * Memory and undefined-behaviour check of the CPU oracle (TEST INFRASTRUCTURE
 * ONLY).  Built by the test-suite with gcc's AddressSanitizer and
 * UndefinedBehaviorSanitizer (no recovery) together with the oracle's sources,
 * it calls every entry point of the oracle on small ragged inputs: the
 * right-hand sides and monitors of every system, the periodic Runge-Kutta runs,
 * the sub-cycled hierarchy step (RK4 and SSP-RK3, every time-refinement mode,
 * periodic and radiative), regrid, the prolongation and restriction pieces,
 * the wave adjoint, dense output and BOR, the one-dimensional stencils and
 * reconstructions, and the sphere integral.  It exits 0 when every call ran
 * clean and every result is finite; the sanitizers abort on the first fault.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* compiled from orc_ccz4_jvp.cpp (dual-number right-hand side) */
void orc_ccz4_rhs_jvp(const double* U, const double* V, double* R, double* RV, int nx, int ny, int nz,
                      const double h[3], const orc_params* p);

static int failures = 0;

static void check_finite(const char* what, const double* a, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            fprintf(stderr, "%s: non-finite value at %ld\n", what, i);
            ++failures;
            return;
        }
}

static orc_params defaults(void)
{
    orc_params p;
    p.sigma = 0.1; p.gamma_ad = 5.0 / 3.0; p.weno_eps = -1.0; p.weno_q = 2.0;
    p.kappa_z = 0.1; p.kappa_c = 0.1; p.bm_f0 = 0.0; p.bm_f1 = 2.0;
    p.gd_g = 0.75; p.gd_eta = 2.0; p.upwind = 1.0;
    p.mhd_recon = 0.0; p.mhd_riemann = 0.0; p.mhd_ch = 1.0; p.mhd_kpsi = 0.0;
    return p;
}

static long vol(const int n[3])
{
    return (long)(n[0] + 2 * ORC_G) * (n[1] + 2 * ORC_G) * (n[2] + 2 * ORC_G);
}

/* smooth, physical values of every field at every point of a ghosted patch
 * whose first interior point sits at x0 with spacing h */
static void fill(int system, double* U, const int n[3], const double x0[3], double h)
{
    const int nf = orc_nfields(system);
    const int sx = n[0] + 2 * ORC_G, sy = n[1] + 2 * ORC_G, sz = n[2] + 2 * ORC_G;
    static const double flat[25] = {1, 1, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0};
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < sz; ++k)
            for (int j = 0; j < sy; ++j)
                for (int i = 0; i < sx; ++i) {
                    const double x = x0[0] + (i - ORC_G) * h, y = x0[1] + (j - ORC_G) * h, z = x0[2] + (k - ORC_G) * h;
                    const double s = sin(3.14159 * x + 0.3 * f) * cos(3.14159 * y) + 0.5 * sin(3.14159 * z + 0.1 * f);
                    double v;
                    if (system == ORC_CCZ4)
                        v = flat[f] + 0.01 * s;
                    else if (system == ORC_WAVE)
                        v = s;
                    else {
                        static const double base[9] = {1.0, 0.0, 0.0, 0.0, 3.0, 0.2, 0.1, -0.1, 0.0};
                        v = base[f] + (f == 8 ? 0.01 : 0.1) * s;
                    }
                    U[(((long)f * sz + k) * sy + j) * sx + i] = v;
                }
}

static void patch_checks(int system)
{
    const int n[3] = {7, 5, 6};
    const double h3[3] = {0.1, 0.1, 0.1}, x0[3] = {-0.3, 0.2, 0.1};
    const int nf = orc_nfields(system);
    const long V = vol(n), N = nf * V;
    double* U = calloc(N, sizeof(double));
    double* R = calloc(N, sizeof(double));
    double* M = calloc(5 * V, sizeof(double));
    orc_params p = defaults();
    fill(system, U, n, x0, 0.1);
    orc_fill_periodic(U, nf, n[0], n[1], n[2]);
    orc_rhs(system, U, R, n[0], n[1], n[2], h3, &p);
    check_finite("rhs", R, N);
    orc_ko_monitor(system, U, M, n[0], n[1], n[2], h3, &p);
    check_finite("ko monitor", M, V);
    if (system == ORC_CCZ4) {
        double* Vt = calloc(N, sizeof(double));
        double* RV = calloc(N, sizeof(double));
        fill(system, Vt, n, x0, 0.37);
        orc_ccz4_monitor(U, M, n[0], n[1], n[2], h3, &p);
        check_finite("ccz4 monitor", M, 5 * V);
        orc_ccz4_rhs_jvp(U, Vt, R, RV, n[0], n[1], n[2], h3, &p);
        check_finite("ccz4 jvp", RV, N);
        free(Vt);
        free(RV);
    }
    if (system == ORC_MHD || system == ORC_MHD_GLM)
        for (int rec = 0; rec < 3; ++rec)
            for (int rie = 0; rie < 3; ++rie) {
                p.mhd_recon = rec;
                p.mhd_riemann = rie;
                orc_rhs(system, U, R, n[0], n[1], n[2], h3, &p);
                check_finite("mhd rhs variant", R, N);
            }
    p = defaults();
    for (int scheme = ORC_RK4; scheme <= ORC_SSPRK3; ++scheme) {
        double* W = malloc(N * sizeof(double));
        memcpy(W, U, N * sizeof(double));
        orc_rk_run(system, scheme, W, n[0], n[1], n[2], h3, 0.01, 2, &p);
        check_finite("rk run", W, N);
        free(W);
    }
    free(U);
    free(R);
    free(M);
}

/* three levels (ratios 2 then 3) of ragged patches on a periodic 12^3 level 0 */
static const int RATIO[3] = {1, 2, 3};
static const int NPATCH[3] = {3, 3, 2};
static const int BOXES[] = {
    0, 0, 0, 4, 6, 11,    5, 0, 0, 11, 6, 11,    0, 7, 0, 11, 11, 11,
    3, 3, 3, 11, 20, 20,  12, 3, 3, 20, 12, 20,  12, 13, 3, 20, 20, 20,
    27, 27, 27, 35, 44, 44,  36, 27, 27, 44, 44, 44,
};
static const int BOXES2[] = {  /* the same levels regridded: other level-1 and level-2 boxes */
    0, 0, 0, 4, 6, 11,    5, 0, 0, 11, 6, 11,    0, 7, 0, 11, 11, 11,
    3, 4, 3, 12, 20, 19,  13, 4, 3, 20, 14, 19,  13, 15, 3, 20, 20, 19,
    27, 30, 27, 35, 44, 41,  36, 30, 27, 44, 44, 41,
};

static orc_hier* make_hier(int system, const int* boxes, double dx0)
{
    const int N0[3] = {12, 12, 12};
    const double xlo[3] = {-1.0, -1.0, -1.0};
    orc_hier* H = orc_hier_create(system, 3, RATIO, N0, xlo, dx0, NPATCH, boxes);
    const int nf = orc_nfields(system);
    double h = dx0;
    int q = 0;
    for (int l = 0; l < 3; ++l) {
        if (l) h /= RATIO[l];
        for (int p = 0; p < NPATCH[l]; ++p, ++q) {
            const int* b = boxes + 6 * q;
            const int n[3] = {b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
            const double x0[3] = {xlo[0] + b[0] * h, xlo[1] + b[1] * h, xlo[2] + b[2] * h};
            double* U = malloc(nf * vol(n) * sizeof(double));
            fill(system, U, n, x0, h);
            orc_hier_set(H, l, p, U);
            free(U);
        }
        orc_hier_fill_same(H, l);
    }
    return H;
}

static void hier_check_finite(const orc_hier* H, int system, const int* boxes, const char* what)
{
    const int nf = orc_nfields(system);
    int q = 0;
    for (int l = 0; l < 3; ++l)
        for (int p = 0; p < NPATCH[l]; ++p, ++q) {
            const int* b = boxes + 6 * q;
            const int n[3] = {b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
            double* U = malloc(nf * vol(n) * sizeof(double));
            orc_hier_get(H, l, p, U);
            /* interior points only: ghosts at coarse-fine faces are stale by design */
            const int sx = n[0] + 6, sy = n[1] + 6, sz = n[2] + 6;
            for (int f = 0; f < nf; ++f)
                for (int k = 3; k < sz - 3; ++k)
                    for (int j = 3; j < sy - 3; ++j)
                        check_finite(what, U + (((long)f * sz + k) * sy + j) * sx + 3, n[0]);
            free(U);
        }
}

static void hierarchy_checks(int system)
{
    const double dx0 = 2.0 / 12.0;
    orc_params p = defaults();
    /* every time-refinement mode on the wave; BOR alone on the others (the
     * modes differ only in the system-independent state formulas) */
    const int last_mode = system == ORC_WAVE ? ORC_TIME_NOSUB : ORC_TIME_BOR;
    for (int scheme = ORC_RK4; scheme <= ORC_SSPRK3; ++scheme)
        for (int mode = ORC_TIME_BOR; mode <= last_mode; ++mode) {
            orc_hier* H = make_hier(system, BOXES, dx0);
            orc_hier_set_scheme(H, scheme);
            orc_hier_set_time_mode(H, mode);
            orc_hier_step(H, 0.1 * dx0, &p);
            hier_check_finite(H, system, BOXES, "hierarchy step");
            if (scheme == ORC_RK4 && mode == ORC_TIME_BOR) {
                orc_hier* Hn = make_hier(system, BOXES2, dx0);
                orc_hier_regrid(Hn, H);
                hier_check_finite(Hn, system, BOXES2, "regrid");
                orc_hier_destroy(Hn);
            }
            orc_hier_destroy(H);
        }
    /* prolongation and restriction pieces: level 1, patch 0 gets its
     * parent-region data from arrays the size of the level-0 patches */
    orc_hier* H = make_hier(system, BOXES, dx0);
    const int nf = orc_nfields(system);
    for (int p0 = 0; p0 < NPATCH[0]; ++p0) {
        const int* b = BOXES + 6 * p0;
        const int n[3] = {b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
        const long N = nf * vol(n);
        double* a[5];
        for (int s = 0; s < 5; ++s) {
            a[s] = malloc(N * sizeof(double));
            orc_hier_get(H, 0, p0, a[s]);
        }
        orc_hier_set_parent_data(H, 0, p0, a[0], a[1], a[2], a[3], a[4]);
        for (int s = 0; s < 5; ++s) free(a[s]);
    }
    for (int r = 0; r < 2; ++r)
        for (int s = 1; s <= 4; ++s) orc_hier_prolong(H, 1, r, s, 0.1 * dx0);
    orc_hier_restrict(H, 1);
    hier_check_finite(H, system, BOXES, "prolong/restrict");
    orc_hier_destroy(H);
}

static void open_checks(void)
{
    /* wave and CCZ4 on a radiative single patch with one refined level */
    const int sys[2] = {ORC_WAVE, ORC_CCZ4};
    for (int t = 0; t < 2; ++t) {
        const int system = sys[t], nf = orc_nfields(system);
        const int ratio[2] = {1, 2}, npatch[2] = {1, 1}, N0[3] = {16, 15, 14};
        const int boxes[12] = {0, 0, 0, 15, 14, 13, 12, 12, 12, 19, 17, 15};
        const double xlo[3] = {-1.0, -0.9, -0.8}, dx0 = 0.2;
        orc_hier* H = orc_hier_create(system, 2, ratio, N0, xlo, dx0, npatch, boxes);
        double h = dx0;
        for (int l = 0; l < 2; ++l) {
            if (l) h /= 2;
            const int* b = boxes + 6 * l;
            const int n[3] = {b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
            const double x0[3] = {xlo[0] + b[0] * h, xlo[1] + b[1] * h, xlo[2] + b[2] * h};
            double* U = malloc(nf * vol(n) * sizeof(double));
            fill(system, U, n, x0, h);
            orc_hier_set(H, l, 0, U);
            free(U);
        }
        double v[25], uinf[25];
        static const double flat[25] = {1, 1, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0};
        for (int f = 0; f < nf; ++f) {
            v[f] = 1.0;
            uinf[f] = system == ORC_CCZ4 ? flat[f] : 0.0;
        }
        orc_hier_set_open(H, v, uinf);
        orc_params p = defaults();
        orc_hier_step(H, 0.05, &p);
        orc_hier_step(H, 0.05, &p);
        orc_hier_destroy(H);
    }
}

static void adjoint_checks(void)
{
    const int n[3] = {8, 6, 5};
    const double h3[3] = {0.125, 0.125, 0.125}, x0[3] = {-0.5, -0.4, -0.3};
    const long V = vol(n);
    orc_params p = defaults();
    double* lam = calloc(2 * V, sizeof(double));
    double* out = calloc(2 * V, sizeof(double));
    fill(ORC_WAVE, lam, n, x0, 0.125);
    orc_wave_rhs_adjoint(lam, out, n[0], n[1], n[2], h3, &p);
    orc_fill_periodic_adjoint(out, 2, n[0], n[1], n[2]);
    check_finite("wave rhs adjoint", out, 2 * V);
    orc_wave_adjoint_run(out, n[0], n[1], n[2], h3, x0, 0.02, 3, 0.3, &p);
    check_finite("wave adjoint run", out, 2 * V);
    fill(ORC_WAVE, lam, n, x0, 0.125);
    const double s = orc_sphere_integral(lam, 0, n[0], n[1], n[2], x0, h3, 0.35, 0.0);
    check_finite("sphere integral", &s, 1);
    free(lam);
    free(out);
}

static void scalar_checks(void)
{
    double u[16];
    for (int i = 0; i < 16; ++i) u[i] = sin(0.7 * i) + 2.0;
    double acc = 0.0;
    acc += orc_d1(u + 8, 1, 0.1) + orc_d2(u + 8, 1, 0.1) + orc_adv(u + 8, 1, 0.1, 0.4) +
           orc_adv(u + 8, 1, 0.1, -0.4) + orc_ko(u + 8, 1, 0.1, 0.2) + orc_dmix(u + 8, 1, 0.1, 1, 0.2);
    acc += orc_weno5z_left(u + 8, 1e-6, 2.0) + orc_weno5z_right(u + 8, 1e-6, 2.0) +
           orc_weno5js_left(u + 8, 1e-6) + orc_weno5js_right(u + 8, 1e-6) +
           orc_weno3_left(u + 8, 1e-6) + orc_weno3_right(u + 8, 1e-6);
    const double UL[8] = {1.0, 0.1, 0.0, 0.0, 3.0, 0.2, 0.1, 0.0};
    const double UR[8] = {0.5, -0.1, 0.0, 0.1, 1.5, 0.2, -0.1, 0.05};
    double F[8];
    for (int d = 0; d < 3; ++d)
        for (int rie = 0; rie < 2; ++rie) {
            orc_mhd_interface_flux(UL, UR, d, 5.0 / 3.0, rie, F);
            check_finite("interface flux", F, 8);
        }
    acc += orc_mhd_fast_speed(UL, 0, 5.0 / 3.0);
    double w[6];
    orc_lagrange6(0.5, w);
    acc += w[0] + w[5];
    double zr, zi;
    orc_rk_scalar(ORC_RK4, -1.0, 0.5, &zr, &zi);
    acc += zr + zi;
    orc_rk_scalar(ORC_SSPRK3, -1.0, 0.5, &zr, &zi);
    acc += zr + zi;
    for (int j = 0; j < 4; ++j)
        for (int m = 0; m < 4; ++m) acc += orc_dense_rk4(j, m, 0.3);
    for (int j = 0; j < 3; ++j)
        for (int m = 0; m < 3; ++m) acc += orc_dense_ssp3(j, m, 0.3);
    enum { NP = 13 };
    double Un[NP], k1[NP], k2[NP], k3[NP], k4[NP], out[NP];
    for (int i = 0; i < NP; ++i) {
        Un[i] = i; k1[i] = 0.1 * i; k2[i] = -0.2 * i; k3[i] = 0.3; k4[i] = 1.0 / (i + 1);
    }
    const double* k[4] = {k1, k2, k3, k4};
    for (int R = 1; R <= 4; ++R)
        for (int r = 0; r < R; ++r) {
            for (int s = 1; s <= 4; ++s) {
                orc_bor_rk4(R, r, s, 0.1, Un, k, out, NP);
                check_finite("bor rk4", out, NP);
                for (int mode = ORC_TIME_BOR; mode <= ORC_TIME_NOSUB; ++mode) {
                    orc_time_state(mode, R, r, s, 0.1, Un, k, out, NP);
                    check_finite("time state", out, NP);
                }
            }
            for (int s = 1; s <= 3; ++s) {
                orc_bor_ssp3(R, r, s, 0.1, Un, k, out, NP);
                check_finite("bor ssp3", out, NP);
                for (int mode = ORC_TIME_BOR; mode <= ORC_TIME_NOSUB; ++mode) {
                    orc_time_state_ssp3(mode, R, r, s, 0.1, Un, k, out, NP);
                    check_finite("time state ssp3", out, NP);
                }
            }
        }
    check_finite("scalar results", &acc, 1);
}

int main(void)
{
    scalar_checks();
    const int systems[4] = {ORC_WAVE, ORC_MHD, ORC_MHD_GLM, ORC_CCZ4};
    for (int s = 0; s < 4; ++s) {
        patch_checks(systems[s]);
        hierarchy_checks(systems[s]);
        printf("system %d clean\n", systems[s]);
        fflush(stdout);
    }
    open_checks();
    adjoint_checks();
    printf("%s (%d failures)\n", failures ? "FAILED" : "clean", failures);
    return failures ? 1 : 0;
}
