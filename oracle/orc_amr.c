/*
 * Oracle: dense output (App. C), Berger-Oliger without order reduction
 * (App. D, RK4), Lagrange prolongation (Sec. III.A), injection restriction
 * and the sub-cycled time step of the AMR skeleton (Sec. III).
 * TEST INFRASTRUCTURE ONLY.
 *
 * Readings:
 *  - grids are vertex centred: fine point R*i coincides with coarse point i
 *    for any integer ratio R, so injection is a copy for R = 2 and R = 3;
 *  - the RK4 dense-output coefficient b_4 is taken as -theta^2/2 + 2 theta^3/3,
 *    the sign that makes b(1) equal the RK4 weights (1,2,2,1)/6 (the printed
 *    minus sign would give b_4(1) = -7/6);
 *  - a fine ghost point at fine index g (per axis) sits at coarse position
 *    g/R = i0 + m/R; for m = 0 it copies the coarse point, otherwise it uses
 *    the 6-point Lagrange polynomial through coarse nodes i0-2 .. i0+3
 *    (three on each side), as a tensor product over the three axes;
 *  - same-level sources (including periodic images: the domain is periodic
 *    on every level) take precedence over prolongation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* App. C, RK(4,4) dense output b_j(theta), j = 0..3 (b_1..b_4), and its
 * derivatives d^m/dtheta^m. */
double orc_dense_rk4(int j, int m, double t)
{
    /* coefficients of theta, theta^2, theta^3 */
    static const double cf[4][3] = {
        {1.0, -1.5, 2.0 / 3.0},
        {0.0, 1.0, -2.0 / 3.0},
        {0.0, 1.0, -2.0 / 3.0},
        {0.0, -0.5, 2.0 / 3.0},
    };
    const double* a = cf[j];
    switch (m) {
    case 0: return a[0] * t + a[1] * t * t + a[2] * t * t * t;
    case 1: return a[0] + 2.0 * a[1] * t + 3.0 * a[2] * t * t;
    case 2: return 2.0 * a[1] + 6.0 * a[2] * t;
    case 3: return 6.0 * a[2];
    }
    return 0.0;
}

/* App. D, standard RK4 with ratio R, fine step r, fine stage s:
 *  1. U_{n+r/R} from the dense output at theta = r/R;
 *  2. U', U'', U''' from the theta-derivatives of the dense output and
 *     f_U U'' = 4 (k_3 - k_2) / dt^3;
 *  3. the fine k_1 .. k_3 with dt_F = dt / R;
 *  4. the fine stage states U, U + k1/2, U + k2/2, U + k3. */
void orc_bor_rk4(int R, int r, int s, double dt, const double* Un,
                 const double* const* k, double* out, long n)
{
    double th = (double)r / (double)R;
    double dtF = dt / R;
    double b[4][4]; /* b[m][j] = d^m b_j / dtheta^m at theta */
    for (int m = 0; m < 4; ++m)
        for (int j = 0; j < 4; ++j) b[m][j] = orc_dense_rk4(j, m, th);
    for (long i = 0; i < n; ++i) {
        double U = Un[i], U1 = 0.0, U2 = 0.0, U3 = 0.0;
        for (int j = 0; j < 4; ++j) {
            U += b[0][j] * k[j][i];
            U1 += b[1][j] * k[j][i];
            U2 += b[2][j] * k[j][i];
            U3 += b[3][j] * k[j][i];
        }
        U1 /= dt;
        U2 /= dt * dt;
        U3 /= dt * dt * dt;
        double fUU2 = 4.0 * (k[2][i] - k[1][i]) / (dt * dt * dt);
        double k1 = dtF * U1;
        double k2 = dtF * U1 + 0.5 * dtF * dtF * U2 + 0.125 * dtF * dtF * dtF * (U3 - fUU2);
        double k3 = dtF * U1 + 0.5 * dtF * dtF * U2 + 0.125 * dtF * dtF * dtF * (U3 + fUU2);
        switch (s) {
        case 1: out[i] = U; break;
        case 2: out[i] = U + 0.5 * k1; break;
        case 3: out[i] = U + 0.5 * k2; break;
        default: out[i] = U + k3; break;
        }
    }
}

/* App. C, SSP-RK(3,3) dense output b_j(theta), j = 0..2, and its derivatives. */
double orc_dense_ssp3(int j, int m, double t)
{
    /* coefficients of theta, theta^2 */
    static const double cf[3][2] = {{1.0, -5.0 / 6.0}, {0.0, 1.0 / 6.0}, {0.0, 4.0 / 6.0}};
    const double* a = cf[j];
    switch (m) {
    case 0: return a[0] * t + a[1] * t * t;
    case 1: return a[0] + 2.0 * a[1] * t;
    case 2: return 2.0 * a[1];
    }
    return 0.0;
}

/* App. D, SSP-RK3 with ratio R, fine step r, fine stage s:
 *  1. U_{n+r/R} from the dense output at theta = r/R;
 *  2. U', U'' from its theta-derivatives;
 *  3. the fine k_1 = dt_F U', k_2 = dt_F U' + dt_F^2 U'',
 *     k_3 = dt_F U' + dt_F^2 U''/2, dt_F = dt / R;
 *  4. the fine stage states U, U + k_1, U + (k_1 + k_2)/4 (the stage states
 *     of the SSP-RK3 tableau). */
void orc_bor_ssp3(int R, int r, int s, double dt, const double* Un,
                  const double* const* k, double* out, long n)
{
    double th = (double)r / (double)R;
    double dtF = dt / R;
    double b[3][3];
    for (int m = 0; m < 3; ++m)
        for (int j = 0; j < 3; ++j) b[m][j] = orc_dense_ssp3(j, m, th);
    for (long i = 0; i < n; ++i) {
        double U = Un[i], U1 = 0.0, U2 = 0.0;
        for (int j = 0; j < 3; ++j) {
            U += b[0][j] * k[j][i];
            U1 += b[1][j] * k[j][i];
            U2 += b[2][j] * k[j][i];
        }
        U1 /= dt;
        U2 /= dt * dt;
        double k1 = dtF * U1;
        double k2 = dtF * U1 + dtF * dtF * U2;
        switch (s) {
        case 1: out[i] = U; break;
        case 2: out[i] = U + k1; break;
        default: out[i] = U + 0.25 * k1 + 0.25 * k2; break;
        }
    }
}

/* Sec. III.B for SSP-RK3 (stage times c = (0, 1, 1/2), weights (1, 1, 4)/6):
 * BOR (orc_bor_ssp3), BO (its dense output at the stage time), BO1 (linear
 * between U^n and U^{n+1}) and no sub-cycling (the parent's stage states
 * U^n, U^n + k_1, U^n + (k_1 + k_2)/4). */
void orc_time_state_ssp3(int mode, int R, int r, int s, double dt, const double* Un,
                         const double* const* k, double* out, long n)
{
    static const double cs[3] = {0.0, 1.0, 0.5};
    static const double cw[3] = {1.0 / 6.0, 1.0 / 6.0, 4.0 / 6.0};
    if (mode == ORC_TIME_BOR) {
        orc_bor_ssp3(R, r, s, dt, Un, k, out, n);
        return;
    }
    const double th = (r + cs[s - 1]) / (double)R;
    for (long i = 0; i < n; ++i) {
        double u = Un[i];
        switch (mode) {
        case ORC_TIME_BO:
            for (int j = 0; j < 3; ++j) u += orc_dense_ssp3(j, 0, th) * k[j][i];
            break;
        case ORC_TIME_BO1: {
            double inc = 0.0;
            for (int j = 0; j < 3; ++j) inc += cw[j] * k[j][i];
            u += th * inc;
            break;
        }
        default: /* ORC_TIME_NOSUB */
            if (s == 2) u += k[0][i];
            if (s == 3) u += 0.25 * k[0][i] + 0.25 * k[1][i];
            break;
        }
        out[i] = u;
    }
}

/* Sec. III.B: the parent's state that feeds the ghost points of fine step r,
 * stage s, for each time-refinement strategy (the parent stepped from U^n
 * with increments k_1..k_4 over dt; the fine stage s of step r sits at
 * theta = (r + c_s)/R, c = (0, 1/2, 1/2, 1)):
 *  - BOR: App. D (orc_bor_rk4);
 *  - BO, dense output: U^n + sum_j b_j(theta) k_j (App. C), the parent's
 *    solution at the stage time;
 *  - BO1: linear in time between U^n and U^{n+1} = U^n + sum_j c_j k_j,
 *    c = (1, 2, 2, 1)/6;
 *  - no sub-cycling (the fine level takes the parent's dt, R = 1 in time):
 *    the parent's own stage states U^n, U^n + k_1/2, U^n + k_2/2, U^n + k_3. */
void orc_time_state(int mode, int R, int r, int s, double dt, const double* Un,
                    const double* const* k, double* out, long n)
{
    static const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    static const double cw[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    if (mode == ORC_TIME_BOR) {
        orc_bor_rk4(R, r, s, dt, Un, k, out, n);
        return;
    }
    const double th = (r + cs[s - 1]) / (double)R;
    for (long i = 0; i < n; ++i) {
        double u = Un[i];
        switch (mode) {
        case ORC_TIME_BO:
            for (int j = 0; j < 4; ++j) u += orc_dense_rk4(j, 0, th) * k[j][i];
            break;
        case ORC_TIME_BO1: {
            double inc = 0.0;
            for (int j = 0; j < 4; ++j) inc += cw[j] * k[j][i];
            u += th * inc;
            break;
        }
        default: /* ORC_TIME_NOSUB */
            if (s > 1) u += (s == 4 ? 1.0 : 0.5) * k[s - 2][i];
            break;
        }
        out[i] = u;
    }
}

/* Sec. III.A: l_j(x) = prod_{m != j} (x - x_m)/(x_j - x_m), nodes x_m = -2..3. */
void orc_lagrange6(double xi, double w[6])
{
    for (int j = 0; j < 6; ++j) {
        double xj = j - 2.0, v = 1.0;
        for (int m = 0; m < 6; ++m) {
            if (m == j) continue;
            double xm = m - 2.0;
            v *= (xi - xm) / (xj - xm);
        }
        w[j] = v;
    }
}

/* ------------------------------------------------------------------------ */

#define MAXLEV 8

typedef struct {
    int ratio;
    int np;
    int* box;       /* lo[3], hi[3] per patch */
    double** U;     /* current state */
    double** Un;    /* state at the start of the level's step */
    double** Us;    /* stage state */
    double** k[4];  /* stage increments of the level's current step */
    double** R;     /* rhs scratch */
    int step_r;     /* index of the level's step inside its parent's step */
    int hint;       /* patch that answered the last owner query (search starts there) */
    int per[3];     /* period in level index space: N0 * R_1 * .. * R_l per axis */
} olevel;

struct orc_hier {
    int system, nf, nlev;
    int tmode;  /* time refinement (ORC_TIME_*) */
    int scheme; /* ORC_RK4 or ORC_SSPRK3 */
    int open;   /* radiative outer boundary instead of periodic level 0 */
    double rad_v[32], rad_uinf[32];
    int N0[3];
    double xlo[3], dx0;
    olevel L[MAXLEV];
};

static void radiative_rhs(orc_hier* H, const double* U, double* R, double h);

static int wrapi(int a, int n)
{
    int m = a % n;
    return m < 0 ? m + n : m;
}

static long pvol(const int* b)
{
    return (long)(b[3] - b[0] + 1 + 2 * ORC_G) * (b[4] - b[1] + 1 + 2 * ORC_G)
           * (b[5] - b[2] + 1 + 2 * ORC_G);
}

static double** alloc_set(const olevel* L, int nf)
{
    double** a = (double**)calloc(L->np, sizeof(double*));
    for (int p = 0; p < L->np; ++p) a[p] = (double*)calloc(pvol(L->box + 6 * p) * nf, sizeof(double));
    return a;
}

orc_hier* orc_hier_create(int system, int nlev, const int* ratio, const int N0[3],
                          const double xlo[3], double dx0, const int* npatch,
                          const int* boxes)
{
    orc_hier* H = (orc_hier*)calloc(1, sizeof(orc_hier));
    H->system = system;
    H->nf = orc_nfields(system);
    H->nlev = nlev;
    for (int d = 0; d < 3; ++d) { H->N0[d] = N0[d]; H->xlo[d] = xlo[d]; }
    H->dx0 = dx0;
    const int* b = boxes;
    for (int l = 0; l < nlev; ++l) {
        olevel* L = &H->L[l];
        L->ratio = l == 0 ? 1 : ratio[l];
        L->np = npatch[l];
        for (int d = 0; d < 3; ++d) L->per[d] = (l == 0 ? N0[d] : H->L[l - 1].per[d] * L->ratio);
        L->box = (int*)malloc(sizeof(int) * 6 * L->np);
        memcpy(L->box, b, sizeof(int) * 6 * L->np);
        b += 6 * L->np;
        L->U = alloc_set(L, H->nf);
        L->Un = alloc_set(L, H->nf);
        L->Us = alloc_set(L, H->nf);
        L->R = alloc_set(L, H->nf);
        for (int j = 0; j < 4; ++j) L->k[j] = alloc_set(L, H->nf);
    }
    return H;
}

static void free_set(double** a, int np)
{
    for (int p = 0; p < np; ++p) free(a[p]);
    free(a);
}

void orc_hier_destroy(orc_hier* H)
{
    for (int l = 0; l < H->nlev; ++l) {
        olevel* L = &H->L[l];
        free_set(L->U, L->np);
        free_set(L->Un, L->np);
        free_set(L->Us, L->np);
        free_set(L->R, L->np);
        for (int j = 0; j < 4; ++j) free_set(L->k[j], L->np);
        free(L->box);
    }
    free(H);
}

int orc_hier_npatch(const orc_hier* H, int l) { return H->L[l].np; }

void orc_hier_set(orc_hier* H, int l, int p, const double* src)
{
    memcpy(H->L[l].U[p], src, sizeof(double) * pvol(H->L[l].box + 6 * p) * H->nf);
}

void orc_hier_get(const orc_hier* H, int l, int p, double* dst)
{
    memcpy(dst, H->L[l].U[p], sizeof(double) * pvol(H->L[l].box + 6 * p) * H->nf);
}

void orc_hier_set_parent_data(orc_hier* H, int l, int p, const double* Un,
                              const double* k1, const double* k2,
                              const double* k3, const double* k4)
{
    olevel* L = &H->L[l];
    long n = pvol(L->box + 6 * p) * H->nf;
    memcpy(L->Un[p], Un, sizeof(double) * n);
    memcpy(L->k[0][p], k1, sizeof(double) * n);
    memcpy(L->k[1][p], k2, sizeof(double) * n);
    memcpy(L->k[2][p], k3, sizeof(double) * n);
    memcpy(L->k[3][p], k4, sizeof(double) * n);
}

/* patch of level l whose interior holds global index g, taken modulo the
 * level's period (the domain is periodic with N0 * R_1 * .. * R_l points per
 * axis on level l); writes the local (ghosted) index into *loc. */
static int owner(const orc_hier* H, int l, const int g0[3], long* loc)
{
    const olevel* L = &H->L[l];
    int g[3] = {g0[0], g0[1], g0[2]};
    if (!H->open)
        for (int d = 0; d < 3; ++d)
            if (g[d] < 0 || g[d] >= L->per[d]) g[d] = wrapi(g[d], L->per[d]);
    /* patches are disjoint, so at most one holds g: start the search at the
     * patch that answered the previous query (consecutive queries are
     * usually neighbours) and go round the list once */
    int* hint = (int*)&L->hint;
    for (int t = 0; t < L->np; ++t) {
        int p = (*hint + t) % L->np;
        const int* b = L->box + 6 * p;
        if (g[0] < b[0] || g[0] > b[3] || g[1] < b[1] || g[1] > b[4] || g[2] < b[2] || g[2] > b[5])
            continue;
        long NX = b[3] - b[0] + 1 + 2 * ORC_G, NY = b[4] - b[1] + 1 + 2 * ORC_G;
        *loc = ((long)(g[2] - b[2] + ORC_G) * NY + (g[1] - b[1] + ORC_G)) * NX + (g[0] - b[0] + ORC_G);
        *hint = p;
        return p;
    }
    return -1;
}

/* Visit the ghost points of patch p on level l that the stencils can read:
 * the centred, lop-sided and KO stencils reach 3 points along one axis and
 * the cross derivatives 2 points along two axes, so faces are visited to
 * depth 3, edges to depth 2 and corners (outside along all three axes) never. */
typedef void (*ghost_fn)(orc_hier* H, int l, int p, long loc, const int g[3], void* ctx);

static void for_ghosts(orc_hier* H, int l, int p, ghost_fn fn, void* ctx)
{
    const int* b = H->L[l].box + 6 * p;
    int n[3] = {b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
    long NX = n[0] + 2 * ORC_G, NY = n[1] + 2 * ORC_G, NZ = n[2] + 2 * ORC_G;
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                int li[3] = {i - ORC_G, j - ORC_G, k - ORC_G};
                int nout = 0, deep = 0;
                for (int d = 0; d < 3; ++d) {
                    int depth = li[d] < 0 ? -li[d] : (li[d] >= n[d] ? li[d] - n[d] + 1 : 0);
                    if (depth > 0) ++nout;
                    if (depth > 2) deep = 1;
                }
                if (nout == 0 || nout == 3 || (nout == 2 && deep)) continue;
                int g[3] = {b[0] + li[0], b[1] + li[1], b[2] + li[2]};
                fn(H, l, p, ((long)k * NY + j) * NX + i, g, ctx);
            }
}

typedef struct { double** A; } set_ctx;

static void fill_one(orc_hier* H, int l, int p, long loc, const int g[3], void* ctx)
{
    double** A = ((set_ctx*)ctx)->A;
    long sloc;
    int q = owner(H, l, g, &sloc);
    if (q < 0) return;
    long vd = pvol(H->L[l].box + 6 * p), vs = pvol(H->L[l].box + 6 * q);
    for (int f = 0; f < H->nf; ++f) A[p][f * vd + loc] = A[q][f * vs + sloc];
}

static void fill_same_set(orc_hier* H, int l, double** A)
{
    set_ctx c = {A};
    for (int p = 0; p < H->L[l].np; ++p) for_ghosts(H, l, p, fill_one, &c);
}

void orc_hier_fill_same(orc_hier* H, int l) { fill_same_set(H, l, H->L[l].U); }

typedef struct {
    double** A;
    double** T;        /* parent's BOR stage state, one array per parent patch */
    unsigned char** D; /* which entries of T have been computed */
    int R, r, s;
    double dtp;
} pro_ctx;

/* value of the parent's BOR stage state at entry `off` of parent patch q
 * (App. D applied at that coarse point, computed once per call) */
static double parent_state(orc_hier* H, int lp, pro_ctx* c, int q, long off)
{
    const olevel* P = &H->L[lp];
    if (!c->D[q][off]) {
        const double* kk[4] = {P->k[0][q] + off, P->k[1][q] + off, P->k[2][q] + off,
                               P->k[3][q] + off};
        if (H->scheme == ORC_SSPRK3)
            orc_time_state_ssp3(H->tmode, c->R, c->r, c->s, c->dtp, P->Un[q] + off, kk, c->T[q] + off, 1);
        else
            orc_time_state(H->tmode, c->R, c->r, c->s, c->dtp, P->Un[q] + off, kk, c->T[q] + off, 1);
        c->D[q][off] = 1;
    }
    return c->T[q][off];
}

static void prolong_one(orc_hier* H, int l, int p, long loc, const int g[3], void* ctx)
{
    pro_ctx* c = (pro_ctx*)ctx;
    long dummy;
    if (owner(H, l, g, &dummy) >= 0) return; /* same-level source has precedence */
    int R = H->L[l].ratio;
    int i0[3], cnt[3];
    double w[3][6];
    for (int d = 0; d < 3; ++d) {
        int m = wrapi(g[d], R);
        i0[d] = (g[d] - m) / R;
        if (m == 0) {
            cnt[d] = 1;
            w[d][0] = 1.0;
        } else {
            cnt[d] = 6;
            orc_lagrange6((double)m / R, w[d]);
        }
    }
    long vd = pvol(H->L[l].box + 6 * p);
    double v[64];
    for (int f = 0; f < H->nf; ++f) v[f] = 0.0;
    /* every field sums the same stencil in the same (z, y, x) order */
    for (int a = 0; a < cnt[2]; ++a)
        for (int b2 = 0; b2 < cnt[1]; ++b2)
            for (int e = 0; e < cnt[0]; ++e) {
                int gc[3] = {i0[0] + (cnt[0] == 1 ? 0 : e - 2),
                             i0[1] + (cnt[1] == 1 ? 0 : b2 - 2),
                             i0[2] + (cnt[2] == 1 ? 0 : a - 2)};
                long ploc;
                int q = owner(H, l - 1, gc, &ploc);
                if (q < 0) {
                    fprintf(stderr, "oracle: prolongation stencil leaves the parent level\n");
                    abort();
                }
                long pv = pvol(H->L[l - 1].box + 6 * q);
                double wt = w[0][e] * w[1][b2] * w[2][a];
                for (int f = 0; f < H->nf; ++f)
                    v[f] += wt * parent_state(H, l - 1, c, q, f * pv + ploc);
            }
    for (int f = 0; f < H->nf; ++f) c->A[p][f * vd + loc] = v[f];
}

static void prolong_set(orc_hier* H, int l, double** A, int r, int s, double dtp)
{
    olevel* P = &H->L[l - 1];
    pro_ctx c;
    c.A = A;
    c.R = H->tmode == ORC_TIME_NOSUB ? 1 : H->L[l].ratio;
    c.r = r;
    c.s = s;
    c.dtp = dtp;
    c.T = (double**)calloc(P->np, sizeof(double*));
    c.D = (unsigned char**)calloc(P->np, sizeof(unsigned char*));
    for (int q = 0; q < P->np; ++q) {
        long n = pvol(P->box + 6 * q) * H->nf;
        c.T[q] = (double*)malloc(sizeof(double) * n);
        c.D[q] = (unsigned char*)calloc(n, 1);
    }
    for (int p = 0; p < H->L[l].np; ++p) for_ghosts(H, l, p, prolong_one, &c);
    for (int q = 0; q < P->np; ++q) {
        free(c.T[q]);
        free(c.D[q]);
    }
    free(c.T);
    free(c.D);
}

void orc_hier_prolong(orc_hier* H, int l, int r, int s, double dt_parent)
{
    prolong_set(H, l, H->L[l].U, r, s, dt_parent);
}

/* injection: every coarse interior point that coincides with a fine interior
 * point takes the fine value */
void orc_hier_restrict(orc_hier* H, int l)
{
    olevel* C = &H->L[l - 1];
    olevel* F = &H->L[l];
    int R = F->ratio;
    for (int q = 0; q < C->np; ++q) {
        const int* b = C->box + 6 * q;
        long NX = b[3] - b[0] + 1 + 2 * ORC_G, NY = b[4] - b[1] + 1 + 2 * ORC_G;
        long vc = pvol(b);
        for (int k = b[2]; k <= b[5]; ++k)
            for (int j = b[1]; j <= b[4]; ++j)
                for (int i = b[0]; i <= b[3]; ++i) {
                    int gf[3] = {R * i, R * j, R * k};
                    long floc;
                    int p = owner(H, l, gf, &floc);
                    if (p < 0) continue;
                    long cloc = ((long)(k - b[2] + ORC_G) * NY + (j - b[1] + ORC_G)) * NX + (i - b[0] + ORC_G);
                    long vf = pvol(F->box + 6 * p);
                    for (int f = 0; f < H->nf; ++f) C->U[q][f * vc + cloc] = F->U[p][f * vf + floc];
                }
    }
}

/* Sec. III.A: when a level grows, the points it gains are set by prolongation
 * from the next coarser level (here taken at the synchronised time, so the
 * parent state is its current U); points that the old level already held keep
 * their values. */
void orc_hier_regrid(orc_hier* Hn, const orc_hier* Ho)
{
    for (int p = 0; p < Hn->L[0].np; ++p)
        memcpy(Hn->L[0].U[p], Ho->L[0].U[p], sizeof(double) * pvol(Hn->L[0].box + 6 * p) * Hn->nf);
    for (int l = 1; l < Hn->nlev; ++l) {
        const olevel* F = &Hn->L[l];
        const olevel* P = &Hn->L[l - 1];
        const int R = F->ratio;
        for (int p = 0; p < F->np; ++p) {
            const int* b = F->box + 6 * p;
            long NX = b[3] - b[0] + 1 + 2 * ORC_G, NY = b[4] - b[1] + 1 + 2 * ORC_G;
            long vd = pvol(b);
            for (int k = b[2]; k <= b[5]; ++k)
                for (int j = b[1]; j <= b[4]; ++j)
                    for (int i = b[0]; i <= b[3]; ++i) {
                        int g[3] = {i, j, k};
                        long dloc = ((long)(k - b[2] + ORC_G) * NY + (j - b[1] + ORC_G)) * NX + (i - b[0] + ORC_G);
                        long sloc;
                        int q = owner(Ho, l, g, &sloc);
                        if (q >= 0) {
                            long vs = pvol(Ho->L[l].box + 6 * q);
                            for (int f = 0; f < Hn->nf; ++f) F->U[p][f * vd + dloc] = Ho->L[l].U[q][f * vs + sloc];
                            continue;
                        }
                        int i0[3], cnt[3];
                        double w[3][6];
                        for (int d = 0; d < 3; ++d) {
                            int m = wrapi(g[d], R);
                            i0[d] = (g[d] - m) / R;
                            if (m == 0) {
                                cnt[d] = 1;
                                w[d][0] = 1.0;
                            } else {
                                cnt[d] = 6;
                                orc_lagrange6((double)m / R, w[d]);
                            }
                        }
                        for (int f = 0; f < Hn->nf; ++f) {
                            double v = 0.0;
                            for (int a = 0; a < cnt[2]; ++a)
                                for (int b2 = 0; b2 < cnt[1]; ++b2)
                                    for (int e = 0; e < cnt[0]; ++e) {
                                        int gc[3] = {i0[0] + (cnt[0] == 1 ? 0 : e - 2),
                                                     i0[1] + (cnt[1] == 1 ? 0 : b2 - 2),
                                                     i0[2] + (cnt[2] == 1 ? 0 : a - 2)};
                                        long cloc;
                                        int qc = owner(Hn, l - 1, gc, &cloc);
                                        if (qc < 0) {
                                            fprintf(stderr, "oracle: regrid stencil leaves the parent level\n");
                                            abort();
                                        }
                                        v += w[0][e] * w[1][b2] * w[2][a]
                                             * P->U[qc][f * pvol(P->box + 6 * qc) + cloc];
                                    }
                            F->U[p][f * vd + dloc] = v;
                        }
                    }
        }
    }
}

/* Sec. III skeleton with sub-cycling: level l takes one step of size dt (RK4
 * or SSP-RK3, U^(s) = U^n + sum_j a_sj k_j); its children then take R steps of
 * dt/R using ghost values built from this step's U^n and k's; the children's
 * result is injected back. */
static void advance(orc_hier* H, int l, double dt, const orc_params* prm)
{
    olevel* L = &H->L[l];
    int nf = H->nf;
    static const double a4[4][3] = {{0, 0, 0}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 1.0}};
    static const double w4[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    static const double a3[4][3] = {{0, 0, 0}, {1.0, 0, 0}, {0.25, 0.25, 0}, {0, 0, 0}};
    static const double w3[4] = {1.0 / 6.0, 1.0 / 6.0, 4.0 / 6.0, 0.0};
    const int ns = H->scheme == ORC_SSPRK3 ? 3 : 4;
    const double (*a)[3] = H->scheme == ORC_SSPRK3 ? a3 : a4;
    const double* cw = H->scheme == ORC_SSPRK3 ? w3 : w4;
    double hh[3];
    double dxl = H->dx0;
    for (int m = 1; m <= l; ++m) dxl /= H->L[m].ratio;
    hh[0] = hh[1] = hh[2] = dxl;

    for (int p = 0; p < L->np; ++p)
        memcpy(L->Un[p], L->U[p], sizeof(double) * pvol(L->box + 6 * p) * nf);
    for (int s = 0; s < ns; ++s) {
        for (int p = 0; p < L->np; ++p) {
            long n = pvol(L->box + 6 * p) * nf;
            for (long i = 0; i < n; ++i) {
                double u = L->Un[p][i];
                for (int j = 0; j < s; ++j) u += a[s][j] * L->k[j][p][i];
                L->Us[p][i] = u;
            }
        }
        fill_same_set(H, l, L->Us);
        if (l > 0) {
            const int Rt = H->tmode == ORC_TIME_NOSUB ? 1 : L->ratio;
            prolong_set(H, l, L->Us, L->step_r, s + 1, dt * Rt);
        }
        for (int p = 0; p < L->np; ++p) {
            const int* b = L->box + 6 * p;
            long n = pvol(b) * nf;
            orc_rhs(H->system, L->Us[p], L->R[p], b[3] - b[0] + 1, b[4] - b[1] + 1,
                    b[5] - b[2] + 1, hh, prm);
            if (l == 0 && H->open) radiative_rhs(H, L->Us[p], L->R[p], dxl);
            for (long i = 0; i < n; ++i) L->k[s][p][i] = dt * L->R[p][i];
        }
    }
    for (int p = 0; p < L->np; ++p) {
        long n = pvol(L->box + 6 * p) * nf;
        for (long i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int s = 0; s < ns; ++s) acc += cw[s] * L->k[s][p][i];
            L->U[p][i] = L->Un[p][i] + acc;
        }
    }
    if (l + 1 < H->nlev) {
        /* sub-cycling: R fine steps of dt/R; without it, one of dt */
        int R = H->tmode == ORC_TIME_NOSUB ? 1 : H->L[l + 1].ratio;
        for (int r = 0; r < R; ++r) {
            H->L[l + 1].step_r = r;
            advance(H, l + 1, dt / R, prm);
        }
        orc_hier_restrict(H, l + 1);
    }
    fill_same_set(H, l, L->U);
}

void orc_hier_set_time_mode(orc_hier* H, int mode) { H->tmode = mode; }
void orc_hier_set_scheme(orc_hier* H, int scheme) { H->scheme = scheme; }

void orc_hier_set_open(orc_hier* H, const double* v, const double* uinf)
{
    H->open = 1;
    for (int f = 0; f < H->nf; ++f) {
        H->rad_v[f] = v[f];
        H->rad_uinf[f] = uinf[f];
    }
}

/* derivative along d at local ghosted index a of a line of extent n (with
 * stride st): centred where a-1 and a+1 exist, else one-sided inward */
static double rad_d1(const double* u, long st, int a, int n, double h)
{
    if (a == 0) return (-3.0 * u[0] + 4.0 * u[st] - u[2 * st]) / (2.0 * h);
    if (a == n - 1) return (3.0 * u[0] - 4.0 * u[-st] + u[-2 * st]) / (2.0 * h);
    return (u[st] - u[-st]) / (2.0 * h);
}

/* radiative right-hand side at every ghost point of the level-0 patch */
static void radiative_rhs(orc_hier* H, const double* U, double* R, double h)
{
    const int* b = H->L[0].box;
    int NX = b[3] - b[0] + 1 + 2 * ORC_G, NY = b[4] - b[1] + 1 + 2 * ORC_G, NZ = b[5] - b[2] + 1 + 2 * ORC_G;
    long vol = (long)NX * NY * NZ, st[3] = {1, NX, (long)NX * NY};
    int N[3] = {NX, NY, NZ};
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                if (i >= ORC_G && i < NX - ORC_G && j >= ORC_G && j < NY - ORC_G && k >= ORC_G && k < NZ - ORC_G)
                    continue;
                int a[3] = {i, j, k};
                double x[3], r2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    x[d] = H->xlo[d] + (b[d] + a[d] - ORC_G) * h;
                    r2 += x[d] * x[d];
                }
                double r = sqrt(r2);
                long c = ((long)k * NY + j) * NX + i;
                for (int f = 0; f < H->nf; ++f) {
                    const double* u = U + f * vol + c;
                    double adv = 0.0;
                    for (int d = 0; d < 3; ++d) adv += x[d] / r * rad_d1(u, st[d], a[d], N[d], h);
                    R[f * vol + c] = -H->rad_v[f] * adv - H->rad_v[f] * (u[0] - H->rad_uinf[f]) / r;
                }
            }
}

void orc_hier_step(orc_hier* H, double dt0, const orc_params* p)
{
    /* the k arrays hold zero on ghost points: rhs and increments are interior only */
    advance(H, 0, dt0, p);
}
