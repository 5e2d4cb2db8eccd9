/*
 * Oracle: Newtonian ideal MHD right-hand side (Sec. IV.B) with the
 * conservative finite-difference form (eq. conservative_discretization),
 * reconstruction of the evolved fields by WENO5-Z (default), WENO5-JS
 * (App. B) or WENO3 (App. A), and the local Lax-Friedrichs flux (eq. LLF,
 * default) or the HLL flux (Sec. II.B.2).  TEST INFRASTRUCTURE ONLY.
 *
 * Conserved fields, in this order: rho, S_x, S_y, S_z, E, B^x, B^y, B^z
 * (the eight-field ideal core: the cleaning scalar psi is identically zero).
 *
 * Readings (the paper leaves these open):
 *  - the reconstruction acts on the evolved (conserved) fields, as the text
 *    states for its tests; the flux is then evaluated on U^L and U^R;
 *  - S in the LLF formula is max over the L and R states of |v_d| + c_f, with
 *    the fast magnetosonic speed c_f^2 = ((a^2+b^2) + sqrt((a^2+b^2)^2 - 4 a^2 b_d^2))/2,
 *    a^2 = Gamma p / rho, b^2 = B^2/rho, b_d^2 = B_d^2/rho (units where the
 *    magnetic pressure is B^2/2, as in the paper's energy density); the
 *    discriminant is evaluated as (a^2 - b^2)^2 + 4 a^2 b_t^2, b_t^2 the sum
 *    of the two transverse components' squares over rho (the same number as
 *    a sum of non-negative terms, which does not cancel where the sound and
 *    Alfven speeds meet with B nearly along d);
 *  - S is taken per interface;
 *  - HLL: the printed formula misses a "+" before S^R S^L (U^R - U^L); the
 *    speeds are S^L = min(v_d - c_f) and S^R = max(v_d + c_f) over the two
 *    states, clamped to S^L <= 0 <= S^R, which gives the textbook flux (F^L
 *    when every wave moves right, F^R when every wave moves left) in one
 *    formula;
 *  - epsilon: dx^4 for the fifth-order reconstructions (App. B), dx^2 for
 *    WENO3 (App. A), unless set;
 *  - reading R2 (mhd_riemann 2): the interface flux is the left-biased
 *    reconstruction of F+ = (F + alpha U)/2 plus the right-biased one of
 *    F- = (F - alpha U)/2, cell by cell from the physical fluxes, with alpha
 *    the largest |v_d| + c_f (and c_h) over the six cells of the stencil;
 *  - divergence cleaning (nine fields, psi last): the B^i flux along d gains
 *    delta^{di} psi, psi has the flux c_h^2 B^d and the source -kappa_psi psi;
 *    the cleaning waves move at -c_h and +c_h, so LLF takes S = max(..., c_h)
 *    and HLL S^L = min(..., -c_h), S^R = max(..., c_h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Table of c_{r,j} for k = 3 (Sec. II.B.2), rows r = -1, 0, 1, 2. */
static const double C3[4][3] = {
    {11.0 / 6.0, -7.0 / 6.0, 1.0 / 3.0},
    {1.0 / 3.0, 5.0 / 6.0, -1.0 / 6.0},
    {-1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0},
    {1.0 / 3.0, -7.0 / 6.0, 11.0 / 6.0},
};
static const double D3[3] = {3.0 / 10.0, 6.0 / 10.0, 1.0 / 10.0};

static double sq(double x) { return x * x; }

/* Smoothness indicators of App. B for the left state at i+1/2; u points at U_i. */
static void beta_left(const double* u, double b[3])
{
    b[0] = 13.0 / 12.0 * sq(u[0] - 2.0 * u[1] + u[2]) + 0.25 * sq(3.0 * u[0] - 4.0 * u[1] + u[2]);
    b[1] = 13.0 / 12.0 * sq(u[-1] - 2.0 * u[0] + u[1]) + 0.25 * sq(u[-1] - u[1]);
    b[2] = 13.0 / 12.0 * sq(u[-2] - 2.0 * u[-1] + u[0]) + 0.25 * sq(u[-2] - 4.0 * u[-1] + 3.0 * u[0]);
}

/* Smoothness indicators of App. B for the right state at i-1/2; u points at U_i. */
static void beta_right(const double* u, double b[3])
{
    b[0] = 13.0 / 12.0 * sq(u[2] - 2.0 * u[1] + u[0]) + 0.25 * sq(u[2] - 4.0 * u[1] + 3.0 * u[0]);
    b[1] = 13.0 / 12.0 * sq(u[1] - 2.0 * u[0] + u[-1]) + 0.25 * sq(u[1] - u[-1]);
    b[2] = 13.0 / 12.0 * sq(u[0] - 2.0 * u[-1] + u[-2]) + 0.25 * sq(3.0 * u[0] - 4.0 * u[-1] + u[-2]);
}

static double powq(double x, double q)
{
    return q == 2.0 ? x * x : pow(x, q);
}

/* Candidate values: ^L U^(r)_{i+1/2} = sum_j c_{r,j} U_{i-r+j};
 *                   ^R U^(r)_{i-1/2} = sum_j c_{r-1,j} U_{i-r+j}. */
static void cand_left(const double* u, double v[3])
{
    for (int r = 0; r < 3; ++r) {
        v[r] = 0.0;
        for (int j = 0; j < 3; ++j) v[r] += C3[r + 1][j] * u[-r + j];
    }
}

static void cand_right(const double* u, double v[3])
{
    for (int r = 0; r < 3; ++r) {
        v[r] = 0.0;
        for (int j = 0; j < 3; ++j) v[r] += C3[r][j] * u[-r + j];
    }
}

/* WENO-Z weights (App. B): alpha_r = d_r (1 + [tau/(eps + beta_r)]^q),
 * tau = |beta_0 - beta_2|, omega_r = alpha_r / sum_s alpha_s. */
static double combine_z(const double v[3], const double b[3], const double d[3],
                        double eps, double q)
{
    double tau = fabs(b[0] - b[2]);
    double a[3], sum = 0.0;
    for (int r = 0; r < 3; ++r) {
        a[r] = d[r] * (1.0 + powq(tau / (eps + b[r]), q));
        sum += a[r];
    }
    double out = 0.0;
    for (int r = 0; r < 3; ++r) out += (a[r] / sum) * v[r];
    return out;
}

double orc_weno5z_left(const double* u, double eps, double q)
{
    double v[3], b[3];
    cand_left(u, v);
    beta_left(u, b);
    return combine_z(v, b, D3, eps, q);
}

double orc_weno5z_right(const double* u, double eps, double q)
{
    double v[3], b[3];
    double dt[3] = {D3[2], D3[1], D3[0]}; /* tilde d_r = d_{k-1-r} */
    cand_right(u, v);
    beta_right(u, b);
    return combine_z(v, b, dt, eps, q);
}

/* Classic (JS) weights of Sec. II.B.2: alpha_r = d_r / (eps + beta_r)^2. */
double orc_weno5js_left(const double* u, double eps)
{
    double v[3], b[3], a[3], sum = 0.0, out = 0.0;
    cand_left(u, v);
    beta_left(u, b);
    for (int r = 0; r < 3; ++r) { a[r] = D3[r] / sq(eps + b[r]); sum += a[r]; }
    for (int r = 0; r < 3; ++r) out += (a[r] / sum) * v[r];
    return out;
}

double orc_weno5js_right(const double* u, double eps)
{
    double v[3], b[3], a[3], sum = 0.0, out = 0.0;
    double dt[3] = {D3[2], D3[1], D3[0]}; /* tilde d_r = d_{k-1-r} */
    cand_right(u, v);
    beta_right(u, b);
    for (int r = 0; r < 3; ++r) { a[r] = dt[r] / sq(eps + b[r]); sum += a[r]; }
    for (int r = 0; r < 3; ++r) out += (a[r] / sum) * v[r];
    return out;
}

/* WENO3 (App. A): the two candidates, smoothness indicators and weights as
 * printed, omega_r = alpha_r / sum_s alpha_s; u points at U_i. */
double orc_weno3_left(const double* u, double eps)
{
    double v[2] = {0.5 * u[0] + 0.5 * u[1], -0.5 * u[-1] + 1.5 * u[0]};
    double b[2] = {sq(u[1] - u[0]), sq(u[0] - u[-1])};
    double a[2] = {(2.0 / 3.0) / sq(eps + b[0]), (1.0 / 3.0) / sq(eps + b[1])};
    double sum = a[0] + a[1];
    return (a[0] / sum) * v[0] + (a[1] / sum) * v[1];
}

double orc_weno3_right(const double* u, double eps)
{
    double v[2] = {-0.5 * u[1] + 1.5 * u[0], 0.5 * u[0] + 0.5 * u[-1]};
    double b[2] = {sq(u[0] - u[1]), sq(u[-1] - u[0])};
    double a[2] = {(1.0 / 3.0) / sq(eps + b[0]), (2.0 / 3.0) / sq(eps + b[1])};
    double sum = a[0] + a[1];
    return (a[0] / sum) * v[0] + (a[1] / sum) * v[1];
}

/* Physical flux along direction d, the normal velocity v_d and the fast
 * magnetosonic speed c_f. */
static void mhd_flux_vc(const double U[8], int d, double gam, double F[8], double* vd, double* cf)
{
    double rho = U[0];
    double v[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
    double E = U[4];
    double B[3] = {U[5], U[6], U[7]};
    double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double S2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    double p = (gam - 1.0) * (E - 0.5 * S2 / rho - 0.5 * B2);
    double vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    double ptot = p + 0.5 * B2;
    F[0] = rho * v[d];
    for (int i = 0; i < 3; ++i)
        F[1 + i] = rho * v[d] * v[i] + (i == d ? ptot : 0.0) - B[d] * B[i];
    F[4] = (E + ptot) * v[d] - vB * B[d];
    for (int i = 0; i < 3; ++i) F[5 + i] = v[d] * B[i] - v[i] * B[d];
    double Bt2 = 0.0;
    for (int i = 0; i < 3; ++i)
        if (i != d) Bt2 += B[i] * B[i];
    double a2 = gam * p / rho, b2 = B2 / rho, bt2 = Bt2 / rho;
    double cf2 = 0.5 * (a2 + b2 + sqrt(sq(a2 - b2) + 4.0 * a2 * bt2));
    *vd = v[d];
    *cf = sqrt(cf2);
}

double orc_mhd_fast_speed(const double U[8], int d, double gam)
{
    double F[8], vd, cf;
    mhd_flux_vc(U, d, gam, F, &vd, &cf);
    return cf;
}

/* interface flux of nf = 8 or 9 fields (9: with the cleaning scalar and speed ch) */
static void interface_flux(const double* UL, const double* UR, int d, double gam, int riemann, int nf,
                           double ch, double* F)
{
    double FL[9], FR[9], vL, cL, vR, cR;
    mhd_flux_vc(UL, d, gam, FL, &vL, &cL);
    mhd_flux_vc(UR, d, gam, FR, &vR, &cR);
    if (nf == 9) {
        FL[5 + d] += UL[8];
        FR[5 + d] += UR[8];
        FL[8] = ch * ch * UL[5 + d];
        FR[8] = ch * ch * UR[5 + d];
    }
    if (riemann == 1) {
        /* HLL: F = (S^R F^L - S^L F^R + S^R S^L (U^R - U^L)) / (S^R - S^L) */
        double SL = fmin(vL - cL, vR - cR), SR = fmax(vL + cL, vR + cR);
        if (nf == 9) {
            SL = fmin(SL, -ch);
            SR = fmax(SR, ch);
        }
        SL = fmin(SL, 0.0);
        SR = fmax(SR, 0.0);
        for (int f = 0; f < nf; ++f) F[f] = (SR * FL[f] - SL * FR[f] + SR * SL * (UR[f] - UL[f])) / (SR - SL);
    } else {
        /* LLF with S = max over the two states of |v_d| + c_f (and c_h) */
        double sL = fabs(vL) + cL, sR = fabs(vR) + cR;
        double S = sL > sR ? sL : sR;
        if (nf == 9 && ch > S) S = ch;
        for (int f = 0; f < nf; ++f) F[f] = 0.5 * (FL[f] + FR[f] - S * (UR[f] - UL[f]));
    }
}

void orc_mhd_interface_flux(const double UL[8], const double UR[8], int d, double gam, int riemann,
                            double F[8])
{
    interface_flux(UL, UR, d, gam, riemann, 8, 0.0, F);
}

/* physical flux of nf fields at one cell and its largest signal speed */
static void cell_flux(const double* U, int d, double gam, int nf, double ch, double* F, double* speed)
{
    double vd, cf;
    mhd_flux_vc(U, d, gam, F, &vd, &cf);
    *speed = fabs(vd) + cf;
    if (nf == 9) {
        F[5 + d] += U[8];
        F[8] = ch * ch * U[5 + d];
        if (ch > *speed) *speed = ch;
    }
}

static double recon_left(int recon, const double* u, double eps, double q)
{
    return recon == 2 ? orc_weno3_left(u, eps) : recon == 1 ? orc_weno5js_left(u, eps) : orc_weno5z_left(u, eps, q);
}

static double recon_right(int recon, const double* u, double eps, double q)
{
    return recon == 2 ? orc_weno3_right(u, eps) : recon == 1 ? orc_weno5js_right(u, eps) : orc_weno5z_right(u, eps, q);
}

static void mhd_rhs_nf(const double* U, double* R, int nx, int ny, int nz, const double h[3],
                       const orc_params* p, int nf)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    long st[3] = {1, NX, NX * NY};
    int n[3] = {nx, ny, nz};
    for (int k = ORC_G; k < nz + ORC_G; ++k)
        for (int j = ORC_G; j < ny + ORC_G; ++j)
            for (int i = ORC_G; i < nx + ORC_G; ++i)
                for (int f = 0; f < nf; ++f) R[f * vol + (k * NY + j) * NX + i] = 0.0;
    const int recon = (int)p->mhd_recon, riemann = (int)p->mhd_riemann;
    for (int d = 0; d < 3; ++d) {
        double eps = p->weno_eps > 0.0 ? p->weno_eps : (recon == 2 ? h[d] * h[d] : h[d] * h[d] * h[d] * h[d]);
        /* every interface i+1/2 with i = -1 .. n_d - 1 along d (interior coords) */
        int lo[3] = {ORC_G, ORC_G, ORC_G}, hi[3] = {nx + ORC_G, ny + ORC_G, nz + ORC_G};
        lo[d] = ORC_G - 1;
        (void)n;
        for (int k = lo[2]; k < hi[2]; ++k)
            for (int j = lo[1]; j < hi[1]; ++j)
                for (int i = lo[0]; i < hi[0]; ++i) {
                    long c = (k * NY + j) * NX + i;
                    double UL[9], UR[9], Fi[9];
                    if (riemann == 2) {
                        /* cells i-2 .. i+3: physical fluxes, alpha, split fluxes */
                        double Uc[6][9], Fc[6][9], sp[6], alpha = 0.0;
                        for (int m = 0; m < 6; ++m) {
                            for (int f = 0; f < nf; ++f) Uc[m][f] = U[f * vol + c + (m - 2) * st[d]];
                            cell_flux(Uc[m], d, p->gamma_ad, nf, p->mhd_ch, Fc[m], &sp[m]);
                            if (sp[m] > alpha) alpha = sp[m];
                        }
                        for (int f = 0; f < nf; ++f) {
                            double gp[6], gm[6];
                            for (int m = 0; m < 6; ++m) {
                                gp[m] = 0.5 * (Fc[m][f] + alpha * Uc[m][f]);
                                gm[m] = 0.5 * (Fc[m][f] - alpha * Uc[m][f]);
                            }
                            Fi[f] = recon_left(recon, gp + 2, eps, p->weno_q) + recon_right(recon, gm + 3, eps, p->weno_q);
                        }
                    } else {
                    for (int f = 0; f < nf; ++f) {
                        double line[6];
                        for (int m = 0; m < 6; ++m) line[m] = U[f * vol + c + (m - 2) * st[d]];
                        /* line[2] is U_i; the left state at i+1/2 is
                         * reconstructed around cell i, the right state at
                         * i+1/2 is the right state at (i+1)-1/2 of cell i+1 */
                        if (recon == 2) {
                            UL[f] = orc_weno3_left(line + 2, eps);
                            UR[f] = orc_weno3_right(line + 3, eps);
                        } else if (recon == 1) {
                            UL[f] = orc_weno5js_left(line + 2, eps);
                            UR[f] = orc_weno5js_right(line + 3, eps);
                        } else {
                            UL[f] = orc_weno5z_left(line + 2, eps, p->weno_q);
                            UR[f] = orc_weno5z_right(line + 3, eps, p->weno_q);
                        }
                    }
                    interface_flux(UL, UR, d, p->gamma_ad, riemann, nf, p->mhd_ch, Fi);
                    }
                    for (int f = 0; f < nf; ++f) {
                        double Fh = Fi[f];
                        /* interface i+1/2 closes cell i (if interior) on the right
                         * and opens cell i+1 (if interior) on the left */
                        int ii[3] = {i, j, k};
                        if (ii[d] >= ORC_G) R[f * vol + c] -= Fh / h[d];
                        if (ii[d] + 1 < n[d] + ORC_G) R[f * vol + c + st[d]] += Fh / h[d];
                    }
                }
    }
    if (nf == 9)
        for (int k = ORC_G; k < nz + ORC_G; ++k)
            for (int j = ORC_G; j < ny + ORC_G; ++j)
                for (int i = ORC_G; i < nx + ORC_G; ++i) {
                    long c = (k * NY + j) * NX + i;
                    R[8 * vol + c] -= p->mhd_kpsi * U[8 * vol + c];
                }
}

void orc_mhd_rhs(const double* U, double* R, int nx, int ny, int nz,
                 const double h[3], const orc_params* p)
{
    mhd_rhs_nf(U, R, nx, ny, nz, h, p, 8);
}

void orc_mhd_glm_rhs(const double* U, double* R, int nx, int ny, int nz,
                     const double h[3], const orc_params* p)
{
    mhd_rhs_nf(U, R, nx, ny, nz, h, p, 9);
}
