/*
 * Oracle: CCZ4 right-hand side in vacuum (Sec. V, eqs. syseq1 .. syseq2, the
 * Ricci split below them, the Bona-Masso slicing and the Gamma-driver shift),
 * with 4th-order centred derivatives, lop-sided advection and KO dissipation
 * on every field (Sec. II.B.1).  TEST INFRASTRUCTURE ONLY.
 *
 * Field order: chi, gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz, trKhat,
 *              At_xx .. At_zz, Ghat^x Ghat^y Ghat^z, Theta, alpha,
 *              beta^x beta^y beta^z, B^x B^y B^z  (25 fields).
 *
 * Readings of the printed equations:
 *  - vacuum: tau = S_i = S_ij = 0;
 *  - Z^i = chi (Ghat^i - Gt^i) / 2 follows from Ghat^i = Gt^i + 2 Z^i / chi,
 *    with Gt^i = gt^{jk} Gt^i_{jk};
 *  - R_ij + 2 nabla_(i Z_j) = Rhat_ij + Rhat^chi_ij as printed;
 *    R + 2 nabla_i Z^i is its trace chi gt^{ij}(...), and
 *    nabla_i nabla^i alpha = chi gt^{ij} nabla_i nabla_j alpha;
 *  - [.]^TF removes the trace with respect to gt_ij;
 *  - the shift terms of the Ghat equation use Ghat as printed;
 *  - Bona-Masso f = f0 + f1/alpha (f1 = 2, f0 = 0 is "1+log");
 *  - the B^i equation uses d_t Ghat^i without its advection term and without
 *    dissipation (dissipation is added to every field separately);
 *  - ln det gt is evaluated as log1p(d) with d = det(I+h) - 1 expanded in
 *    h = gt - I, which is the same number written without cancellation.
 *  The terms proportional to Theta or Z vanish on the constraint surface;
 *  they are pinned off it by the covariant Z4 equation of Sec. V on a
 *  time-symmetric slice (Z^i from Ghat != Gt, the kappa_z, Theta-gradient and
 *  Z.grad(alpha) terms) and on a homogeneous, spatially flat metric (the terms
 *  quadratic in trK and Theta), and the shift terms by the Lie derivative.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

enum {
    F_CHI = 0, F_GT = 1, F_KH = 7, F_AT = 8, F_GH = 14, F_TH = 17,
    F_ALP = 18, F_BETA = 19, F_B = 22, NF_CCZ4 = 25
};

/* symmetric index pair (i,j) -> 0..5 for xx xy xz yy yz zz */
static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

/* The right-hand side at point c of the patch array U (field stride vol,
 * axis strides st): out[f] = rhs of field f + its KO term.  When mon is not
 * NULL it also receives the constraint monitors of Sec. V at that point:
 * mon[0] = Theta, mon[1] = gamma_ij Z^i Z^j = gt_ij Z^i Z^j / chi, mon[2] =
 * H_Z, the bracket of the Theta equation (R + 2 nabla_i Z^i + 2/3 trKhat^2 +
 * 2/3 Theta (trKhat - 2 Theta) - At_ij At^ij), mon[3] = ln det gt, mon[4] =
 * tr At = gt^ij At_ij; each is the value the right-hand side itself uses. */
static void ccz4_point(const double* U, long vol, long c, const long st[3], const double h[3],
                       const orc_params* p, double out[NF_CCZ4], double* mon)
{
    const double kz = p->kappa_z, kc = p->kappa_c;
    {
        {
            {
#define FLD(f) (U + (long)(f) * vol + c)
                /* ---- point values ---- */
                double chi = *FLD(F_CHI), Kh = *FLD(F_KH), Th = *FLD(F_TH), alp = *FLD(F_ALP);
                double gt[3][3], At[3][3], Gh[3], beta[3], Bv[3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        gt[i][j] = *FLD(F_GT + SYM[i][j]);
                        At[i][j] = *FLD(F_AT + SYM[i][j]);
                    }
                for (int i = 0; i < 3; ++i) {
                    Gh[i] = *FLD(F_GH + i);
                    beta[i] = *FLD(F_BETA + i);
                    Bv[i] = *FLD(F_B + i);
                }
                /* ---- centred first derivatives: d[k] = d_k ---- */
                double dchi[3], dKh[3], dTh[3], dalp[3], dgt[3][3][3], dGh[3][3], dbeta[3][3];
                for (int k = 0; k < 3; ++k) {
                    dchi[k] = orc_d1(FLD(F_CHI), st[k], h[k]);
                    dKh[k] = orc_d1(FLD(F_KH), st[k], h[k]);
                    dTh[k] = orc_d1(FLD(F_TH), st[k], h[k]);
                    dalp[k] = orc_d1(FLD(F_ALP), st[k], h[k]);
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            dgt[k][i][j] = orc_d1(FLD(F_GT + SYM[i][j]), st[k], h[k]);
                    for (int i = 0; i < 3; ++i) {
                        dGh[k][i] = orc_d1(FLD(F_GH + i), st[k], h[k]);   /* d_k Ghat^i */
                        dbeta[k][i] = orc_d1(FLD(F_BETA + i), st[k], h[k]); /* d_k beta^i */
                    }
                }
                /* ---- second derivatives: dd[k][l] = d_k d_l ---- */
                double ddchi[3][3], ddalp[3][3], ddgt[3][3][3][3], ddbeta[3][3][3];
                for (int k = 0; k < 3; ++k)
                    for (int l = k; l < 3; ++l) {
                        if (k == l) {
                            ddchi[k][l] = orc_d2(FLD(F_CHI), st[k], h[k]);
                            ddalp[k][l] = orc_d2(FLD(F_ALP), st[k], h[k]);
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j)
                                    ddgt[k][l][i][j] = orc_d2(FLD(F_GT + SYM[i][j]), st[k], h[k]);
                            for (int i = 0; i < 3; ++i)
                                ddbeta[k][l][i] = orc_d2(FLD(F_BETA + i), st[k], h[k]);
                        } else {
                            /* D_kl = D_l(D_k U), k < l */
                            ddchi[k][l] = orc_dmix(FLD(F_CHI), st[k], h[k], st[l], h[l]);
                            ddalp[k][l] = orc_dmix(FLD(F_ALP), st[k], h[k], st[l], h[l]);
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j)
                                    ddgt[k][l][i][j] = orc_dmix(FLD(F_GT + SYM[i][j]), st[k], h[k], st[l], h[l]);
                            for (int i = 0; i < 3; ++i)
                                ddbeta[k][l][i] = orc_dmix(FLD(F_BETA + i), st[k], h[k], st[l], h[l]);
                            /* D_lk = D_kl (the paper's D_xy = D_yx = D_y(D_x U)) */
                            ddchi[l][k] = ddchi[k][l];
                            ddalp[l][k] = ddalp[k][l];
                            for (int i = 0; i < 3; ++i) {
                                ddbeta[l][k][i] = ddbeta[k][l][i];
                                for (int j = 0; j < 3; ++j) ddgt[l][k][i][j] = ddgt[k][l][i][j];
                            }
                        }
                    }
                /* ---- advection beta^k d_k U of every field, and KO ---- */
                double adv[NF_CCZ4], ko[NF_CCZ4];
                for (int f = 0; f < NF_CCZ4; ++f) {
                    adv[f] = 0.0;
                    ko[f] = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        double dk = p->upwind != 0.0 ? orc_adv(FLD(f), st[k], h[k], beta[k])
                                                     : orc_d1(FLD(f), st[k], h[k]);
                        adv[f] += beta[k] * dk;
                        ko[f] += orc_ko(FLD(f), st[k], h[k], p->sigma);
                    }
                }
#undef FLD
                /* ---- inverse conformal metric, ln det ---- */
                double hx = gt[0][0] - 1.0, hy = gt[1][1] - 1.0, hz = gt[2][2] - 1.0;
                double hxy = gt[0][1], hxz = gt[0][2], hyz = gt[1][2];
                double dmin = (hx + hy + hz)
                              + (hx * hy - hxy * hxy + hx * hz - hxz * hxz + hy * hz - hyz * hyz)
                              + (hx * (hy * hz - hyz * hyz) - hxy * (hxy * hz - hyz * hxz)
                                 + hxz * (hxy * hyz - hy * hxz));
                double det = 1.0 + dmin;
                double lndet = log1p(dmin);
                double gu[3][3];
                gu[0][0] = (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) / det;
                gu[0][1] = (gt[0][2] * gt[2][1] - gt[0][1] * gt[2][2]) / det;
                gu[0][2] = (gt[0][1] * gt[1][2] - gt[0][2] * gt[1][1]) / det;
                gu[1][1] = (gt[0][0] * gt[2][2] - gt[0][2] * gt[2][0]) / det;
                gu[1][2] = (gt[0][2] * gt[1][0] - gt[0][0] * gt[1][2]) / det;
                gu[2][2] = (gt[0][0] * gt[1][1] - gt[0][1] * gt[1][0]) / det;
                gu[1][0] = gu[0][1];
                gu[2][0] = gu[0][2];
                gu[2][1] = gu[1][2];

                /* ---- Christoffel symbols of gt ----
                 * Gl[i][j][k] = Gt_{ijk} = (d_j gt_ik + d_k gt_ij - d_i gt_jk)/2
                 * Gu[i][j][k] = Gt^i_{jk} = gt^{il} Gt_{ljk}                    */
                double Gl[3][3][3], Gu[3][3][3], Gtc[3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k)
                            Gl[i][j][k] = 0.5 * (dgt[j][i][k] + dgt[k][i][j] - dgt[i][j][k]);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k) {
                            double s = 0.0;
                            for (int l = 0; l < 3; ++l) s += gu[i][l] * Gl[l][j][k];
                            Gu[i][j][k] = s;
                        }
                for (int i = 0; i < 3; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k) s += gu[j][k] * Gu[i][j][k];
                    Gtc[i] = s;
                }
                double Z[3];
                for (int i = 0; i < 3; ++i) Z[i] = 0.5 * chi * (Gh[i] - Gtc[i]);

                /* ---- Rhat^chi_ij ---- */
                double Rchi[3][3];
                {
                    double trdd = 0.0;
                    for (int k = 0; k < 3; ++k)
                        for (int m = 0; m < 3; ++m)
                            trdd += gu[k][m] * (ddchi[k][m] - 1.5 / chi * dchi[k] * dchi[m]);
                    double Ghd = 0.0;
                    for (int k = 0; k < 3; ++k) Ghd += Gh[k] * dchi[k];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) {
                            double Gd = 0.0;
                            for (int k = 0; k < 3; ++k) Gd += Gu[k][i][j] * dchi[k];
                            double zsym = 0.0;
                            for (int k = 0; k < 3; ++k)
                                zsym += Z[k] * 0.5 * (gt[k][i] * dchi[j] + gt[k][j] * dchi[i]);
                            Rchi[i][j] = 0.5 / chi * ddchi[i][j] - 0.5 / chi * Gd
                                         - 0.25 / (chi * chi) * dchi[i] * dchi[j]
                                         + 2.0 / (chi * chi) * zsym
                                         + 0.5 / chi * gt[i][j] * (trdd - Ghd);
                        }
                }
                /* ---- Rhat_ij ---- */
                double Rh[3][3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int m = 0; m < 3; ++m)
                            for (int n = 0; n < 3; ++n) s += -0.5 * gu[m][n] * ddgt[m][n][i][j];
                        for (int k = 0; k < 3; ++k)
                            s += 0.5 * (gt[k][i] * dGh[j][k] + gt[k][j] * dGh[i][k]);
                        for (int k = 0; k < 3; ++k)
                            s += Gh[k] * 0.5 * (Gl[i][j][k] + Gl[j][i][k]);
                        for (int m = 0; m < 3; ++m)
                            for (int n = 0; n < 3; ++n)
                                for (int k = 0; k < 3; ++k)
                                    s += gu[m][n] * (Gu[k][m][i] * Gl[j][k][n]
                                                     + Gu[k][m][j] * Gl[i][k][n]
                                                     + Gu[k][m][i] * Gl[k][n][j]);
                        Rh[i][j] = s;
                    }
                /* ---- nabla_i nabla_j alpha ---- */
                double DDa[3][3];
                {
                    double cross = 0.0;
                    for (int k = 0; k < 3; ++k)
                        for (int m = 0; m < 3; ++m) cross += gu[k][m] * dalp[k] * dchi[m];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) {
                            double Gd = 0.0;
                            for (int k = 0; k < 3; ++k) Gd += Gu[k][i][j] * dalp[k];
                            DDa[i][j] = ddalp[i][j] - Gd
                                        + 0.5 / chi * (dalp[i] * dchi[j] + dalp[j] * dchi[i]
                                                       - gt[i][j] * cross);
                        }
                }
                double Ric[3][3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) Ric[i][j] = Rh[i][j] + Rchi[i][j];
                double trRic = 0.0, lapa = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        trRic += chi * gu[i][j] * Ric[i][j];
                        lapa += chi * gu[i][j] * DDa[i][j];
                    }
                /* ---- raised traceless curvature ---- */
                double Amix[3][3], Aup[3][3], trA = 0.0, AA = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int l = 0; l < 3; ++l) s += gu[i][l] * At[l][j];
                        Amix[i][j] = s; /* At^i_j */
                    }
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int l = 0; l < 3; ++l) s += Amix[i][l] * gu[l][j];
                        Aup[i][j] = s; /* At^{ij} */
                    }
                for (int i = 0; i < 3; ++i) {
                    trA += Amix[i][i];
                    for (int j = 0; j < 3; ++j) AA += At[i][j] * Aup[i][j];
                }
                double divb = dbeta[0][0] + dbeta[1][1] + dbeta[2][2];
                double Zda = Z[0] * dalp[0] + Z[1] * dalp[1] + Z[2] * dalp[2];

                double rhs[NF_CCZ4];
                /* ---- d_t gt_ij ---- */
                for (int i = 0; i < 3; ++i)
                    for (int j = i; j < 3; ++j) {
                        double s = adv[F_GT + SYM[i][j]];
                        for (int k = 0; k < 3; ++k)
                            s += gt[i][k] * dbeta[j][k] + gt[k][j] * dbeta[i][k];
                        s += -2.0 / 3.0 * gt[i][j] * divb
                             - 2.0 * alp * (At[i][j] - 1.0 / 3.0 * gt[i][j] * trA)
                             - kc / 3.0 * alp * gt[i][j] * lndet;
                        rhs[F_GT + SYM[i][j]] = s;
                    }
                /* ---- d_t At_ij ---- */
                {
                    double X[3][3], trX = 0.0;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) X[i][j] = alp * Ric[i][j] - DDa[i][j];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) trX += gu[i][j] * X[i][j];
                    for (int i = 0; i < 3; ++i)
                        for (int j = i; j < 3; ++j) {
                            double s = adv[F_AT + SYM[i][j]];
                            for (int k = 0; k < 3; ++k)
                                s += At[i][k] * dbeta[j][k] + At[k][j] * dbeta[i][k];
                            s += -2.0 / 3.0 * At[i][j] * divb
                                 - kc / 3.0 * alp * gt[i][j] * trA
                                 + chi * (X[i][j] - 1.0 / 3.0 * gt[i][j] * trX);
                            double AAij = 0.0;
                            for (int k = 0; k < 3; ++k) AAij += At[i][k] * Amix[k][j];
                            s += alp * (Kh * At[i][j] - 2.0 * AAij);
                            rhs[F_AT + SYM[i][j]] = s;
                        }
                }
                /* ---- d_t chi ---- */
                rhs[F_CHI] = adv[F_CHI] + 2.0 / 3.0 * chi * (alp * (Kh + 2.0 * Th) - divb);
                /* ---- d_t trKhat ---- */
                rhs[F_KH] = adv[F_KH] - lapa
                            + alp * (1.0 / 3.0 * (Kh + 2.0 * Th) * (Kh + 2.0 * Th) + AA + kz * Th)
                            + 2.0 * Zda;
                /* ---- d_t Theta ---- */
                rhs[F_TH] = adv[F_TH]
                            + 0.5 * alp * (trRic + 2.0 / 3.0 * Kh * Kh
                                           + 2.0 / 3.0 * Th * (Kh - 2.0 * Th) - AA)
                            - Zda - alp * (2.0 * kz * Th);
                /* ---- d_t Ghat^i (and its part without advection, for B^i) ---- */
                double dtG_noadv[3];
                for (int i = 0; i < 3; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < 3; ++j) s += -Gh[j] * dbeta[j][i];
                    s += 2.0 / 3.0 * Gh[i] * divb;
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k) s += gu[j][k] * ddbeta[j][k][i];
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k) s += 1.0 / 3.0 * gu[i][j] * ddbeta[j][k][k];
                    for (int j = 0; j < 3; ++j) s += -2.0 * Aup[i][j] * dalp[j];
                    double b1 = 0.0;
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k) b1 += Gu[i][j][k] * Aup[j][k];
                    for (int j = 0; j < 3; ++j) b1 += -1.5 / chi * Aup[i][j] * dchi[j];
                    for (int j = 0; j < 3; ++j) b1 += -2.0 / 3.0 * gu[i][j] * dKh[j];
                    s += 2.0 * alp * b1;
                    double b2 = 0.0;
                    for (int j = 0; j < 3; ++j)
                        b2 += -gu[i][j] * (1.0 / 3.0 * dTh[j] + Th / alp * dalp[j]);
                    b2 += -1.0 / chi * Z[i] * (kz + 2.0 / 3.0 * (Kh + 2.0 * Th));
                    s += 2.0 * alp * b2;
                    dtG_noadv[i] = s;
                    rhs[F_GH + i] = adv[F_GH + i] + s;
                }
                /* ---- gauge ---- */
                double f = p->bm_f0 + p->bm_f1 / alp;
                rhs[F_ALP] = adv[F_ALP] - alp * alp * f * Kh;
                for (int i = 0; i < 3; ++i) {
                    rhs[F_BETA + i] = adv[F_BETA + i] + p->gd_g * Bv[i];
                    rhs[F_B + i] = adv[F_B + i] - p->gd_eta * Bv[i] + dtG_noadv[i];
                }
                for (int fld = 0; fld < NF_CCZ4; ++fld) out[fld] = rhs[fld] + ko[fld];
                if (mon) {
                    double zz = 0.0;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) zz += gt[i][j] * Z[i] * Z[j];
                    mon[0] = Th;
                    mon[1] = zz / chi;
                    mon[2] = trRic + 2.0 / 3.0 * Kh * Kh + 2.0 / 3.0 * Th * (Kh - 2.0 * Th) - AA;
                    mon[3] = lndet;
                    mon[4] = trA;
                }
            }
        }
    }
}

void orc_ccz4_rhs(const double* U, double* R, int nx, int ny, int nz,
                  const double h[3], const orc_params* p)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    long st[3] = {1, NX, NX * NY};
    double out[NF_CCZ4];
    for (int kk = ORC_G; kk < nz + ORC_G; ++kk)
        for (int jj = ORC_G; jj < ny + ORC_G; ++jj)
            for (int ii = ORC_G; ii < nx + ORC_G; ++ii) {
                long c = (kk * NY + jj) * NX + ii;
                ccz4_point(U, vol, c, st, h, p, out, 0);
                for (int fld = 0; fld < NF_CCZ4; ++fld) R[(long)fld * vol + c] = out[fld];
            }
}

/* Constraint monitors (see ccz4_point) at every interior point: M holds
 * five fields in the patch-array layout. */
void orc_ccz4_monitor(const double* U, double* M, int nx, int ny, int nz,
                      const double h[3], const orc_params* p)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    long st[3] = {1, NX, NX * NY};
    double out[NF_CCZ4], mon[5];
    for (int kk = ORC_G; kk < nz + ORC_G; ++kk)
        for (int jj = ORC_G; jj < ny + ORC_G; ++jj)
            for (int ii = ORC_G; ii < nx + ORC_G; ++ii) {
                long c = (kk * NY + jj) * NX + ii;
                ccz4_point(U, vol, c, st, h, p, out, mon);
                for (int q = 0; q < 5; ++q) M[(long)q * vol + c] = mon[q];
            }
}
