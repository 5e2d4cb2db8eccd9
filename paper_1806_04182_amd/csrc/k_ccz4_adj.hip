// Transpose of the CCZ4 right-hand side (project addition, for the adjoint):
// lamU = (dR/dU)^T lam on a periodic level, R the CCZ4 right-hand side of
// Sec. V with the stencils of Sec. II.B.1 (centred first and second
// derivatives, lop-sided advection, KO dissipation).
//
// R at an interior point c is R(c) = F(P(c)) + adv(c) + ko(c), where P(c)
// holds the point values of the 25 fields, the centred first derivatives of
// the 16 fields whose gradients enter the equations and the second
// derivatives of the 11 fields whose Hessians enter them, and F is pointwise
// algebra.  Two kernels:
//  1. per interior point: recompute P(c) and F's intermediates, then run F in
//     reverse to get Pbar(c) = (dF/dP)^T lam(c) (139 numbers), plus the
//     derivative of the advection term with respect to beta^k(c); written to
//     a workspace;
//  2. per point p of the ghosted box: gather the transposed stencils,
//     lamU(p) = ubar(p) + sum_c (dD(c)/dU(p)) Dbar(c) + advection and KO
//     transposes of lam, over interior points c only.  Ghost entries of lamU
//     are contributions to ghost values; the transpose of the ghost fill folds
//     them into their owners.
// The sign branch of the lop-sided stencils is taken from beta at c, as in the
// forward right-hand side (frozen at U).
#include "k_common.h"

namespace mol {

namespace {

enum { CHI = 0, GT = 1, KH = 7, AT = 8, GH = 14, TH = 17, ALP = 18, BETA = 19, BB = 22, NF = 25 };

// workspace slots: point-value adjoints of the 25 fields; then adjoints of the
// first derivatives (3 directions each) of the 16 fields gt_ij, chi, alpha,
// Ghat^i, beta^i, Khat, Theta; then adjoints of the second derivatives (6
// packed pairs each) of the 11 fields gt_ij, chi, alpha, beta^i
constexpr int ND1 = 16, ND2 = 11;
constexpr int W_U = 0, W_D1 = NF, W_D2 = NF + 3 * ND1, NW = NF + 3 * ND1 + 6 * ND2;
// slot of field f among those 16 / 11 fields, or -1
__device__ constexpr int d1_slot(int f)
{
    return f >= GT && f < GT + 6 ? f - GT : f == CHI ? 6 : f == ALP ? 7 : f >= GH && f < GH + 3 ? 8 + f - GH
           : f >= BETA && f < BETA + 3 ? 11 + f - BETA : f == KH ? 14 : f == TH ? 15 : -1;
}
__device__ constexpr int d2_slot(int f)
{
    return f >= GT && f < GT + 6 ? f - GT : f == CHI ? 6 : f == ALP ? 7 : f >= BETA && f < BETA + 3 ? 8 + f - BETA : -1;
}

__device__ constexpr int SI(int i, int j)
{
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

struct AdjConst {
    double i12h, i12h2, i144h2, ko;
    double kz, kc, f0, f1, g, eta;
    int upwind;
};

// ---------------------------------------------------------------- kernel 1
__global__ __launch_bounds__(256) void ccz4_adj_point_kernel(const PatchDev* __restrict__ patches,
                                                             const Tile* __restrict__ tiles, int ntiles,
                                                             const double* __restrict__ Ug,
                                                             const double* __restrict__ lamg,
                                                             double* __restrict__ W,
                                                             const int64_t* __restrict__ wofs, AdjConst C)
{
    const Tile t = tiles[blockIdx.x];
    const PatchDev P = patches[t.patch];
    const int ii = t.o[0] + threadIdx.x, jj = t.o[1] + threadIdx.y, kk = t.o[2] + threadIdx.z;
    if (ii >= P.n[0] || jj >= P.n[1] || kk >= P.n[2]) return;
    const int64_t loc = (int64_t)(kk + G) * P.pitch_z + (int64_t)(jj + G) * P.pitch_y + (ii + G);
    const int64_t fs = P.fs;
    const double* u = Ug + P.off + loc;
    const double* lm = lamg + P.off + loc;
    double* w = W + wofs[t.patch] + loc;
    const int S[3] = {1, P.pitch_y, P.pitch_z};
    auto F = [&](int f) { return u + (int64_t)f * fs; };
    auto d1 = [&](int f, int k) { return C.i12h * fd1(F(f), S[k]); };
    auto dd = [&](int f, int k, int l) {
        return k == l ? C.i12h2 * fd2(F(f), S[k]) : C.i144h2 * fmix(F(f), S[k], S[l]);
    };

    // ---- forward recomputation (full symmetric tensors) ----
    const double chi = F(CHI)[0], Kh = F(KH)[0], Th = F(TH)[0], alp = F(ALP)[0];
    double g[3][3], A[3][3], Gh[3], be[3], Bv[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            g[i][j] = F(GT + SI(i, j))[0];
            A[i][j] = F(AT + SI(i, j))[0];
        }
    for (int i = 0; i < 3; ++i) {
        Gh[i] = F(GH + i)[0];
        be[i] = F(BETA + i)[0];
        Bv[i] = F(BB + i)[0];
    }
    double dg[3][3][3], dchi[3], dalp[3], dGh[3][3], db[3][3], dKh[3], dTh[3];
    for (int k = 0; k < 3; ++k) {
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) dg[k][i][j] = dg[k][j][i] = d1(GT + SI(i, j), k);
        dchi[k] = d1(CHI, k);
        dalp[k] = d1(ALP, k);
        dKh[k] = d1(KH, k);
        dTh[k] = d1(TH, k);
        for (int i = 0; i < 3; ++i) {
            dGh[k][i] = d1(GH + i, k);
            db[k][i] = d1(BETA + i, k);
        }
    }
    double ddc[3][3], dda[3][3], ddb[3][3][3];
    for (int k = 0; k < 3; ++k)
        for (int l = k; l < 3; ++l) {
            ddc[k][l] = ddc[l][k] = dd(CHI, k, l);
            dda[k][l] = dda[l][k] = dd(ALP, k, l);
            for (int i = 0; i < 3; ++i) ddb[i][k][l] = ddb[i][l][k] = dd(BETA + i, k, l);
        }
    double gu[3][3], lndet;
    {
        const double hx = g[0][0] - 1.0, hy = g[1][1] - 1.0, hz = g[2][2] - 1.0;
        const double hxy = g[0][1], hxz = g[0][2], hyz = g[1][2];
        const double m2 = hx * hy - hxy * hxy + hx * hz - hxz * hxz + hy * hz - hyz * hyz;
        const double m3 = hx * (hy * hz - hyz * hyz) - hxy * (hxy * hz - hyz * hxz) + hxz * (hxy * hyz - hy * hxz);
        const double dm = (hx + hy + hz) + m2 + m3;
        lndet = log1p(dm);
        const double idet = 1.0 / (1.0 + dm);
        gu[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[1][2]) * idet;
        gu[0][1] = gu[1][0] = (g[0][2] * g[1][2] - g[0][1] * g[2][2]) * idet;
        gu[0][2] = gu[2][0] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) * idet;
        gu[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[0][2]) * idet;
        gu[1][2] = gu[2][1] = (g[0][2] * g[0][1] - g[0][0] * g[1][2]) * idet;
        gu[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[0][1]) * idet;
    }
    double Gl[3][3][3], Gu[3][3][3], Gc[3], Z[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) Gl[i][j][k] = 0.5 * (dg[j][i][k] + dg[k][i][j] - dg[i][j][k]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) Gu[i][j][k] = gu[i][0] * Gl[0][j][k] + gu[i][1] * Gl[1][j][k] + gu[i][2] * Gl[2][j][k];
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += gu[j][k] * Gu[i][j][k];
        Gc[i] = s;
        Z[i] = 0.5 * chi * (Gh[i] - Gc[i]);
    }
    const double ic = 1.0 / chi;
    double trc = 0.0, Ghd = 0.0;
    for (int k = 0; k < 3; ++k) {
        Ghd += Gh[k] * dchi[k];
        for (int m = 0; m < 3; ++m) trc += gu[k][m] * (ddc[k][m] - 1.5 * ic * dchi[k] * dchi[m]);
    }
    // gt^{mn} d_m d_n gt_q, once per packed component q
    double lapg[6];
    for (int q = 0; q < 6; ++q) {
        double t = 0.0;
        for (int m = 0; m < 3; ++m)
            for (int n = m; n < 3; ++n) t += (m == n ? 1.0 : 2.0) * gu[m][n] * dd(GT + q, m, n);
        lapg[q] = t;
    }
    double Ric[3][3], Gd[3][3], zs[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            double gd = 0.0, z = 0.0;
            for (int k = 0; k < 3; ++k) {
                gd += Gu[k][i][j] * dchi[k];
                z += Z[k] * 0.5 * (g[k][i] * dchi[j] + g[k][j] * dchi[i]);
            }
            Gd[i][j] = gd;
            zs[i][j] = z;
            double r = 0.5 * ic * ddc[i][j] - 0.5 * ic * gd - 0.25 * ic * ic * dchi[i] * dchi[j] + 2.0 * ic * ic * z +
                       0.5 * ic * g[i][j] * (trc - Ghd);
            r += -0.5 * lapg[SI(i, j)];
            for (int k = 0; k < 3; ++k) {
                r += 0.5 * (g[k][i] * dGh[j][k] + g[k][j] * dGh[i][k]);
                r += Gh[k] * 0.5 * (Gl[i][j][k] + Gl[j][i][k]);
            }
            for (int m = 0; m < 3; ++m)
                for (int n = 0; n < 3; ++n)
                    for (int k = 0; k < 3; ++k)
                        r += gu[m][n] * (Gu[k][m][i] * Gl[j][k][n] + Gu[k][m][j] * Gl[i][k][n] + Gu[k][m][i] * Gl[k][n][j]);
            Ric[i][j] = Ric[j][i] = r;
            Gd[j][i] = gd;
            zs[j][i] = z;
        }
    double cr = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) cr += gu[k][m] * dalp[k] * dchi[m];
    const double hic = 0.5 * ic;
    double DDa[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            DDa[i][j] = dda[i][j] - (Gu[0][i][j] * dalp[0] + Gu[1][i][j] * dalp[1] + Gu[2][i][j] * dalp[2]) +
                        hic * (dalp[i] * dchi[j] + dalp[j] * dchi[i] - g[i][j] * cr);
    double Am[3][3], Au[3][3], trA = 0.0, AA = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Am[i][j] = gu[i][0] * A[0][j] + gu[i][1] * A[1][j] + gu[i][2] * A[2][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Au[i][j] = Am[i][0] * gu[0][j] + Am[i][1] * gu[1][j] + Am[i][2] * gu[2][j];
    for (int i = 0; i < 3; ++i) {
        trA += Am[i][i];
        for (int j = 0; j < 3; ++j) AA += A[i][j] * Au[i][j];
    }
    double X[3][3], trX = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X[i][j] = alp * Ric[i][j] - DDa[i][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) trX += gu[i][j] * X[i][j];
    const double divb = db[0][0] + db[1][1] + db[2][2];
    const double Kt = Kh + 2.0 * Th;
    double gdiv[3];
    for (int l = 0; l < 3; ++l) gdiv[l] = ddb[0][0][l] + ddb[1][1][l] + ddb[2][2][l];
    double b1[3], rG[3], b2[3];
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += Gu[i][j][k] * Au[j][k];
        for (int j = 0; j < 3; ++j) s += -1.5 * ic * Au[i][j] * dchi[j];
        b1[i] = s;
        double r = 0.0;
        for (int j = 0; j < 3; ++j) r += -(2.0 / 3.0) * gu[i][j] * dKh[j] - gu[i][j] * ((1.0 / 3.0) * dTh[j] + Th / alp * dalp[j]);
        rG[i] = r;
        b2[i] = -Z[i] * ic * (C.kz + (2.0 / 3.0) * Kt);
    }

    // ---- reverse sweep ----
    double lGT[3][3], lAT[3][3], lGH[3], lBB[3], lBE[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            lGT[i][j] = lm[(int64_t)(GT + SI(i, j)) * fs];
            lAT[i][j] = lm[(int64_t)(AT + SI(i, j)) * fs];
        }
    for (int i = 0; i < 3; ++i) {
        lGH[i] = lm[(int64_t)(GH + i) * fs];
        lBB[i] = lm[(int64_t)(BB + i) * fs];
        lBE[i] = lm[(int64_t)(BETA + i) * fs];
    }
    const double lCHI = lm[(int64_t)CHI * fs], lKH = lm[(int64_t)KH * fs], lTH = lm[(int64_t)TH * fs],
                 lALP = lm[(int64_t)ALP * fs];

    double a_g[3][3] = {}, a_A[3][3] = {}, a_gu[3][3] = {}, a_Gl[3][3][3] = {}, a_Gu[3][3][3] = {};
    double a_Ric[3][3] = {}, a_DDa[3][3] = {}, a_Am[3][3] = {}, a_Au[3][3] = {}, a_X[3][3] = {};
    double a_dg[3][3][3] = {}, a_dGh[3][3] = {}, a_db[3][3] = {}, a_ddc[3][3] = {}, a_dda[3][3] = {}, a_ddb[3][3][3] = {};
    double a_lapg[6] = {};
    double a_chi = 0.0, a_Kh = 0.0, a_Th = 0.0, a_alp = 0.0, a_ic = 0.0, a_lndet = 0.0, a_trA = 0.0, a_AA = 0.0;
    double a_divb = 0.0, a_Zda = 0.0, a_Kt = 0.0, a_trX = 0.0, a_trRic = 0.0, a_lapa = 0.0;
    double a_Gh[3] = {}, a_Bv[3] = {}, a_Z[3] = {}, a_dchi[3] = {}, a_dalp[3] = {}, a_dKh[3] = {}, a_dTh[3] = {};
    double a_gdiv[3] = {}, a_gddb[3] = {};

    // (7) alpha: -(f0 alp^2 + f1 alp) Kh
    a_alp += -(2.0 * C.f0 * alp + C.f1) * Kh * lALP;
    a_Kh += -(C.f0 * alp * alp + C.f1 * alp) * lALP;
    // (6) beta^i = g B^i; B^i = -eta B^i + S_i; Ghat^i = S_i
    for (int i = 0; i < 3; ++i) {
        a_Bv[i] += C.g * lBE[i] - C.eta * lBB[i];
        const double aS = lGH[i] + lBB[i];
        a_Gh[i] += (2.0 / 3.0) * divb * aS;
        a_divb += (2.0 / 3.0) * Gh[i] * aS;
        a_gddb[i] += aS;
        for (int j = 0; j < 3; ++j) {
            a_Gh[j] += -db[j][i] * aS;
            a_db[j][i] += -Gh[j] * aS;
            a_gu[i][j] += (1.0 / 3.0) * gdiv[j] * aS;
            a_gdiv[j] += (1.0 / 3.0) * gu[i][j] * aS;
            a_Au[i][j] += -2.0 * dalp[j] * aS;
            a_dalp[j] += -2.0 * Au[i][j] * aS;
        }
        a_alp += 2.0 * (b1[i] + rG[i] + b2[i]) * aS;
        const double ab = 2.0 * alp * aS;  // adjoint of b1, rG and b2
        // b1
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                a_Gu[i][j][k] += Au[j][k] * ab;
                a_Au[j][k] += Gu[i][j][k] * ab;
            }
        for (int j = 0; j < 3; ++j) {
            a_ic += -1.5 * Au[i][j] * dchi[j] * ab;
            a_Au[i][j] += -1.5 * ic * dchi[j] * ab;
            a_dchi[j] += -1.5 * ic * Au[i][j] * ab;
        }
        // rG
        for (int j = 0; j < 3; ++j) {
            a_gu[i][j] += (-(2.0 / 3.0) * dKh[j] - (1.0 / 3.0) * dTh[j] - Th / alp * dalp[j]) * ab;
            a_dKh[j] += -(2.0 / 3.0) * gu[i][j] * ab;
            a_dTh[j] += -(1.0 / 3.0) * gu[i][j] * ab;
            a_dalp[j] += -gu[i][j] * Th / alp * ab;
            a_Th += -gu[i][j] * dalp[j] / alp * ab;
            a_alp += gu[i][j] * Th * dalp[j] / (alp * alp) * ab;
        }
        // b2
        a_Z[i] += -ic * (C.kz + (2.0 / 3.0) * Kt) * ab;
        a_ic += -Z[i] * (C.kz + (2.0 / 3.0) * Kt) * ab;
        a_Kt += -Z[i] * ic * (2.0 / 3.0) * ab;
    }
    // (5) Theta
    {
        double trRic = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) trRic += chi * gu[i][j] * Ric[i][j];
        const double Zda = Z[0] * dalp[0] + Z[1] * dalp[1] + Z[2] * dalp[2];
        a_alp += (0.5 * (trRic + (2.0 / 3.0) * Kh * Kh + (2.0 / 3.0) * Th * (Kh - 2.0 * Th) - AA) - 2.0 * C.kz * Th) * lTH;
        a_trRic += 0.5 * alp * lTH;
        a_Kh += 0.5 * alp * ((4.0 / 3.0) * Kh + (2.0 / 3.0) * Th) * lTH;
        a_Th += (0.5 * alp * (2.0 / 3.0) * (Kh - 4.0 * Th) - 2.0 * alp * C.kz) * lTH;
        a_AA += -0.5 * alp * lTH;
        a_Zda += -lTH;
        // (4) Khat
        a_lapa += -lKH;
        a_alp += ((1.0 / 3.0) * Kt * Kt + AA + C.kz * Th) * lKH;
        a_Kt += alp * (2.0 / 3.0) * Kt * lKH;
        a_AA += alp * lKH;
        a_Th += alp * C.kz * lKH;
        a_Zda += 2.0 * lKH;
        (void)Zda;
    }
    // (3) chi
    a_chi += (2.0 / 3.0) * (alp * Kt - divb) * lCHI;
    a_alp += (2.0 / 3.0) * chi * Kt * lCHI;
    a_Kt += (2.0 / 3.0) * chi * alp * lCHI;
    a_divb += -(2.0 / 3.0) * chi * lCHI;
    // (2) At_ij and (1) gt_ij, i <= j
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const double la = lAT[i][j], lg = lGT[i][j];
            double AAm = 0.0;
            for (int k = 0; k < 3; ++k) AAm += A[i][k] * Am[k][j];
            for (int k = 0; k < 3; ++k) {
                a_A[i][k] += db[j][k] * la;
                a_db[j][k] += A[i][k] * la;
                a_A[k][j] += db[i][k] * la;
                a_db[i][k] += A[k][j] * la;
                a_g[i][k] += db[j][k] * lg;
                a_db[j][k] += g[i][k] * lg;
                a_g[k][j] += db[i][k] * lg;
                a_db[i][k] += g[k][j] * lg;
                a_A[i][k] += -2.0 * alp * Am[k][j] * la;
                a_Am[k][j] += -2.0 * alp * A[i][k] * la;
            }
            a_A[i][j] += -(2.0 / 3.0) * divb * la + alp * Kh * la;
            a_divb += -(2.0 / 3.0) * A[i][j] * la - (2.0 / 3.0) * g[i][j] * lg;
            a_alp += -(C.kc / 3.0) * g[i][j] * trA * la + (Kh * A[i][j] - 2.0 * AAm) * la;
            a_g[i][j] += -(C.kc / 3.0) * alp * trA * la - (1.0 / 3.0) * chi * trX * la;
            a_trA += -(C.kc / 3.0) * alp * g[i][j] * la;
            a_chi += (X[i][j] - (1.0 / 3.0) * g[i][j] * trX) * la;
            a_X[i][j] += chi * la;
            a_trX += -(1.0 / 3.0) * chi * g[i][j] * la;
            a_Kh += alp * A[i][j] * la;
            // gt
            a_g[i][j] += -(2.0 / 3.0) * divb * lg + (2.0 / 3.0) * alp * trA * lg - (C.kc / 3.0) * alp * lndet * lg;
            a_alp += -2.0 * (A[i][j] - (1.0 / 3.0) * g[i][j] * trA) * lg - (C.kc / 3.0) * g[i][j] * lndet * lg;
            a_A[i][j] += -2.0 * alp * lg;
            a_trA += (2.0 / 3.0) * alp * g[i][j] * lg;
            a_lndet += -(C.kc / 3.0) * alp * g[i][j] * lg;
        }
    // trX, X
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a_gu[i][j] += X[i][j] * a_trX;
            a_X[i][j] += gu[i][j] * a_trX;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a_alp += Ric[i][j] * a_X[i][j];
            a_Ric[i][j] += alp * a_X[i][j];
            a_DDa[i][j] += -a_X[i][j];
        }
    // Kt, Zda, divb, AA, trA, Au, Am
    a_Kh += a_Kt;
    a_Th += 2.0 * a_Kt;
    for (int i = 0; i < 3; ++i) {
        a_Z[i] += dalp[i] * a_Zda;
        a_dalp[i] += Z[i] * a_Zda;
        a_db[i][i] += a_divb;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a_A[i][j] += Au[i][j] * a_AA;
            a_Au[i][j] += A[i][j] * a_AA;
        }
    for (int i = 0; i < 3; ++i) a_Am[i][i] += a_trA;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) {
                a_Am[i][l] += gu[l][j] * a_Au[i][j];
                a_gu[l][j] += Am[i][l] * a_Au[i][j];
            }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) {
                a_gu[i][l] += A[l][j] * a_Am[i][j];
                a_A[l][j] += gu[i][l] * a_Am[i][j];
            }
    // lapa = chi gu.DDa, trRic = chi gu.Ric
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a_chi += gu[i][j] * (DDa[i][j] * a_lapa + Ric[i][j] * a_trRic);
            a_gu[i][j] += chi * (DDa[i][j] * a_lapa + Ric[i][j] * a_trRic);
            a_DDa[i][j] += chi * gu[i][j] * a_lapa;
            a_Ric[i][j] += chi * gu[i][j] * a_trRic;
        }
    // gddb, gdiv
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
                a_gu[k][l] += ddb[i][k][l] * a_gddb[i];
                a_ddb[i][k][l] += gu[k][l] * a_gddb[i];
            }
    for (int l = 0; l < 3; ++l)
        for (int i = 0; i < 3; ++i) a_ddb[i][i][l] += a_gdiv[l];
    // DDa
    {
        double a_cr = 0.0, a_hic = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double a = a_DDa[i][j];
                a_dda[i][j] += a;
                for (int k = 0; k < 3; ++k) {
                    a_Gu[k][i][j] += -dalp[k] * a;
                    a_dalp[k] += -Gu[k][i][j] * a;
                }
                a_hic += (dalp[i] * dchi[j] + dalp[j] * dchi[i] - g[i][j] * cr) * a;
                a_dalp[i] += hic * dchi[j] * a;
                a_dchi[j] += hic * dalp[i] * a;
                a_dalp[j] += hic * dchi[i] * a;
                a_dchi[i] += hic * dalp[j] * a;
                a_g[i][j] += -hic * cr * a;
                a_cr += -hic * g[i][j] * a;
            }
        for (int k = 0; k < 3; ++k)
            for (int m = 0; m < 3; ++m) {
                a_gu[k][m] += dalp[k] * dchi[m] * a_cr;
                a_dalp[k] += gu[k][m] * dchi[m] * a_cr;
                a_dchi[m] += gu[k][m] * dalp[k] * a_cr;
            }
        a_ic += 0.5 * a_hic;
    }
    // Ric = Rh + Rchi (computed once per pair i <= j)
    {
        double a_trc = 0.0, a_Ghd = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                const double a = i == j ? a_Ric[i][i] : a_Ric[i][j] + a_Ric[j][i];
                // Rchi
                a_ic += (0.5 * ddc[i][j] - 0.5 * Gd[i][j] - 0.5 * ic * dchi[i] * dchi[j] + 4.0 * ic * zs[i][j] +
                         0.5 * g[i][j] * (trc - Ghd)) * a;
                a_ddc[i][j] += 0.5 * ic * a;
                a_dchi[i] += -0.25 * ic * ic * dchi[j] * a;
                a_dchi[j] += -0.25 * ic * ic * dchi[i] * a;
                a_g[i][j] += 0.5 * ic * (trc - Ghd) * a;
                a_trc += 0.5 * ic * g[i][j] * a;
                a_Ghd += -0.5 * ic * g[i][j] * a;
                const double aGd = -0.5 * ic * a, azs = 2.0 * ic * ic * a;
                for (int k = 0; k < 3; ++k) {
                    a_Gu[k][i][j] += dchi[k] * aGd;
                    a_dchi[k] += Gu[k][i][j] * aGd;
                    a_Z[k] += 0.5 * (g[k][i] * dchi[j] + g[k][j] * dchi[i]) * azs;
                    a_g[k][i] += 0.5 * Z[k] * dchi[j] * azs;
                    a_dchi[j] += 0.5 * Z[k] * g[k][i] * azs;
                    a_g[k][j] += 0.5 * Z[k] * dchi[i] * azs;
                    a_dchi[i] += 0.5 * Z[k] * g[k][j] * azs;
                }
                // Rh
                a_lapg[SI(i, j)] += -0.5 * a;
                for (int k = 0; k < 3; ++k) {
                    a_g[k][i] += 0.5 * dGh[j][k] * a;
                    a_dGh[j][k] += 0.5 * g[k][i] * a;
                    a_g[k][j] += 0.5 * dGh[i][k] * a;
                    a_dGh[i][k] += 0.5 * g[k][j] * a;
                    a_Gh[k] += 0.5 * (Gl[i][j][k] + Gl[j][i][k]) * a;
                    a_Gl[i][j][k] += 0.5 * Gh[k] * a;
                    a_Gl[j][i][k] += 0.5 * Gh[k] * a;
                }
                for (int m = 0; m < 3; ++m)
                    for (int n = 0; n < 3; ++n)
                        for (int k = 0; k < 3; ++k) {
                            a_gu[m][n] += (Gu[k][m][i] * Gl[j][k][n] + Gu[k][m][j] * Gl[i][k][n] + Gu[k][m][i] * Gl[k][n][j]) * a;
                            a_Gu[k][m][i] += gu[m][n] * (Gl[j][k][n] + Gl[k][n][j]) * a;
                            a_Gu[k][m][j] += gu[m][n] * Gl[i][k][n] * a;
                            a_Gl[j][k][n] += gu[m][n] * Gu[k][m][i] * a;
                            a_Gl[i][k][n] += gu[m][n] * Gu[k][m][j] * a;
                            a_Gl[k][n][j] += gu[m][n] * Gu[k][m][i] * a;
                        }
            }
        // lapg[q] = gt^{mn} d_m d_n gt_q: the second derivatives go to the
        // workspace now (packed pairs), gt^{mn} collects the rest
        for (int q = 0; q < 6; ++q)
            for (int m = 0; m < 3; ++m)
                for (int n = m; n < 3; ++n) {
                    const double v = dd(GT + q, m, n);
                    a_gu[m][n] += v * a_lapg[q];
                    if (m != n) a_gu[n][m] += v * a_lapg[q];
                    w[(int64_t)(W_D2 + 6 * d2_slot(GT + q) + SI(m, n)) * fs] = (m == n ? 1.0 : 2.0) * gu[m][n] * a_lapg[q];
                }
        for (int k = 0; k < 3; ++k)
            for (int m = 0; m < 3; ++m) {
                a_gu[k][m] += (ddc[k][m] - 1.5 * ic * dchi[k] * dchi[m]) * a_trc;
                a_ddc[k][m] += gu[k][m] * a_trc;
                a_ic += -1.5 * gu[k][m] * dchi[k] * dchi[m] * a_trc;
                a_dchi[k] += -1.5 * ic * gu[k][m] * dchi[m] * a_trc;
                a_dchi[m] += -1.5 * ic * gu[k][m] * dchi[k] * a_trc;
            }
        for (int k = 0; k < 3; ++k) {
            a_Gh[k] += dchi[k] * a_Ghd;
            a_dchi[k] += Gh[k] * a_Ghd;
        }
    }
    // Z = chi (Ghat - Gc) / 2, Gc = gu.Gu
    for (int i = 0; i < 3; ++i) {
        a_chi += 0.5 * (Gh[i] - Gc[i]) * a_Z[i];
        a_Gh[i] += 0.5 * chi * a_Z[i];
        const double aGc = -0.5 * chi * a_Z[i];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                a_gu[j][k] += Gu[i][j][k] * aGc;
                a_Gu[i][j][k] += gu[j][k] * aGc;
            }
    }
    // Gu = gu Gl
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    a_gu[i][l] += Gl[l][j][k] * a_Gu[i][j][k];
                    a_Gl[l][j][k] += gu[i][l] * a_Gu[i][j][k];
                }
    // Gl from dg
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                a_dg[j][i][k] += 0.5 * a_Gl[i][j][k];
                a_dg[k][i][j] += 0.5 * a_Gl[i][j][k];
                a_dg[i][j][k] += -0.5 * a_Gl[i][j][k];
            }
    // lndet, gu = g^-1, ic = 1/chi
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s += gu[i][a] * a_gu[a][b] * gu[b][j];
            a_g[i][j] += gu[i][j] * a_lndet - s;
        }
    a_chi += -ic * ic * a_ic;

    // advection: d/d beta^k of sum_f lam_f beta^k L_k u_f
    double a_be[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < NF; ++f) {
        const double lf = lm[(int64_t)f * fs];
        for (int k = 0; k < 3; ++k)
            a_be[k] += lf * C.i12h * (C.upwind ? fadv(F(f), S[k], be[k]) : fd1(F(f), S[k]));
    }

    // ---- write Pbar(c) ----
    auto put = [&](int q, double v) { w[(int64_t)q * fs] = v; };
    auto sym = [&](const double (&a)[3][3], int i, int j) { return i == j ? a[i][i] : a[i][j] + a[j][i]; };
    put(W_U + CHI, a_chi);
    put(W_U + KH, a_Kh);
    put(W_U + TH, a_Th);
    put(W_U + ALP, a_alp);
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            put(W_U + GT + SI(i, j), sym(a_g, i, j));
            put(W_U + AT + SI(i, j), sym(a_A, i, j));
        }
    for (int i = 0; i < 3; ++i) {
        put(W_U + GH + i, a_Gh[i]);
        put(W_U + BETA + i, a_be[i]);
        put(W_U + BB + i, a_Bv[i]);
    }
    for (int k = 0; k < 3; ++k) {
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) put(W_D1 + 3 * d1_slot(GT + SI(i, j)) + k, sym(a_dg[k], i, j));
        put(W_D1 + 3 * d1_slot(CHI) + k, a_dchi[k]);
        put(W_D1 + 3 * d1_slot(ALP) + k, a_dalp[k]);
        put(W_D1 + 3 * d1_slot(KH) + k, a_dKh[k]);
        put(W_D1 + 3 * d1_slot(TH) + k, a_dTh[k]);
        for (int i = 0; i < 3; ++i) {
            put(W_D1 + 3 * d1_slot(GH + i) + k, a_dGh[k][i]);
            put(W_D1 + 3 * d1_slot(BETA + i) + k, a_db[k][i]);
        }
    }
    for (int k = 0; k < 3; ++k)
        for (int l = k; l < 3; ++l) {
            const int m = SI(k, l);
            put(W_D2 + 6 * d2_slot(CHI) + m, sym(a_ddc, k, l));
            put(W_D2 + 6 * d2_slot(ALP) + m, sym(a_dda, k, l));
            for (int i = 0; i < 3; ++i) put(W_D2 + 6 * d2_slot(BETA + i) + m, sym(a_ddb[i], k, l));
        }
}

// ---------------------------------------------------------------- kernel 2
__global__ __launch_bounds__(256) void ccz4_adj_gather_kernel(const PatchDev* __restrict__ patches,
                                                              const Tile* __restrict__ tiles,
                                                              const double* __restrict__ Ug,
                                                              const double* __restrict__ lamg,
                                                              const double* __restrict__ W,
                                                              const int64_t* __restrict__ wofs, AdjConst C,
                                                              double* __restrict__ lamU)
{
    const Tile t = tiles[blockIdx.x];
    const PatchDev P = patches[t.patch];
    const int q[3] = {t.o[0] + (int)threadIdx.x, t.o[1] + (int)threadIdx.y, t.o[2] + (int)threadIdx.z};
    if (q[0] >= P.n[0] + G || q[1] >= P.n[1] + G || q[2] >= P.n[2] + G) return;
    const int64_t loc = (int64_t)(q[2] + G) * P.pitch_z + (int64_t)(q[1] + G) * P.pitch_y + (q[0] + G);
    const int64_t fs = P.fs;
    const int S[3] = {1, P.pitch_y, P.pitch_z};
    const double* lp = lamg + P.off + loc;
    const double* bp = Ug + P.off + loc + (int64_t)BETA * fs;
    const double* wp = W + wofs[t.patch] + loc;
    // c = p + off along axis d (and e along axis d2) is an interior point
    auto inside = [&](int d, int off, int d2 = 0, int e = 0) {
        int c[3] = {q[0], q[1], q[2]};
        c[d] += off;
        c[d2] += e;
        return c[0] >= 0 && c[0] < P.n[0] && c[1] >= 0 && c[1] < P.n[1] && c[2] >= 0 && c[2] < P.n[2];
    };
    const bool self = inside(0, 0);
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};   // D1: coefficient of u(c+o), o = -2..2
    const double w2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    const double wko[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};
    const double wlp[7] = {0.0, 0.0, -3.0, -10.0, 18.0, -6.0, 1.0};  // beta >= 0: o = -3..3
    const double wlm[7] = {-1.0, 6.0, -18.0, 10.0, 3.0, 0.0, 0.0};   // beta < 0
    double acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = self ? wp[(int64_t)(W_U + f) * fs] : 0.0;
    // u(p) enters the stencils of the interior points c = p - o e_k
    for (int k = 0; k < 3; ++k)
        for (int o = -3; o <= 3; ++o) {
            if (!inside(k, -o)) continue;
            const int64_t cof = -(int64_t)o * S[k];
            const double bk = bp[(int64_t)k * fs + cof];
            const double wa = C.upwind ? (bk >= 0.0 ? wlp[o + 3] : wlm[o + 3]) : (o >= -2 && o <= 2 ? w1[o + 2] : 0.0);
            // KO and advection act on lam of every field
            const double wl = C.ko * wko[o + 3] + C.i12h * wa * bk;
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] += wl * lp[(int64_t)f * fs + cof];
            if (o < -2 || o > 2) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int s1 = d1_slot(f), s2 = d2_slot(f);
                if (s1 >= 0) acc[f] += C.i12h * w1[o + 2] * wp[(int64_t)(W_D1 + 3 * s1 + k) * fs + cof];
                if (s2 >= 0) acc[f] += C.i12h2 * w2[o + 2] * wp[(int64_t)(W_D2 + 6 * s2 + SI(k, k)) * fs + cof];
            }
        }
    for (int k = 0; k < 3; ++k)
        for (int l = k + 1; l < 3; ++l)
            for (int a = -2; a <= 2; ++a)
                for (int b = -2; b <= 2; ++b) {
                    if (a == 0 || b == 0 || !inside(k, -a, l, -b)) continue;
                    const int64_t cof = -(int64_t)a * S[k] - (int64_t)b * S[l];
                    const double wm = C.i144h2 * w1[a + 2] * w1[b + 2];
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        const int s2 = d2_slot(f);
                        if (s2 >= 0) acc[f] += wm * wp[(int64_t)(W_D2 + 6 * s2 + SI(k, l)) * fs + cof];
                    }
                }
#pragma unroll
    for (int f = 0; f < NF; ++f) lamU[P.off + loc + (int64_t)f * fs] = acc[f];
}

}  // namespace

int ccz4_adjoint_slots() { return NW; }

hipError_t launch_ccz4_adjoint(const SysParams& sp, const PatchDev* patches, const Tile* tiles, int ntiles,
                               const int td[3], const Tile* gtiles, int ngtiles, const int gtd[3],
                               const double* U, const double* lam, double* W, const int64_t* wofs, double* lamU,
                               hipStream_t s)
{
    AdjConst C;
    C.i12h = 1.0 / (12.0 * sp.h);
    C.i12h2 = 1.0 / (12.0 * sp.h * sp.h);
    C.i144h2 = 1.0 / (144.0 * sp.h * sp.h);
    C.ko = sp.sigma / (64.0 * sp.h);
    C.kz = sp.kappa_z;
    C.kc = sp.kappa_c;
    C.f0 = sp.bm_f0;
    C.f1 = sp.bm_f1;
    C.g = sp.gd_g;
    C.eta = sp.gd_eta;
    C.upwind = sp.upwind;
    if (ntiles > 0) {
        ccz4_adj_point_kernel<<<ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, ntiles, U, lam, W, wofs, C);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ngtiles > 0)
        ccz4_adj_gather_kernel<<<ngtiles, dim3(gtd[0], gtd[1], gtd[2]), 0, s>>>(patches, gtiles, U, lam, W, wofs, C, lamU);
    return hipGetLastError();
}

}  // namespace mol
