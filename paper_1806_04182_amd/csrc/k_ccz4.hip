// CCZ4 in vacuum (Sec. V): evolution of chi, gt_ij, trKhat, At_ij, Ghat^i,
// Theta (eqs. syseq1 .. syseq2 with the Ricci split and nabla_i nabla_j alpha
// printed below them), Bona-Masso slicing and Gamma-driver shift, with
// 4th-order centred derivatives, lop-sided advection and Kreiss-Oliger
// dissipation on every field (Sec. II.B.1), fused with the Runge-Kutta stage
// update.  One thread evaluates one grid point.
//
// Conventions: symmetric pairs are packed xx xy xz yy yz zz; Z^i =
// chi (Ghat^i - Gt^i)/2; R + 2 nabla Z and nabla^i nabla_i alpha are traces
// with the physical inverse metric chi gt^{ij}; [.]^TF is taken with gt;
// ln det gt = log1p(det(I + h) - 1) expanded in h = gt - I.
#include "k_common.h"

namespace mol {

namespace {

enum { CHI = 0, GT = 1, KH = 7, AT = 8, GH = 14, TH = 17, ALP = 18, BETA = 19, BB = 22, NF = 25 };

__device__ constexpr int SI(int i, int j)
{
    return i > j ? SI(j, i) : (i == 0 ? j : (i == 1 ? 2 + j : 5));
}

struct CczConst {
    double i12h;    // 1 / (12 h)
    double i12h2;   // 1 / (12 h^2)
    double i144h2;  // 1 / (144 h^2)
    double ko;      // sigma / (64 h)
    double kz, kc, f0, f1, g, eta;
    int upwind;
};

template <bool UPWIND>
__global__ __launch_bounds__(128) void ccz4_stage_kernel(StageArgs a, CczConst C)
{
    PointRef pr;
    int pi, pj, pk, pp;
    if (!tile_point(a, blockIdx.x, pr, pi, pj, pk, pp)) return;
    const double* __restrict__ u = a.Us + pr.c;
    const int64_t fs = pr.fs;
    const int s[3] = {1, pr.sy, pr.sz};
#define FLD(f) (u + (int64_t)(f) * fs)

    // ---- point values and the inverse conformal metric ----
    const double chi = FLD(CHI)[0], Kh = FLD(KH)[0], Th = FLD(TH)[0], alp = FLD(ALP)[0];
    double g[6], A[6], Gh[3], be[3], Bv[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        g[q] = FLD(GT + q)[0];
        A[q] = FLD(AT + q)[0];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Gh[i] = FLD(GH + i)[0];
        be[i] = FLD(BETA + i)[0];
        Bv[i] = FLD(BB + i)[0];
    }
    double gu[6], lndet;
    {
        const double hx = g[0] - 1.0, hy = g[3] - 1.0, hz = g[5] - 1.0;
        const double hxy = g[1], hxz = g[2], hyz = g[4];
        const double m2 = hx * hy - hxy * hxy + hx * hz - hxz * hxz + hy * hz - hyz * hyz;
        const double m3 = hx * (hy * hz - hyz * hyz) - hxy * (hxy * hz - hyz * hxz) + hxz * (hxy * hyz - hy * hxz);
        const double dm = (hx + hy + hz) + m2 + m3;
        lndet = log1p(dm);
        const double idet = 1.0 / (1.0 + dm);
        gu[0] = (g[3] * g[5] - g[4] * g[4]) * idet;
        gu[1] = (g[2] * g[4] - g[1] * g[5]) * idet;
        gu[2] = (g[1] * g[4] - g[2] * g[3]) * idet;
        gu[3] = (g[0] * g[5] - g[2] * g[2]) * idet;
        gu[4] = (g[2] * g[1] - g[0] * g[4]) * idet;
        gu[5] = (g[0] * g[3] - g[1] * g[1]) * idet;
    }

    // ---- first derivatives ----
    double dchi[3], dalp[3], dK[3], dTh[3], db[3][3], dG[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dchi[k] = C.i12h * fd1(FLD(CHI), s[k]);
        dalp[k] = C.i12h * fd1(FLD(ALP), s[k]);
        dK[k] = C.i12h * fd1(FLD(KH), s[k]);
        dTh[k] = C.i12h * fd1(FLD(TH), s[k]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            db[k][i] = C.i12h * fd1(FLD(BETA + i), s[k]);
            dG[k][i] = C.i12h * fd1(FLD(GH + i), s[k]);
        }
    }
    // Christoffel symbols of gt: Gl[i][jk] = (d_j g_ik + d_k g_ij - d_i g_jk)/2,
    // Gu[i][jk] = gt^{il} Gl[l][jk], contracted Gc^i = gt^{jk} Gu[i][jk]
    double Gl[3][6], Gu[3][6], Gc[3];
    {
        double dg[3][6];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < 6; ++q) dg[k][q] = C.i12h * fd1(FLD(GT + q), s[k]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int k = j; k < 3; ++k)
                    Gl[i][SI(j, k)] = 0.5 * (dg[j][SI(i, k)] + dg[k][SI(i, j)] - dg[i][SI(j, k)]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int q = 0; q < 6; ++q)
            Gu[i][q] = gu[SI(i, 0)] * Gl[0][q] + gu[SI(i, 1)] * Gl[1][q] + gu[SI(i, 2)] * Gl[2][q];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        Gc[i] = gu[0] * Gu[i][0] + gu[3] * Gu[i][3] + gu[5] * Gu[i][5] +
                2.0 * (gu[1] * Gu[i][1] + gu[2] * Gu[i][2] + gu[4] * Gu[i][4]);
    double Z[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Z[i] = 0.5 * chi * (Gh[i] - Gc[i]);

    // ---- second derivatives, contracted as soon as possible ----
    double ddchi[6], ddalp[6], lapg[6], gddb[3], gdiv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = k; l < 3; ++l) {
            if (k == l) {
                ddchi[SI(k, k)] = C.i12h2 * fd2(FLD(CHI), s[k]);
                ddalp[SI(k, k)] = C.i12h2 * fd2(FLD(ALP), s[k]);
            } else {
                ddchi[SI(k, l)] = C.i144h2 * fmix(FLD(CHI), s[k], s[l]);
                ddalp[SI(k, l)] = C.i144h2 * fmix(FLD(ALP), s[k], s[l]);
            }
        }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double* w = FLD(GT + q);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = k; l < 3; ++l) {
                const double dd = k == l ? C.i12h2 * fd2(w, s[k]) : C.i144h2 * fmix(w, s[k], s[l]);
                acc += (k == l ? 1.0 : 2.0) * gu[SI(k, l)] * dd;
            }
        lapg[q] = acc;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) gdiv[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double* w = FLD(BETA + i);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = k; l < 3; ++l) {
                const double dd = k == l ? C.i12h2 * fd2(w, s[k]) : C.i144h2 * fmix(w, s[k], s[l]);
                acc += (k == l ? 1.0 : 2.0) * gu[SI(k, l)] * dd;
                // sum_k d_j d_k beta^k: beta^i contributes d_j d_i beta^i to row j
                if (k == i) gdiv[l] += dd;
                if (l == i && k != l) gdiv[k] += dd;
            }
        gddb[i] = acc;
    }

    // ---- Ricci tensor pieces ----
    double Ric[6];
    {
        // H[k][i][n] = sum_m gt^{nm} Gt^k_{mi}
        double H[3][3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int n = 0; n < 3; ++n)
                    H[k][i][n] = gu[SI(n, 0)] * Gu[k][SI(0, i)] + gu[SI(n, 1)] * Gu[k][SI(1, i)] +
                                 gu[SI(n, 2)] * Gu[k][SI(2, i)];
        double trdd = 0.0, Ghd = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Ghd += Gh[k] * dchi[k];
#pragma unroll
            for (int m = 0; m < 3; ++m)
                trdd += gu[SI(k, m)] * (ddchi[SI(k, m)] - 1.5 / chi * dchi[k] * dchi[m]);
        }
        const double ic = 1.0 / chi;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const int q = SI(i, j);
                // Rhat_ij
                double r = -0.5 * lapg[q];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    r += 0.5 * (g[SI(k, i)] * dG[j][k] + g[SI(k, j)] * dG[i][k]);
                    r += Gh[k] * 0.5 * (Gl[i][SI(j, k)] + Gl[j][SI(i, k)]);
#pragma unroll
                    for (int n = 0; n < 3; ++n)
                        r += H[k][i][n] * Gl[j][SI(k, n)] + H[k][j][n] * Gl[i][SI(k, n)] +
                             H[k][i][n] * Gl[k][SI(n, j)];
                }
                // Rhat^chi_ij
                double Gd = 0.0, zs = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Gd += Gu[k][q] * dchi[k];
                    zs += Z[k] * 0.5 * (g[SI(k, i)] * dchi[j] + g[SI(k, j)] * dchi[i]);
                }
                r += 0.5 * ic * ddchi[q] - 0.5 * ic * Gd - 0.25 * ic * ic * dchi[i] * dchi[j] +
                     2.0 * ic * ic * zs + 0.5 * ic * g[q] * (trdd - Ghd);
                Ric[q] = r;
            }
    }
    // nabla_i nabla_j alpha
    double DDa[6];
    {
        double cr = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m) cr += gu[SI(k, m)] * dalp[k] * dchi[m];
        const double hic = 0.5 / chi;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const int q = SI(i, j);
                DDa[q] = ddalp[q] - (Gu[0][q] * dalp[0] + Gu[1][q] * dalp[1] + Gu[2][q] * dalp[2]) +
                         hic * (dalp[i] * dchi[j] + dalp[j] * dchi[i] - g[q] * cr);
            }
    }
    auto tr = [&](const double* T) {  // gt^{ij} T_ij
        return gu[0] * T[0] + gu[3] * T[3] + gu[5] * T[5] + 2.0 * (gu[1] * T[1] + gu[2] * T[2] + gu[4] * T[4]);
    };
    const double trRic = chi * tr(Ric);
    const double lapa = chi * tr(DDa);
    // raised At
    double Am[3][3], Au[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Am[i][j] = gu[SI(i, 0)] * A[SI(0, j)] + gu[SI(i, 1)] * A[SI(1, j)] + gu[SI(i, 2)] * A[SI(2, j)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            Au[SI(i, j)] = Am[i][0] * gu[SI(0, j)] + Am[i][1] * gu[SI(1, j)] + Am[i][2] * gu[SI(2, j)];
    const double trA = Am[0][0] + Am[1][1] + Am[2][2];
    double AA = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) AA += A[SI(i, j)] * Au[SI(i, j)];
    const double divb = db[0][0] + db[1][1] + db[2][2];
    const double Zda = Z[0] * dalp[0] + Z[1] * dalp[1] + Z[2] * dalp[2];
    const double Kt = Kh + 2.0 * Th;

    double rhs[NF];
    // d_t gt_ij
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int q = SI(i, j);
            double r = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) r += g[SI(i, k)] * db[j][k] + g[SI(k, j)] * db[i][k];
            rhs[GT + q] = r - (2.0 / 3.0) * g[q] * divb - 2.0 * alp * (A[q] - (1.0 / 3.0) * g[q] * trA) -
                          (C.kc / 3.0) * alp * g[q] * lndet;
        }
    // d_t At_ij
    {
        double X[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) X[q] = alp * Ric[q] - DDa[q];
        const double trX = tr(X);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const int q = SI(i, j);
                double r = 0.0, aa = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    r += A[SI(i, k)] * db[j][k] + A[SI(k, j)] * db[i][k];
                    aa += A[SI(i, k)] * Am[k][j];
                }
                rhs[AT + q] = r - (2.0 / 3.0) * A[q] * divb - (C.kc / 3.0) * alp * g[q] * trA +
                              chi * (X[q] - (1.0 / 3.0) * g[q] * trX) + alp * (Kh * A[q] - 2.0 * aa);
            }
    }
    rhs[CHI] = (2.0 / 3.0) * chi * (alp * Kt - divb);
    rhs[KH] = -lapa + alp * ((1.0 / 3.0) * Kt * Kt + AA + C.kz * Th) + 2.0 * Zda;
    rhs[TH] = 0.5 * alp * (trRic + (2.0 / 3.0) * Kh * Kh + (2.0 / 3.0) * Th * (Kh - 2.0 * Th) - AA) - Zda -
              alp * (2.0 * C.kz * Th);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double r = (2.0 / 3.0) * Gh[i] * divb + gddb[i];
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r += -Gh[j] * db[j][i] + (1.0 / 3.0) * gu[SI(i, j)] * gdiv[j] - 2.0 * Au[SI(i, j)] * dalp[j];
            b1 += -1.5 / chi * Au[SI(i, j)] * dchi[j] - (2.0 / 3.0) * gu[SI(i, j)] * dK[j];
            b2 += -gu[SI(i, j)] * ((1.0 / 3.0) * dTh[j] + Th / alp * dalp[j]);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) b1 += (q == 0 || q == 3 || q == 5 ? 1.0 : 2.0) * Gu[i][q] * Au[q];
        b2 += -Z[i] / chi * (C.kz + (2.0 / 3.0) * Kt);
        r += 2.0 * alp * b1 + 2.0 * alp * b2;
        rhs[GH + i] = r;
        rhs[BB + i] = -C.eta * Bv[i] + r;  // d_t Ghat^i without its advection term
        rhs[BETA + i] = C.g * Bv[i];
    }
    rhs[ALP] = -alp * alp * (C.f0 + C.f1 / alp) * Kh;

    // ---- advection (every field) and KO dissipation, then the RK update ----
#pragma unroll 1
    for (int f = 0; f < NF; ++f) {
        const double* w = FLD(f);
        double adv = 0.0, ko = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            adv += be[k] * (UPWIND ? fadv(w, s[k], be[k]) : fd1(w, s[k]));
            ko += fko(w, s[k]);
        }
        stage_store(a, pr.c + (int64_t)f * fs, (rhs[f] + C.i12h * adv) + C.ko * ko);
    }
#undef FLD
}

}  // namespace

hipError_t launch_stage_ccz4(const SysParams& sp, const StageArgs& a, const int td[3], hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    CczConst C;
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
    dim3 blk(td[0], td[1], td[2]);
    if (sp.upwind)
        ccz4_stage_kernel<true><<<a.ntiles, blk, 0, s>>>(a, C);
    else
        ccz4_stage_kernel<false><<<a.ntiles, blk, 0, s>>>(a, C);
    return hipGetLastError();
}

}  // namespace mol
