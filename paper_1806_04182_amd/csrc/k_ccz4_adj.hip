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

// Further workspace slots, after the NW stencil-input adjoints: forward
// intermediates stored by the first kernel, then adjoints of intermediates
// handed from one kernel to the next.  Symmetric tensors are packed by SI;
// an adjoint of a packed component is the derivative with respect to that one
// variable (both orders of an off-diagonal pair together).
constexpr int F_GU = NW;              // inverse conformal metric gt^{ij} (6)
constexpr int F_GL = F_GU + 6;        // Gamma_{i jk}, packed in jk (18)
constexpr int F_GUU = F_GL + 18;      // Gamma^i_{jk}, packed in jk (18)
constexpr int F_Z = F_GUU + 18;       // Z^i (3)
constexpr int F_RIC = F_Z + 3;        // R_ij = Rt_ij + R^chi_ij (6)
constexpr int F_DDA = F_RIC + 6;      // D_i D_j alpha (6)
constexpr int F_LNDET = F_DDA + 6;    // ln det gt (1)
constexpr int F_DDG = F_LNDET + 1;    // d_m d_n gt_p, [p][mn packed] (36)
constexpr int F_DGH = F_DDG + 36;     // d_j Ghat^k, [j][k] (9)
constexpr int H_ARIC = F_DGH + 9;     // adjoint of R_ij (6)
constexpr int H_ADDA = H_ARIC + 6;    // adjoint of D_i D_j alpha (6)
constexpr int H_AGU = H_ADDA + 6;     // adjoint of gt^{ij} (6)
constexpr int H_AGUU = H_AGU + 6;     // adjoint of Gamma^i_{jk} (18)
constexpr int H_AZ = H_AGUU + 18;     // adjoint of Z^i (3)
constexpr int H_AGL = H_AZ + 3;       // adjoint of Gamma_{i jk} (18)
constexpr int NWX = H_AGL + 18;

// multiplicity of a packed pair in a full double sum, and its indices
__device__ constexpr double MU(int p) { return p == 0 || p == 3 || p == 5 ? 1.0 : 2.0; }
__device__ constexpr int PI_(int p) { return p < 3 ? 0 : (p < 5 ? 1 : 2); }
__device__ constexpr int PJ_(int p) { return p < 3 ? p : (p < 5 ? p - 2 : 2); }

// One interior point of a tile and its views of U, lam and the workspace.
struct Pt {
    const double* u;
    const double* lm;
    double* w;
    int64_t fs;
    int64_t wfs;  // slot stride of the workspace (interior-only layout)
    int S[3];
    __device__ double U(int f) const { return u[(int64_t)f * fs]; }
    __device__ double L(int f) const { return lm[(int64_t)f * fs]; }
    __device__ double& Wq(int q) const { return w[(int64_t)q * wfs]; }
    __device__ double d1(const AdjConst& C, int f, int k) const { return C.i12h * fd1(u + (int64_t)f * fs, S[k]); }
    __device__ double dd(const AdjConst& C, int f, int k, int l) const
    {
        const double* v = u + (int64_t)f * fs;
        return k == l ? C.i12h2 * fd2(v, S[k]) : C.i144h2 * fmix(v, S[k], S[l]);
    }
};

__device__ __forceinline__ bool pt_init(Pt& q, const PatchDev* __restrict__ patches, const Tile* __restrict__ tiles,
                                        const double* Ug, const double* lamg, double* W,
                                        const int64_t* __restrict__ wofs)
{
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const PatchDev P = patches[t.patch];
    const int ii = t.o[0] + threadIdx.x, jj = t.o[1] + threadIdx.y, kk = t.o[2] + threadIdx.z;
    if (ii >= P.n[0] || jj >= P.n[1] || kk >= P.n[2]) return false;
    const int64_t loc = (int64_t)(kk + G) * P.pitch_z + (int64_t)(jj + G) * P.pitch_y + (ii + G);
    q.fs = P.fs;
    q.u = Ug + P.off + loc;
    q.lm = lamg + P.off + loc;
    q.wfs = adj_wfs(P.n);
    q.w = W + wofs[t.patch] + ((int64_t)kk * P.n[1] + jj) * adj_wpitch(P.n[0]) + ii;
    q.S[0] = 1;
    q.S[1] = P.pitch_y;
    q.S[2] = P.pitch_z;
    return true;
}

// waves per SIMD the gauge reverse is held to: two cost it 116 bytes per
// lane of scratch; with the interior-only workspace one wave without
// scratch measured slightly faster (reverse RK4 step at 48^3 1.961 against
// 1.975 ms)
#ifndef MOL_ADJ_GAUGE_WAVES
#define MOL_ADJ_GAUGE_WAVES 1
#endif
#define ADJ_KERNEL2(name, waves)                                                                           \
    __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves))) void name(                \
        const PatchDev* __restrict__ patches, const Tile* __restrict__ tiles, const double* __restrict__ Ug,  \
        const double* __restrict__ lamg, double* __restrict__ W, const int64_t* __restrict__ wofs, AdjConst C)
#define ADJ_KERNEL(name)                                                                                   \
    __global__ __launch_bounds__(256) void name(const PatchDev* __restrict__ patches,                      \
                                                const Tile* __restrict__ tiles, const double* __restrict__ Ug, \
                                                const double* __restrict__ lamg, double* __restrict__ W,   \
                                                const int64_t* __restrict__ wofs, AdjConst C)

// inverse and ln det of the conformal metric (det expanded about the identity)
__device__ __forceinline__ void metric_inverse(const double g[6], double gu[6], double& lndet)
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

// ------------------------------------------------------------ kernel K0
// The derivative of the advection terms sum_f lam_f beta^k L_k u_f with
// respect to beta^k (first writer of those three slots).
__device__ __forceinline__ void advection_body(const Pt& q, const AdjConst& C)
{
    double be[3], a_be[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k) be[k] = q.U(BETA + k);
    for (int f = 0; f < NF; ++f) {
        const double lf = q.L(f);
        const double* v = q.u + (int64_t)f * q.fs;
        for (int k = 0; k < 3; ++k) a_be[k] += lf * (C.upwind ? fadv(v, q.S[k], be[k]) : fd1(v, q.S[k]));
    }
    for (int k = 0; k < 3; ++k) q.Wq(W_U + BETA + k) = C.i12h * a_be[k];
}
ADJ_KERNEL(ccz4_adj_advection_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    advection_body(q, C);
}

// The advection reverse runs inside the forward-intermediates kernel (after
// its stores) instead of as a launch of its own: 1 saves a launch and a
// pass over the points' stencil neighbourhoods of U.
#ifndef MOL_ADJ_FUSE_ADV
#define MOL_ADJ_FUSE_ADV 1
#endif

// ------------------------------------------------------------ kernel K1
// Forward intermediates (stored): inverse metric, Christoffel symbols, Z^i,
// ln det, d Ghat, D_iD_j alpha.  The Ricci tensor follows in K1b.
ADJ_KERNEL(ccz4_adj_forward_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    double g[6], gu[6], lndet;
    for (int p = 0; p < 6; ++p) g[p] = q.U(GT + p);
    metric_inverse(g, gu, lndet);
    const double chi = q.U(CHI), ic = 1.0 / chi;
    double Gh[3], dchi[3], dalp[3];
    for (int i = 0; i < 3; ++i) {
        Gh[i] = q.U(GH + i);
        dchi[i] = q.d1(C, CHI, i);
        dalp[i] = q.d1(C, ALP, i);
    }
    double Gl[3][6], Gu[3][6];
    {
        double dg[3][6];
        for (int k = 0; k < 3; ++k)
            for (int p = 0; p < 6; ++p) dg[k][p] = q.d1(C, GT + p, k);
        for (int i = 0; i < 3; ++i)
            for (int p = 0; p < 6; ++p) {
                const int j = PI_(p), k = PJ_(p);
                Gl[i][p] = 0.5 * (dg[j][SI(i, k)] + dg[k][SI(i, j)] - dg[i][p]);
            }
    }
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p)
            Gu[i][p] = gu[SI(i, 0)] * Gl[0][p] + gu[SI(i, 1)] * Gl[1][p] + gu[SI(i, 2)] * Gl[2][p];
    double Z[3];
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int p = 0; p < 6; ++p) s += MU(p) * gu[p] * Gu[i][p];
        Z[i] = 0.5 * chi * (Gh[i] - s);
    }
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) q.Wq(F_DGH + 3 * j + k) = q.d1(C, GH + k, j);
    // D_i D_j alpha
    {
        double cr = 0.0;
        for (int p = 0; p < 6; ++p)
            cr += gu[p] * (p == 0 || p == 3 || p == 5 ? dalp[PI_(p)] * dchi[PJ_(p)]
                                                      : dalp[PI_(p)] * dchi[PJ_(p)] + dalp[PJ_(p)] * dchi[PI_(p)]);
        const double hic = 0.5 * ic;
        for (int p = 0; p < 6; ++p) {
            const int i = PI_(p), j = PJ_(p);
            q.Wq(F_DDA + p) = q.dd(C, ALP, i, j) - (Gu[0][p] * dalp[0] + Gu[1][p] * dalp[1] + Gu[2][p] * dalp[2]) +
                              hic * (dalp[i] * dchi[j] + dalp[j] * dchi[i] - g[p] * cr);
        }
    }
    for (int p = 0; p < 6; ++p) q.Wq(F_GU + p) = gu[p];
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p) {
            q.Wq(F_GL + 6 * i + p) = Gl[i][p];
            q.Wq(F_GUU + 6 * i + p) = Gu[i][p];
        }
    for (int i = 0; i < 3; ++i) q.Wq(F_Z + i) = Z[i];
    q.Wq(F_LNDET) = lndet;
#if MOL_ADJ_FUSE_ADV
    advection_body(q, C);
#endif
}

// ------------------------------------------------------------ kernel K1b
// Forward intermediates (stored): the Ricci tensor R_ij = Rt_ij + R^chi_ij
// and the second derivatives of gt_ij, from the stored gt^{ij}, Gamma_ijk,
// Gamma^i_jk, Z^i and d Ghat (split from K1 so that each half holds two
// waves per SIMD).
// held to two waves per SIMD (20 bytes per lane of scratch): left alone the
// compiler takes 4 registers more than half the file and runs one wave
// (reverse RK4 step at 48^3 1.954 -> 1.926 ms)
ADJ_KERNEL2(ccz4_adj_ricci_fwd_kernel, 2)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    double g[6], gu[6];
    for (int p = 0; p < 6; ++p) {
        g[p] = q.U(GT + p);
        gu[p] = q.Wq(F_GU + p);
    }
    const double chi = q.U(CHI), ic = 1.0 / chi;
    double Gh[3], dchi[3], Z[3];
    for (int i = 0; i < 3; ++i) {
        Gh[i] = q.U(GH + i);
        dchi[i] = q.d1(C, CHI, i);
        Z[i] = q.Wq(F_Z + i);
    }
    double Gl[3][6];
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p) Gl[i][p] = q.Wq(F_GL + 6 * i + p);
    double ddc[6], trc = 0.0, Ghd = 0.0;
    for (int p = 0; p < 6; ++p) {
        ddc[p] = q.dd(C, CHI, PI_(p), PJ_(p));
        trc += MU(p) * gu[p] * (ddc[p] - 1.5 * ic * dchi[PI_(p)] * dchi[PJ_(p)]);
    }
    for (int k = 0; k < 3; ++k) Ghd += Gh[k] * dchi[k];
    // Gamma-Gamma terms through Q_i^{kn} = gt^{mn} Gamma^k_{mi}:
    // sum_kn Q_i^{kn} (Gamma_jkn + Gamma_knj) + Q_j^{kn} Gamma_ikn; and
    // gd_ij = Gamma^k_ij d_k chi.  Gamma^i_jk is needed for these only.
    double Q[3][3][3], gdv[6];
    {
        double Gu[3][6];
        for (int i = 0; i < 3; ++i)
            for (int p = 0; p < 6; ++p) Gu[i][p] = q.Wq(F_GUU + 6 * i + p);
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k)
                for (int n = 0; n < 3; ++n)
                    Q[i][k][n] = gu[SI(0, n)] * Gu[k][SI(0, i)] + gu[SI(1, n)] * Gu[k][SI(1, i)] + gu[SI(2, n)] * Gu[k][SI(2, i)];
        for (int p = 0; p < 6; ++p) {
            double gd = 0.0;
            for (int k = 0; k < 3; ++k) gd += Gu[k][p] * dchi[k];
            gdv[p] = gd;
        }
    }
    double dGh[3][3];  // [j][k] = d_j Ghat^k
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) dGh[j][k] = q.Wq(F_DGH + 3 * j + k);
    // Ricci tensor, one packed component at a time
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        const double gd = gdv[p];
        double zs = 0.0;
        for (int k = 0; k < 3; ++k) zs += Z[k] * 0.5 * (g[SI(k, i)] * dchi[j] + g[SI(k, j)] * dchi[i]);
        double lap = 0.0;
        for (int m = 0; m < 6; ++m) {
            const double v = q.dd(C, GT + p, PI_(m), PJ_(m));
            q.Wq(F_DDG + 6 * p + m) = v;
            lap += MU(m) * gu[m] * v;
        }
        double r = 0.5 * ic * ddc[p] - 0.5 * ic * gd - 0.25 * ic * ic * dchi[i] * dchi[j] + 2.0 * ic * ic * zs +
                   0.5 * ic * g[p] * (trc - Ghd) - 0.5 * lap;
        for (int k = 0; k < 3; ++k) {
            r += 0.5 * (g[SI(k, i)] * dGh[j][k] + g[SI(k, j)] * dGh[i][k]);
            r += Gh[k] * 0.5 * (Gl[i][SI(j, k)] + Gl[j][SI(i, k)]);
        }
        for (int k = 0; k < 3; ++k)
            for (int n = 0; n < 3; ++n)
                r += Q[i][k][n] * (Gl[j][SI(k, n)] + Gl[k][SI(n, j)]) + Q[j][k][n] * Gl[i][SI(k, n)];
        q.Wq(F_RIC + p) = r;
    }
}

// ------------------------------------------------------------ kernel K2
// Reverse of the gt_ij and At_ij equations, with X_ij = alpha R_ij - D_iD_j alpha,
// its trace, Am = gt^{-1} At, tr At and ln det gt.
ADJ_KERNEL(ccz4_adj_metric_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    double g[6], A[6], gu[6], X[6];
    for (int p = 0; p < 6; ++p) {
        g[p] = q.U(GT + p);
        A[p] = q.U(AT + p);
        gu[p] = q.Wq(F_GU + p);
    }
    const double alp = q.U(ALP), Kh = q.U(KH), chi = q.U(CHI), lndet = q.Wq(F_LNDET);
    double db[3][3];  // db[k][i] = d_k beta^i
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) db[k][i] = q.d1(C, BETA + i, k);
    const double divb = db[0][0] + db[1][1] + db[2][2];
    double Am[3][3], trA = 0.0, trX = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Am[i][j] = gu[SI(i, 0)] * A[SI(0, j)] + gu[SI(i, 1)] * A[SI(1, j)] + gu[SI(i, 2)] * A[SI(2, j)];
    for (int i = 0; i < 3; ++i) trA += Am[i][i];
    for (int p = 0; p < 6; ++p) {
        X[p] = alp * q.Wq(F_RIC + p) - q.Wq(F_DDA + p);
        trX += MU(p) * gu[p] * X[p];
    }
    double a_A[6] = {}, a_g[6] = {}, a_X[6] = {}, a_gu[6] = {}, a_db[3][3] = {}, a_Am[3][3] = {};
    double a_divb = 0.0, a_alp = 0.0, a_trA = 0.0, a_chi = 0.0, a_trX = 0.0, a_Kh = 0.0, a_lndet = 0.0;
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        const double la = q.L(AT + p), lg = q.L(GT + p);
        double AAm = 0.0;
        for (int k = 0; k < 3; ++k) AAm += A[SI(i, k)] * Am[k][j];
        for (int k = 0; k < 3; ++k) {
            a_A[SI(i, k)] += db[j][k] * la;
            a_db[j][k] += A[SI(i, k)] * la + g[SI(i, k)] * lg;
            a_A[SI(k, j)] += db[i][k] * la;
            a_db[i][k] += A[SI(k, j)] * la + g[SI(k, j)] * lg;
            a_g[SI(i, k)] += db[j][k] * lg;
            a_g[SI(k, j)] += db[i][k] * lg;
            a_A[SI(i, k)] += -2.0 * alp * Am[k][j] * la;
            a_Am[k][j] += -2.0 * alp * A[SI(i, k)] * la;
        }
        a_A[p] += (-(2.0 / 3.0) * divb + alp * Kh) * la - 2.0 * alp * lg;
        a_divb += -(2.0 / 3.0) * A[p] * la - (2.0 / 3.0) * g[p] * lg;
        a_alp += -(C.kc / 3.0) * g[p] * trA * la + (Kh * A[p] - 2.0 * AAm) * la;
        a_alp += -2.0 * (A[p] - (1.0 / 3.0) * g[p] * trA) * lg - (C.kc / 3.0) * g[p] * lndet * lg;
        a_g[p] += -(C.kc / 3.0) * alp * trA * la - (1.0 / 3.0) * chi * trX * la;
        a_g[p] += -(2.0 / 3.0) * divb * lg + (2.0 / 3.0) * alp * trA * lg - (C.kc / 3.0) * alp * lndet * lg;
        a_trA += -(C.kc / 3.0) * alp * g[p] * la + (2.0 / 3.0) * alp * g[p] * lg;
        a_chi += (X[p] - (1.0 / 3.0) * g[p] * trX) * la;
        a_X[p] += chi * la;
        a_trX += -(1.0 / 3.0) * chi * g[p] * la;
        a_Kh += alp * A[p] * la;
        a_lndet += -(C.kc / 3.0) * alp * g[p] * lg;
    }
    // trX = sum gt^{ij} X_ij; X = alpha R - DDa
    for (int p = 0; p < 6; ++p) {
        a_gu[p] += MU(p) * X[p] * a_trX;
        a_X[p] += MU(p) * gu[p] * a_trX;
        a_alp += q.Wq(F_RIC + p) * a_X[p];
    }
    // tr At = sum_i Am_ii; Am = gt^{-1} At
    for (int i = 0; i < 3; ++i) a_Am[i][i] += a_trA;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) {
                a_gu[SI(i, l)] += A[SI(l, j)] * a_Am[i][j];
                a_A[SI(l, j)] += gu[SI(i, l)] * a_Am[i][j];
            }
    // ln det gt; div beta
    for (int p = 0; p < 6; ++p) a_g[p] += MU(p) * gu[p] * a_lndet;
    for (int i = 0; i < 3; ++i) a_db[i][i] += a_divb;
    for (int p = 0; p < 6; ++p) {
        q.Wq(W_U + AT + p) = a_A[p];
        q.Wq(W_U + GT + p) = a_g[p];
        q.Wq(H_ARIC + p) = alp * a_X[p];
        q.Wq(H_ADDA + p) = -a_X[p];
        q.Wq(H_AGU + p) = a_gu[p];
    }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) q.Wq(W_D1 + 3 * d1_slot(BETA + i) + k) = a_db[k][i];
    q.Wq(W_U + CHI) = a_chi;
    q.Wq(W_U + KH) = a_Kh;
    q.Wq(W_U + ALP) = a_alp;
}

// ------------------------------------------------------------ kernel K3
// Reverse of the chi, Khat, Theta, Ghat^i, B^i, beta^i and alpha equations.
ADJ_KERNEL2(ccz4_adj_gauge_kernel, MOL_ADJ_GAUGE_WAVES)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    double A[6], gu[6];
    for (int p = 0; p < 6; ++p) {
        A[p] = q.U(AT + p);
        gu[p] = q.Wq(F_GU + p);
    }
    const double chi = q.U(CHI), Kh = q.U(KH), Th = q.U(TH), alp = q.U(ALP), ic = 1.0 / chi;
    const double Kt = Kh + 2.0 * Th;
    double Gh[3], Z[3], dalp[3], dchi[3], dKh[3], dTh[3];
    for (int i = 0; i < 3; ++i) {
        Gh[i] = q.U(GH + i);
        Z[i] = q.Wq(F_Z + i);
        dalp[i] = q.d1(C, ALP, i);
        dchi[i] = q.d1(C, CHI, i);
        dKh[i] = q.d1(C, KH, i);
        dTh[i] = q.d1(C, TH, i);
    }
    double db[3][3];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) db[k][i] = q.d1(C, BETA + i, k);
    const double divb = db[0][0] + db[1][1] + db[2][2];
    double Am[3][3], Au[6], AA = 0.0, trRic = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Am[i][j] = gu[SI(i, 0)] * A[SI(0, j)] + gu[SI(i, 1)] * A[SI(1, j)] + gu[SI(i, 2)] * A[SI(2, j)];
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        Au[p] = Am[i][0] * gu[SI(0, j)] + Am[i][1] * gu[SI(1, j)] + Am[i][2] * gu[SI(2, j)];
        AA += MU(p) * A[p] * Au[p];
        trRic += MU(p) * gu[p] * q.Wq(F_RIC + p);
    }
    trRic *= chi;

    double a_alp = 0.0, a_Kh = 0.0, a_Th = 0.0, a_chi = 0.0, a_Kt = 0.0, a_AA = 0.0, a_trRic = 0.0, a_lapa = 0.0;
    double a_Zda = 0.0, a_divb = 0.0, a_ic = 0.0;
    double a_Au[6] = {}, a_gu[6] = {}, a_Gh[3] = {}, a_dalp[3] = {}, a_dchi[3] = {}, a_Z[3] = {}, a_db[3][3] = {};
    {
        const double lALP = q.L(ALP), lKH = q.L(KH), lTH = q.L(TH), lCHI = q.L(CHI);
        // alpha: -(f0 alpha^2 + f1 alpha) Khat
        a_alp += -(2.0 * C.f0 * alp + C.f1) * Kh * lALP;
        a_Kh += -(C.f0 * alp * alp + C.f1 * alp) * lALP;
        // Theta
        a_alp += (0.5 * (trRic + (2.0 / 3.0) * Kh * Kh + (2.0 / 3.0) * Th * (Kh - 2.0 * Th) - AA) - 2.0 * C.kz * Th) * lTH;
        a_trRic += 0.5 * alp * lTH;
        a_Kh += 0.5 * alp * ((4.0 / 3.0) * Kh + (2.0 / 3.0) * Th) * lTH;
        a_Th += (0.5 * alp * (2.0 / 3.0) * (Kh - 4.0 * Th) - 2.0 * alp * C.kz) * lTH;
        a_AA += -0.5 * alp * lTH;
        a_Zda += -lTH;
        // Khat
        a_lapa += -lKH;
        a_alp += ((1.0 / 3.0) * Kt * Kt + AA + C.kz * Th) * lKH;
        a_Kt += alp * (2.0 / 3.0) * Kt * lKH;
        a_AA += alp * lKH;
        a_Th += alp * C.kz * lKH;
        a_Zda += 2.0 * lKH;
        // chi
        a_chi += (2.0 / 3.0) * (alp * Kt - divb) * lCHI;
        a_alp += (2.0 / 3.0) * chi * Kt * lCHI;
        a_Kt += (2.0 / 3.0) * chi * alp * lCHI;
        a_divb += -(2.0 / 3.0) * chi * lCHI;
    }
    // Ghat^i = S^i, B^i = S^i - eta B^i, beta^i = g B^i (the second
    // derivatives of beta in S^i are reversed by the shift kernel)
    double ab[3];
    for (int i = 0; i < 3; ++i) {
        q.Wq(W_U + BB + i) = C.g * q.L(BETA + i) - C.eta * q.L(BB + i);
        const double aS = q.L(GH + i) + q.L(BB + i);
        a_Gh[i] += (2.0 / 3.0) * divb * aS;
        a_divb += (2.0 / 3.0) * Gh[i] * aS;
        for (int j = 0; j < 3; ++j) {
            a_Gh[j] += -db[j][i] * aS;
            a_db[j][i] += -Gh[j] * aS;
            a_Au[SI(i, j)] += -2.0 * dalp[j] * aS;
            a_dalp[j] += -2.0 * Au[SI(i, j)] * aS;
        }
        ab[i] = 2.0 * alp * aS;
    }
    // 2 alpha (b1 + rG + b2)
    for (int i = 0; i < 3; ++i) {
        double b1 = 0.0, rG = 0.0;
        for (int p = 0; p < 6; ++p) b1 += MU(p) * q.Wq(F_GUU + 6 * i + p) * Au[p];
        for (int j = 0; j < 3; ++j) {
            b1 += -1.5 * ic * Au[SI(i, j)] * dchi[j];
            rG += -(2.0 / 3.0) * gu[SI(i, j)] * dKh[j] - gu[SI(i, j)] * ((1.0 / 3.0) * dTh[j] + Th / alp * dalp[j]);
        }
        const double b2 = -Z[i] * ic * (C.kz + (2.0 / 3.0) * Kt);
        a_alp += (b1 + rG + b2) * (q.L(GH + i) + q.L(BB + i)) * 2.0;
    }
    double a_dKh[3] = {}, a_dTh[3] = {};
    for (int i = 0; i < 3; ++i) {
        const double abi = ab[i];
        for (int p = 0; p < 6; ++p) {
            a_Au[p] += MU(p) * q.Wq(F_GUU + 6 * i + p) * abi;
            q.Wq(H_AGUU + 6 * i + p) = MU(p) * Au[p] * abi;
        }
        for (int j = 0; j < 3; ++j) {
            a_ic += -1.5 * Au[SI(i, j)] * dchi[j] * abi;
            a_Au[SI(i, j)] += -1.5 * ic * dchi[j] * abi;
            a_dchi[j] += -1.5 * ic * Au[SI(i, j)] * abi;
            a_gu[SI(i, j)] += (-(2.0 / 3.0) * dKh[j] - (1.0 / 3.0) * dTh[j] - Th / alp * dalp[j]) * abi;
            a_dKh[j] += -(2.0 / 3.0) * gu[SI(i, j)] * abi;
            a_dTh[j] += -(1.0 / 3.0) * gu[SI(i, j)] * abi;
            a_dalp[j] += -gu[SI(i, j)] * Th / alp * abi;
            a_Th += -gu[SI(i, j)] * dalp[j] / alp * abi;
            a_alp += gu[SI(i, j)] * Th * dalp[j] / (alp * alp) * abi;
        }
        a_Z[i] += -ic * (C.kz + (2.0 / 3.0) * Kt) * abi;
        a_ic += -Z[i] * (C.kz + (2.0 / 3.0) * Kt) * abi;
        a_Kt += -Z[i] * ic * (2.0 / 3.0) * abi;
    }
    a_Kh += a_Kt;
    a_Th += 2.0 * a_Kt;
    for (int i = 0; i < 3; ++i) {
        a_Z[i] += dalp[i] * a_Zda;
        a_dalp[i] += Z[i] * a_Zda;
        a_db[i][i] += a_divb;
    }
    // AA = At_ij At^ij; At^ij = Am gt^{-1}; Am = gt^{-1} At
    double a_A[6];
    for (int p = 0; p < 6; ++p) {
        a_A[p] = MU(p) * Au[p] * a_AA;
        a_Au[p] += MU(p) * A[p] * a_AA;
    }
    double a_Am[3][3] = {};
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        for (int l = 0; l < 3; ++l) {
            a_Am[i][l] += gu[SI(l, j)] * a_Au[p];
            a_gu[SI(l, j)] += Am[i][l] * a_Au[p];
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) {
                a_gu[SI(i, l)] += A[SI(l, j)] * a_Am[i][j];
                a_A[SI(l, j)] += gu[SI(i, l)] * a_Am[i][j];
            }
    // lapa = chi gt^{ij} D_iD_j alpha, trRic = chi gt^{ij} R_ij
    for (int p = 0; p < 6; ++p) {
        const double dda = q.Wq(F_DDA + p), ric = q.Wq(F_RIC + p);
        a_chi += MU(p) * gu[p] * (dda * a_lapa + ric * a_trRic);
        a_gu[p] += MU(p) * chi * (dda * a_lapa + ric * a_trRic);
        q.Wq(H_ADDA + p) += MU(p) * chi * gu[p] * a_lapa;
        q.Wq(H_ARIC + p) += MU(p) * chi * gu[p] * a_trRic;
        q.Wq(H_AGU + p) += a_gu[p];
        q.Wq(W_U + AT + p) += a_A[p];
    }
    a_chi += -ic * ic * a_ic;
    q.Wq(W_U + CHI) += a_chi;
    q.Wq(W_U + KH) += a_Kh;
    q.Wq(W_U + ALP) += a_alp;
    q.Wq(W_U + TH) = a_Th;
    for (int i = 0; i < 3; ++i) {
        q.Wq(W_U + GH + i) = a_Gh[i];
        q.Wq(H_AZ + i) = a_Z[i];
        q.Wq(W_D1 + 3 * d1_slot(ALP) + i) = a_dalp[i];
        q.Wq(W_D1 + 3 * d1_slot(CHI) + i) = a_dchi[i];
        q.Wq(W_D1 + 3 * d1_slot(KH) + i) = a_dKh[i];
        q.Wq(W_D1 + 3 * d1_slot(TH) + i) = a_dTh[i];
    }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) q.Wq(W_D1 + 3 * d1_slot(BETA + i) + k) += a_db[k][i];
}

// ------------------------------------------------------------ kernel K3b
// Reverse of the second-derivative terms of the shift in S^i:
// gt^{kl} d_k d_l beta^i + (1/3) gt^{ij} d_j d_k beta^k (first writer of the
// second-derivative slots of beta).
__device__ __forceinline__ void shift_body(const Pt& q, const AdjConst& C)
{
    double gu[6], aS[3], a_gu[6] = {};
    for (int p = 0; p < 6; ++p) gu[p] = q.Wq(F_GU + p);
    for (int i = 0; i < 3; ++i) aS[i] = q.L(GH + i) + q.L(BB + i);
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p) {
            a_gu[p] += MU(p) * q.dd(C, BETA + i, PI_(p), PJ_(p)) * aS[i];
            q.Wq(W_D2 + 6 * d2_slot(BETA + i) + p) = MU(p) * gu[p] * aS[i];
        }
    // gdiv[l] = d_l d_m beta^m enters S^i as (1/3) gt^{il} gdiv[l]
    for (int l = 0; l < 3; ++l) {
        double gdiv = 0.0, a = 0.0;
        for (int m = 0; m < 3; ++m) gdiv += q.dd(C, BETA + m, m, l);
        for (int i = 0; i < 3; ++i) {
            a_gu[SI(i, l)] += (1.0 / 3.0) * gdiv * aS[i];
            a += (1.0 / 3.0) * gu[SI(i, l)] * aS[i];
        }
        for (int m = 0; m < 3; ++m) q.Wq(W_D2 + 6 * d2_slot(BETA + m) + SI(m, l)) += a;
    }
    for (int p = 0; p < 6; ++p) q.Wq(H_AGU + p) += a_gu[p];
}
ADJ_KERNEL(ccz4_adj_shift_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    shift_body(q, C);
}

// ------------------------------------------------------------ kernel K4
// Reverse of D_iD_j alpha and of the chi part of the Ricci tensor
// (R^chi_ij, with the traces trc and Ghd).
__device__ __forceinline__ void chi_body(const Pt& q, const AdjConst& C)
{
    double g[6], gu[6], aR[6], aD[6];
    for (int p = 0; p < 6; ++p) {
        g[p] = q.U(GT + p);
        gu[p] = q.Wq(F_GU + p);
        aR[p] = q.Wq(H_ARIC + p);
        aD[p] = q.Wq(H_ADDA + p);
    }
    const double chi = q.U(CHI), ic = 1.0 / chi, hic = 0.5 * ic;
    double Gh[3], Z[3], dchi[3], dalp[3];
    for (int i = 0; i < 3; ++i) {
        Gh[i] = q.U(GH + i);
        Z[i] = q.Wq(F_Z + i);
        dchi[i] = q.d1(C, CHI, i);
        dalp[i] = q.d1(C, ALP, i);
    }
    double ddc[6], trc = 0.0, Ghd = 0.0, cr = 0.0;
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        ddc[p] = q.dd(C, CHI, i, j);
        trc += MU(p) * gu[p] * (ddc[p] - 1.5 * ic * dchi[i] * dchi[j]);
        cr += gu[p] * (i == j ? dalp[i] * dchi[j] : dalp[i] * dchi[j] + dalp[j] * dchi[i]);
    }
    for (int k = 0; k < 3; ++k) Ghd += Gh[k] * dchi[k];
    double a_g[6] = {}, a_gu[6] = {}, a_dchi[3] = {}, a_dalp[3] = {}, a_Z[3] = {};
    double a_ic = 0.0, a_hic = 0.0, a_cr = 0.0, a_trc = 0.0, a_Ghd = 0.0;
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        // D_iD_j alpha = dd alpha - Gamma^k_ij d_k alpha + (1/2chi)(d_i alpha d_j chi + d_j alpha d_i chi - gt_ij cr)
        const double a = aD[p];
        q.Wq(W_D2 + 6 * d2_slot(ALP) + p) = a;
        double Gd = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double Gkp = q.Wq(F_GUU + 6 * k + p);
            Gd += Gkp * dchi[k];
            a_dalp[k] += -Gkp * a;
        }
        a_hic += (dalp[i] * dchi[j] + dalp[j] * dchi[i] - g[p] * cr) * a;
        a_dalp[i] += hic * dchi[j] * a;
        a_dchi[j] += hic * dalp[i] * a;
        a_dalp[j] += hic * dchi[i] * a;
        a_dchi[i] += hic * dalp[j] * a;
        a_g[p] += -hic * cr * a;
        a_cr += -hic * g[p] * a;
        // R^chi_ij
        const double r = aR[p];
        double zs = 0.0;
        for (int k = 0; k < 3; ++k) zs += Z[k] * 0.5 * (g[SI(k, i)] * dchi[j] + g[SI(k, j)] * dchi[i]);
        a_ic += (0.5 * ddc[p] - 0.5 * Gd - 0.5 * ic * dchi[i] * dchi[j] + 4.0 * ic * zs + 0.5 * g[p] * (trc - Ghd)) * r;
        a_dchi[i] += -0.25 * ic * ic * dchi[j] * r;
        a_dchi[j] += -0.25 * ic * ic * dchi[i] * r;
        a_g[p] += 0.5 * ic * (trc - Ghd) * r;
        a_trc += 0.5 * ic * g[p] * r;
        a_Ghd += -0.5 * ic * g[p] * r;
        const double aGd = -0.5 * ic * r, azs = 2.0 * ic * ic * r;
        for (int k = 0; k < 3; ++k) {
            const double Gkp = q.Wq(F_GUU + 6 * k + p);
            // Gamma^k_ij enters D_iD_j alpha (-d_k alpha) and Gd (d_k chi)
            q.Wq(H_AGUU + 6 * k + p) += -dalp[k] * a + dchi[k] * aGd;
            a_dchi[k] += Gkp * aGd;
            a_Z[k] += 0.5 * (g[SI(k, i)] * dchi[j] + g[SI(k, j)] * dchi[i]) * azs;
            a_g[SI(k, i)] += 0.5 * Z[k] * dchi[j] * azs;
            a_dchi[j] += 0.5 * Z[k] * g[SI(k, i)] * azs;
            a_g[SI(k, j)] += 0.5 * Z[k] * dchi[i] * azs;
            a_dchi[i] += 0.5 * Z[k] * g[SI(k, j)] * azs;
        }
    }
    // cr = gt^{km} d_k alpha d_m chi
    for (int p = 0; p < 6; ++p) {
        const int k = PI_(p), m = PJ_(p);
        a_gu[p] += (k == m ? dalp[k] * dchi[m] : dalp[k] * dchi[m] + dalp[m] * dchi[k]) * a_cr;
    }
    for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) {
            a_dalp[k] += gu[SI(k, m)] * dchi[m] * a_cr;
            a_dchi[m] += gu[SI(k, m)] * dalp[k] * a_cr;
        }
    a_ic += 0.5 * a_hic;
    // trc = gt^{km} (dd chi_km - 3/2 d_k chi d_m chi / chi); Ghd = Ghat^k d_k chi
    for (int p = 0; p < 6; ++p) {
        const int k = PI_(p), m = PJ_(p);
        a_gu[p] += MU(p) * (ddc[p] - 1.5 * ic * dchi[k] * dchi[m]) * a_trc;
        q.Wq(W_D2 + 6 * d2_slot(CHI) + p) = 0.5 * ic * aR[p] + MU(p) * gu[p] * a_trc;
        a_ic += -1.5 * MU(p) * gu[p] * dchi[k] * dchi[m] * a_trc;
        a_dchi[k] += -1.5 * ic * MU(p) * gu[p] * dchi[m] * a_trc;
        a_dchi[m] += -1.5 * ic * MU(p) * gu[p] * dchi[k] * a_trc;
    }
    for (int k = 0; k < 3; ++k) {
        q.Wq(W_U + GH + k) += dchi[k] * a_Ghd;
        a_dchi[k] += Gh[k] * a_Ghd;
    }
    for (int p = 0; p < 6; ++p) {
        q.Wq(W_U + GT + p) += a_g[p];
        q.Wq(H_AGU + p) += a_gu[p];
    }
    q.Wq(W_U + CHI) += -ic * ic * a_ic;
    for (int i = 0; i < 3; ++i) {
        q.Wq(W_D1 + 3 * d1_slot(ALP) + i) += a_dalp[i];
        q.Wq(W_D1 + 3 * d1_slot(CHI) + i) += a_dchi[i];
        q.Wq(H_AZ + i) += a_Z[i];
    }
}
ADJ_KERNEL(ccz4_adj_chi_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    chi_body(q, C);
}

// ------------------------------------------------------------ kernel K5
// Reverse of the conformal Ricci tensor Rt_ij: -1/2 gt^{mn} d_m d_n gt_ij,
// gt_k(i d_j) Ghat^k, Ghat^k Gamma_(ij)k and the Gamma-Gamma products.
__device__ __forceinline__ void ricci_body(const Pt& q, const AdjConst& C)
{
    double gu[6], aR[6], Gl[3][6], Gu[3][6];
    for (int p = 0; p < 6; ++p) {
        gu[p] = q.Wq(F_GU + p);
        aR[p] = q.Wq(H_ARIC + p);
    }
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p) {
            Gl[i][p] = q.Wq(F_GL + 6 * i + p);
            Gu[i][p] = q.Wq(F_GUU + 6 * i + p);
        }
    double a_gu[6] = {}, a_Gl[3][6] = {}, a_Gu[3][6] = {};
    {
        // Q_i^{kn} = gt^{mn} Gamma^k_{mi}; T_ij = sum_kn Q_i^{kn} (Gamma_jkn + Gamma_knj) + Q_j^{kn} Gamma_ikn
        double Q[3][3][3], aQ[3][3][3] = {};
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k)
                for (int n = 0; n < 3; ++n)
                    Q[i][k][n] = gu[SI(0, n)] * Gu[k][SI(0, i)] + gu[SI(1, n)] * Gu[k][SI(1, i)] + gu[SI(2, n)] * Gu[k][SI(2, i)];
        for (int p = 0; p < 6; ++p) {
            const int i = PI_(p), j = PJ_(p);
            const double a = aR[p];
            for (int k = 0; k < 3; ++k)
                for (int n = 0; n < 3; ++n) {
                    aQ[i][k][n] += (Gl[j][SI(k, n)] + Gl[k][SI(n, j)]) * a;
                    aQ[j][k][n] += Gl[i][SI(k, n)] * a;
                    a_Gl[j][SI(k, n)] += Q[i][k][n] * a;
                    a_Gl[k][SI(n, j)] += Q[i][k][n] * a;
                    a_Gl[i][SI(k, n)] += Q[j][k][n] * a;
                }
        }
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k)
                for (int n = 0; n < 3; ++n)
                    for (int m = 0; m < 3; ++m) {
                        a_gu[SI(m, n)] += Gu[k][SI(m, i)] * aQ[i][k][n];
                        a_Gu[k][SI(m, i)] += gu[SI(m, n)] * aQ[i][k][n];
                    }
    }
    // Ghat^k Gamma_(ij)k; gt_k(i d_j) Ghat^k
    double a_g[6] = {}, a_Gh[3] = {}, Gh[3], g[6];
    for (int k = 0; k < 3; ++k) Gh[k] = q.U(GH + k);
    for (int p = 0; p < 6; ++p) g[p] = q.U(GT + p);
    double a_dGh[3][3] = {};  // [j][k] = adjoint of d_j Ghat^k
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        const double a = aR[p];
        for (int k = 0; k < 3; ++k) {
            a_g[SI(k, i)] += 0.5 * q.Wq(F_DGH + 3 * j + k) * a;
            a_dGh[j][k] += 0.5 * g[SI(k, i)] * a;
            a_g[SI(k, j)] += 0.5 * q.Wq(F_DGH + 3 * i + k) * a;
            a_dGh[i][k] += 0.5 * g[SI(k, j)] * a;
            a_Gh[k] += 0.5 * (Gl[i][SI(j, k)] + Gl[j][SI(i, k)]) * a;
            a_Gl[i][SI(j, k)] += 0.5 * Gh[k] * a;
            a_Gl[j][SI(i, k)] += 0.5 * Gh[k] * a;
        }
    }
    // -1/2 gt^{mn} d_m d_n gt_ij: the second derivatives of gt are written here
    for (int p = 0; p < 6; ++p) {
        const double al = -0.5 * aR[p];
        for (int m = 0; m < 6; ++m) {
            a_gu[m] += MU(m) * q.Wq(F_DDG + 6 * p + m) * al;
            q.Wq(W_D2 + 6 * d2_slot(GT + p) + m) = MU(m) * gu[m] * al;
        }
    }
    for (int p = 0; p < 6; ++p) {
        q.Wq(W_U + GT + p) += a_g[p];
        q.Wq(H_AGU + p) += a_gu[p];
    }
    for (int i = 0; i < 3; ++i) {
        q.Wq(W_U + GH + i) += a_Gh[i];
        for (int k = 0; k < 3; ++k) q.Wq(W_D1 + 3 * d1_slot(GH + k) + i) = a_dGh[i][k];
        for (int p = 0; p < 6; ++p) {
            q.Wq(H_AGUU + 6 * i + p) += a_Gu[i][p];
            q.Wq(H_AGL + 6 * i + p) = a_Gl[i][p];
        }
    }
}
ADJ_KERNEL(ccz4_adj_ricci_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    ricci_body(q, C);
}

// The reverses of the shift Hessian, of D_iD_j alpha with the chi part of
// the Ricci tensor, and of the conformal Ricci tensor run one after the other
// in one launch: one launch and one point set-up instead of three.  Alone
// each fits two waves per SIMD; together the kernel takes more than half the
// register file and runs one wave without scratch (held to two waves it
// spills 560 bytes per lane), and is still slightly faster than the three
// (reverse RK4 step at 48^3 1.886 against 1.897 ms).
#ifndef MOL_ADJ_FUSE_SCR
#define MOL_ADJ_FUSE_SCR 1
#endif
ADJ_KERNEL(ccz4_adj_shift_chi_ricci_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    // the bodies pass their results through the workspace; the fences keep
    // the compiler from hoisting one body's loads into the one before it,
    // which would hold both bodies' values live at once
    shift_body(q, C);
    asm volatile("" ::: "memory");
    chi_body(q, C);
    asm volatile("" ::: "memory");
    ricci_body(q, C);
}

// ------------------------------------------------------------ kernel K6
// Chain to the stencil inputs: Z = chi (Ghat - gt^{jk} Gamma^i_jk)/2,
// Gamma^i_jk = gt^{il} Gamma_ljk, Gamma_ijk from d gt, gt^{ij} = inverse of gt_ij.
ADJ_KERNEL(ccz4_adj_chain_kernel)
{
    Pt q;
    if (!pt_init(q, patches, tiles, Ug, lamg, W, wofs)) return;
    double gu[6], a_gu[6], a_Gu[3][6], a_Gl[3][6];
    for (int p = 0; p < 6; ++p) {
        gu[p] = q.Wq(F_GU + p);
        a_gu[p] = q.Wq(H_AGU + p);
    }
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p) {
            a_Gu[i][p] = q.Wq(H_AGUU + 6 * i + p);
            a_Gl[i][p] = q.Wq(H_AGL + 6 * i + p);
        }
    const double chi = q.U(CHI);
    double a_chi = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double aZ = q.Wq(H_AZ + i);
        double Gc = 0.0;
        for (int p = 0; p < 6; ++p) Gc += MU(p) * gu[p] * q.Wq(F_GUU + 6 * i + p);
        a_chi += 0.5 * (q.U(GH + i) - Gc) * aZ;
        q.Wq(W_U + GH + i) += 0.5 * chi * aZ;
        const double aGc = -0.5 * chi * aZ;
        for (int p = 0; p < 6; ++p) {
            a_gu[p] += MU(p) * q.Wq(F_GUU + 6 * i + p) * aGc;
            a_Gu[i][p] += MU(p) * gu[p] * aGc;
        }
    }
    q.Wq(W_U + CHI) += a_chi;
    // Gamma^i_p = sum_l gt^{il} Gamma_l p
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p)
            for (int l = 0; l < 3; ++l) {
                a_gu[SI(i, l)] += q.Wq(F_GL + 6 * l + p) * a_Gu[i][p];
                a_Gl[l][p] += gu[SI(i, l)] * a_Gu[i][p];
            }
    // Gamma_i(jk) = (d_j gt_ik + d_k gt_ij - d_i gt_jk)/2
    double a_dg[3][6] = {};
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 6; ++p) {
            const int j = PI_(p), k = PJ_(p);
            const double a = 0.5 * a_Gl[i][p];
            a_dg[j][SI(i, k)] += a;
            a_dg[k][SI(i, j)] += a;
            a_dg[i][p] -= a;
        }
    for (int k = 0; k < 3; ++k)
        for (int p = 0; p < 6; ++p) q.Wq(W_D1 + 3 * d1_slot(GT + p) + k) = a_dg[k][p];
    // gt^{-1}: a(gt) = -gt^{-1} a(gt^{-1}) gt^{-1} on the full symmetric adjoint
    double Af[3][3];
    for (int p = 0; p < 6; ++p) {
        const double v = MU(p) == 1.0 ? a_gu[p] : 0.5 * a_gu[p];
        Af[PI_(p)][PJ_(p)] = Af[PJ_(p)][PI_(p)] = v;
    }
    for (int p = 0; p < 6; ++p) {
        const int i = PI_(p), j = PJ_(p);
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) s += gu[SI(i, a)] * Af[a][b] * gu[SI(b, j)];
        q.Wq(W_U + GT + p) += -MU(p) * s;
    }
}

// ---------------------------------------------------------------- kernel 2
#ifndef MOL_ADJ_GATHER_GROUP
#define MOL_ADJ_GATHER_GROUP 13
#endif

// Epilogue of the periodic (WRAP) gather inside a reverse RK4 step: with v the
// transposed value at p, wsum = v (first) or wsum + v; then either
// wnext = a lam + b v (the next stage's input), or lam += wsum (last).
struct GatherEpi {
    const double* lam0;  // lam of the step (read)
    double* lam;         // lam of the step, updated in place by the last stage
    double* wsum;
    double* wnext;
    double a, b;
    int first, last;
};

// WRAP = false: every point p of the ghosted box, interior stencil points c
// only; the ghost entries of lamU are then folded into their owners by the
// fill transpose.  WRAP = true (one periodic patch of at least 7 points per
// axis): every interior point p, with the stencil points c taken at their
// periodic images, so no ghost entry arises; the result goes through the
// epilogue instead of lamU.
template <bool WRAP>
__global__ __launch_bounds__(256) void ccz4_adj_gather_kernel(const PatchDev* __restrict__ patches,
                                                              const Tile* __restrict__ tiles,
                                                              const double* __restrict__ Ug,
                                                              const double* __restrict__ lamg,
                                                              const double* __restrict__ W,
                                                              const int64_t* __restrict__ wofs, AdjConst C,
                                                              double* __restrict__ lamU, GatherEpi E)
{
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const PatchDev P = patches[t.patch];
    const int q[3] = {t.o[0] + (int)threadIdx.x, t.o[1] + (int)threadIdx.y, t.o[2] + (int)threadIdx.z};
    if (WRAP ? (q[0] >= P.n[0] || q[1] >= P.n[1] || q[2] >= P.n[2])
             : (q[0] >= P.n[0] + G || q[1] >= P.n[1] + G || q[2] >= P.n[2] + G))
        return;
    const int64_t loc = (int64_t)(q[2] + G) * P.pitch_z + (int64_t)(q[1] + G) * P.pitch_y + (q[0] + G);
    const int64_t fs = P.fs;
    const int S[3] = {1, P.pitch_y, P.pitch_z};
    const double* lp = lamg + P.off + loc;
    const double* bp = Ug + P.off + loc + (int64_t)BETA * fs;
    // the workspace holds interior points only (its own row and plane
    // pitches): wb is p's index there, which for a ghost point p lies outside
    // the patch's block; only wb plus the offset of an interior c is read
    const int64_t wpy = adj_wpitch(P.n[0]), wfs = adj_wfs(P.n);
    const int64_t SW[3] = {1, wpy, wpy * P.n[1]};
    const int64_t wb = wofs[t.patch] + ((int64_t)q[2] * P.n[1] + q[1]) * wpy + q[0];
    // c = p + off along axis d (and e along axis d2) is an interior point
    // (always, at its periodic image, when WRAP)
    auto inside = [&](int d, int off, int d2 = 0, int e = 0) {
        if constexpr (WRAP) return true;
        int c[3] = {q[0], q[1], q[2]};
        c[d] += off;
        c[d2] += e;
        return c[0] >= 0 && c[0] < P.n[0] && c[1] >= 0 && c[1] < P.n[1] && c[2] >= 0 && c[2] < P.n[2];
    };
    // offset of p + off along axis d from p (at the periodic image when WRAP),
    // in points; then in the level buffer and in the workspace
    auto tapv = [&](int d, int off) -> int {
        int v = off;
        if constexpr (WRAP) {
            const int c = q[d] + off;
            v = c < 0 ? off + P.n[d] : (c >= P.n[d] ? off - P.n[d] : off);
        }
        return v;
    };
    auto shift = [&](int d, int off) -> int64_t { return (int64_t)tapv(d, off) * S[d]; };
    auto shiftw = [&](int d, int off) -> int64_t { return (int64_t)tapv(d, off) * SW[d]; };
    const bool self = inside(0, 0);
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};   // D1: coefficient of u(c+o), o = -2..2
    const double w2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    const double wko[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};
    const double wlp[7] = {0.0, 0.0, -3.0, -10.0, 18.0, -6.0, 1.0};  // beta >= 0: o = -3..3
    const double wlm[7] = {-1.0, 6.0, -18.0, 10.0, 3.0, 0.0, 0.0};   // beta < 0
    // fields in groups of MOL_ADJ_GATHER_GROUP (13: the 25 fields in two
    // sweeps, at about 150 VGPRs; three sweeps of 9 and one of 25, at 240
    // VGPRs, measured slower), one accumulator per field of the group; the
    // taps are swept once per group (rolled loops keep the code small) and
    // the terms of each field are summed in the same order whatever the
    // grouping
#pragma unroll
    for (int f0 = 0; f0 < NF; f0 += MOL_ADJ_GATHER_GROUP) {
        constexpr int GF = MOL_ADJ_GATHER_GROUP;
        double acc[GF];
#pragma unroll
        for (int g = 0; g < GF; ++g)
            if (f0 + g < NF) acc[g] = self ? W[wb + (int64_t)(W_U + f0 + g) * wfs] : 0.0;
        // u(p) enters the stencils of the interior points c = p - o e_k
#pragma unroll 1
        for (int k = 0; k < 3; ++k)
#pragma unroll 1
            for (int o = -3; o <= 3; ++o) {
                if (!inside(k, -o)) continue;
                const int64_t cof = shift(k, -o);
                const double bk = bp[(int64_t)k * fs + cof];
                const double wa = C.upwind ? (bk >= 0.0 ? wlp[o + 3] : wlm[o + 3]) : (o >= -2 && o <= 2 ? w1[o + 2] : 0.0);
                // KO and advection act on lam of every field
                const double wl = C.ko * wko[o + 3] + C.i12h * wa * bk;
#pragma unroll
                for (int g = 0; g < GF; ++g)
                    if (f0 + g < NF) acc[g] += wl * lp[(int64_t)(f0 + g) * fs + cof];
                if (o < -2 || o > 2) continue;
                const int64_t cofw = wb + shiftw(k, -o);
#pragma unroll
                for (int g = 0; g < GF; ++g) {
                    const int f = f0 + g;
                    if (f >= NF) continue;
                    const int s1 = d1_slot(f), s2 = d2_slot(f);
                    if (s1 >= 0) acc[g] += C.i12h * w1[o + 2] * W[(int64_t)(W_D1 + 3 * s1 + k) * wfs + cofw];
                    if (s2 >= 0) acc[g] += C.i12h2 * w2[o + 2] * W[(int64_t)(W_D2 + 6 * s2 + SI(k, k)) * wfs + cofw];
                }
            }
#pragma unroll 1
        for (int k = 0; k < 3; ++k)
#pragma unroll 1
            for (int l = k + 1; l < 3; ++l)
#pragma unroll 1
                for (int ia = 0; ia < 4; ++ia)
#pragma unroll 1
                    for (int ib = 0; ib < 4; ++ib) {
                        // the mixed stencil's taps: offsets -2, -1, 1, 2 on both axes
                        const int a = ia < 2 ? ia - 2 : ia - 1, b = ib < 2 ? ib - 2 : ib - 1;
                        if (!inside(k, -a, l, -b)) continue;
                        const int64_t cofw = wb + shiftw(k, -a) + shiftw(l, -b);
                        const double wm = C.i144h2 * w1[a + 2] * w1[b + 2];
#pragma unroll
                        for (int g = 0; g < GF; ++g) {
                            const int f = f0 + g;
                            if (f >= NF) continue;
                            const int s2 = d2_slot(f);
                            if (s2 >= 0) acc[g] += wm * W[(int64_t)(W_D2 + 6 * s2 + SI(k, l)) * wfs + cofw];
                        }
                    }
#pragma unroll
        for (int g = 0; g < GF; ++g) {
            if (f0 + g >= NF) continue;
            const int64_t idx = P.off + loc + (int64_t)(f0 + g) * fs;
            if constexpr (!WRAP) {
                lamU[idx] = acc[g];
            } else {
                const double s = E.first ? acc[g] : E.wsum[idx] + acc[g];
                if (E.last) {
                    E.lam[idx] = E.lam0[idx] + s;
                } else {
                    E.wsum[idx] = s;
                    E.wnext[idx] = E.a * E.lam0[idx] + E.b * acc[g];
                }
            }
        }
    }
}

AdjConst adj_const(const SysParams& sp)
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
    return C;
}

}  // namespace

int ccz4_adjoint_slots() { return NWX; }

hipError_t launch_ccz4_adjoint(const SysParams& sp, const PatchDev* patches, const Tile* tiles, int ntiles,
                               const int td[3], const Tile* gtiles, int ngtiles, const int gtd[3],
                               const double* U, const double* lam, double* W, const int64_t* wofs, double* lamU,
                               hipStream_t s)
{
    const AdjConst C = adj_const(sp);
    if (ntiles > 0) {
        // every pointwise kernel covers the same interior points; each writes
        // or accumulates only the workspace slots listed in its comment
        const dim3 b(td[0], td[1], td[2]);
        if (!MOL_ADJ_FUSE_ADV) ccz4_adj_advection_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        ccz4_adj_forward_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        ccz4_adj_ricci_fwd_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        ccz4_adj_metric_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        ccz4_adj_gauge_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        if (MOL_ADJ_FUSE_SCR) {
            ccz4_adj_shift_chi_ricci_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        } else {
            ccz4_adj_shift_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
            ccz4_adj_chi_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
            ccz4_adj_ricci_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        }
        ccz4_adj_chain_kernel<<<ntiles, b, 0, s>>>(patches, tiles, U, lam, W, wofs, C);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ngtiles > 0)
        ccz4_adj_gather_kernel<false>
            <<<ngtiles, dim3(gtd[0], gtd[1], gtd[2]), 0, s>>>(patches, gtiles, U, lam, W, wofs, C, lamU, GatherEpi{});
    return hipGetLastError();
}

hipError_t launch_ccz4_adjoint_stage(const SysParams& sp, const PatchDev* patches, const Tile* tiles, int ntiles,
                                     const int td[3], const Tile* itiles, int nitiles, const int itd[3],
                                     const double* U, const double* lam_in, double* W, const int64_t* wofs,
                                     const double* lam0, double* lam, double* wsum, double* wnext, double a,
                                     double b, int first, int last, hipStream_t s)
{
    // the point-wise kernels as in launch_ccz4_adjoint (no gather), then the
    // periodic gather with the reverse-RK4 epilogue
    hipError_t e = launch_ccz4_adjoint(sp, patches, tiles, ntiles, td, nullptr, 0, itd, U, lam_in, W, wofs, nullptr, s);
    if (e != hipSuccess || nitiles <= 0) return e;
    AdjConst C = adj_const(sp);
    GatherEpi E{lam0, lam, wsum, wnext, a, b, first, last};
    ccz4_adj_gather_kernel<true>
        <<<nitiles, dim3(itd[0], itd[1], itd[2]), 0, s>>>(patches, itiles, U, lam_in, W, wofs, C, nullptr, E);
    return hipGetLastError();
}

}  // namespace mol
