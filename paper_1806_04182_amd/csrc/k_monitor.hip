// Constraint and dissipation monitors of a level (Sec. V: Theta, Z^i,
// the bracket H_Z of the Theta equation, the conformal constraints
// ln det gt = 0 and tr At = 0; Sec. II.B.1: the size of the KO term), one
// thread per interior point, reduced deterministically (fixed tile walk,
// fixed LDS tree, one final block) like the norms.
//
// The Ricci part of H_Z is evaluated in contracted form: with
// Gt_ijk = (d_j gt_ik + d_k gt_ij - d_i gt_jk)/2 and Gt^k_ij = gt^kl Gt_lij,
//   gt^ij Rhat_ij = -1/2 gt^mn (gt^ij d_m d_n gt_ij) + d_k Ghat^k
//                   + 1/2 Ghat^k gt^ij d_k gt_ij
//                   + gt^ij gt^mn (2 Gt^k_mi Gt_jkn + Gt^k_mi Gt_knj),
//   gt^ij Rhat^chi_ij = 2/chi gt^ij d_i d_j chi - 5/(2 chi^2) gt^ij d_i chi d_j chi
//                       - 3/(2 chi) Gt^k d_k chi - 1/(2 chi) Ghat^k d_k chi,
// the traces of the printed Rhat_ij and Rhat^chi_ij with
// Z^k = chi (Ghat^k - Gt^k)/2 substituted; R + 2 nabla_i Z^i is chi times
// their sum.
#include "k_common.h"

namespace mol {

namespace {

constexpr int RB = 256;
constexpr int NQ = 3 * MOL_MON_COUNT + 1;

struct MonRed {
    double v[NQ];
};

__device__ __forceinline__ bool is_max(int q) { return q < 3 * MOL_MON_COUNT && q % 3 == 2; }

// Block reduction: each wave reduces its 64 lanes (wave_sum / wave_max), lane
// 0 of each wave parks the result in LDS, then the RB / 64 wave results are
// folded in wave order.  Fixed order throughout: the same bits on every run.
constexpr int NWV = RB / 64;
__device__ __forceinline__ void block_reduce(MonRed& r, double* sh)
{
    const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int lane = t & 63, wv = t >> 6;
    for (int q = 0; q < NQ; ++q) {
        const double v = is_max(q) ? wave_max(r.v[q]) : wave_sum(r.v[q]);
        if (lane == 0) sh[q * NWV + wv] = v;
    }
    __syncthreads();
    for (int q = 0; q < NQ; ++q) {
        double v = sh[q * NWV];
        for (int w = 1; w < NWV; ++w) v = is_max(q) ? fmax(v, sh[q * NWV + w]) : v + sh[q * NWV + w];
        r.v[q] = v;
    }
}

// 4th-order stencils of Sec. II.B.1 along stride s (weighted differences)
__device__ __forceinline__ double d1(const double* u, int64_t s, double i12h)
{
    return (8.0 * (u[s] - u[-s]) - (u[2 * s] - u[-2 * s])) * i12h;
}
__device__ __forceinline__ double d2(const double* u, int64_t s, double i12h2)
{
    const double c = u[0];
    return (16.0 * ((u[s] - c) + (u[-s] - c)) - ((u[2 * s] - c) + (u[-2 * s] - c))) * i12h2;
}
// D_b(D_a u)
__device__ __forceinline__ double dmix(const double* u, int64_t sa, int64_t sb, double i12h)
{
    return (8.0 * (d1(u + sb, sa, i12h) - d1(u - sb, sa, i12h)) - (d1(u + 2 * sb, sa, i12h) - d1(u - 2 * sb, sa, i12h))) *
           i12h;
}
__device__ __forceinline__ double ko(const double* u, int64_t s, double kc)
{
    const double c = u[0];
    const double a1 = (u[s] - c) + (u[-s] - c), a2 = (u[2 * s] - c) + (u[-2 * s] - c),
                 a3 = (u[3 * s] - c) + (u[-3 * s] - c);
    return (a3 - 6.0 * a2 + 15.0 * a1) * kc;
}

// CCZ4 field order
enum { F_CHI = 0, F_GT = 1, F_KH = 7, F_AT = 8, F_GH = 14, F_TH = 17 };
__device__ __forceinline__ int sym(int i, int j)
{
    // xx xy xz yy yz zz
    return i == j ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : (i + j == 1 ? 1 : (i + j == 2 ? 2 : 4));
}

struct MonArgs {
    const PatchDev* patches;
    const Tile* tiles;
    int ntiles;
    int nf;
    int ccz4;
    unsigned which;
    double h, sigma;
    const double* U;
    double* point;  // nullable: requested monitors at interior points, field k = k-th requested
    double* partial;
};

__global__ __launch_bounds__(RB) void monitor_kernel(MonArgs a)
{
    __shared__ double sh[NQ * NWV];
    MonRed r;
    for (int q = 0; q < NQ; ++q) r.v[q] = 0.0;
    const double h = a.h, dV = h * h * h;
    const double i12h = 1.0 / (12.0 * h), i12h2 = 1.0 / (12.0 * h * h), kcoef = a.sigma / (64.0 * h);
    for (int tt = blockIdx.x; tt < a.ntiles; tt += gridDim.x) {
        const Tile t = a.tiles[tt];
        const PatchDev P = a.patches[t.patch];
        const int i = t.o[0] + threadIdx.x, j = t.o[1] + threadIdx.y, k = t.o[2] + threadIdx.z;
        if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) continue;
        const int64_t c = P.off + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + i + G;
        const int64_t st[3] = {1, P.pitch_y, P.pitch_z};
        const double* U = a.U + c;
        for (int f = 0; f < a.nf; ++f)
            if (!isfinite(U[f * P.fs])) r.v[3 * MOL_MON_COUNT] += 1.0;
        double mon[MOL_MON_COUNT];
        if (a.which & MOL_MON_KO) {
            double s = 0.0;
            for (int f = 0; f < a.nf; ++f) {
                const double* u = U + f * P.fs;
                const double q = ko(u, st[0], kcoef) + ko(u, st[1], kcoef) + ko(u, st[2], kcoef);
                s += q * q;
            }
            mon[5] = sqrt(s);
        }
        if (a.ccz4 && (a.which & (MOL_MON_ALL & ~MOL_MON_KO))) {
            const int64_t fs = P.fs;
            double g[3][3], A[3][3];
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) {
                    g[p][q] = U[(F_GT + sym(p, q)) * fs];
                    A[p][q] = U[(F_AT + sym(p, q)) * fs];
                }
            const double chi = U[F_CHI * fs], Kh = U[F_KH * fs], Th = U[F_TH * fs];
            // ln det gt from h = gt - I (no cancellation), and the inverse
            const double hx = g[0][0] - 1.0, hy = g[1][1] - 1.0, hz = g[2][2] - 1.0;
            const double cxx = g[1][1] * g[2][2] - g[1][2] * g[1][2], cxy = g[0][2] * g[1][2] - g[0][1] * g[2][2],
                         cxz = g[0][1] * g[1][2] - g[0][2] * g[1][1], cyy = g[0][0] * g[2][2] - g[0][2] * g[0][2],
                         cyz = g[0][1] * g[0][2] - g[0][0] * g[1][2], czz = g[0][0] * g[1][1] - g[0][1] * g[0][1];
            const double dm = (hx + hy + hz) +
                              ((hx * hy - g[0][1] * g[0][1]) + (hx * hz - g[0][2] * g[0][2]) +
                               (hy * hz - g[1][2] * g[1][2])) +
                              (hx * (hy * hz - g[1][2] * g[1][2]) - g[0][1] * (g[0][1] * hz - g[1][2] * g[0][2]) +
                               g[0][2] * (g[0][1] * g[1][2] - hy * g[0][2]));
            const double idet = 1.0 / (1.0 + dm);
            double gi[3][3];
            gi[0][0] = cxx * idet;
            gi[0][1] = gi[1][0] = cxy * idet;
            gi[0][2] = gi[2][0] = cxz * idet;
            gi[1][1] = cyy * idet;
            gi[1][2] = gi[2][1] = cyz * idet;
            gi[2][2] = czz * idet;
            mon[0] = Th;
            mon[3] = log1p(dm);
            double trA = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) trA += gi[p][q] * A[p][q];
            mon[4] = trA;
            if (a.which & (MOL_MON_Z | MOL_MON_HZ)) {
                // first derivatives of gt: dg[m][p][q] = d_m gt_pq
                double dg[3][3][3];
                for (int p = 0; p < 3; ++p)
                    for (int q = p; q < 3; ++q) {
                        const double* u = U + (F_GT + sym(p, q)) * fs;
                        for (int m = 0; m < 3; ++m) dg[m][p][q] = dg[m][q][p] = d1(u, st[m], i12h);
                    }
                // Gl[l][p][q] = Gt_lpq, Gu[k][p][q] = Gt^k_pq, Gc^k = gt^pq Gt^k_pq
                double Gl[3][3][3], Gu[3][3][3], Gc[3];
                for (int l = 0; l < 3; ++l)
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) Gl[l][p][q] = 0.5 * (dg[p][l][q] + dg[q][l][p] - dg[l][p][q]);
                for (int kk = 0; kk < 3; ++kk) {
                    Gc[kk] = 0.0;
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) {
                            Gu[kk][p][q] = gi[kk][0] * Gl[0][p][q] + gi[kk][1] * Gl[1][p][q] + gi[kk][2] * Gl[2][p][q];
                            Gc[kk] += gi[p][q] * Gu[kk][p][q];
                        }
                }
                double Gh[3], Z[3];
                for (int p = 0; p < 3; ++p) {
                    Gh[p] = U[(F_GH + p) * fs];
                    Z[p] = 0.5 * chi * (Gh[p] - Gc[p]);
                }
                double zz = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) zz += g[p][q] * Z[p] * Z[q];
                mon[1] = sqrt(zz / chi);
                if (a.which & MOL_MON_HZ) {
                    // -1/2 gt^mn gt^ij d_m d_n gt_ij, and gt^mn d_m d_n chi
                    double lapg = 0.0, lapchi = 0.0;
                    const double* uc = U + F_CHI * fs;
                    for (int m = 0; m < 3; ++m)
                        for (int n = m; n < 3; ++n) {
                            const double wmn = (m == n ? 1.0 : 2.0) * gi[m][n];
                            double s = 0.0;
                            for (int p = 0; p < 3; ++p)
                                for (int q = p; q < 3; ++q) {
                                    const double* u = U + (F_GT + sym(p, q)) * fs;
                                    const double dd = m == n ? d2(u, st[m], i12h2) : dmix(u, st[m], st[n], i12h);
                                    s += (p == q ? 1.0 : 2.0) * gi[p][q] * dd;
                                }
                            lapg += wmn * s;
                            lapchi += wmn * (m == n ? d2(uc, st[m], i12h2) : dmix(uc, st[m], st[n], i12h));
                        }
                    double divGh = 0.0, dchi[3];
                    for (int m = 0; m < 3; ++m) {
                        divGh += d1(U + (F_GH + m) * fs, st[m], i12h);
                        dchi[m] = d1(uc, st[m], i12h);
                    }
                    double trdg = 0.0, gg = 0.0, cc = 0.0, Gtd = 0.0, Ghd = 0.0;
                    for (int kk = 0; kk < 3; ++kk) {
                        double s = 0.0;
                        for (int p = 0; p < 3; ++p)
                            for (int q = 0; q < 3; ++q) s += gi[p][q] * dg[kk][p][q];
                        trdg += Gh[kk] * s;
                        Gtd += Gc[kk] * dchi[kk];
                        Ghd += Gh[kk] * dchi[kk];
                        for (int p = 0; p < 3; ++p) cc += gi[kk][p] * dchi[kk] * dchi[p];
                    }
                    // gt^ij gt^mn (2 Gt^k_mi Gt_jkn + Gt^k_mi Gt_knj)
                    for (int m = 0; m < 3; ++m)
                        for (int ii = 0; ii < 3; ++ii)
                            for (int kk = 0; kk < 3; ++kk) {
                                double s = 0.0;
                                for (int jj = 0; jj < 3; ++jj)
                                    for (int n = 0; n < 3; ++n)
                                        s += gi[ii][jj] * gi[m][n] * (2.0 * Gl[jj][kk][n] + Gl[kk][n][jj]);
                                gg += Gu[kk][m][ii] * s;
                            }
                    const double trRh = -0.5 * lapg + divGh + 0.5 * trdg + gg;
                    const double trRc = 2.0 / chi * lapchi - 2.5 / (chi * chi) * cc - 1.5 / chi * Gtd - 0.5 / chi * Ghd;
                    double AA = 0.0;
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) {
                            double Aup = 0.0;
                            for (int l = 0; l < 3; ++l)
                                for (int n = 0; n < 3; ++n) Aup += gi[p][l] * gi[q][n] * A[l][n];
                            AA += A[p][q] * Aup;
                        }
                    mon[2] = chi * (trRh + trRc) + 2.0 / 3.0 * Kh * Kh + 2.0 / 3.0 * Th * (Kh - 2.0 * Th) - AA;
                }
            }
        }
        int rank = 0;
        for (int q = 0; q < MOL_MON_COUNT; ++q) {
            if (!(a.which >> q & 1u)) continue;
            const double v = mon[q];
            if (a.point) a.point[c + rank * P.fs] = v;
            ++rank;
            if (!isfinite(v)) continue;
            r.v[3 * q] += fabs(v) * dV;
            r.v[3 * q + 1] += v * v * dV;
            r.v[3 * q + 2] = fmax(r.v[3 * q + 2], fabs(v));
        }
    }
    block_reduce(r, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0)
        for (int q = 0; q < NQ; ++q) a.partial[blockIdx.x * NQ + q] = r.v[q];
}

__global__ __launch_bounds__(RB) void monitor_final_kernel(const double* __restrict__ partial, int nb,
                                                           double* __restrict__ out)
{
    __shared__ double sh[NQ * NWV];
    MonRed r;
    for (int q = 0; q < NQ; ++q) r.v[q] = 0.0;
    const int t = threadIdx.x;
    for (int b = t; b < nb; b += RB)
        for (int q = 0; q < NQ; ++q) {
            const double v = partial[b * NQ + q];
            r.v[q] = is_max(q) ? fmax(r.v[q], v) : r.v[q] + v;
        }
    block_reduce(r, sh);
    if (t == 0)
        for (int q = 0; q < NQ; ++q) out[q] = r.v[q];
}

}  // namespace

int monitor_partials() { return NQ; }

hipError_t launch_monitor(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], int nf, int ccz4,
                          unsigned which, double h, double sigma, const double* U, double* point, double* partial,
                          int nblocks, double* out, hipStream_t s)
{
    MonArgs a{patches, tiles, ntiles, nf, ccz4, which, h, sigma, U, point, partial};
    monitor_kernel<<<nblocks, dim3(td[0], td[1], td[2]), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    monitor_final_kernel<<<1, RB, 0, s>>>(partial, nblocks, out);
    return hipGetLastError();
}

}  // namespace mol
