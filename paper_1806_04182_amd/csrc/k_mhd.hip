// Newtonian ideal MHD (Sec. IV.B, eight-field core: rho, S, E, B) in the
// conservative finite-difference form (eq. conservative_discretization):
//   L = - sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d,
// with the evolved fields reconstructed at every interface by WENO5-Z
// (App. B; q = 2, eps = dx^4 unless set), WENO5-JS (App. B) or WENO3 (App. A,
// eps = dx^2 unless set), and the local Lax-Friedrichs flux (eq. LLF)
// F = (F(U^L) + F(U^R) - S (U^R - U^L)) / 2, S the larger of |v_d| + c_f over
// the two states (fast magnetosonic speed c_f), or the HLL flux
// F = (S^R F^L - S^L F^R + S^R S^L (U^R - U^L)) / (S^R - S^L) with
// S^L = min(v_d - c_f, 0), S^R = max(v_d + c_f, 0) over the two states.  With
// the divergence-cleaning scalar psi (nine fields) the B^i flux along d gains
// delta^{di} psi, psi has the flux c_h^2 B^d and the source -kappa_psi psi, and
// the cleaning speeds -c_h, +c_h join the signal speeds.  Fused with the
// Runge-Kutta stage update.
#include "k_common.h"

namespace mol {

namespace {

struct MhdConst {
    double gam;
    double eps[3];
    double q;
    double ih;  // 1 / dx
    double ch2, ch, kpsi;  // cleaning: c_h^2, c_h, kappa_psi
};

// WENO5-Z value at the interface to the right of v[2] reconstructed from the
// left, using one division: alpha_r = d_r (e_r^2 + tau^2) / e_r^2 with
// e_r = eps + beta_r, scaled by e_0^2 e_1^2 e_2^2.  The right state at the
// interface to the left of a cell is the same formula on mirrored values.
template <bool Q2>
__device__ __forceinline__ double weno5z(double v0, double v1, double v2, double v3, double v4,
                                         double eps, double q)
{
    const double p0 = (2.0 * v2 + 5.0 * v3 - v4) * (1.0 / 6.0);
    const double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) * (1.0 / 6.0);
    const double p2 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * (1.0 / 6.0);
    const double a0 = v2 - 2.0 * v3 + v4, b0 = 3.0 * v2 - 4.0 * v3 + v4;
    const double a1 = v1 - 2.0 * v2 + v3, b1 = v1 - v3;
    const double a2 = v0 - 2.0 * v1 + v2, b2 = v0 - 4.0 * v1 + 3.0 * v2;
    const double be0 = (13.0 / 12.0) * a0 * a0 + 0.25 * b0 * b0;
    const double be1 = (13.0 / 12.0) * a1 * a1 + 0.25 * b1 * b1;
    const double be2 = (13.0 / 12.0) * a2 * a2 + 0.25 * b2 * b2;
    const double tau = fabs(be0 - be2);
    const double e0 = eps + be0, e1 = eps + be1, e2 = eps + be2;
    double w0, w1, w2;
    if constexpr (Q2) {
        const double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2, t2 = tau * tau;
        w0 = 0.3 * (s0 + t2) * (s1 * s2);
        w1 = 0.6 * (s1 + t2) * (s0 * s2);
        w2 = 0.1 * (s2 + t2) * (s0 * s1);
    } else {
        w0 = 0.3 * (1.0 + pow(tau / e0, q));
        w1 = 0.6 * (1.0 + pow(tau / e1, q));
        w2 = 0.1 * (1.0 + pow(tau / e2, q));
    }
    return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

// WENO5-JS value at the interface to the right of v[2] from the left:
// alpha_r = d_r / e_r^2, e_r = eps + beta_r, scaled by e_0^2 e_1^2 e_2^2.
__device__ __forceinline__ double weno5js(double v0, double v1, double v2, double v3, double v4, double eps)
{
    const double p0 = (2.0 * v2 + 5.0 * v3 - v4) * (1.0 / 6.0);
    const double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) * (1.0 / 6.0);
    const double p2 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * (1.0 / 6.0);
    const double a0 = v2 - 2.0 * v3 + v4, b0 = 3.0 * v2 - 4.0 * v3 + v4;
    const double a1 = v1 - 2.0 * v2 + v3, b1 = v1 - v3;
    const double a2 = v0 - 2.0 * v1 + v2, b2 = v0 - 4.0 * v1 + 3.0 * v2;
    const double e0 = eps + ((13.0 / 12.0) * a0 * a0 + 0.25 * b0 * b0);
    const double e1 = eps + ((13.0 / 12.0) * a1 * a1 + 0.25 * b1 * b1);
    const double e2 = eps + ((13.0 / 12.0) * a2 * a2 + 0.25 * b2 * b2);
    const double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
    const double w0 = 0.3 * (s1 * s2), w1 = 0.6 * (s0 * s2), w2 = 0.1 * (s0 * s1);
    return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

// WENO3 value at the interface to the right of v2 from the left (cells v1,
// v2, v3): alpha_0 = (2/3) / e_0^2, alpha_1 = (1/3) / e_1^2, scaled by e_0^2 e_1^2.
__device__ __forceinline__ double weno3(double v1, double v2, double v3, double eps)
{
    const double p0 = 0.5 * (v2 + v3), p1 = 1.5 * v2 - 0.5 * v1;
    const double d0 = v3 - v2, d1 = v2 - v1;
    const double e0 = eps + d0 * d0, e1 = eps + d1 * d1;
    const double w0 = (2.0 / 3.0) * (e1 * e1), w1 = (1.0 / 3.0) * (e0 * e0);
    return (w0 * p0 + w1 * p1) / (w0 + w1);
}

enum { REC_W5Z = 0, REC_W5JS = 1, REC_W3 = 2 };
enum { RS_LLF = 0, RS_HLL = 1, RS_SPLIT = 2 };

// reconstructed value at the interface to the right of v2 from the left
template <int REC, bool Q2>
__device__ __forceinline__ double recon(double v0, double v1, double v2, double v3, double v4, double eps, double q)
{
    if constexpr (REC == REC_W3)
        return weno3(v1, v2, v3, eps);
    else if constexpr (REC == REC_W5JS)
        return weno5js(v0, v1, v2, v3, v4, eps);
    else
        return weno5z<Q2>(v0, v1, v2, v3, v4, eps, q);
}

// physical flux along d, the normal velocity v_d and the fast speed c_f
__device__ __forceinline__ void flux(const double U[8], int d, double gam, double F[8], double& vdo, double& cf)
{
    const double rho = U[0], ir = 1.0 / rho;
    const double vx = U[1] * ir, vy = U[2] * ir, vz = U[3] * ir;
    const double Bx = U[5], By = U[6], Bz = U[7];
    const double B2 = Bx * Bx + By * By + Bz * Bz;
    const double S2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    const double p = (gam - 1.0) * (U[4] - 0.5 * S2 * ir - 0.5 * B2);
    const double pt = p + 0.5 * B2;
    const double vB = vx * Bx + vy * By + vz * Bz;
    const double vd = d == 0 ? vx : d == 1 ? vy : vz;
    const double Bd = d == 0 ? Bx : d == 1 ? By : Bz;
    F[0] = U[1 + d];
    F[1] = U[1] * vd - Bd * Bx + (d == 0 ? pt : 0.0);
    F[2] = U[2] * vd - Bd * By + (d == 1 ? pt : 0.0);
    F[3] = U[3] * vd - Bd * Bz + (d == 2 ? pt : 0.0);
    F[4] = (U[4] + pt) * vd - vB * Bd;
    F[5] = vd * Bx - vx * Bd;
    F[6] = vd * By - vy * Bd;
    F[7] = vd * Bz - vz * Bd;
    // (a^2 + b^2)^2 - 4 a^2 b_d^2 as (a^2 - b^2)^2 + 4 a^2 b_t^2: no cancellation
    // where the sound and Alfven speeds meet with B nearly along d
    const double Bt2 = d == 0 ? By * By + Bz * Bz : d == 1 ? Bx * Bx + Bz * Bz : Bx * Bx + By * By;
    const double a2 = gam * p * ir, b2 = B2 * ir, bt2 = Bt2 * ir;
    const double dab = a2 - b2;
    const double cf2 = 0.5 * (a2 + b2 + sqrt(dab * dab + 4.0 * a2 * bt2));
    vdo = vd;
    cf = sqrt(cf2);
}

// Interface flux between cells 2 and 3 of a six-cell line; get(f, m) returns
// cell m (0..5) of field f.  Left state reconstructed around cell 2, right
// state around cell 3 (the left formula on mirrored cells).
template <int NF, int REC, int RS, bool Q2, class Get>
__device__ __forceinline__ void riemann6(Get get, int d, const MhdConst& C, double Fh[NF])
{
    if constexpr (RS == RS_SPLIT) {
        // (F +- alpha U)/2 of the six cells, alpha the largest signal speed
        // among them; left-biased reconstruction of the + part around cell 2,
        // right-biased (mirrored) of the - part around cell 3
        double gp[NF][6], gm[NF][6], alpha = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            double U[NF], F[NF], vd, cf;
#pragma unroll
            for (int f = 0; f < NF; ++f) U[f] = get(f, m);
            flux(U, d, C.gam, F, vd, cf);
            double sp = fabs(vd) + cf;
            if constexpr (NF == 9) {
                F[5 + d] += U[8];
                F[8] = C.ch2 * U[5 + d];
                sp = fmax(sp, C.ch);
            }
            alpha = fmax(alpha, sp);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                gp[f][m] = F[f];
                gm[f][m] = U[f];
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double p[6], q[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                p[m] = 0.5 * (gp[f][m] + alpha * gm[f][m]);
                q[m] = 0.5 * (gp[f][m] - alpha * gm[f][m]);
            }
            Fh[f] = recon<REC, Q2>(p[0], p[1], p[2], p[3], p[4], C.eps[d], C.q) +
                    recon<REC, Q2>(q[5], q[4], q[3], q[2], q[1], C.eps[d], C.q);
        }
        return;
    }
    double UL[NF], UR[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double c0 = get(f, 0), c1 = get(f, 1), c2 = get(f, 2), c3 = get(f, 3), c4 = get(f, 4),
                     c5 = get(f, 5);
        UL[f] = recon<REC, Q2>(c0, c1, c2, c3, c4, C.eps[d], C.q);
        UR[f] = recon<REC, Q2>(c5, c4, c3, c2, c1, C.eps[d], C.q);
    }
    double FL[NF], FR[NF], vL, cL, vR, cR;
    flux(UL, d, C.gam, FL, vL, cL);
    flux(UR, d, C.gam, FR, vR, cR);
    if constexpr (NF == 9) {
        FL[5 + d] += UL[8];
        FR[5 + d] += UR[8];
        FL[8] = C.ch2 * UL[5 + d];
        FR[8] = C.ch2 * UR[5 + d];
    }
    if constexpr (RS == RS_HLL) {
        double SL = fmin(vL - cL, vR - cR), SR = fmax(vL + cL, vR + cR);
        if constexpr (NF == 9) {
            SL = fmin(SL, -C.ch);
            SR = fmax(SR, C.ch);
        }
        SL = fmin(SL, 0.0);
        SR = fmax(SR, 0.0);
        const double id = 1.0 / (SR - SL), SRL = SR * SL;
#pragma unroll
        for (int f = 0; f < NF; ++f) Fh[f] = (SR * FL[f] - SL * FR[f] + SRL * (UR[f] - UL[f])) * id;
    } else {
        double S = fmax(fabs(vL) + cL, fabs(vR) + cR);
        if constexpr (NF == 9) S = fmax(S, C.ch);
#pragma unroll
        for (int f = 0; f < NF; ++f) Fh[f] = 0.5 * (FL[f] + FR[f] - S * (UR[f] - UL[f]));
    }
}

// One workgroup of 16 x 16 threads owns a tile of 15 x 15 columns and marches
// along z over ZC planes.  Per plane: the plane (with a 3-cell halo in x and
// y) is staged in LDS; thread (tx, ty) computes the x-interface flux to the
// left of column (tx, ty) and the y-interface flux below it (the extra row and
// column of threads supply the fluxes on the far side of the tile), so every
// interface flux is computed once; the z-interface flux above the plane comes
// from a 6-cell register window carried along the column, the one below from
// the previous plane.  Then the flux differences form the right-hand side and
// the RK stage update is applied.
constexpr int MT = 15;           // columns per tile edge
constexpr int MB = MT + 1;       // threads per tile edge
constexpr int MH = MT + 6;       // plane width with halo
constexpr int MP = MH + 1;       // LDS row pitch

template <int NF, int REC, int RS, bool Q2>
__global__ __launch_bounds__(MB * MB) void mhd_stage_kernel(StageArgs a, MhdConst C, int zc)
{
    __shared__ double pl[NF][MH][MP];
    __shared__ double fx[NF][MT][MB];
    __shared__ double fy[NF][MB][MT];
    const Tile tile = a.tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const PatchDev P = a.patches[tile.patch];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + MB * ty;
    const int x0 = tile.o[0], y0 = tile.o[1], z0 = tile.o[2];
    const int z1 = min(z0 + zc, P.n[2]);
    const int64_t fs = P.fs;
    const int sz = P.pitch_z;
    const bool col = tx < MT && ty < MT && x0 + tx < P.n[0] && y0 + ty < P.n[1];
    // ghosted-box coordinates of this thread's column
    const int64_t colbase = P.off + (int64_t)(y0 + ty + G) * P.pitch_y + (x0 + tx + G);
    const double* __restrict__ Us = a.Us;

    double w[NF][6];  // cells k-2 .. k+3 of the own column
    double Fm[NF];    // z-flux below the current plane
    if (col) {
        double c7[NF][7];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < 7; ++m) c7[f][m] = Us[colbase + f * fs + (int64_t)(z0 - 3 + m + G) * sz];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < 6; ++m) w[f][m] = c7[f][m + 1];
        riemann6<NF, REC, RS, Q2>([&](int f, int m) { return c7[f][m]; }, 2, C, Fm);
    }
    for (int k = z0; k < z1; ++k) {
        // stage plane k with its x/y halo
        const int64_t pbase = P.off + (int64_t)(k + G) * sz + (int64_t)y0 * P.pitch_y + x0;
        for (int e = tid; e < NF * MH * MH; e += MB * MB) {
            const int f = e / (MH * MH), r = e - f * MH * MH, hy = r / MH, hx = r - hy * MH;
            const bool ok = x0 + hx < P.n[0] + 2 * G && y0 + hy < P.n[1] + 2 * G;
            pl[f][hy][hx] = ok ? Us[pbase + f * fs + (int64_t)hy * P.pitch_y + hx] : 0.0;
        }
        __syncthreads();
        // x-interface to the left of column (tx, ty): cells tx-3 .. tx+2 of row ty
        double Fp[NF];
        if (col) riemann6<NF, REC, RS, Q2>([&](int f, int m) { return w[f][m]; }, 2, C, Fp);
        if (ty < MT && x0 + tx <= P.n[0] && y0 + ty < P.n[1]) {
            double F[NF];
            riemann6<NF, REC, RS, Q2>([&](int f, int m) { return pl[f][ty + G][tx + m]; }, 0, C, F);
#pragma unroll
            for (int f = 0; f < NF; ++f) fx[f][ty][tx] = F[f];
        }
        // y-interface below column (tx, ty)
        if (tx < MT && y0 + ty <= P.n[1] && x0 + tx < P.n[0]) {
            double F[NF];
            riemann6<NF, REC, RS, Q2>([&](int f, int m) { return pl[f][ty + m][tx + G]; }, 1, C, F);
#pragma unroll
            for (int f = 0; f < NF; ++f) fy[f][ty][tx] = F[f];
        }
        __syncthreads();
        if (col) {
            const int64_t cidx = colbase + (int64_t)(k + G) * sz;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double div = (fx[f][ty][tx + 1] - fx[f][ty][tx]) + (fy[f][ty + 1][tx] - fy[f][ty][tx]) +
                                   (Fp[f] - Fm[f]);
                // psi: the damping source at the cell (w[8][2] is plane k of the column)
                const double rhs = f == 8 ? -div * C.ih - C.kpsi * w[f][2] : -div * C.ih;
                stage_store(a, cidx + f * fs, rhs);
            }
            if (k + 1 < z1) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
#pragma unroll
                    for (int m = 0; m < 5; ++m) w[f][m] = w[f][m + 1];
                    w[f][5] = Us[colbase + f * fs + (int64_t)(k + 4 + G) * sz];
                    Fm[f] = Fp[f];
                }
            }
        }
        __syncthreads();
    }
}

template <int NF>
hipError_t dispatch(const SysParams& sp, const StageArgs& a, const MhdConst& C, int zc, hipStream_t s)
{
    const dim3 g(a.ntiles), b(MB, MB, 1);
    const bool hll = sp.mhd_flux == MOL_FLUX_HLL;
    if (sp.mhd_flux == MOL_FLUX_SPLIT) {
        switch (sp.mhd_recon) {
        case MOL_RECON_WENO3: mhd_stage_kernel<NF, REC_W3, RS_SPLIT, true><<<g, b, 0, s>>>(a, C, zc); break;
        case MOL_RECON_WENO5JS: mhd_stage_kernel<NF, REC_W5JS, RS_SPLIT, true><<<g, b, 0, s>>>(a, C, zc); break;
        default:
            if (C.q == 2.0) mhd_stage_kernel<NF, REC_W5Z, RS_SPLIT, true><<<g, b, 0, s>>>(a, C, zc);
            else mhd_stage_kernel<NF, REC_W5Z, RS_SPLIT, false><<<g, b, 0, s>>>(a, C, zc);
        }
        return hipGetLastError();
    }
    switch (sp.mhd_recon) {
    case MOL_RECON_WENO3:
        if (hll) mhd_stage_kernel<NF, REC_W3, RS_HLL, true><<<g, b, 0, s>>>(a, C, zc);
        else mhd_stage_kernel<NF, REC_W3, RS_LLF, true><<<g, b, 0, s>>>(a, C, zc);
        break;
    case MOL_RECON_WENO5JS:
        if (hll) mhd_stage_kernel<NF, REC_W5JS, RS_HLL, true><<<g, b, 0, s>>>(a, C, zc);
        else mhd_stage_kernel<NF, REC_W5JS, RS_LLF, true><<<g, b, 0, s>>>(a, C, zc);
        break;
    default:
        if (C.q == 2.0) {
            if (hll) mhd_stage_kernel<NF, REC_W5Z, RS_HLL, true><<<g, b, 0, s>>>(a, C, zc);
            else mhd_stage_kernel<NF, REC_W5Z, RS_LLF, true><<<g, b, 0, s>>>(a, C, zc);
        } else {
            if (hll) mhd_stage_kernel<NF, REC_W5Z, RS_HLL, false><<<g, b, 0, s>>>(a, C, zc);
            else mhd_stage_kernel<NF, REC_W5Z, RS_LLF, false><<<g, b, 0, s>>>(a, C, zc);
        }
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage_mhd(const SysParams& sp, const StageArgs& a, const int td[3], hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    MhdConst C;
    C.gam = sp.gamma_ad;
    const double h2 = sp.h * sp.h;
    const double e = sp.weno_eps > 0.0 ? sp.weno_eps : (sp.mhd_recon == MOL_RECON_WENO3 ? h2 : h2 * h2);
    C.eps[0] = C.eps[1] = C.eps[2] = e;
    C.q = sp.weno_q;
    C.ih = 1.0 / sp.h;
    if (td[0] != MT || td[1] != MT) return hipErrorInvalidConfiguration;
    C.ch = sp.mhd_ch;
    C.ch2 = sp.mhd_ch * sp.mhd_ch;
    C.kpsi = sp.mhd_kpsi;
    if (sp.system == MOL_MHD_GLM) return dispatch<9>(sp, a, C, td[2], s);
    return dispatch<8>(sp, a, C, td[2], s);
}

}  // namespace mol
