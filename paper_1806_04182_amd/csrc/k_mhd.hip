// Newtonian ideal MHD (Sec. IV.B, eight-field core: rho, S, E, B) in the
// conservative finite-difference form (eq. conservative_discretization):
//   L = - sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d,
// with the evolved fields reconstructed at every interface by WENO5-Z
// (App. B; q = 2, eps = dx^4 unless set) and the local Lax-Friedrichs flux
// (eq. LLF) F = (F(U^L) + F(U^R) - S (U^R - U^L)) / 2, where S is the larger
// of |v_d| + c_f over the two states (fast magnetosonic speed c_f).  Fused with
// the Runge-Kutta stage update.
#include "k_common.h"

namespace mol {

namespace {

struct MhdConst {
    double gam;
    double eps[3];
    double q;
    double ih;  // 1 / dx
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

// physical flux along d and the signal speed |v_d| + c_f
__device__ __forceinline__ void flux(const double U[8], int d, double gam, double F[8], double& spd)
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
    const double a2 = gam * p * ir, b2 = B2 * ir, bd2 = Bd * Bd * ir;
    const double sm = a2 + b2;
    const double cf2 = 0.5 * (sm + sqrt(sm * sm - 4.0 * a2 * bd2));
    spd = fabs(vd) + sqrt(cf2);
}

// LLF flux at the interface between cells 2 and 3 of a six-cell line; get(f, m)
// returns cell m (0..5) of field f.  Left state reconstructed around cell 2,
// right state around cell 3 (the left formula on mirrored cells).
template <bool Q2, class Get>
__device__ __forceinline__ void llf6(Get get, int d, const MhdConst& C, double Fh[8])
{
    double UL[8], UR[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) {
        const double c0 = get(f, 0), c1 = get(f, 1), c2 = get(f, 2), c3 = get(f, 3), c4 = get(f, 4),
                     c5 = get(f, 5);
        UL[f] = weno5z<Q2>(c0, c1, c2, c3, c4, C.eps[d], C.q);
        UR[f] = weno5z<Q2>(c5, c4, c3, c2, c1, C.eps[d], C.q);
    }
    double FL[8], FR[8], sL, sR;
    flux(UL, d, C.gam, FL, sL);
    flux(UR, d, C.gam, FR, sR);
    const double S = fmax(sL, sR);
#pragma unroll
    for (int f = 0; f < 8; ++f) Fh[f] = 0.5 * (FL[f] + FR[f] - S * (UR[f] - UL[f]));
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

template <bool Q2>
__global__ __launch_bounds__(MB * MB) void mhd_stage_kernel(StageArgs a, MhdConst C, int zc)
{
    __shared__ double pl[8][MH][MP];
    __shared__ double fx[8][MT][MB];
    __shared__ double fy[8][MB][MT];
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

    double w[8][6];  // cells k-2 .. k+3 of the own column
    double Fm[8];    // z-flux below the current plane
    if (col) {
        double c7[8][7];
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int m = 0; m < 7; ++m) c7[f][m] = Us[colbase + f * fs + (int64_t)(z0 - 3 + m + G) * sz];
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int m = 0; m < 6; ++m) w[f][m] = c7[f][m + 1];
        llf6<Q2>([&](int f, int m) { return c7[f][m]; }, 2, C, Fm);
    }
    for (int k = z0; k < z1; ++k) {
        // stage plane k with its x/y halo
        const int64_t pbase = P.off + (int64_t)(k + G) * sz + (int64_t)y0 * P.pitch_y + x0;
        for (int e = tid; e < 8 * MH * MH; e += MB * MB) {
            const int f = e / (MH * MH), r = e - f * MH * MH, hy = r / MH, hx = r - hy * MH;
            const bool ok = x0 + hx < P.n[0] + 2 * G && y0 + hy < P.n[1] + 2 * G;
            pl[f][hy][hx] = ok ? Us[pbase + f * fs + (int64_t)hy * P.pitch_y + hx] : 0.0;
        }
        __syncthreads();
        // x-interface to the left of column (tx, ty): cells tx-3 .. tx+2 of row ty
        double Fp[8];
        if (col) llf6<Q2>([&](int f, int m) { return w[f][m]; }, 2, C, Fp);
        if (ty < MT && x0 + tx <= P.n[0] && y0 + ty < P.n[1]) {
            double F[8];
            llf6<Q2>([&](int f, int m) { return pl[f][ty + G][tx + m]; }, 0, C, F);
#pragma unroll
            for (int f = 0; f < 8; ++f) fx[f][ty][tx] = F[f];
        }
        // y-interface below column (tx, ty)
        if (tx < MT && y0 + ty <= P.n[1] && x0 + tx < P.n[0]) {
            double F[8];
            llf6<Q2>([&](int f, int m) { return pl[f][ty + m][tx + G]; }, 1, C, F);
#pragma unroll
            for (int f = 0; f < 8; ++f) fy[f][ty][tx] = F[f];
        }
        __syncthreads();
        if (col) {
            const int64_t cidx = colbase + (int64_t)(k + G) * sz;
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const double div = (fx[f][ty][tx + 1] - fx[f][ty][tx]) + (fy[f][ty + 1][tx] - fy[f][ty][tx]) +
                                   (Fp[f] - Fm[f]);
                stage_store(a, cidx + f * fs, -div * C.ih);
            }
            if (k + 1 < z1) {
#pragma unroll
                for (int f = 0; f < 8; ++f) {
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

}  // namespace

hipError_t launch_stage_mhd(const SysParams& sp, const StageArgs& a, const int td[3], hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    MhdConst C;
    C.gam = sp.gamma_ad;
    const double e = sp.weno_eps > 0.0 ? sp.weno_eps : sp.h * sp.h * sp.h * sp.h;
    C.eps[0] = C.eps[1] = C.eps[2] = e;
    C.q = sp.weno_q;
    C.ih = 1.0 / sp.h;
    if (td[0] != MT || td[1] != MT) return hipErrorInvalidConfiguration;
    if (C.q == 2.0)
        mhd_stage_kernel<true><<<a.ntiles, dim3(MB, MB, 1), 0, s>>>(a, C, td[2]);
    else
        mhd_stage_kernel<false><<<a.ntiles, dim3(MB, MB, 1), 0, s>>>(a, C, td[2]);
    return hipGetLastError();
}

}  // namespace mol
