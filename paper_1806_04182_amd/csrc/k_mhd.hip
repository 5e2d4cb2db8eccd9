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
    if (q == 2.0) {
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

// LLF flux at the interface between u[0] and u[st] along d (u: field 0 at the
// left cell; fields fs apart)
__device__ __forceinline__ void llf(const double* __restrict__ u, int64_t fs, int st, int d,
                                    const MhdConst& C, double Fh[8])
{
    double UL[8], UR[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) {
        const double* w = u + f * fs;
        const double m2 = w[-2 * st], m1 = w[-st], c0 = w[0], p1 = w[st], p2 = w[2 * st], p3 = w[3 * st];
        UL[f] = weno5z(m2, m1, c0, p1, p2, C.eps[d], C.q);
        UR[f] = weno5z(p3, p2, p1, c0, m1, C.eps[d], C.q);
    }
    double FL[8], FR[8], sL, sR;
    flux(UL, d, C.gam, FL, sL);
    flux(UR, d, C.gam, FR, sR);
    const double S = fmax(sL, sR);
#pragma unroll
    for (int f = 0; f < 8; ++f) Fh[f] = 0.5 * (FL[f] + FR[f] - S * (UR[f] - UL[f]));
}

__global__ __launch_bounds__(256) void mhd_stage_kernel(StageArgs a, MhdConst C)
{
    PointRef pr;
    int i, j, k, p;
    if (!tile_point(a, xcd_tile(blockIdx.x, gridDim.x), pr, i, j, k, p)) return;
    const double* u = a.Us + pr.c;
    const int s[3] = {1, pr.sy, pr.sz};
    double rhs[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) rhs[f] = 0.0;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        double Fp[8], Fm[8];
        llf(u, pr.fs, s[d], d, C, Fp);
        llf(u - s[d], pr.fs, s[d], d, C, Fm);
#pragma unroll
        for (int f = 0; f < 8; ++f) rhs[f] -= (Fp[f] - Fm[f]) * C.ih;
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) stage_store(a, pr.c + f * pr.fs, rhs[f]);
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
    mhd_stage_kernel<<<a.ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(a, C);
    return hipGetLastError();
}

}  // namespace mol
