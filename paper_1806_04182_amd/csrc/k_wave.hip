// Scalar wave (Sec. IV.A, first order in time):
//   d_t phi = -Pi + Q phi,   d_t Pi = -(D_xx + D_yy + D_zz) phi + Q Pi,
// with the 4th-order D_xx of Sec. II.B.1 and KO dissipation Q on both fields,
// fused with the Runge-Kutta stage update; and the transpose of the
// right-hand side (project addition, for the adjoint).
#include "k_common.h"

namespace mol {

namespace {

__global__ __launch_bounds__(256) void wave_stage_kernel(StageArgs a, double ih2, double ko)
{
    PointRef pr;
    int i, j, k, p;
    if (!tile_point(a, xcd_tile(blockIdx.x, gridDim.x), pr, i, j, k, p)) return;
    const double* phi = a.Us + pr.c;
    const double* pi = phi + pr.fs;
    const int s[3] = {1, pr.sy, pr.sz};
    double lap = 0.0, qphi = 0.0, qpi = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lap += fd2(phi, s[d]);
        qphi += fko(phi, s[d]);
        qpi += fko(pi, s[d]);
    }
    stage_store(a, pr.c, -pi[0] + ko * qphi);
    stage_store(a, pr.c + pr.fs, -ih2 * lap + ko * qpi);
}

// lamU(p) = sum_c lam(c) dR(c)/dU(p): the stencils are symmetric, so the
// transpose reads lam at the same offsets, restricted to interior points.
__global__ __launch_bounds__(256) void wave_adjoint_kernel(const PatchDev* __restrict__ patches,
                                                           const Tile* __restrict__ tiles,
                                                           const double* __restrict__ lam,
                                                           double* __restrict__ lamU, double ih2,
                                                           double ko)
{
    const Tile t = tiles[blockIdx.x];
    const PatchDev P = patches[t.patch];
    const int i = t.o[0] + (int)threadIdx.x, j = t.o[1] + (int)threadIdx.y,
              k = t.o[2] + (int)threadIdx.z;
    if (i >= P.n[0] + G || j >= P.n[1] + G || k >= P.n[2] + G) return;
    const int64_t c = P.off + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + (i + G);
    const double* lp = lam + c;
    const double* lq = lam + c + P.fs;
    const int q[3] = {i, j, k};
    const int s[3] = {1, P.pitch_y, P.pitch_z};
    const double kow[4] = {-20.0, 15.0, -6.0, 1.0};
    const double d2w[3] = {-30.0, 16.0, -1.0};
    auto inside = [&](int d, int off) {
        int a0 = q[0], a1 = q[1], a2 = q[2];
        if (d == 0) a0 += off;
        if (d == 1) a1 += off;
        if (d == 2) a2 += off;
        return a0 >= 0 && a0 < P.n[0] && a1 >= 0 && a1 < P.n[1] && a2 >= 0 && a2 < P.n[2];
    };
    double gphi = 0.0, gpi = 0.0, gd2 = 0.0;
    const bool self = inside(0, 0);
    const double lp0 = self ? lp[0] : 0.0, lq0 = self ? lq[0] : 0.0;
    // the centre weight appears once per axis
    gphi += 3.0 * kow[0] * lp0;
    gpi += 3.0 * kow[0] * lq0;
    gd2 += 3.0 * d2w[0] * lq0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int m = 1; m <= 3; ++m) {
            // offsets of points outside the interior are replaced by 0 (the
            // point itself, always addressable) and the value loaded there is
            // discarded
            const bool up = inside(d, m), dn = inside(d, -m);
            const int ou = up ? m * s[d] : 0, od = dn ? -m * s[d] : 0;
            const double pu = lp[ou], pd = lp[od], qu = lq[ou], qd = lq[od];
            const double sp = (up ? pu : 0.0) + (dn ? pd : 0.0);
            const double sq = (up ? qu : 0.0) + (dn ? qd : 0.0);
            gphi += kow[m] * sp;
            gpi += kow[m] * sq;
            if (m <= 2) gd2 += d2w[m] * sq;
        }
    }
    lamU[c] = ko * gphi - ih2 * gd2;
    lamU[c + P.fs] = -lp0 + ko * gpi;
}

}  // namespace

hipError_t launch_stage_wave(const SysParams& sp, const StageArgs& a, const int td[3], hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    const double ih2 = 1.0 / (12.0 * sp.h * sp.h);
    const double ko = sp.sigma / (64.0 * sp.h);
    wave_stage_kernel<<<a.ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(a, ih2, ko);
    return hipGetLastError();
}

hipError_t launch_wave_adjoint(const SysParams& sp, const PatchDev* patches, const Tile* tiles, int ntiles,
                               const int td[3], const double* lam, double* lamU, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const double ih2 = 1.0 / (12.0 * sp.h * sp.h);
    const double ko = sp.sigma / (64.0 * sp.h);
    wave_adjoint_kernel<<<ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, lam, lamU, ih2, ko);
    return hipGetLastError();
}

}  // namespace mol
