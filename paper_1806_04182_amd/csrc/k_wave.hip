// Scalar wave (Sec. IV.A, first order in time):
//   d_t phi = -Pi + Q phi,   d_t Pi = -(D_xx + D_yy + D_zz) phi + Q Pi,
// with the 4th-order D_xx of Sec. II.B.1 and KO dissipation Q on both fields,
// fused with the Runge-Kutta stage update; and the transpose of the
// right-hand side (project addition, for the adjoint).
#include "k_common.h"

namespace mol {

namespace {

// WRAP: the patch is the whole periodic domain (at least 4 points per axis)
// and the neighbours are read at the periodic images of interior points, so
// that the stage needs no ghost fill; the stencils see the same values.
template <bool WRAP>
__global__ __launch_bounds__(256) void wave_stage_kernel(StageArgs a, double ih2, double ko)
{
    PointRef pr;
    int i, j, k, p;
    if (!tile_point(a, xcd_tile(blockIdx.x, gridDim.x), pr, i, j, k, p)) return;
    const double* phi = a.Us + pr.c;
    const double* pi = phi + pr.fs;
    const int s[3] = {1, pr.sy, pr.sz};
    double lap = 0.0, qphi = 0.0, qpi = 0.0;
    if constexpr (WRAP) {
        const int q[3] = {i, j, k};
        const int* n = a.patches[p].n;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double vp[7], vq[7];
#pragma unroll
            for (int o = -3; o <= 3; ++o) {
                int c = q[d] + o;
                c = c < 0 ? c + n[d] : (c >= n[d] ? c - n[d] : c);
                const int64_t off = (int64_t)(c - q[d]) * s[d];
                vp[o + 3] = phi[off];
                vq[o + 3] = pi[off];
            }
            lap += fd2(vp + 3, 1);
            qphi += fko(vp + 3, 1);
            qpi += fko(vq + 3, 1);
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lap += fd2(phi, s[d]);
            qphi += fko(phi, s[d]);
            qpi += fko(pi, s[d]);
        }
    }
    stage_store(a, pr.c, -pi[0] + ko * qphi);
    stage_store(a, pr.c + pr.fs, -ih2 * lap + ko * qpi);
}

// Large levels: a workgroup of WX x WY threads owns WX x WY columns and marches
// along z over zc planes.  z-neighbours come from a 7-value register queue per
// field (each value is read from memory once per column); x/y neighbours from
// the current plane staged in LDS, whose interior part is written from the
// queues and whose 3-point halo is loaded from memory.  The halo cells of a
// plane are dealt out to the threads once (NH cells each, fixed offsets), so
// the per-plane loop has no index arithmetic; columns beyond the patch
// interior (ragged tail) load their own cell like a halo cell.
constexpr int WX = MOL_WAVE_WX, WY = MOL_WAVE_WY, WHX = WX + 6, WHY = WY + 6, WPX = WHX + 2;
constexpr int WNH = 6 * WHX + 6 * WY;                   // halo cells per plane
constexpr int WT = WX * WY, NH = (WNH + WT - 1) / WT;  // halo cells per thread

// WRAP: the patch is the whole periodic domain; every cell outside the
// interior (halo cells, the column queue's planes, ragged-tail cells) is read
// at its periodic image, so the stage needs no ghost fill.
template <bool NT, bool WRAP>
__global__ __launch_bounds__(WT) void wave_zmarch_kernel(StageArgs a, double ih2, double ko, int zc)
{
    __shared__ double pl[2][WHY][WPX];
    const Tile tile = a.tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const PatchDev P = a.patches[tile.patch];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + WX * ty;
    const int x0 = tile.o[0], y0 = tile.o[1], z0 = tile.o[2];
    const int z1 = min(z0 + zc, P.n[2]);
    const int sz = P.pitch_z;
    const bool col = x0 + tx < P.n[0] && y0 + ty < P.n[1];
    // own cell in the ghosted box (ragged-tail columns may lie beyond it)
    const bool cin = x0 + tx < P.n[0] + G && y0 + ty < P.n[1] + G;
    const int64_t cb = P.off + (int64_t)(y0 + ty + G) * P.pitch_y + (x0 + tx + G);
    const double* __restrict__ U = a.Us;
    // periodic image of interior coordinate v in [-3, n + 3)
    auto wrapc = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    // plane offset of interior plane z (its image when WRAP)
    auto plane = [&](int z) -> int64_t { return (int64_t)((WRAP ? wrapc(z, P.n[2]) : z) + G) * sz; };
    // in-plane offset (from the patch start) of a ragged-tail column's own
    // cell: its image when WRAP (-1: beyond the reach of the stencils)
    const int64_t cwo = !WRAP ? cb - P.off
                        : cin ? (int64_t)(wrapc(y0 + ty, P.n[1]) + G) * P.pitch_y + wrapc(x0 + tx, P.n[0]) + G
                              : -1;
    // this thread's halo cells: LDS slot (-1: none) and offset in the plane
    // (-1: outside the ghosted box)
    int hl[NH], hg[NH];
#pragma unroll
    for (int r = 0; r < NH; ++r) {
        const int e = tid + r * WT;
        int hx = 0, hy = 0;
        if (e < 6 * WHX) {  // three rows below and three above the columns
            hy = e / WHX;
            hx = e - hy * WHX;
            if (hy >= 3) hy += WY;
        } else {            // three cells left and right of every column row
            const int q = e - 6 * WHX, row = q / 6, c = q - row * 6;
            hy = G + row;
            hx = c < 3 ? c : WX + c;
        }
        const bool ok = e < WNH && x0 + hx < P.n[0] + 2 * G && y0 + hy < P.n[1] + 2 * G;
        hl[r] = e < WNH ? hy * WPX + hx : -1;
        if constexpr (WRAP)  // offset from the patch start, at the image
            hg[r] = ok ? (wrapc(y0 + hy - G, P.n[1]) + G) * P.pitch_y + wrapc(x0 + hx - G, P.n[0]) + G : -1;
        else                 // offset from the tile's ghosted-box corner
            hg[r] = ok ? hy * P.pitch_y + hx : -1;
    }
    double qp[7], qq[7];  // phi and Pi at z = k-3 .. k+3
    if (col)
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            qp[m] = U[cb + plane(z0 - 3 + m)];
            qq[m] = U[cb + P.fs + plane(z0 - 3 + m)];
        }
    // halo cells and stage-update inputs are fetched one plane ahead
    double hp[NH], hq[NH];
    StageIn sp, sq;
    auto fetch = [&](int k, double* np, double* nq, StageIn& s0, StageIn& s1) __attribute__((always_inline)) {
        const int64_t hb = P.off + (int64_t)(k + G) * sz + (WRAP ? 0 : (int64_t)y0 * P.pitch_y + x0);
#pragma unroll
        for (int r = 0; r < NH; ++r) {
            const bool ok = hg[r] >= 0;
            np[r] = ok ? U[hb + hg[r]] : 0.0;
            nq[r] = ok ? U[hb + P.fs + hg[r]] : 0.0;
        }
        if (col) {
            const int64_t c = cb + (int64_t)(k + G) * sz;
            s0 = stage_load<NT>(a, c);
            s1 = stage_load<NT>(a, c + P.fs);
        }
    };
    if (z0 < z1) fetch(z0, hp, hq, sp, sq);
    for (int k = z0; k < z1; ++k) {
        const int64_t pc = (int64_t)(k + G) * sz;
        if (col) {
            qp[6] = U[cb + plane(k + 3)];
            qq[6] = U[cb + P.fs + plane(k + 3)];
            pl[0][ty + G][tx + G] = qp[3];
            pl[1][ty + G][tx + G] = qq[3];
        } else {
            pl[0][ty + G][tx + G] = cwo >= 0 && cin ? U[P.off + pc + cwo] : 0.0;
            pl[1][ty + G][tx + G] = cwo >= 0 && cin ? U[P.off + P.fs + pc + cwo] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < NH; ++r)
            if (hl[r] >= 0) {
                (&pl[0][0][0])[hl[r]] = hp[r];
                (&pl[1][0][0])[hl[r]] = hq[r];
            }
        const StageIn cp = sp, cq = sq;
        if (k + 1 < z1) fetch(k + 1, hp, hq, sp, sq);
        __syncthreads();
        if (col) {
            const double* p = &pl[0][ty + G][tx + G];
            const double* q = &pl[1][ty + G][tx + G];
            double lap = fd2(p, 1) + fd2(p, WPX) + fd2(qp + 3, 1);
            double qphi = fko(p, 1) + fko(p, WPX) + fko(qp + 3, 1);
            double qpi = fko(q, 1) + fko(q, WPX) + fko(qq + 3, 1);
            stage_apply<NT>(a, cb + pc, -q[0] + ko * qphi, cp);
            stage_apply<NT>(a, cb + pc + P.fs, -ih2 * lap + ko * qpi, cq);
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                qp[m] = qp[m + 1];
                qq[m] = qq[m + 1];
            }
        }
        __syncthreads();
    }
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
    if (td[0] == WX && td[1] == WY && td[2] > 1) {
        // levels larger than the caches: the point loads and stores of the
        // stage update are non-temporal (6-7% faster at 256^3 and 512^3,
        // 18% slower at 128^3, where the arrays stay in the caches)
        const dim3 g(a.ntiles), b(WX, WY, 1);
        if (a.stream)
            a.wrap ? wave_zmarch_kernel<true, true><<<g, b, 0, s>>>(a, ih2, ko, td[2])
                   : wave_zmarch_kernel<true, false><<<g, b, 0, s>>>(a, ih2, ko, td[2]);
        else
            a.wrap ? wave_zmarch_kernel<false, true><<<g, b, 0, s>>>(a, ih2, ko, td[2])
                   : wave_zmarch_kernel<false, false><<<g, b, 0, s>>>(a, ih2, ko, td[2]);
    } else if (a.wrap) {
        wave_stage_kernel<true><<<a.ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(a, ih2, ko);
    } else {
        wave_stage_kernel<false><<<a.ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(a, ih2, ko);
    }
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
