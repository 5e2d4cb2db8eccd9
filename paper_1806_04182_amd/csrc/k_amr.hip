// Ghost fill, its transpose, coarse-fine prolongation and injection kernels
// (the data movement of the Sec. III skeleton), plus a vector update used
// by the RK4 adjoint.
#include "k_common.h"

namespace mol {

namespace {

constexpr int BLK = 256;

int grid_for(int64_t n)
{
    int64_t b = (n + BLK - 1) / BLK;
    return (int)(b < 1 ? 1 : (b > 65535 * 8 ? 65535 * 8 : b));
}

// Copies of nf fields between two points: the loads of up to FC fields are
// issued together before their stores.
constexpr int FC = 8;
__device__ __forceinline__ void copy_fields(const double* __restrict__ src, int64_t sfs, double* __restrict__ dst,
                                            int64_t dfs, int nf)
{
    for (int f0 = 0; f0 < nf; f0 += FC) {
        double v[FC];
#pragma unroll
        for (int j = 0; j < FC; ++j)
            if (f0 + j < nf) v[j] = src[(f0 + j) * sfs];
#pragma unroll
        for (int j = 0; j < FC; ++j)
            if (f0 + j < nf) dst[(f0 + j) * dfs] = v[j];
    }
}

// same-level / periodic copy: ghost <- interior point of the owning patch.
// One thread per (ghost point, group of FC fields), the group the slow index,
// so that a launch has ceil(nf / FC) times as many threads, each with one
// batch of loads in flight, and consecutive threads still copy consecutive
// points.
__global__ __launch_bounds__(BLK) void fill_kernel(const GhostCopy* __restrict__ e, int64_t n, int nf,
                                                   double* __restrict__ U)
{
    const int ng = (nf + FC - 1) / FC;
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * ng; t += (int64_t)gridDim.x * BLK) {
        const int64_t gi = t / n;
        const GhostCopy c = e[t - gi * n];
        const int f0 = (int)gi * FC;
        copy_fields(U + c.src + f0 * c.sfs, c.sfs, U + c.dst + f0 * c.dfs, c.dfs, min(FC, nf - f0));
    }
}

// transpose of the copy: source += its images, images <- 0; one thread per
// (source point, field), the field the slow index (every address is touched
// by exactly one thread)
__global__ __launch_bounds__(BLK) void fill_adjoint_kernel(const GhostSource* __restrict__ src, int64_t n,
                                                           const GhostImage* __restrict__ img, int nf,
                                                           double* __restrict__ A)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * nf; t += (int64_t)gridDim.x * BLK) {
        const int64_t f = t / n;
        const GhostSource s = src[t - f * n];
        double acc = A[s.src + f * s.sfs];
        for (int q = s.beg; q < s.end; ++q) {
            const int64_t d = img[q].dst + f * img[q].dfs;
            acc += A[d];
            A[d] = 0.0;
        }
        A[s.src + f * s.sfs] = acc;
    }
}

struct BorW {
    double w[4];
};

// parent BOR stage state (App. D) T = U^n + sum_j w_j k_j on the band of
// parent points that the prolongation stencils read.  A band entry writes T at
// its position in some parent patch's ghosted box (dst) from the interior
// point that owns it (src), so the parent's k arrays need no ghost fill.
// One thread per (point, field).
__global__ __launch_bounds__(BLK) void bor_band_kernel(const GhostCopy* __restrict__ band, int64_t n, int nf,
                                                       BorW W, const double* __restrict__ Un,
                                                       const double* __restrict__ k0,
                                                       const double* __restrict__ k1,
                                                       const double* __restrict__ k2,
                                                       const double* __restrict__ k3, double* __restrict__ T)
{
    const int64_t tot = n * nf;
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < tot; t += (int64_t)gridDim.x * BLK) {
        const int f = (int)(t / n);
        const GhostCopy b = band[t - (int64_t)f * n];
        const int64_t q = b.src + f * b.sfs;
        T[b.dst + f * b.dfs] = Un[q] + W.w[0] * k0[q] + W.w[1] * k1[q] + W.w[2] * k2[q] + W.w[3] * k3[q];
    }
}

// Lagrange weights at xi = m / R, m = 0 .. R-1
struct LagW {
    double w[4][6];
};

// Coarse-fine ghost points: tensor-product quintic Lagrange interpolation
// (Sec. III.A) of the parent's BOR stage state.  One thread per (parent cell,
// field) loads the cell's stencil once and forms every present fine point of
// the cell, axis by axis (x, then y, then z).  On a fractional axis a point
// with m = 0 takes the node i0 itself (selected, not weighted), so only the
// nodes of its own stencil enter its value.
template <int R>
__global__ __launch_bounds__(BLK) void prolong_kernel(const ProlongCell* __restrict__ e, int64_t n, int nf, LagW L,
                                                      const double* __restrict__ T, double* __restrict__ U)
{
    const int64_t tot = n * nf;
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < tot; t += (int64_t)gridDim.x * BLK) {
        const int f = (int)(t / n);
        const ProlongCell c = e[t - (int64_t)f * n];
        const bool fx = c.frac & 1, fy = c.frac & 2, fz = c.frac & 4;
        const double* __restrict__ base = T + c.cbase + f * c.cfs;
        double out[R][R][R];  // [mz][my][mx]
#pragma unroll
        for (int kc = 0; kc < 6; ++kc) {
            if (kc > 0 && !fz) break;
            double Y[R][R];  // [my][mx] at this z node
#pragma unroll
            for (int kb = 0; kb < 6; ++kb) {
                if (kb > 0 && !fy) break;
                const double* row = base + kc * c.cpz + kb * c.cpy;
                double X[R];
                if (fx) {
                    double r[6];
#pragma unroll
                    for (int a = 0; a < 6; ++a) r[a] = row[a];
                    X[0] = r[2];
#pragma unroll
                    for (int mx = 1; mx < R; ++mx) {
                        double sx = 0.0;
#pragma unroll
                        for (int a = 0; a < 6; ++a) sx += L.w[mx][a] * r[a];
                        X[mx] = sx;
                    }
                } else {
#pragma unroll
                    for (int mx = 0; mx < R; ++mx) X[mx] = row[0];
                }
#pragma unroll
                for (int my = 0; my < R; ++my)
#pragma unroll
                    for (int mx = 0; mx < R; ++mx) {
                        if (!fy) {
                            Y[my][mx] = X[mx];
                        } else if (my == 0) {
                            if (kb == 2) Y[0][mx] = X[mx];
                        } else {
                            Y[my][mx] = (kb == 0 ? 0.0 : Y[my][mx]) + L.w[my][kb] * X[mx];
                        }
                    }
            }
#pragma unroll
            for (int mz = 0; mz < R; ++mz)
#pragma unroll
                for (int my = 0; my < R; ++my)
#pragma unroll
                    for (int mx = 0; mx < R; ++mx) {
                        if (!fz) {
                            out[mz][my][mx] = Y[my][mx];
                        } else if (mz == 0) {
                            if (kc == 2) out[0][my][mx] = Y[my][mx];
                        } else {
                            out[mz][my][mx] = (kc == 0 ? 0.0 : out[mz][my][mx]) + L.w[mz][kc] * Y[my][mx];
                        }
                    }
        }
        double* __restrict__ d = U + c.dbase + f * c.dfs;
#pragma unroll
        for (int mz = 0; mz < R; ++mz)
#pragma unroll
            for (int my = 0; my < R; ++my)
#pragma unroll
                for (int mx = 0; mx < R; ++mx)
                    if (c.mask >> ((mz * R + my) * R + mx) & 1)
                        d[(int64_t)mz * c.dpz + (int64_t)my * c.dpy + mx] = out[mz][my][mx];
    }
}

__global__ __launch_bounds__(BLK) void restrict_kernel(const RestrictPt* __restrict__ e, int64_t n, int nf,
                                                       const double* __restrict__ Uf, double* __restrict__ Uc)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) {
        const RestrictPt r = e[t];
        copy_fields(Uf + r.f, r.ffs, Uc + r.c, r.cfs, nf);
    }
}

__global__ __launch_bounds__(BLK) void axpby_kernel(int64_t n, double a, const double* x,
                                                    double b, const double* y, double* z)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK)
        z[t] = a * x[t] + b * y[t];
}

}  // namespace

hipError_t launch_fill(const GhostCopy* e, int64_t n, int nf, double* U, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    fill_kernel<<<grid_for(n * ((nf + FC - 1) / FC)), BLK, 0, s>>>(e, n, nf, U);
    return hipGetLastError();
}

hipError_t launch_fill_adjoint(const GhostSource* src, int64_t n, const GhostImage* img, int nf, double* A,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    fill_adjoint_kernel<<<grid_for(n * nf), BLK, 0, s>>>(src, n, img, nf, A);
    return hipGetLastError();
}

// Radiative outer boundary (open domain): one thread per (boundary point,
// field); the right-hand side -v (x^i/r) d_i U - v (U - U_inf)/r with 2nd-order
// differences (centred inside the ghosted array, one-sided at its edge), then
// the same Runge-Kutta stage update as the interior.
__global__ __launch_bounds__(BLK) void radiative_kernel(StageArgs a, PatchDev P, const RadPt* __restrict__ pts,
                                                        int64_t n, int nf, RadParams rp, double x0, double y0,
                                                        double z0, double h)
{
    const int N[3] = {P.n[0] + 2 * G, P.n[1] + 2 * G, P.n[2] + 2 * G};
    const int64_t S[3] = {1, P.pitch_y, P.pitch_z};
    const double xl[3] = {x0, y0, z0}, i2h = 0.5 / h;
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * nf; t += (int64_t)gridDim.x * BLK) {
        const int f = (int)(t / n);
        const RadPt q = pts[t - (int64_t)f * n];
        const int64_t idx = P.off + f * P.fs + q.a[2] * S[2] + q.a[1] * S[1] + q.a[0];
        const double* u = a.Us + idx;
        double x[3], r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            x[d] = xl[d] + (P.lo[d] + q.a[d] - G) * h;
            r2 += x[d] * x[d];
        }
        const double ir = 1.0 / sqrt(r2);
        double adv = 0.0;
        for (int d = 0; d < 3; ++d) {
            const int64_t s = S[d];
            double du;
            if (q.a[d] == 0)
                du = (-3.0 * u[0] + 4.0 * u[s] - u[2 * s]) * i2h;
            else if (q.a[d] == N[d] - 1)
                du = (3.0 * u[0] - 4.0 * u[-s] + u[-2 * s]) * i2h;
            else
                du = (u[s] - u[-s]) * i2h;
            adv += x[d] * ir * du;
        }
        const double rhs = -rp.v[f] * adv - rp.v[f] * (u[0] - rp.uinf[f]) * ir;
        stage_apply(a, idx, rhs, stage_load(a, idx));
    }
}

// copy between two level buffers (regrid): dst[e.dst + f dfs] = src[e.src + f sfs]
__global__ __launch_bounds__(BLK) void copy2_kernel(const GhostCopy* __restrict__ e, int64_t n, int nf,
                                                    const double* __restrict__ src, double* __restrict__ dst)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * nf; t += (int64_t)gridDim.x * BLK) {
        const int64_t f = t / n;
        const GhostCopy c = e[t - f * n];
        dst[c.dst + f * c.dfs] = src[c.src + f * c.sfs];
    }
}

hipError_t launch_copy2(const GhostCopy* e, int64_t n, int nf, const double* src, double* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    copy2_kernel<<<grid_for(n * nf), BLK, 0, s>>>(e, n, nf, src, dst);
    return hipGetLastError();
}

hipError_t launch_radiative(const StageArgs& a, const PatchDev& P, const RadPt* pts, int64_t n, int nf,
                            const RadParams& rp, const double xlo[3], double h, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    radiative_kernel<<<grid_for(n * nf), BLK, 0, s>>>(a, P, pts, n, nf, rp, xlo[0], xlo[1], xlo[2], h);
    return hipGetLastError();
}

hipError_t launch_bor_band(const GhostCopy* band, int64_t n, int nf, const double w[4], const double* Un,
                           const double* k0, const double* k1, const double* k2, const double* k3, double* T,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    BorW W;
    for (int j = 0; j < 4; ++j) W.w[j] = w[j];
    bor_band_kernel<<<grid_for(n * nf), BLK, 0, s>>>(band, n, nf, W, Un, k0, k1, k2, k3, T);
    return hipGetLastError();
}

hipError_t launch_prolong(const ProlongCell* e, int64_t n, int nf, int R, const double* lw_host, const double* T,
                          double* U, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    LagW L{};
    if (R < 2 || R > 4) return hipErrorInvalidValue;
    for (int m = 0; m < R; ++m)
        for (int j = 0; j < 6; ++j) L.w[m][j] = lw_host[m * 6 + j];
    switch (R) {
    case 2: prolong_kernel<2><<<grid_for(n * nf), BLK, 0, s>>>(e, n, nf, L, T, U); break;
    case 3: prolong_kernel<3><<<grid_for(n * nf), BLK, 0, s>>>(e, n, nf, L, T, U); break;
    default: prolong_kernel<4><<<grid_for(n * nf), BLK, 0, s>>>(e, n, nf, L, T, U); break;
    }
    return hipGetLastError();
}

hipError_t launch_restrict(const RestrictPt* e, int64_t n, int nf, const double* Uf, double* Uc, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    restrict_kernel<<<grid_for(n), BLK, 0, s>>>(e, n, nf, Uf, Uc);
    return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                        hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    axpby_kernel<<<grid_for(n), BLK, 0, s>>>(n, a, x, b, y, z);
    return hipGetLastError();
}

}  // namespace mol
