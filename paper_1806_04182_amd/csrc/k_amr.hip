// Ghost fill, its transpose, coarse-fine prolongation and injection kernels
// (the data movement of the Sec. III skeleton), plus a vector update used
// by the RK4 adjoint.
#include "molamr_int.h"

namespace mol {

namespace {

constexpr int BLK = 256;

int grid_for(int64_t n)
{
    int64_t b = (n + BLK - 1) / BLK;
    return (int)(b < 1 ? 1 : (b > 65535 * 8 ? 65535 * 8 : b));
}

// same-level / periodic copy: ghost <- interior point of the owning patch
__global__ __launch_bounds__(BLK) void fill_kernel(const GhostCopy* __restrict__ e, int64_t n, int nf,
                                                   double* __restrict__ U)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) {
        const GhostCopy c = e[t];
        for (int f = 0; f < nf; ++f) U[c.dst + f * c.dfs] = U[c.src + f * c.sfs];
    }
}

// transpose of the copy: source += its images, images <- 0
__global__ __launch_bounds__(BLK) void fill_adjoint_kernel(const GhostSource* __restrict__ src, int64_t n,
                                                           const GhostImage* __restrict__ img, int nf,
                                                           double* __restrict__ A)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) {
        const GhostSource s = src[t];
        for (int f = 0; f < nf; ++f) {
            double acc = A[s.src + f * s.sfs];
            for (int q = s.beg; q < s.end; ++q) {
                const int64_t d = img[q].dst + f * img[q].dfs;
                acc += A[d];
                A[d] = 0.0;
            }
            A[s.src + f * s.sfs] = acc;
        }
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

// Lagrange weights at xi = m / R, m = 0 .. R-1 (row 0: the coincident copy)
struct LagW {
    double w[4][6];
};

// coarse-fine ghost point: tensor-product Lagrange interpolation (Sec. III.A)
// of the parent's BOR stage state; one thread per (ghost point, field)
__global__ __launch_bounds__(BLK) void prolong_kernel(const ProlongPt* __restrict__ e, int64_t n, int nf, LagW L,
                                                      const double* __restrict__ T, double* __restrict__ U)
{
    const int64_t tot = n * nf;
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < tot; t += (int64_t)gridDim.x * BLK) {
        const int f = (int)(t / n);
        const ProlongPt p = e[t - (int64_t)f * n];
        const int cx = p.m[0] ? 6 : 1, cy = p.m[1] ? 6 : 1, cz = p.m[2] ? 6 : 1;
        const double* wx = L.w[p.m[0]];
        const double* wy = L.w[p.m[1]];
        const double* wz = L.w[p.m[2]];
        const int64_t base = p.cbase + f * p.cfs;
        double sz = 0.0;
        for (int c = 0; c < cz; ++c) {
            double sy = 0.0;
            for (int b = 0; b < cy; ++b) {
                const double* row = T + base + (int64_t)c * p.cpz + (int64_t)b * p.cpy;
                double sx = 0.0;
                if (cx == 6) {
#pragma unroll
                    for (int a = 0; a < 6; ++a) sx += wx[a] * row[a];
                } else {
                    sx = row[0];
                }
                sy += wy[b] * sx;
            }
            sz += wz[c] * sy;
        }
        U[p.dst + f * p.dfs] = sz;
    }
}

__global__ __launch_bounds__(BLK) void restrict_kernel(const RestrictPt* __restrict__ e, int64_t n, int nf,
                                                       const double* __restrict__ Uf, double* __restrict__ Uc)
{
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) {
        const RestrictPt r = e[t];
        for (int f = 0; f < nf; ++f) Uc[r.c + f * r.cfs] = Uf[r.f + f * r.ffs];
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
    fill_kernel<<<grid_for(n), BLK, 0, s>>>(e, n, nf, U);
    return hipGetLastError();
}

hipError_t launch_fill_adjoint(const GhostSource* src, int64_t n, const GhostImage* img, int nf, double* A,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    fill_adjoint_kernel<<<grid_for(n), BLK, 0, s>>>(src, n, img, nf, A);
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

hipError_t launch_prolong(const ProlongPt* e, int64_t n, int nf, int R, const double* lw_host, const double* T,
                          double* U, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (R < 1 || R > 4) return hipErrorInvalidValue;
    LagW L{};
    for (int m = 0; m < R; ++m)
        for (int j = 0; j < 6; ++j) L.w[m][j] = lw_host[m * 6 + j];
    prolong_kernel<<<grid_for(n * nf), BLK, 0, s>>>(e, n, nf, L, T, U);
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
