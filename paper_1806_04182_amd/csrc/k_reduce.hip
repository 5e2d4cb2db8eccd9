// Deterministic reductions over the interior of a level (norms, the sphere
// integral objective, the Gaussian initial data and its vector-Jacobian
// product).  Order of summation is fixed: each thread walks a fixed set of
// tiles, blocks reduce with a fixed tree in LDS, and one final block reduces
// the per-block partials with the same tree.
#include "k_common.h"

// Sphere membership |x| < R decides which points enter the objective: the
// coordinates and x^2 + y^2 + z^2 are evaluated without FMA contraction so
// that points on the sphere are classified exactly as by a plain C evaluation
// of the same expressions.
#pragma clang fp contract(off)

namespace mol {

namespace {

constexpr int RB = 256;  // threads per reduction block (one tile of 32 x 4 x 2)
constexpr int NQ = 5;    // reduced quantities per launch

struct Red {
    double v[NQ];
};

// q < 2, 3: sums; q == 2: max
// Block reduction: each wave reduces its 64 lanes (wave_sum, or wave_max for
// entry nmaxq), lane 0 of each wave parks the result in LDS, then the RB / 64
// wave results are folded in wave order.  Fixed order throughout: the same
// bits on every run.
constexpr int NWV = RB / 64;
__device__ __forceinline__ void block_reduce(Red& r, double* sh, int nmaxq)
{
    const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int lane = t & 63, wv = t >> 6;
    for (int q = 0; q < NQ; ++q) {
        const double v = q == nmaxq ? wave_max(r.v[q]) : wave_sum(r.v[q]);
        if (lane == 0) sh[q * NWV + wv] = v;
    }
    __syncthreads();
    for (int q = 0; q < NQ; ++q) {
        double v = sh[q * NWV];
        for (int w = 1; w < NWV; ++w) v = q == nmaxq ? fmax(v, sh[q * NWV + w]) : v + sh[q * NWV + w];
        r.v[q] = v;
    }
}

__global__ __launch_bounds__(RB) void norms_kernel(const PatchDev* __restrict__ patches,
                                                   const Tile* __restrict__ tiles, int ntiles,
                                                   const double* __restrict__ U, int field, double shift,
                                                   double r2max, double h, double x0, double y0, double z0,
                                                   CoordBox box, double* __restrict__ partial)
{
    __shared__ double sh[NQ * NWV];
    Red r;
    for (int q = 0; q < NQ; ++q) r.v[q] = 0.0;
    const double dV = h * h * h;
    for (int tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        const Tile t = tiles[tt];
        const PatchDev P = patches[t.patch];
        const int i = t.o[0] + threadIdx.x, j = t.o[1] + threadIdx.y, k = t.o[2] + threadIdx.z;
        if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) continue;
        const double x = x0 + (P.lo[0] + i) * h, y = y0 + (P.lo[1] + j) * h, z = z0 + (P.lo[2] + k) * h;
        if (!(x >= box.lo[0] && x <= box.hi[0] && y >= box.lo[1] && y <= box.hi[1] && z >= box.lo[2] &&
              z <= box.hi[2]))
            continue;
        const double v =
            U[P.off + (int64_t)field * P.fs + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + i + G] -
            shift;
        if (!isfinite(v)) {
            r.v[4] += 1.0;
            continue;
        }
        r.v[0] += fabs(v) * dV;
        r.v[1] += v * v * dV;
        r.v[2] = fmax(r.v[2], fabs(v));
        if (x * x + y * y + z * z < r2max) r.v[3] += v * dV;
    }
    block_reduce(r, sh, 2);
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0)
        for (int q = 0; q < NQ; ++q) partial[blockIdx.x * NQ + q] = r.v[q];
}

__global__ __launch_bounds__(RB) void final_kernel(const double* __restrict__ partial, int nb, int nmaxq,
                                                   double* __restrict__ out)
{
    __shared__ double sh[NQ * NWV];
    Red r;
    for (int q = 0; q < NQ; ++q) r.v[q] = 0.0;
    const int t = threadIdx.x;
    for (int b = t; b < nb; b += RB)
        for (int q = 0; q < NQ; ++q) {
            const double a = partial[b * NQ + q];
            r.v[q] = q == nmaxq ? fmax(r.v[q], a) : r.v[q] + a;
        }
    block_reduce(r, sh, nmaxq);
    if (t == 0)
        for (int q = 0; q < NQ; ++q) out[q] = r.v[q];
}

// Gaussian initial data: field fg = base + A exp(-|d|^2 / w^2), d the
// minimum-image displacement from c; the other nf - 1 fields are constants
// (field f is 1 where bit f of `ones` is set, else 0, as is the base of fg).
// With lam: the vector-Jacobian product sum_points lam[fg] d(A exp(..))/dprm.
__global__ __launch_bounds__(RB) void gaussian_kernel(const PatchDev* __restrict__ patches,
                                                      const Tile* __restrict__ tiles, int ntiles, Red prm,
                                                      double h, double x0, double y0, double z0, double Lx,
                                                      double Ly, double Lz, int nf, int fg, unsigned ones,
                                                      double* __restrict__ U, const double* __restrict__ lam,
                                                      double* __restrict__ partial)
{
    __shared__ double sh[NQ * NWV];
    Red r;
    for (int q = 0; q < NQ; ++q) r.v[q] = 0.0;
    const double A = prm.v[0], w = prm.v[1];
    for (int tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        const Tile t = tiles[tt];
        const PatchDev P = patches[t.patch];
        const int i = t.o[0] + threadIdx.x, j = t.o[1] + threadIdx.y, k = t.o[2] + threadIdx.z;
        if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) continue;
        double d[3] = {x0 + (P.lo[0] + i) * h - prm.v[2], y0 + (P.lo[1] + j) * h - prm.v[3],
                       z0 + (P.lo[2] + k) * h - prm.v[4]};
        const double L[3] = {Lx, Ly, Lz};
        for (int a = 0; a < 3; ++a) d[a] -= L[a] * rint(d[a] / L[a]);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double E = exp(-r2 / (w * w));
        const int64_t c = P.off + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + i + G;
        if (U)
            for (int f = 0; f < nf; ++f) {
                const double base = (ones >> f & 1u) ? 1.0 : 0.0;
                U[c + (int64_t)f * P.fs] = f == fg ? base + A * E : base;
            }
        if (lam) {
            const double l = lam[c + (int64_t)fg * P.fs];
            r.v[0] += l * E;
            r.v[1] += l * A * E * 2.0 * r2 / (w * w * w);
            for (int a = 0; a < 3; ++a) r.v[2 + a] += l * A * E * 2.0 * d[a] / (w * w);
        }
    }
    if (!lam) return;
    block_reduce(r, sh, -1);
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0)
        for (int q = 0; q < NQ; ++q) partial[blockIdx.x * NQ + q] = r.v[q];
}

__global__ __launch_bounds__(RB) void sphere_adjoint_kernel(const PatchDev* __restrict__ patches,
                                                            const Tile* __restrict__ tiles, int nf, int field,
                                                            double r2max, double w, double h, double x0,
                                                            double y0, double z0, double* __restrict__ lam)
{
    const Tile t = tiles[blockIdx.x];
    const PatchDev P = patches[t.patch];
    const int i = t.o[0] + threadIdx.x, j = t.o[1] + threadIdx.y, k = t.o[2] + threadIdx.z;
    if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) return;
    const int64_t c = P.off + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + i + G;
    const double x = x0 + (P.lo[0] + i) * h, y = y0 + (P.lo[1] + j) * h, z = z0 + (P.lo[2] + k) * h;
    const double v = x * x + y * y + z * z < r2max ? w : 0.0;
    for (int f = 0; f < nf; ++f) lam[c + f * P.fs] = f == field ? v : 0.0;
}

}  // namespace

hipError_t launch_sphere_adjoint(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], int nf,
                                 int field, double radius, double scale, double h, const double xlo[3], double* lam,
                                 hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    sphere_adjoint_kernel<<<ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, nf, field, radius * radius,
                                                                       scale * h * h * h, h, xlo[0], xlo[1],
                                                                       xlo[2], lam);
    return hipGetLastError();
}

namespace {
// refinement tagging: flags[(gz * py + gy) * px + gx] = 1 where |U[field]| >= thr
__global__ __launch_bounds__(RB) void tag_kernel(const PatchDev* __restrict__ patches, const Tile* __restrict__ tiles,
                                                 const double* __restrict__ U, int field, double thr, int px, int py,
                                                 uint8_t* __restrict__ flags)
{
    const Tile t = tiles[blockIdx.x];
    const PatchDev P = patches[t.patch];
    const int i = t.o[0] + threadIdx.x, j = t.o[1] + threadIdx.y, k = t.o[2] + threadIdx.z;
    if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) return;
    const double v =
        U[P.off + (int64_t)field * P.fs + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + i + G];
    if (fabs(v) >= thr)
        flags[((int64_t)(P.lo[2] + k) * py + (P.lo[1] + j)) * px + (P.lo[0] + i)] = 1;
}
}  // namespace

hipError_t launch_tag(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], const double* U,
                      int field, double thr, const int period[3], uint8_t* flags, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    tag_kernel<<<ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, U, field, thr, period[0], period[1], flags);
    return hipGetLastError();
}

hipError_t launch_norms(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], const double* U,
                        int field, double shift, double radius, double h, const double xlo[3], const CoordBox& box,
                        double* partial, int nblocks, double* out, hipStream_t s)
{
    if (td[0] * td[1] * td[2] != RB) return hipErrorInvalidValue;
    norms_kernel<<<nblocks, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, ntiles, U, field, shift,
                                                               radius * radius, h, xlo[0], xlo[1], xlo[2], box,
                                                               partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    final_kernel<<<1, RB, 0, s>>>(partial, nblocks, 2, out);
    return hipGetLastError();
}

hipError_t launch_gaussian(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3],
                           const double prm5[5], double h, const double xlo[3], const double per[3], int nf, int fg,
                           unsigned ones, double* U, const double* lam, double* partial, int nblocks, double* grad,
                           hipStream_t s)
{
    if (td[0] * td[1] * td[2] != RB) return hipErrorInvalidValue;
    Red prm;
    for (int q = 0; q < NQ; ++q) prm.v[q] = prm5[q];
    const int nb = lam ? nblocks : (ntiles < 1 ? 1 : ntiles);
    gaussian_kernel<<<nb, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, ntiles, prm, h, xlo[0], xlo[1],
                                                             xlo[2], per[0], per[1], per[2], nf, fg, ones, U, lam,
                                                             partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !lam) return e;
    final_kernel<<<1, RB, 0, s>>>(partial, nblocks, -1, grad);
    return hipGetLastError();
}

}  // namespace mol
