// Puncture initial data of Sec. V (eq. conformal_factor and the Bowen-York
// extrinsic curvature below it): one thread per point of a level, interior
// points only or the whole ghosted boxes.
//   psi = 1 + sum_A m_A / (2 r_A),  chi = psi^-4,  alpha = psi^-2,
//   gt_ij = delta_ij,  At_ij = psi^-6 sum_A [ 3/(2 r^2) (P_i n_j + P_j n_i
//        - (delta_ij - n_i n_j) P.n) + 3/r^3 (n_j w_i + n_i w_j) ],
// with w = S x n (so that eps_kil S^l n^k = w_i), every other field zero.
#include "molamr_int.h"

namespace mol {

namespace {

struct Holes {
    int n;
    double v[MOL_MAX_HOLES * 10];  // m, c[3], P[3], S[3] per hole
};

__global__ __launch_bounds__(256) void puncture_kernel(const PatchDev* __restrict__ patches,
                                                       const Tile* __restrict__ tiles, int ntiles, Holes H,
                                                       double h, double x0, double y0, double z0, int whole,
                                                       double* __restrict__ U)
{
    const int tt = blockIdx.x;
    if (tt >= ntiles) return;
    const Tile t = tiles[tt];
    const PatchDev P = patches[t.patch];
    const int i = t.o[0] + threadIdx.x, j = t.o[1] + threadIdx.y, k = t.o[2] + threadIdx.z;
    const int g = whole ? G : 0;
    if (i < -g || j < -g || k < -g || i >= P.n[0] + g || j >= P.n[1] + g || k >= P.n[2] + g) return;
    const double x[3] = {x0 + (P.lo[0] + i) * h, y0 + (P.lo[1] + j) * h, z0 + (P.lo[2] + k) * h};
    double psi = 1.0, A[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < H.n; ++a) {
        const double* hv = H.v + 10 * a;
        const double d[3] = {x[0] - hv[1], x[1] - hv[2], x[2] - hv[3]};
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double ir = 1.0 / r;
        psi += hv[0] * 0.5 * ir;
        const double n[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
        const double* Pm = hv + 4;
        const double* S = hv + 7;
        const double Pn = Pm[0] * n[0] + Pm[1] * n[1] + Pm[2] * n[2];
        const double w[3] = {S[1] * n[2] - S[2] * n[1], S[2] * n[0] - S[0] * n[2], S[0] * n[1] - S[1] * n[0]};
        const double cp = 1.5 * ir * ir, cs = 3.0 * ir * ir * ir;
        int q = 0;
        for (int p = 0; p < 3; ++p)
            for (int s = p; s < 3; ++s, ++q) {
                const double dps = p == s ? 1.0 : 0.0;
                A[q] += cp * (Pm[p] * n[s] + Pm[s] * n[p] - (dps - n[p] * n[s]) * Pn) + cs * (n[s] * w[p] + n[p] * w[s]);
            }
    }
    const double ip2 = 1.0 / (psi * psi), ip4 = ip2 * ip2, ip6 = ip4 * ip2;
    const int64_t c = P.off + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + i + G;
    // chi, gt_ij (6), trKhat, At_ij (6), Ghat^i (3), Theta, alpha, beta^i (3), B^i (3)
    U[c] = ip4;
    for (int q = 0; q < 6; ++q) {
        U[c + (1 + q) * P.fs] = (q == 0 || q == 3 || q == 5) ? 1.0 : 0.0;
        U[c + (8 + q) * P.fs] = A[q] * ip6;
    }
    U[c + 7 * P.fs] = 0.0;
    for (int f = 14; f < 18; ++f) U[c + f * P.fs] = 0.0;
    U[c + 18 * P.fs] = ip2;
    for (int f = 19; f < 25; ++f) U[c + f * P.fs] = 0.0;
}

}  // namespace

hipError_t launch_puncture(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], int nholes,
                           const double* holes, double h, const double xlo[3], int whole, double* U, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (td[0] * td[1] * td[2] > 256 || nholes > MOL_MAX_HOLES) return hipErrorInvalidValue;
    Holes H;
    H.n = nholes;
    for (int q = 0; q < 10 * nholes; ++q) H.v[q] = holes[q];
    puncture_kernel<<<ntiles, dim3(td[0], td[1], td[2]), 0, s>>>(patches, tiles, ntiles, H, h, xlo[0], xlo[1],
                                                                 xlo[2], whole, U);
    return hipGetLastError();
}

}  // namespace mol
