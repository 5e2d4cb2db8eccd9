// CCZ4 in vacuum (Sec. V): evolution of chi, gt_ij, trKhat, At_ij, Ghat^i,
// Theta (eqs. syseq1 .. syseq2 with the Ricci split and nabla_i nabla_j alpha
// printed below them), Bona-Masso slicing and Gamma-driver shift, with
// 4th-order centred derivatives, lop-sided advection and Kreiss-Oliger
// dissipation on every field (Sec. II.B.1), fused with the Runge-Kutta stage
// update.
//
// Conventions: symmetric pairs are packed xx xy xz yy yz zz; Z^i =
// chi (Ghat^i - Gt^i)/2; R + 2 nabla Z and nabla^i nabla_i alpha are traces
// with the physical inverse metric chi gt^{ij}; [.]^TF is taken with gt;
// ln det gt = log1p(det(I + h) - 1) expanded in h = gt - I.
//
// Kernel organisation (gfx950): one workgroup of 256 threads owns a tile of
// TX x TY x TZ points.  The 25 fields are streamed through LDS one at a time
// (tile plus a 3-point halo, brought in by 16-byte LDS-DMA loads that write
// LDS without passing through registers; the next field's halo lands in a
// second buffer while the current one is differentiated).  Each field's derivatives are
// consumed as soon as they arrive (Christoffel symbols after the six metric
// components, Ricci terms after chi and Ghat, the lapse Hessian after alpha,
// ...), and point values that are needed only late are taken from LDS when
// their field passes, so that only partial sums stay live (the kernel keeps
// to 256 registers per lane, two waves per SIMD).  Advection and dissipation of
// every field are parked in LDS until the algebra that needs all fields is
// done; then the RK stage update writes the results.
#include <utility>

#include <algorithm>

#include "k_common.h"

namespace mol {

namespace {

enum { CHI = 0, GT = 1, KH = 7, AT = 8, GH = 14, TH = 17, ALP = 18, BETA = 19, BB = 22, NF = 25 };

// packed index of the symmetric pair (i, j); written without recursion so
// that it folds to a constant wherever i and j are constants
__device__ constexpr int SI(int i, int j)
{
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

// Neighbour combinations along stride s: e_m = (u_m - u_0) + (u_-m - u_0),
// o_m = u_m - u_-m (m = 1, 2, 3).  In these, 12 h D1 = 8 o1 - o2,
// 12 h^2 D2 = 16 e1 - e2, the sixth-order dissipation stencil is
// e3 - 6 e2 + 15 e1, and b times the lop-sided derivative (the b >= 0
// stencil reading i-1 .. i+3, its mirror for b < 0) is
// b (o3/2 - 3 o2 + 21 o1/2) + |b| (e3/2 - 3 e2 + 15 e1/2), which needs no
// branch on the sign of b.
struct Axis {
    double e1, e2, e3, o1, o2, o3;
};
__device__ __forceinline__ Axis axis(const double* __restrict__ u, int s)
{
    const double c = u[0];
    Axis a;
    a.e1 = (u[s] - c) + (u[-s] - c);
    a.e2 = (u[2 * s] - c) + (u[-2 * s] - c);
    a.e3 = (u[3 * s] - c) + (u[-3 * s] - c);
    a.o1 = u[s] - u[-s];
    a.o2 = u[2 * s] - u[-2 * s];
    a.o3 = u[3 * s] - u[-3 * s];
    return a;
}

struct CczConst {
    double i12h;    // 1 / (12 h)
    double i12h2;   // 1 / (12 h^2)
    double i144h2;  // 1 / (144 h^2)
    double ko;      // sigma / (64 h)
    double kz, kc, f0, f1, g, eta;
};

// order in which the fields pass through LDS
constexpr int ORDER[NF] = {GT + 0, GT + 1, GT + 2,   GT + 3,   GT + 4,   GT + 5, CHI,    ALP, AT + 0,
                           AT + 1, AT + 2, AT + 3,   AT + 4,   AT + 5,   GH + 0, GH + 1, GH + 2,
                           BETA + 0, BETA + 1, BETA + 2, KH,     TH,     BB + 0, BB + 1, BB + 2};

// LDS geometry of the stage kernel for a TX x TY x TZ tile.  Two load paths
// are compiled: LDS-DMA (the default, MOL_CCZ4_DMA = 1, described below
// DMA) and loads staged through registers (MOL_CCZ4_DMA = 0), in which the
// halo tile's rows are padded to a pitch of PX doubles: a wave reads 8 rows
// of 8 doubles; with PX = 24 (= 8 mod 16 doubles) every group of rows served
// in one LDS cycle starts on distinct banks.  There only the halo points a
// field's stencils read are loaded (below); NR, the passes of a whole-box
// load with 16 lanes per row, bounds the loads per thread and sizes the
// staging registers.
#ifndef MOL_CCZ4_PERSISTENT
#define MOL_CCZ4_PERSISTENT 0
#endif
#ifndef MOL_CCZ4_DMA
#define MOL_CCZ4_DMA 1
#endif

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt immediate that waits until at most n vector-memory loads of this
// wave are outstanding (expcnt and lgkmcnt left unconstrained)
__device__ constexpr int vm_wait(int n) { return 0x0F70 | n; }

// Workgroup barrier after this wave's LDS accesses have completed.  Unlike
// __syncthreads() it does not wait for the wave's outstanding vector-memory
// loads, so LDS-DMA loads of later passes stay in flight across it (the
// caller waits for the ones the next pass reads); the memory clobber keeps the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int TX, int TY, int TZ>
struct CczLds {
    static constexpr int HX = TX + 2 * G, HY = TY + 2 * G, HZ = TZ + 2 * G;
    static constexpr int PX = TX == 8 ? 24 : HX;
    static constexpr int NT = TX * TY * TZ;
    static constexpr int LW = 16, PP = (NT / LW) / HY, NR = (HZ + PP - 1) / PP;
    static_assert(HX <= LW && PP >= 1 && HZ % PP == 0, "halo tile does not fit the load pattern");
    static constexpr int LV = PX * HY * HZ;
    // Cross of a single-axis field: the tile's columns over all HZ planes
    // (z slab, NT / (TX TY) planes per pass) and, on the tile's own planes,
    // the three points beyond each x face and each y face (wings)
    static constexpr int ZS = TX * TY * HZ, NZ = (ZS + NT - 1) / NT, ZPP = NT / (TX * TY);
    static constexpr int XW = 2 * G * TY * TZ, YW = 2 * G * TX * TZ, NW = (XW + YW + NT - 1) / NT;
    static_assert(NT % (TX * TY) == 0 && NZ + NW <= NR, "cross does not fit the load pattern");
    // The rest of the halo that a field with second derivatives reads: its
    // cross plus the reach-2 squares of the mixed derivatives, i.e. the z slab
    // and, on each of the tile's planes, the wings and the four 2 x 2 corners
    // (TPE points), and on the two planes below and above the tile, reach-2
    // strips beyond the x faces and beyond the y faces (OPE points).  The
    // reach-3 edges and the corners off the tile's planes are never read.
    static constexpr int TPE = 6 * TY + 6 * TX + 16, OPE = 4 * TY + 4 * TX;
    static constexpr int BE = TZ * TPE + 4 * OPE, NB = (BE + NT - 1) / NT;
    static_assert(NZ + NB <= NR, "reduced box does not fit the load pattern");
    // Direct loads into LDS: the halo box in two buffers of rows of HX
    // doubles at pitch HX, written by 16-byte LDS-DMA loads (a wave's load
    // fills 64 consecutive 16-byte chunks, lane l the l-th) while the other
    // buffer is read.  Each buffer holds the window from row G of the first
    // plane to row G + TY - 1 of the last, the two planes being read only in
    // the tile's columns: NCH chunks, NI loads per thread.
    static constexpr bool DMA = MOL_CCZ4_DMA;
    static constexpr int CPR = HX / 2, C0 = G * CPR, NCH = ((HZ - 1) * HY + TY) * CPR;
    static constexpr int NI = (NCH + NT - 1) / NT;
    // loads per thread that every wave issues (the waves past the end of the
    // window skip the last one)
    static constexpr int NIW = (NI - 1) * NT + (NT - 64) < NCH ? NI : NI - 1;
    static constexpr int NBUF = DMA ? MOL_CCZ4_NBUF : 1;
    static_assert(NBUF >= 1 && NBUF <= 3 && (DMA || NBUF == 1), "one to three halo buffers");
    static_assert(HX % 2 == 0, "halo rows must be whole 16-byte chunks");
    static constexpr int LB = DMA ? 2 * NCH : LV;  // doubles per halo buffer
};

// fields whose stencils read only along the axes through the point (first
// derivatives, advection, dissipation): their halo corners are never read
[[maybe_unused]] __device__ constexpr bool single_axis(int f)
{
    return (f >= KH && f < GH + 3) || f == TH || (f >= BB && f < BB + 3);
}

// One tile of the stage: the right-hand side of every interior point of tile
// tidx and its stage update.  buf: the halo tile of the field passing
// through LDS; akx: advection + dissipation of every field.
template <int TX, int TY, int TZ, bool UPWIND>
__device__ __forceinline__ void ccz4_tile(const StageArgs& a, const CczConst& C, int tidx, double* __restrict__ buf,
                                          double* __restrict__ buf2, double* __restrict__ buf3,
                                          double (*__restrict__ akx)[TX * TY * TZ])
{
    using L = CczLds<TX, TY, TZ>;
    constexpr bool DMA = L::DMA;
    constexpr int HY = L::HY, HZ = L::HZ, PX = DMA ? L::HX : L::PX, NT = L::NT, NR = L::NR;

    const Tile tile = a.tiles[tidx];
    const PatchDev P = a.patches[tile.patch];
    const int tx = threadIdx.x, tz = threadIdx.z;
    const int tid = tx + TX * ((int)threadIdx.y + TY * tz);
    // With the halo rows at a pitch of 14 doubles, the two rows that one LDS
    // cycle serves for a wave's 8 x 8 reads (lanes 16 m .. 16 m + 15) are
    // rows y and y + 4, whose 64-byte segments fall on disjoint banks
    const int ty = (DMA && TY == 8) ? (((int)threadIdx.y >> 1) | (((int)threadIdx.y & 1) << 2)) : (int)threadIdx.y;
    const bool valid = tile.o[0] + tx < P.n[0] && tile.o[1] + ty < P.n[1] && tile.o[2] + tz < P.n[2];
    // halo tile origin = tile origin - 3 in interior coordinates = tile origin in ghosted coordinates
    const int64_t hbase = P.off + (int64_t)tile.o[2] * P.pitch_z + (int64_t)tile.o[1] * P.pitch_y + tile.o[0];
    const int64_t c = hbase + (int64_t)(tz + G) * P.pitch_z + (int64_t)(ty + G) * P.pitch_y + (tx + G);
    const int64_t fs = P.fs;

    const int hzmax = P.n[2] + 2 * G - tile.o[2];  // halo planes inside the ghosted box
    double stg[NR];
    // the cross of a single-axis field (fewer loads than the box): z-slab
    // element tid + r NT is column (zx, zy) of plane zz + r ZPP; wing element
    // e = tid + r NT is decoded per pass.  Elements outside the ghosted box
    // load from the tile origin and are never read.
    constexpr int ZS = L::ZS, NZ = L::NZ, ZPP = L::ZPP, XW = L::XW, YW = L::YW, NW = L::NW;
    const int zx = tid % TX + G, zy = (tid / TX) % TY + G, zz = tid / (TX * TY);
    const bool zin = tile.o[0] + zx < P.n[0] + 2 * G && tile.o[1] + zy < P.n[1] + 2 * G;
    auto wing = [&](int e, int& hx, int& hy, int& hz) __attribute__((always_inline)) {
        if (e < XW) {
            const int w = e % (2 * G), r = e / (2 * G);
            hx = w < G ? w : w + TX;
            hy = r % TY + G;
            hz = r / TY + G;
        } else {
            const int e2 = e - XW, r = e2 / TX, w = r % (2 * G);
            hx = e2 % TX + G;
            hy = w < G ? w : w + TY;
            hz = r / (2 * G) + G;
        }
    };
    auto gload_x = [&](int f) __attribute__((always_inline)) {
        const double* src = a.Us + hbase + (int64_t)f * fs;
#pragma unroll
        for (int r = 0; r < NZ; ++r) {
            const int hz = zz + r * ZPP;
            const bool ok = zin && hz < HZ && hz < hzmax;
            stg[r] = src[ok ? hz * P.pitch_z + zy * P.pitch_y + zx : 0];
        }
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const int e = tid + r * NT;
            int hx, hy, hz;
            wing(e, hx, hy, hz);
            const bool ok = e < XW + YW && tile.o[0] + hx < P.n[0] + 2 * G && tile.o[1] + hy < P.n[1] + 2 * G &&
                            hz < hzmax;
            stg[NZ + r] = src[ok ? hz * P.pitch_z + hy * P.pitch_y + hx : 0];
        }
    };
    // the reduced box of a field with second derivatives: the z slab as for
    // the cross, then the extra points decoded per pass
    constexpr int TPE = L::TPE, OPE = L::OPE, BE = L::BE, NB = L::NB;
    auto bextra = [&](int e, int& hx, int& hy, int& hz) __attribute__((always_inline)) {
        // reach-2 positions beyond a face: G - 2, G - 1, G + T, G + T + 1
        auto r2 = [](int c, int T) { return c < 2 ? G - 2 + c : G + T + c - 2; };
        if (e < TZ * TPE) {
            const int pl = e / TPE, w = e - pl * TPE;
            hz = G + pl;
            if (w < 6 * TY) {
                const int c = w % 6;
                hx = c < 3 ? c : c + TX;
                hy = G + w / 6;
            } else if (w < 6 * TY + 6 * TX) {
                const int w2 = w - 6 * TY, r = w2 / TX;
                hx = G + w2 % TX;
                hy = r < 3 ? r : r + TY;
            } else {
                const int w3 = w - 6 * TY - 6 * TX;
                hx = r2(w3 % 4, TX);
                hy = r2(w3 / 4, TY);
            }
        } else {
            const int e2 = e - TZ * TPE, pl = e2 / OPE, w = e2 - pl * OPE;
            hz = r2(pl, TZ);
            if (w < 4 * TY) {
                hx = r2(w % 4, TX);
                hy = G + w / 4;
            } else {
                const int w2 = w - 4 * TY;
                hx = G + w2 % TX;
                hy = r2(w2 / TX, TY);
            }
        }
    };
    auto gload = [&](int f) __attribute__((always_inline)) {
        const double* src = a.Us + hbase + (int64_t)f * fs;
#pragma unroll
        for (int r = 0; r < NZ; ++r) {
            const int hz = zz + r * ZPP;
            const bool ok = zin && hz < HZ && hz < hzmax;
            stg[r] = src[ok ? hz * P.pitch_z + zy * P.pitch_y + zx : 0];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int e = tid + r * NT;
            int hx, hy, hz;
            bextra(e, hx, hy, hz);
            const bool ok = e < BE && tile.o[0] + hx < P.n[0] + 2 * G && tile.o[1] + hy < P.n[1] + 2 * G &&
                            hz < hzmax;
            stg[NZ + r] = src[ok ? hz * P.pitch_z + hy * P.pitch_y + hx : 0];
        }
    };
    auto lstore = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < NZ; ++r) {
            const int hz = zz + r * ZPP;
            if (ZS % NT == 0 || hz < HZ) buf[(hz * HY + zy) * PX + zx] = stg[r];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int e = tid + r * NT;
            int hx, hy, hz;
            bextra(e, hx, hy, hz);
            if (BE % NT == 0 || e < BE) buf[(hz * HY + hy) * PX + hx] = stg[NZ + r];
        }
    };
    auto lstore_x = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < NZ; ++r) {
            const int hz = zz + r * ZPP;
            if (ZS % NT == 0 || hz < HZ) buf[(hz * HY + zy) * PX + zx] = stg[r];
        }
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const int e = tid + r * NT;
            int hx, hy, hz;
            wing(e, hx, hy, hz);
            if ((XW + YW) % NT == 0 || e < XW + YW) buf[(hz * HY + hy) * PX + hx] = stg[NZ + r];
        }
    };

    // LDS-DMA loads of the halo window: chunk j = r NT + tid, offsets from the
    // tile's halo origin (0, the origin itself, for chunks outside the
    // ghosted box, which only the stencils of points outside the patch read)
    int doff[DMA ? L::NI : 1];
    if constexpr (DMA) {
#pragma unroll
        for (int r = 0; r < L::NI; ++r) {
            const int j = r * NT + tid, ac = j + L::C0, row = ac / L::CPR, cc = ac - row * L::CPR;
            const int hz = row / HY, hy = row - hz * HY;
            const bool ok = j < L::NCH && tile.o[0] + 2 * cc < P.n[0] + 2 * G &&
                            tile.o[1] + hy < P.n[1] + 2 * G && hz < hzmax;
            doff[r] = ok ? hz * P.pitch_z + hy * P.pitch_y + 2 * cc : 0;
        }
    }
    auto dma = [&](int f, double* dst) __attribute__((always_inline)) {
        const double* src = a.Us + hbase + (int64_t)f * fs;
        const int wbase = tid & ~63;  // first chunk of this wave's window of 64
#pragma unroll
        for (int r = 0; r < L::NI; ++r)
            if ((r + 1) * NT <= L::NCH || r * NT + tid < L::NCH)
                __builtin_amdgcn_global_load_lds((const void*)(src + doff[r]), (lds_void*)(dst + 2 * (r * NT + wbase)),
                                                 16, 0, 0);
    };

    // ---- point values needed from the first pass on (global loads) ----
    const double* __restrict__ u = a.Us + c;
    const double chi = u[CHI * fs];
    double g[6], Gh[3], be[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = u[(GT + q) * fs];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Gh[i] = u[(GH + i) * fs];
        be[i] = u[(BETA + i) * fs];
    }
    double gu[6], lndet;
    {
        const double hx = g[0] - 1.0, hy = g[3] - 1.0, hz = g[5] - 1.0;
        const double hxy = g[1], hxz = g[2], hyz = g[4];
        const double m2 = hx * hy - hxy * hxy + hx * hz - hxz * hxz + hy * hz - hyz * hyz;
        const double m3 = hx * (hy * hz - hyz * hyz) - hxy * (hxy * hz - hyz * hxz) + hxz * (hxy * hyz - hy * hxz);
        const double dm = (hx + hy + hz) + m2 + m3;
        lndet = log1p(dm);
        const double idet = 1.0 / (1.0 + dm);
        gu[0] = (g[3] * g[5] - g[4] * g[4]) * idet;
        gu[1] = (g[2] * g[4] - g[1] * g[5]) * idet;
        gu[2] = (g[1] * g[4] - g[2] * g[3]) * idet;
        gu[3] = (g[0] * g[5] - g[2] * g[2]) * idet;
        gu[4] = (g[2] * g[1] - g[0] * g[4]) * idet;
        gu[5] = (g[0] * g[3] - g[1] * g[1]) * idet;
    }

    // ---- quantities built while the fields stream through LDS ----
    double dg[3][6], lapg[6];           // metric derivatives (until the Christoffels are formed)
    double Gu[3][6], Z[3], GtAu[3];     // Gt^i_jk (until At^jk is known), Z^i, Gt^i_jk At^jk
    double Ric[6];                      // R_ij + 2 nabla_(i Z_j), accumulated
    double dchi[3], dalp[3], DDa[6];    // chi and alpha gradients, nabla_i nabla_j alpha
    double db[3][3], gddb[3], gdiv[3];  // d_k beta^i, gt^jk d_j d_k beta^i, d_i (d_k beta^k)
    double rG[3];                       // Ghat^i terms with d Khat and d Theta
    double alp, A[6], Au[6], Kh, Th, Bv[3];  // point values taken from LDS, At^{ij}
    const int S[3] = {1, PX, PX * HY};
    // this point in the halo buffer
    const int ctr = ((tz + G) * HY + ty + G) * PX + tx + G - (DMA ? 2 * L::C0 : 0);

    // halo buffer of pass q
    constexpr int NBUF = L::NBUF;
    auto hbuf = [&](int q) __attribute__((always_inline)) {
        return q % NBUF == 0 ? buf : (q % NBUF == 1 ? buf2 : buf3);
    };
    if constexpr (DMA) {
#pragma unroll
        for (int q = 0; q + 1 < NBUF; ++q) dma(ORDER[q], hbuf(q));
        __builtin_amdgcn_s_waitcnt(vm_wait(NBUF == 3 ? L::NIW : 0));
    } else {
        gload(ORDER[0]);
        lstore();
    }
    __syncthreads();
    // one pass per field, expanded at compile time so that every branch and
    // array index below is a constant
    auto pass = [&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        constexpr int f = ORDER[q];
        if constexpr (DMA) {
            if constexpr (q + NBUF - 1 < NF) dma(ORDER[q + NBUF - 1], hbuf(q + NBUF - 1));
        } else if constexpr (q + 1 < NF) {
            if constexpr (single_axis(ORDER[q + 1]))
                gload_x(ORDER[q + 1]);
            else
                gload(ORDER[q + 1]);
        }
        if (valid) {
            const double* t = hbuf(q) + ctr;
            // advection beta^k d_k and KO dissipation of every field; first
            // and pure second derivatives from the same combinations
            constexpr bool second = (f >= GT && f < GT + 6) || f == CHI || f == ALP || (f >= BETA && f < BETA + 3);
            double adv = 0.0, ko = 0.0, d1v[3], d2v[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const Axis x = axis(t, S[k]);
                ko += (x.e3 - 6.0 * x.e2) + 15.0 * x.e1;
                d1v[k] = 8.0 * x.o1 - x.o2;
                if (UPWIND)
                    adv += be[k] * ((0.5 * x.o3 - 3.0 * x.o2) + 10.5 * x.o1) +
                           fabs(be[k]) * ((0.5 * x.e3 - 3.0 * x.e2) + 7.5 * x.e1);
                else
                    adv += be[k] * d1v[k];
                if constexpr (second) d2v[k] = 16.0 * x.e1 - x.e2;
            }
            akx[f][tid] = C.i12h * adv + C.ko * ko;

            auto d1 = [&](int k) __attribute__((always_inline)) { return C.i12h * d1v[k]; };
            auto dd = [&](int k, int l) __attribute__((always_inline)) {
                return k == l ? C.i12h2 * d2v[k] : C.i144h2 * fmix(t, S[k], S[l]);
            };
            // gt^{kl} d_k d_l of the field in LDS
            auto trdd = [&]() __attribute__((always_inline)) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int l = k; l < 3; ++l) s += (k == l ? 1.0 : 2.0) * gu[SI(k, l)] * dd(k, l);
                return s;
            };

            if constexpr (f >= GT && f < GT + 6) {
                constexpr int qq = f - GT;
#pragma unroll
                for (int k = 0; k < 3; ++k) dg[k][qq] = d1(k);
                lapg[qq] = trdd();
                if constexpr (qq == 5) {
                    // Christoffels: Gl[i][jk] = (d_j g_ik + d_k g_ij - d_i g_jk)/2, Gu = gt^-1 Gl
                    double Gl[3][6];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j)
#pragma unroll
                            for (int k = j; k < 3; ++k)
                                Gl[i][SI(j, k)] = 0.5 * (dg[j][SI(i, k)] + dg[k][SI(i, j)] - dg[i][SI(j, k)]);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int m = 0; m < 6; ++m)
                            Gu[i][m] = gu[SI(i, 0)] * Gl[0][m] + gu[SI(i, 1)] * Gl[1][m] + gu[SI(i, 2)] * Gl[2][m];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const double Gc = gu[0] * Gu[i][0] + gu[3] * Gu[i][3] + gu[5] * Gu[i][5] +
                                          2.0 * (gu[1] * Gu[i][1] + gu[2] * Gu[i][2] + gu[4] * Gu[i][4]);
                        Z[i] = 0.5 * chi * (Gh[i] - Gc);
                    }
                    // Rhat_ij without the d Ghat term:
                    //  -gt^mn d_m d_n gt_ij / 2 + Ghat^k Gt_(ij)k
                    //  + gt^mn (Gt^k_mi Gt_jkn + Gt^k_mj Gt_ikn + Gt^k_mi Gt_knj)
                    // built row by row: with H_i[k][n] = gt^{nm} Gt^k_{mi},
                    // P_ij = H_i[k][n] Gt_jkn and Q_ij = H_i[k][n] Gt_knj, the
                    // quadratic part of entry (i, j) is P_ij + P_ji + Q_ij
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = i; j < 3; ++j) {
                            double r = -0.5 * lapg[SI(i, j)];
#pragma unroll
                            for (int k = 0; k < 3; ++k) r += Gh[k] * 0.5 * (Gl[i][SI(j, k)] + Gl[j][SI(i, k)]);
                            Ric[SI(i, j)] = r;
                        }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        double H[3][3];
#pragma unroll
                        for (int k = 0; k < 3; ++k)
#pragma unroll
                            for (int n = 0; n < 3; ++n)
                                H[k][n] = gu[SI(n, 0)] * Gu[k][SI(0, i)] + gu[SI(n, 1)] * Gu[k][SI(1, i)] +
                                          gu[SI(n, 2)] * Gu[k][SI(2, i)];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            double p = 0.0, qv = 0.0;
#pragma unroll
                            for (int k = 0; k < 3; ++k)
#pragma unroll
                                for (int n = 0; n < 3; ++n) {
                                    p += H[k][n] * Gl[j][SI(k, n)];
                                    if (j >= i) qv += H[k][n] * Gl[k][SI(n, j)];
                                }
                            if (j >= i) Ric[SI(i, j)] += p + qv;
                            if (j <= i) Ric[SI(j, i)] += p;
                        }
                    }
                }
            } else if constexpr (f >= GH && f < GH + 3) {
                // gt_k(i d_j) Ghat^k for k = f - GH
                constexpr int kk = f - GH;
                double dG[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) dG[j] = d1(j);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j)
                        Ric[SI(i, j)] += 0.5 * (g[SI(kk, i)] * dG[j] + g[SI(kk, j)] * dG[i]);
            } else if constexpr (f == CHI) {
                double ddc[6];
#pragma unroll
                for (int k = 0; k < 3; ++k) dchi[k] = d1(k);
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int l = k; l < 3; ++l) ddc[SI(k, l)] = dd(k, l);
                const double ic = 1.0 / chi;
                double tr = 0.0, Ghd = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Ghd += Gh[k] * dchi[k];
#pragma unroll
                    for (int m = 0; m < 3; ++m) tr += gu[SI(k, m)] * (ddc[SI(k, m)] - 1.5 * ic * dchi[k] * dchi[m]);
                }
                // Rhat^chi_ij
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j) {
                        const int m = SI(i, j);
                        double Gd = 0.0, zs = 0.0;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            Gd += Gu[k][m] * dchi[k];
                            zs += Z[k] * 0.5 * (g[SI(k, i)] * dchi[j] + g[SI(k, j)] * dchi[i]);
                        }
                        Ric[m] += 0.5 * ic * ddc[m] - 0.5 * ic * Gd - 0.25 * ic * ic * dchi[i] * dchi[j] +
                                  2.0 * ic * ic * zs + 0.5 * ic * g[m] * (tr - Ghd);
                    }
            } else if constexpr (f == ALP) {
                alp = t[0];
#pragma unroll
                for (int k = 0; k < 3; ++k) dalp[k] = d1(k);
                double cr = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int m = 0; m < 3; ++m) cr += gu[SI(k, m)] * dalp[k] * dchi[m];
                const double hic = 0.5 / chi;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j) {
                        const int m = SI(i, j);
                        DDa[m] = dd(i, j) - (Gu[0][m] * dalp[0] + Gu[1][m] * dalp[1] + Gu[2][m] * dalp[2]) +
                                 hic * (dalp[i] * dchi[j] + dalp[j] * dchi[i] - g[m] * cr);
                    }
            } else if constexpr (f >= AT && f < AT + 6) {
                A[f - AT] = t[0];
                if constexpr (f == AT + 5) {
                    // At^{ij} and Gt^i_jk At^jk; the Christoffels are not needed after this
                    double Am[3][3];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            Am[i][j] = gu[SI(i, 0)] * A[SI(0, j)] + gu[SI(i, 1)] * A[SI(1, j)] +
                                       gu[SI(i, 2)] * A[SI(2, j)];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = i; j < 3; ++j)
                            Au[SI(i, j)] = Am[i][0] * gu[SI(0, j)] + Am[i][1] * gu[SI(1, j)] + Am[i][2] * gu[SI(2, j)];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        GtAu[i] = Gu[i][0] * Au[0] + Gu[i][3] * Au[3] + Gu[i][5] * Au[5] +
                                  2.0 * (Gu[i][1] * Au[1] + Gu[i][2] * Au[2] + Gu[i][4] * Au[4]);
                }
            } else if constexpr (f >= BETA && f < BETA + 3) {
                constexpr int i = f - BETA;
                if constexpr (i == 0) gdiv[0] = gdiv[1] = gdiv[2] = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) db[k][i] = d1(k);
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int l = k; l < 3; ++l) {
                        const double v = dd(k, l);
                        s += (k == l ? 1.0 : 2.0) * gu[SI(k, l)] * v;
                        // d_j d_i beta^i goes to row j
                        if (k == i) gdiv[l] += v;
                        if (l == i && k != l) gdiv[k] += v;
                    }
                gddb[i] = s;
            } else if constexpr (f == KH) {
                Kh = t[0];
                double d[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) d[k] = d1(k);
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    rG[i] = -(2.0 / 3.0) * (gu[SI(i, 0)] * d[0] + gu[SI(i, 1)] * d[1] + gu[SI(i, 2)] * d[2]);
            } else if constexpr (f == TH) {
                Th = t[0];
                double d[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) d[k] = d1(k);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        rG[i] += -gu[SI(i, j)] * ((1.0 / 3.0) * d[j] + Th / alp * dalp[j]);
            } else if constexpr (f >= BB && f < BB + 3) {
                Bv[f - BB] = t[0];
            }
        }
        if constexpr (DMA) {
            // the next field's halo has arrived (the loads of the field after
            // it may still be in flight), and every wave is done with this
            // buffer before the load issued in the pass NBUF - 1 ahead refills it
            if constexpr (q + 1 < NF) __builtin_amdgcn_s_waitcnt(vm_wait(NBUF == 3 && q + 2 < NF ? L::NIW : 0));
            lds_barrier();
        } else {
            __syncthreads();
            if constexpr (q + 1 < NF) {
                if constexpr (single_axis(ORDER[q + 1]))
                    lstore_x();
                else
                    lstore();
                __syncthreads();
            }
        }
    };
    [&]<int... Q>(std::integer_sequence<int, Q...>) {
        (pass(std::integral_constant<int, Q>{}), ...);
    }(std::make_integer_sequence<int, NF>{});
    if (!valid) return;

    // ---- algebra with all fields available ----
    auto tr = [&](const double* T) __attribute__((always_inline)) {  // gt^{ij} T_ij
        return gu[0] * T[0] + gu[3] * T[3] + gu[5] * T[5] + 2.0 * (gu[1] * T[1] + gu[2] * T[2] + gu[4] * T[4]);
    };
    // raised traceless curvature At^i_j
    double Am[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Am[i][j] = gu[SI(i, 0)] * A[SI(0, j)] + gu[SI(i, 1)] * A[SI(1, j)] + gu[SI(i, 2)] * A[SI(2, j)];
    const double trRic = chi * tr(Ric);
    const double lapa = chi * tr(DDa);
    const double trA = Am[0][0] + Am[1][1] + Am[2][2];
    double AA = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) AA += A[SI(i, j)] * Au[SI(i, j)];
    const double divb = db[0][0] + db[1][1] + db[2][2];
    const double Zda = Z[0] * dalp[0] + Z[1] * dalp[1] + Z[2] * dalp[2];
    const double Kt = Kh + 2.0 * Th;
    // periodic ghost images of this point in the output (a.images): per axis
    // the offset to the image, 0 when the point is not within G of a face
    int64_t im[3] = {0, 0, 0};
    if (a.images) {
        const int q[3] = {tile.o[0] + tx, tile.o[1] + ty, tile.o[2] + tz};
        const int64_t sd[3] = {1, P.pitch_y, P.pitch_z};
#pragma unroll
        for (int d = 0; d < 3; ++d)
            im[d] = q[d] < G ? (int64_t)P.n[d] * sd[d] : (q[d] >= P.n[d] - G ? -(int64_t)P.n[d] * sd[d] : 0);
    }
    const bool img = (im[0] | im[1] | im[2]) != 0;
    // the stage update of every field as straight-line code (stage_update)
    const StageCoef sc = stage_coef(a);
    double* pout = a.out;
    // Fields in the order of the out() calls below; the stage inputs of the
    // field PD calls ahead are requested before a field's update is stored,
    // so that their memory latency overlaps the algebra in between.
    constexpr int OUTORD[NF] = {GT,     GT + 1, GT + 2, GT + 3, GT + 4,   GT + 5, AT,     AT + 1, AT + 2,
                                AT + 3, AT + 4, AT + 5, CHI,    KH,       TH,     GH,     BB,     BETA,
                                GH + 1, BB + 1, BETA + 1, GH + 2, BB + 2, BETA + 2, ALP};
    constexpr int PD = 3;
    double pu[PD], pv[PD];
    auto pref = [&](int p) __attribute__((always_inline)) {
        if (p < NF) {
            const int64_t i = c + (int64_t)OUTORD[p] * fs;
            pu[p % PD] = sc.pun[i];
            pv[p % PD] = sc.pw[i];
        }
    };
#pragma unroll
    for (int p = 0; p < PD; ++p) pref(p);
    int pos = 0;
    auto out = [&](int f, double phys) __attribute__((always_inline)) {
        const int64_t idx = c + (int64_t)f * fs;
        const double un = pu[pos % PD], w = pv[pos % PD];
        pref(pos + PD);
        ++pos;
        const double v = stage_update(a, sc, idx, phys + akx[f][tid], un, w);
        pout[idx] = v;
        if (img)
#pragma unroll
            for (int m = 1; m < 8; ++m)
                if (((m & 1) == 0 || im[0]) && ((m & 2) == 0 || im[1]) && ((m & 4) == 0 || im[2]))
                    pout[idx + ((m & 1) ? im[0] : 0) + ((m & 2) ? im[1] : 0) + ((m & 4) ? im[2] : 0)] = v;
    };

    // d_t gt_ij
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int m = SI(i, j);
            double r = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) r += g[SI(i, k)] * db[j][k] + g[SI(k, j)] * db[i][k];
            out(GT + m, r - (2.0 / 3.0) * g[m] * divb - 2.0 * alp * (A[m] - (1.0 / 3.0) * g[m] * trA) -
                            (C.kc / 3.0) * alp * g[m] * lndet);
        }
    // d_t At_ij
    {
        double X[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) X[m] = alp * Ric[m] - DDa[m];
        const double trX = tr(X);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const int m = SI(i, j);
                double r = 0.0, aa = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    r += A[SI(i, k)] * db[j][k] + A[SI(k, j)] * db[i][k];
                    aa += A[SI(i, k)] * Am[k][j];
                }
                out(AT + m, r - (2.0 / 3.0) * A[m] * divb - (C.kc / 3.0) * alp * g[m] * trA +
                                chi * (X[m] - (1.0 / 3.0) * g[m] * trX) + alp * (Kh * A[m] - 2.0 * aa));
            }
    }
    out(CHI, (2.0 / 3.0) * chi * (alp * Kt - divb));
    out(KH, -lapa + alp * ((1.0 / 3.0) * Kt * Kt + AA + C.kz * Th) + 2.0 * Zda);
    out(TH, 0.5 * alp * (trRic + (2.0 / 3.0) * Kh * Kh + (2.0 / 3.0) * Th * (Kh - 2.0 * Th) - AA) - Zda -
                alp * (2.0 * C.kz * Th));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double r = (2.0 / 3.0) * Gh[i] * divb + gddb[i];
        double b1 = GtAu[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r += -Gh[j] * db[j][i] + (1.0 / 3.0) * gu[SI(i, j)] * gdiv[j] - 2.0 * Au[SI(i, j)] * dalp[j];
            b1 += -1.5 / chi * Au[SI(i, j)] * dchi[j];
        }
        const double b2 = -Z[i] / chi * (C.kz + (2.0 / 3.0) * Kt);
        r += 2.0 * alp * (b1 + rG[i] + b2);
        out(GH + i, r);
        out(BB + i, -C.eta * Bv[i] + r);  // d_t Ghat^i without its advection term
        out(BETA + i, C.g * Bv[i]);
    }
    out(ALP, -alp * alp * (C.f0 + C.f1 / alp) * Kh);
}

template <int TX, int TY, int TZ, bool UPWIND>
__global__ __launch_bounds__(TX * TY * TZ, MOL_CCZ4_WAVES) void ccz4_stage_kernel(StageArgs a, CczConst C)
{
    using L = CczLds<TX, TY, TZ>;
    __shared__ double buf[L::LB];
    __shared__ double buf2[L::NBUF >= 2 ? L::LB : 1];
    __shared__ double buf3[L::NBUF >= 3 ? L::LB : 1];
    __shared__ double akx[NF][L::NT];
    ccz4_tile<TX, TY, TZ, UPWIND>(a, C, xcd_tile(blockIdx.x, gridDim.x), buf, buf2, buf3, akx);
}

// Persistent form: a grid of at most as many workgroups as are resident at
// once; the workgroups of XCD x (x = blockIdx mod 8) take the tiles of that
// XCD's contiguous range of the tile list in turn, so that concurrently
// running tiles of an XCD stay spatial neighbours, and every workgroup exits
// after its last tile.
template <int TX, int TY, int TZ, bool UPWIND>
__global__ __launch_bounds__(TX * TY * TZ, MOL_CCZ4_WAVES) void ccz4_stage_persistent_kernel(StageArgs a, CczConst C)
{
    using L = CczLds<TX, TY, TZ>;
    __shared__ double buf[L::LB];
    __shared__ double buf2[L::NBUF >= 2 ? L::LB : 1];
    __shared__ double buf3[L::NBUF >= 3 ? L::LB : 1];
    __shared__ double akx[NF][L::NT];
    constexpr int NXCD = 8;
    const int n = a.ntiles, x = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
    const int per = n / NXCD, rem = n % NXCD;
    const int lo = x * per + (x < rem ? x : rem), hi = lo + per + (x < rem ? 1 : 0);
    const int nwg = ((int)gridDim.x - x + NXCD - 1) / NXCD;  // workgroups of this XCD
    for (int t = lo + slot; t < hi; t += nwg) {
        ccz4_tile<TX, TY, TZ, UPWIND>(a, C, t, buf, buf2, buf3, akx);
        __syncthreads();  // the next tile overwrites buf and akx
    }
}

}  // namespace

namespace {
// the tile shapes compiled besides the default (the autotuner picks one per level)
template <int TX, int TY, int TZ>
hipError_t launch_ccz4_tile(const SysParams& sp, const StageArgs& a, const CczConst& C, hipStream_t s)
{
    const dim3 blk(TX, TY, TZ);
    if (sp.upwind)
        ccz4_stage_kernel<TX, TY, TZ, true><<<a.ntiles, blk, 0, s>>>(a, C);
    else
        ccz4_stage_kernel<TX, TY, TZ, false><<<a.ntiles, blk, 0, s>>>(a, C);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_stage_ccz4(const SysParams& sp, const StageArgs& a, const int td[3], hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    const bool dflt = td[0] == MOL_CCZ4_TX && td[1] == MOL_CCZ4_TY && td[2] == MOL_CCZ4_TZ;
    const bool t888 = td[0] == 8 && td[1] == 8 && td[2] == 8, t848 = td[0] == 8 && td[1] == 4 && td[2] == 8;
    if (!dflt && !t888 && !t848) return hipErrorInvalidConfiguration;
    CczConst C;
    C.i12h = 1.0 / (12.0 * sp.h);
    C.i12h2 = 1.0 / (12.0 * sp.h * sp.h);
    C.i144h2 = 1.0 / (144.0 * sp.h * sp.h);
    C.ko = sp.sigma / (64.0 * sp.h);
    C.kz = sp.kappa_z;
    C.kc = sp.kappa_c;
    C.f0 = sp.bm_f0;
    C.f1 = sp.bm_f1;
    C.g = sp.gd_g;
    C.eta = sp.gd_eta;
    if (!dflt) return t888 ? launch_ccz4_tile<8, 8, 8>(sp, a, C, s) : launch_ccz4_tile<8, 4, 8>(sp, a, C, s);
    dim3 blk(MOL_CCZ4_TX, MOL_CCZ4_TY, MOL_CCZ4_TZ);
#if MOL_CCZ4_PERSISTENT
    // as many workgroups as are resident at once: MOL_CCZ4_WAVES waves per
    // SIMD, four SIMDs per compute unit
    static int cus[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!cus[dev] && (e = hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    constexpr int wg_per_cu = MOL_CCZ4_WAVES * 4 / (MOL_CCZ4_TX * MOL_CCZ4_TY * MOL_CCZ4_TZ / 64);
    const int grid = std::min(a.ntiles, cus[dev] * std::max(wg_per_cu, 1));
    if (sp.upwind)
        ccz4_stage_persistent_kernel<MOL_CCZ4_TX, MOL_CCZ4_TY, MOL_CCZ4_TZ, true><<<grid, blk, 0, s>>>(a, C);
    else
        ccz4_stage_persistent_kernel<MOL_CCZ4_TX, MOL_CCZ4_TY, MOL_CCZ4_TZ, false><<<grid, blk, 0, s>>>(a, C);
#else
    if (sp.upwind)
        ccz4_stage_kernel<MOL_CCZ4_TX, MOL_CCZ4_TY, MOL_CCZ4_TZ, true><<<a.ntiles, blk, 0, s>>>(a, C);
    else
        ccz4_stage_kernel<MOL_CCZ4_TX, MOL_CCZ4_TY, MOL_CCZ4_TZ, false><<<a.ntiles, blk, 0, s>>>(a, C);
#endif
    return hipGetLastError();
}

}  // namespace mol
