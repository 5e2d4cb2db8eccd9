// Device helpers shared by the stage kernels: point addressing inside a tile
// and the fused Runge-Kutta update.
#pragma once

#include "molamr_int.h"

namespace mol {

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): workgroup b runs on XCD b % 8.  Giving every XCD a contiguous range of
// the tile list keeps spatially neighbouring tiles, whose halos overlap, in the
// same L2.  Bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    constexpr int NXCD = 8;
    const int per = n / NXCD, rem = n % NXCD;
    const int x = b % NXCD, slot = b / NXCD;
    return x * per + (x < rem ? x : rem) + slot;
}

// Interior point handled by this thread inside tile `tile`; returns false for
// the ragged tail.
struct PointRef {
    int64_t c;     // level-buffer index of field 0 at the point
    int64_t fs;    // field stride
    int sy, sz;    // pitches (x stride is 1)
};

__device__ __forceinline__ bool tile_point(const StageArgs& a, int tile, PointRef& pr, int& i, int& j,
                                           int& k, int& patch)
{
    const Tile t = a.tiles[tile];
    const PatchDev& P = a.patches[t.patch];
    i = t.o[0] + (int)threadIdx.x;
    j = t.o[1] + (int)threadIdx.y;
    k = t.o[2] + (int)threadIdx.z;
    patch = t.patch;
    if (i >= P.n[0] || j >= P.n[1] || k >= P.n[2]) return false;
    pr.sy = P.pitch_y;
    pr.sz = P.pitch_z;
    pr.fs = P.fs;
    pr.c = P.off + (int64_t)(k + G) * P.pitch_z + (int64_t)(j + G) * P.pitch_y + (i + G);
    return true;
}

// Point loads and stores of the stage update; NT = true marks them
// non-temporal (streamed past the caches), for levels whose arrays are far
// larger than the caches.
template <bool NT>
__device__ __forceinline__ double mem_ld(const double* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT>
__device__ __forceinline__ void mem_st(double* p, double v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
// Values the stage update reads at a point besides the right-hand side
// (loaded separately so that kernels can fetch them ahead of use).
struct StageIn {
    double un, ac, us;
};
template <bool NT = false>
__device__ __forceinline__ StageIn stage_load(const StageArgs& a, int64_t idx)
{
    StageIn v{0.0, 0.0, 0.0};
    if (a.mode == ST_RHS) return v;
    v.un = mem_ld<NT>(&a.Un[idx]);
    if (a.stage >= 2) {
        if (a.mode == ST_RK4)
            v.ac = mem_ld<NT>(&a.acc[idx]);
        else
            v.us = mem_ld<NT>(&a.Us[idx]);
    }
    return v;
}

// k = dt * rhs, then the RK4 (Table RK44, accumulator form) or SSP-RK3
// (Shu-Osher form of the App. D scheme) stage update, or plain rhs output:
// writes acc (and k) at idx and returns the value of the output at idx.
template <bool NT = false>
__device__ __forceinline__ double stage_value(const StageArgs& a, int64_t idx, double rhs, const StageIn& v)
{
    if (a.mode == ST_RHS) return rhs;
    const double k = a.dt * rhs;
    if (a.kst) mem_st<NT>(&a.kst[idx], k);
    const double un = v.un;
    if (a.mode == ST_RK4) {
        switch (a.stage) {
        case 1: mem_st<NT>(&a.acc[idx], k * (1.0 / 6.0)); return un + 0.5 * k;
        case 2: mem_st<NT>(&a.acc[idx], v.ac + k * (1.0 / 3.0)); return un + 0.5 * k;
        case 3: mem_st<NT>(&a.acc[idx], v.ac + k * (1.0 / 3.0)); return un + k;
        default: return un + (v.ac + k * (1.0 / 6.0));
        }
    }
    switch (a.stage) {
    case 1: return un + k;
    case 2: return 0.75 * un + 0.25 * (v.us + k);
    default: return (1.0 / 3.0) * un + (2.0 / 3.0) * (v.us + k);
    }
}

// The same updates as straight-line code, for kernels that request a point's
// stage inputs ahead of its right-hand side: with k = dt rhs,
// v = al un + bt (w2 + de k), w2 the accumulator (RK4 stage 4) or the stage
// state (SSP-RK3 stages 2, 3), else 0; the new accumulator of RK4 stages 1-3
// is w3 + ep k, w3 the accumulator (stages 2, 3) or 0.  The coefficients and
// the two arrays read (un from pun, w from pw) are uniform per launch; a read
// that a stage does not use is discarded (w then repeats the read of un, un in
// a right-hand-side launch reads the output array), so that the loads need no
// branch and add no traffic.
struct StageCoef {
    bool rhs_only, use_w2, use_w3, st_acc;
    double al, bt, de, ep;
    const double* pun;
    const double* pw;
};
__device__ __forceinline__ StageCoef stage_coef(const StageArgs& a)
{
    StageCoef s;
    const bool rk4 = a.mode == ST_RK4;
    const int n = a.stage;
    s.rhs_only = a.mode == ST_RHS;
    s.al = rk4 ? 1.0 : (n == 1 ? 1.0 : (n == 2 ? 0.75 : 1.0 / 3.0));
    s.bt = rk4 ? 1.0 : (n == 1 ? 1.0 : (n == 2 ? 0.25 : 2.0 / 3.0));
    s.de = rk4 ? (n <= 2 ? 0.5 : (n == 3 ? 1.0 : 1.0 / 6.0)) : 1.0;
    s.ep = n == 1 ? 1.0 / 6.0 : 1.0 / 3.0;
    s.use_w2 = !s.rhs_only && (rk4 ? n == 4 : n >= 2);
    s.use_w3 = rk4 && (n == 2 || n == 3);
    s.st_acc = rk4 && n <= 3;
    s.pun = s.rhs_only ? a.out : a.Un;
    s.pw = s.use_w2 ? (rk4 ? a.acc : a.Us) : (s.use_w3 ? a.acc : s.pun);
    return s;
}
// stage value at idx from the right-hand side and the inputs un = pun[idx],
// w = pw[idx]; writes k and the accumulator where the stage has them
__device__ __forceinline__ double stage_update(const StageArgs& a, const StageCoef& s, int64_t idx, double rhs,
                                               double un, double w)
{
    const double k = a.dt * rhs;
    const double w2 = s.use_w2 ? w : 0.0, w3 = s.use_w3 ? w : 0.0;
    const double v = s.rhs_only ? rhs : s.al * un + s.bt * (w2 + s.de * k);
    if (a.kst && !s.rhs_only) a.kst[idx] = k;
    if (s.st_acc) a.acc[idx] = w3 + s.ep * k;
    return v;
}

template <bool NT = false>
__device__ __forceinline__ void stage_apply(const StageArgs& a, int64_t idx, double rhs, const StageIn& v)
{
    mem_st<NT>(&a.out[idx], stage_value<NT>(a, idx, rhs, v));
}

__device__ __forceinline__ void stage_store(const StageArgs& a, int64_t idx, double rhs)
{
    stage_apply(a, idx, rhs, stage_load(a, idx));
}

// ---- wavefront reductions: a fixed butterfly of lane exchanges over the 64
// lanes of a wave (the same pairs and order on every run; a + b and b + a are
// the same double, so every lane ends with the same value)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// ---- 4th-order finite differences, evaluated as differences of symmetric
// neighbours / differences from the centre so that a small signal on an
// O(1) background keeps its digits.  Scale factors are applied by callers.

// 12 h * D1
__device__ __forceinline__ double fd1(const double* __restrict__ u, int s)
{
    return 8.0 * (u[s] - u[-s]) - (u[2 * s] - u[-2 * s]);
}
// 12 h^2 * D2
__device__ __forceinline__ double fd2(const double* __restrict__ u, int s)
{
    const double c = u[0];
    return 16.0 * ((u[s] - c) + (u[-s] - c)) - ((u[2 * s] - c) + (u[-2 * s] - c));
}
// 64 h / sigma * KO
__device__ __forceinline__ double fko(const double* __restrict__ u, int s)
{
    const double c = u[0];
    return ((u[3 * s] - c) + (u[-3 * s] - c)) - 6.0 * ((u[2 * s] - c) + (u[-2 * s] - c)) +
           15.0 * ((u[s] - c) + (u[-s] - c));
}
// 12 h * lop-sided derivative for the advection term b d U (b >= 0 reads
// i-1..i+3, b < 0 reads i-3..i+1)
__device__ __forceinline__ double fadv(const double* __restrict__ u, int s, double b)
{
    // the b < 0 stencil is the b >= 0 one mirrored and negated: the lanes of
    // a wave read mirrored addresses instead of taking different branches
    // (negation is exact, so the value is the same bit for bit)
    const int m = b >= 0.0 ? s : -s;
    const double c = u[0];
    const double r = (u[3 * m] - c) - 6.0 * (u[2 * m] - c) + 18.0 * (u[m] - c) - 3.0 * (u[-m] - c);
    return b >= 0.0 ? r : -r;
}
// (12 h)^2 * D_b(D_a U)
__device__ __forceinline__ double fmix(const double* __restrict__ u, int sa, int sb)
{
    return 8.0 * (fd1(u + sb, sa) - fd1(u - sb, sa)) - (fd1(u + 2 * sb, sa) - fd1(u - 2 * sb, sa));
}

}  // namespace mol
