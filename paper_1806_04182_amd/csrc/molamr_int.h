// Internal declarations shared by the host runtime and the HIP kernels of
// libmolamr.  Not part of the public ABI (include/molamr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "molamr.h"

namespace mol {

constexpr int G = MOL_GHOST;

// columns per workgroup of the z-marching wave kernel and the longest z chunk
#ifndef MOL_WAVE_WX
#define MOL_WAVE_WX 64
#define MOL_WAVE_WY 8
#endif
#ifndef MOL_WAVE_ZMAX
#define MOL_WAVE_ZMAX 1024
#endif
// tile of the CCZ4 stage kernel (threads per workgroup = product)
#ifndef MOL_CCZ4_TX
#define MOL_CCZ4_TX 8
#define MOL_CCZ4_TY 8
#define MOL_CCZ4_TZ 4
#endif
// LDS halo buffers of the CCZ4 kernel (the halo of the field NBUF - 1 passes
// ahead is requested while a field is differentiated) and its minimum waves
// per SIMD
#ifndef MOL_CCZ4_NBUF
#define MOL_CCZ4_NBUF 2
#endif
#ifndef MOL_CCZ4_WAVES
#define MOL_CCZ4_WAVES 2
#endif

// One patch of a level, as the kernels see it.
struct PatchDev {
    int64_t off;   // start of the patch block in the level buffer (doubles)
    int64_t fs;    // field stride (doubles)
    int n[3];      // interior size
    int pitch_y;   // row pitch: nx + 6 rounded up to 8
    int pitch_z;   // pitch_y * (ny + 6)
    int lo[3];     // global index of the first interior point
    int pad;
};

// Layout of a patch's block in the CCZ4 adjoint workspace: interior points
// only (no ghost layer), rows of nx rounded up to 16 doubles so that every
// row starts on a 128-byte line, slot stride a multiple of 32 doubles.
__host__ __device__ inline int64_t adj_wpitch(int nx) { return ((int64_t)nx + 15) & ~int64_t(15); }
__host__ __device__ inline int64_t adj_wfs(const int n[3])
{
    return (adj_wpitch(n[0]) * n[1] * n[2] + 31) & ~int64_t(31);
}

// A tile of a patch's interior (or of its ghosted box for the adjoint):
// origin in interior coordinates (may be negative for ghosted-box tiles).
struct Tile {
    int patch;
    int o[3];
};

// Same-level ghost copy: destination and source offsets of field 0 in the
// level buffer and the field strides of both patches.
struct GhostCopy {
    int64_t dst;
    int64_t src;
    int64_t dfs;
    int64_t sfs;
};

// Owner-gather adjoint of the ghost copies: one record per source point with
// the range [beg, end) of its images in a list of (dst, dfs) pairs.
struct GhostSource {
    int64_t src;
    int64_t sfs;
    int32_t beg;
    int32_t end;
};
struct GhostImage {
    int64_t dst;
    int64_t dfs;
};

// Coarse-fine ghost points of one fine patch grouped by parent cell: the
// fine points R i0 + m (m in [0, R)^3) of parent cell i0.  Bit
// (mz R + my) R + mx of mask marks the points present.  Axis d is fractional
// (bit d of frac) when some present point has m_d != 0; the stencil then
// spans parent nodes i0-2 .. i0+3 on that axis, otherwise only i0; cbase is
// the stencil corner.  dbase is the fine-level index of the point m = 0,
// which may lie outside the fine patch's ghosted box.
struct ProlongCell {
    int64_t dbase;
    int64_t cbase;
    int64_t dfs, cfs;  // field strides (fine, parent)
    int32_t dpy, dpz;  // fine pitches
    int32_t cpy, cpz;  // parent pitches
    uint64_t mask;
    int32_t frac;
    int32_t pad;
};

// Injection: fine offset, coarse offset (field 0) and field strides.
struct RestrictPt {
    int64_t f;
    int64_t c;
    int64_t ffs;
    int64_t cfs;
};

struct SysParams {
    int system;
    int nf;
    int upwind;
    double h;  // grid spacing of the level (isotropic)
    double sigma, gamma_ad, weno_eps, weno_q, kappa_z, kappa_c, bm_f0, bm_f1, gd_g, gd_eta;
    int mhd_recon, mhd_flux;
    double mhd_ch, mhd_kpsi;
};

// What the fused stage kernels do after evaluating k = dt * rhs.
enum StageMode { ST_RHS = 0, ST_RK4 = 1, ST_SSP3 = 2 };

struct StageArgs {
    const PatchDev* patches;
    const Tile* tiles;
    int ntiles;
    int mode;
    int stage;
    double dt;
    const double* Un;
    const double* Us;
    double* acc;
    double* out;
    double* kst;
    // 1 when one array of the level exceeds 128 MiB: the z-marching wave
    // kernel then streams its point loads and stores past the caches (the
    // other stage kernels measured slower with that and ignore it)
    int stream;
    // 1 when the driver steps a wave level that is one periodic patch: the
    // wave stage kernels then read stencil neighbours at the periodic images
    // of interior points and the ghost fill before the stage is skipped
    int wrap;
    // 1 when the driver steps a CCZ4 level that is one periodic patch of at
    // least 2G points per axis: the stage kernel also writes its output at
    // the periodic ghost images of every point within G of a face (faces,
    // edges, corners), which is what the ghost fill would copy there, and
    // the fill after the stage is skipped
    int images;
};

// kernel launchers (each returns hipGetLastError() of its launch)
hipError_t launch_stage_wave(const SysParams& sp, const StageArgs& a, const int tdim[3], hipStream_t s);
hipError_t launch_stage_mhd(const SysParams& sp, const StageArgs& a, const int tdim[3], hipStream_t s);
hipError_t launch_stage_ccz4(const SysParams& sp, const StageArgs& a, const int tdim[3], hipStream_t s);
inline hipError_t launch_stage(const SysParams& sp, const StageArgs& a, const int tdim[3], hipStream_t s)
{
    switch (sp.system) {
    case MOL_WAVE: return launch_stage_wave(sp, a, tdim, s);
    case MOL_MHD:
    case MOL_MHD_GLM: return launch_stage_mhd(sp, a, tdim, s);
    default: return launch_stage_ccz4(sp, a, tdim, s);
    }
}
hipError_t launch_fill(const GhostCopy* e, int64_t n, int nf, double* U, hipStream_t s);
hipError_t launch_copy2(const GhostCopy* e, int64_t n, int nf, const double* src, double* dst, hipStream_t s);
hipError_t launch_tag(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], const double* U,
                      int field, double thr, const int period[3], uint8_t* flags, hipStream_t s);
// radiative outer boundary: ghosted-box coordinates of each boundary point of
// the level-0 patch, and the per-field speed and value at infinity
struct RadPt {
    int32_t a[4];
};
struct RadParams {
    double v[32], uinf[32];
};
hipError_t launch_radiative(const StageArgs& a, const PatchDev& P, const RadPt* pts, int64_t n, int nf,
                            const RadParams& rp, const double xlo[3], double h, hipStream_t s);
hipError_t launch_fill_adjoint(const GhostSource* src, int64_t nsrc, const GhostImage* img,
                               int nf, double* A, hipStream_t s);
hipError_t launch_bor_band(const GhostCopy* band, int64_t n, int nf, const double w[4], const double* Un,
                           const double* k0, const double* k1, const double* k2, const double* k3, double* T,
                           hipStream_t s);
hipError_t launch_prolong(const ProlongCell* e, int64_t n, int nf, int R, const double* lw_host, const double* T,
                          double* U, hipStream_t s);
hipError_t launch_restrict(const RestrictPt* e, int64_t n, int nf, const double* Uf, double* Uc,
                           hipStream_t s);
int ccz4_adjoint_slots();
hipError_t launch_ccz4_adjoint(const SysParams& sp, const PatchDev* patches, const Tile* tiles, int ntiles,
                               const int td[3], const Tile* gtiles, int ngtiles, const int gtd[3],
                               const double* U, const double* lam, double* W, const int64_t* wofs, double* lamU,
                               hipStream_t s);
// One stage of the reverse RK4 step on a level that is one periodic patch of
// at least 7 points per axis: the point-wise kernels at Ust, then the gather
// over interior points with periodic stencil images and the epilogue
// wsum = (first ? 0 : wsum) + v, then wnext = a lam0 + b v, or on the last
// stage lam = lam0 + wsum (interior points only; ghost entries untouched).
hipError_t launch_ccz4_adjoint_stage(const SysParams& sp, const PatchDev* patches, const Tile* tiles, int ntiles,
                                     const int td[3], const Tile* itiles, int nitiles, const int itd[3],
                                     const double* U, const double* lam_in, double* W, const int64_t* wofs,
                                     const double* lam0, double* lam, double* wsum, double* wnext, double a,
                                     double b, int first, int last, hipStream_t s);
hipError_t launch_wave_adjoint(const SysParams& sp, const PatchDev* patches, const Tile* tiles,
                               int ntiles, const int tdim[3], const double* lam, double* lamU,
                               hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y,
                        double* z, hipStream_t s);
// Closed coordinate box lo <= x <= hi per axis (infinite bounds: no restriction).
struct CoordBox {
    double lo[3], hi[3];
};
hipError_t launch_norms(const PatchDev* patches, const Tile* tiles, int ntiles, const int tdim[3],
                        const double* U, int field, double shift, double radius, double h,
                        const double xlo[3], const CoordBox& box, double* partial, int nblocks, double* out,
                        hipStream_t s);
int monitor_partials();  // doubles per reduction block of launch_monitor
hipError_t launch_monitor(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], int nf, int ccz4,
                          unsigned which, double h, double sigma, const double* U, double* point, double* partial,
                          int nblocks, double* out, hipStream_t s);
hipError_t launch_puncture(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3], int nholes,
                           const double* holes, double h, const double xlo[3], int whole, double* U, hipStream_t s);
hipError_t launch_sphere_adjoint(const PatchDev* patches, const Tile* tiles, int ntiles, const int tdim[3],
                                int nf, int field, double radius, double scale, double h, const double xlo[3],
                                double* lam, hipStream_t s);
hipError_t launch_gaussian(const PatchDev* patches, const Tile* tiles, int ntiles, const int td[3],
                           const double prm5[5], double h, const double xlo[3], const double per[3], int nf, int fg,
                           unsigned ones, double* U, const double* lam, double* partial, int nblocks, double* grad,
                           hipStream_t s);

}  // namespace mol
