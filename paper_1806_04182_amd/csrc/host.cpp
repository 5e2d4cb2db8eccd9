// Host runtime of libmolamr: patchset construction (layout, ghost / prolong /
// restrict schedules, tile work lists), argument validation, the C ABI entry
// points, the sub-cycled driver and its HIP-graph capture.
//
// The AMR skeleton follows Sec. III of Palenzuela et al. (arXiv:1806.04182);
// BOR sub-cycling follows App. D; the spatial interpolation is the quintic
// Lagrange polynomial of Sec. III.A.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "molamr_int.h"

using namespace mol;

// workgroup tiles of the adjoint (at most 256 threads each): over the
// ghosted box for the transposed stencils (wave adjoint, CCZ4 gather), over
// the interior for the CCZ4 point-wise kernels.  Measured on the 48^3 CCZ4
// adjoint: the gather takes 185 us with 32 x 4 x 2 against 223 us with
// 16 x 4 x 4 (rows of whole cache lines, fewer workgroups than resident
// slots); the eight point-wise kernels 562 - 185 = 377 us with 16 x 16 x 1
// against 411 us with the stage kernel's 8 x 8 x 4
// tile of the CCZ4 adjoint's periodic gather (interior points)
#ifndef MOL_ADJ_WTX
#define MOL_ADJ_WTX 16
#define MOL_ADJ_WTY 8
#define MOL_ADJ_WTZ 2
#endif
#ifndef MOL_ADJ_GTX
#define MOL_ADJ_GTX 32
#define MOL_ADJ_GTY 4
#define MOL_ADJ_GTZ 2
#endif
#ifndef MOL_ADJ_PTX
#define MOL_ADJ_PTX 16
#define MOL_ADJ_PTY 16
#define MOL_ADJ_PTZ 1
#endif

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(MOL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct Box {
    int lo[3], hi[3];
    int n(int d) const { return hi[d] - lo[d] + 1; }
};

int wrapi(int a, int n)
{
    int m = a % n;
    return m < 0 ? m + n : m;
}

int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

// Device tables of one object in one allocation: each table is appended to a
// host staging buffer (256-byte aligned), device-only regions are reserved
// after them, and commit() makes one hipMalloc and one copy, then points
// every registered slot at its place.  Slots must not move before commit.
struct Arena {
    std::vector<unsigned char> host;
    std::vector<std::pair<void**, size_t>> tables;    // slot, offset
    std::vector<std::pair<void**, size_t>> reserved;  // slot, bytes
    struct Adopt {
        void** slot;
        const void* src;
        size_t bytes;
    };
    std::vector<Adopt> adopted;  // device tables copied from elsewhere
    void* dev = nullptr;
    void stage(const void* src, size_t bytes, void** slot)
    {
        const size_t off = (host.size() + 255) / 256 * 256;
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        tables.emplace_back(slot, off);
    }
    void reserve(size_t bytes, void** slot) { reserved.emplace_back(slot, bytes); }
    void adopt(const void* src, size_t bytes, void** slot) { adopted.push_back(Adopt{slot, src, bytes}); }
    int commit()
    {
        size_t total = (host.size() + 255) / 256 * 256;
        std::vector<size_t> roff, aoff;
        for (auto& r : reserved) {
            roff.push_back(total);
            total += (r.second + 255) / 256 * 256;
        }
        for (auto& a : adopted) {
            aoff.push_back(total);
            total += (a.bytes + 255) / 256 * 256;
        }
        if (total == 0) return MOL_OK;
        hipError_t e = hipMalloc(&dev, total);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        unsigned char* d = static_cast<unsigned char*>(dev);
        if (!host.empty() && (e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy");
        for (size_t i = 0; i < adopted.size(); ++i)
            if ((e = hipMemcpy(d + aoff[i], adopted[i].src, adopted[i].bytes, hipMemcpyDeviceToDevice)) != hipSuccess)
                return hip_fail(e, "hipMemcpy");
        for (auto& t : tables) *t.first = d + t.second;
        for (size_t i = 0; i < reserved.size(); ++i) *reserved[i].first = d + roff[i];
        for (size_t i = 0; i < adopted.size(); ++i) *adopted[i].slot = d + aoff[i];
        host.clear();
        host.shrink_to_fit();
        tables.clear();
        reserved.clear();
        adopted.clear();
        return MOL_OK;
    }
    void release()
    {
        if (dev) (void)hipFree(dev);
        dev = nullptr;
    }
};

// device array helper: a block of its own (hipMalloc'd), or a table in an
// arena (placed by the arena's commit, freed with it)
template <class T>
struct DevArr {
    T* p = nullptr;
    int64_t n = 0;
    bool in_arena = false;
    int upload(const std::vector<T>& v, Arena* A = nullptr)
    {
        n = (int64_t)v.size();
        if (n == 0) return MOL_OK;
        if (A) {
            in_arena = true;
            A->stage(v.data(), sizeof(T) * n, reinterpret_cast<void**>(&p));
            return MOL_OK;
        }
        hipError_t e = hipMalloc(&p, sizeof(T) * n);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        e = hipMemcpy(p, v.data(), sizeof(T) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        return MOL_OK;
    }
    void release()
    {
        if (p && !in_arena) (void)hipFree(p);
        p = nullptr;
        n = 0;
        in_arena = false;
    }
    // the same table as `o` (a device copy made by A's commit)
    void adopt(const DevArr& o, Arena* A)
    {
        n = o.n;
        if (n == 0) return;
        in_arena = true;
        A->adopt(o.p, sizeof(T) * n, reinterpret_cast<void**>(&p));
    }
};

struct TileList {
    int tdim[3] = {1, 1, 1};
    DevArr<Tile> dev;
    std::vector<int> by_patch;  // start of each patch's tiles, then the total
    std::vector<int> count;     // tiles of each patch
    int order = 0;              // patch order in the launch: 0 as given, 1 largest first
};

}  // namespace

struct mol_patchset {
    SysParams sp{};
    int nlev = 0;
    int open = 0;                  // radiative outer boundary (level 0 one patch)
    RadParams rad{};               // per-field speed and value at infinity
    DevArr<RadPt> rad_pts;         // the level-0 ghost points it evolves
    int N0[3] = {0, 0, 0};
    double xlo[3] = {0, 0, 0};
    double dx0 = 0;
    struct Level {
        int ratio = 1;
        int period[3] = {0, 0, 0};
        double h = 0;
        std::vector<Box> boxes;
        std::vector<PatchDev> pd;
        int64_t nelems = 0;
        DevArr<PatchDev> d_pd;
        // same-level ghost copies, grouped by destination patch
        DevArr<GhostCopy> fill;
        std::vector<int64_t> fill_by_patch;
        DevArr<GhostSource> fill_src;
        DevArr<GhostImage> fill_img;
        // coarse-fine ghost points (this level is the fine one) grouped by
        // parent cell, by dst patch
        DevArr<ProlongCell> pcell;
        std::vector<int64_t> pcell_by_patch;
        std::vector<double> lagw;  // Lagrange weights [R][6]
        // parent points read by the prolongation stencils of this level: the
        // position in a parent patch's ghosted box (dst) and the interior
        // point that owns it (src)
        DevArr<GhostCopy> band;
        std::vector<int64_t> band_by_patch;
        // injection into the parent level, grouped by fine patch
        DevArr<RestrictPt> rst;
        std::vector<int64_t> rst_by_patch;
        TileList tiles;   // interior tiles for the stage kernels
        TileList gtiles;  // ghosted-box tiles for the adjoint
        TileList ptiles;  // interior tiles for the CCZ4 adjoint's point-wise kernels
        TileList ntiles;  // interior tiles for reductions / initial data
        TileList wtiles;  // interior tiles for the CCZ4 adjoint's periodic gather
        // CCZ4 adjoint workspace: start of each patch's block (slots x fs)
        DevArr<int64_t> wofs;
        int64_t wsize = 0;
    };
    Level L[MOL_MAX_LEVELS];
    Arena arena;                // every device table and buffer below
    std::vector<DevArr<Tile>> retired;  // tile lists replaced by the autotuner (graphs may still use them)
    double* scratch = nullptr;  // reduction partials
    double* tband = nullptr;    // parent-level BOR stage state used by the prolongation
    int red_blocks = 256;
    hipStream_t capture_stream = nullptr;

    ~mol_patchset()
    {
        for (auto& l : L) {
            l.d_pd.release();
            l.fill.release();
            l.fill_src.release();
            l.fill_img.release();
            l.pcell.release();
            l.band.release();
            l.rst.release();
            l.tiles.dev.release();
            l.gtiles.dev.release();
            l.ptiles.dev.release();
            l.wofs.release();
            l.ntiles.dev.release();
            l.wtiles.dev.release();
        }
        rad_pts.release();
        for (auto& t : retired) t.release();
        arena.release();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
    }
};

struct mol_regrid {
    mol_patchset* pn = nullptr;
    const mol_patchset* po = nullptr;
    DevArr<GhostCopy> copy[MOL_MAX_LEVELS];   // new <- old at the same level
    DevArr<ProlongCell> cells[MOL_MAX_LEVELS];  // new points interpolated from the new parent
    ~mol_regrid()
    {
        for (int l = 0; l < MOL_MAX_LEVELS; ++l) {
            copy[l].release();
            cells[l].release();
        }
    }
};

struct mol_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

using Level = mol_patchset::Level;

int64_t local_index(const PatchDev& p, int i, int j, int k)  // ghosted local coords
{
    return (int64_t)k * p.pitch_z + (int64_t)j * p.pitch_y + i;
}

// patch of `lev` whose interior holds global index g (wrapped by the period);
// candidates restrict the search.  Returns -1 when none.
int find_owner(const Level& lev, const int g0[3], const std::vector<int>& cand, int gw[3])
{
    for (int d = 0; d < 3; ++d) gw[d] = wrapi(g0[d], lev.period[d]);
    for (int q : cand) {
        const Box& b = lev.boxes[q];
        if (gw[0] >= b.lo[0] && gw[0] <= b.hi[0] && gw[1] >= b.lo[1] && gw[1] <= b.hi[1] &&
            gw[2] >= b.lo[2] && gw[2] <= b.hi[2])
            return q;
    }
    return -1;
}

// do the periodic images of boxes a (grown by `grow`) and b intersect?
bool periodic_touch(const Box& a, int grow, const Box& b, const int per[3])
{
    for (int d = 0; d < 3; ++d) {
        bool any = false;
        for (int s = -1; s <= 1 && !any; ++s) {
            int lo = b.lo[d] + s * per[d], hi = b.hi[d] + s * per[d];
            if (hi >= a.lo[d] - grow && lo <= a.hi[d] + grow) any = true;
        }
        if (!any) return false;
    }
    return true;
}

std::vector<std::vector<int>> candidates(const Level& a, int grow, const Level& b, int scale)
{
    // scale: a's coordinates are b's coordinates times `scale` (a finer)
    std::vector<std::vector<int>> out(a.boxes.size());
    for (size_t p = 0; p < a.boxes.size(); ++p) {
        Box ab = a.boxes[p];
        for (int d = 0; d < 3; ++d) {
            ab.lo[d] = (int)std::floor((double)(ab.lo[d] - grow) / scale);
            ab.hi[d] = (int)std::floor((double)(ab.hi[d] + grow) / scale);
        }
        for (size_t q = 0; q < b.boxes.size(); ++q)
            if (periodic_touch(ab, 4, b.boxes[q], b.period)) out[p].push_back((int)q);
    }
    return out;
}

// Coarse-fine ghost point (host side, used to build the band and the cells):
// destination (fine level), base of its parent stencil (parent level, field 0,
// lowest corner), field strides, parent pitches and the fine index modulo R.
struct ProlongPt {
    int64_t dst;
    int64_t cbase;
    int64_t dfs;
    int64_t cfs;
    int32_t cpy;
    int32_t cpz;
    int8_t m[3];
};

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// tiles of td[0] x td[1] x td[2] points over every patch (grown by margin),
// each patch's tiles contiguous; patches in the given order (0: as listed,
// 1: largest interior first, so that the small patches fill the tail of the
// launch)
int build_tiles(const Level& lev, const int td[3], int margin, TileList& tl, Arena* A, int order = 0)
{
    tl.tdim[0] = td[0];
    tl.tdim[1] = td[1];
    tl.tdim[2] = td[2];
    tl.order = order;
    const size_t np = lev.pd.size();
    std::vector<int> perm(np);
    for (size_t p = 0; p < np; ++p) perm[p] = (int)p;
    auto vol = [&](int p) { return (int64_t)lev.pd[p].n[0] * lev.pd[p].n[1] * lev.pd[p].n[2]; };
    if (order == 1) std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return vol(a) > vol(b); });
    std::vector<Tile> v;
    tl.by_patch.assign(np + 1, 0);
    tl.count.assign(np, 0);
    for (int p : perm) {
        const PatchDev& pd = lev.pd[p];
        tl.by_patch[p] = (int)v.size();
        if (order == 2 || order == 3) {
            // columns of tiles along z, z fastest (order 2), or grouped in
            // blocks of 2 x 2 columns (order 3): tiles that share z halos run
            // together on one XCD
            const int bw = order == 3 ? 2 : 1;
            for (int jb = -margin; jb < pd.n[1] + margin; jb += bw * td[1])
                for (int ib = -margin; ib < pd.n[0] + margin; ib += bw * td[0])
                    for (int jj = jb; jj < std::min(jb + bw * td[1], pd.n[1] + margin); jj += td[1])
                        for (int ii = ib; ii < std::min(ib + bw * td[0], pd.n[0] + margin); ii += td[0])
                            for (int k = -margin; k < pd.n[2] + margin; k += td[2]) v.push_back(Tile{p, {ii, jj, k}});
        } else {
            for (int k = -margin; k < pd.n[2] + margin; k += td[2])
                for (int j = -margin; j < pd.n[1] + margin; j += td[1])
                    for (int i = -margin; i < pd.n[0] + margin; i += td[0])
                        v.push_back(Tile{p, {i, j, k}});
        }
        tl.count[p] = (int)v.size() - tl.by_patch[p];
    }
    tl.by_patch[np] = (int)v.size();
    return tl.dev.upload(v, A);
}

// Tile of the stage kernels (the autotuner can replace it).  Wave: levels of
// at least 2^21 points march along z (64 x 8 columns; chunk length for about
// 512 workgroups, two per compute unit: the fastest measured at 256^3 (64
// planes) and 512^3 (whole 512-plane columns, no chunk-boundary re-reads));
// smaller levels use one thread per point.  MHD: 15 x 15 columns, 4 planes.
void default_tile(int system, int64_t level_points, int td[3])
{
    switch (system) {
    case MOL_WAVE:
        if (level_points >= (int64_t(1) << 21)) {
            td[0] = MOL_WAVE_WX;
            td[1] = MOL_WAVE_WY;
            td[2] = (int)std::max<int64_t>(
                4, std::min<int64_t>(MOL_WAVE_ZMAX, level_points / (MOL_WAVE_WX * MOL_WAVE_WY * 512)));
        } else {
            td[0] = 32;
            td[1] = 4;
            td[2] = 2;
        }
        break;
    case MOL_MHD:
    case MOL_MHD_GLM: td[0] = 15; td[1] = 15; td[2] = 4; break;  // 15 x 15 columns, 4 planes (z-marching)
    default: td[0] = MOL_CCZ4_TX; td[1] = MOL_CCZ4_TY; td[2] = MOL_CCZ4_TZ; break;
    }
}

bool overlap(const Box& a, const Box& b)
{
    for (int d = 0; d < 3; ++d)
        if (a.hi[d] < b.lo[d] || b.hi[d] < a.lo[d]) return false;
    return true;
}

// level l of ps takes over level l of prev (whose levels 0..l match): the
// host lists are copied and the device tables copied into ps's arena
void reuse_level(mol_patchset* ps, const mol_patchset* prev, int l)
{
    Level& lev = ps->L[l];
    const Level& o = prev->L[l];
    Arena* A = &ps->arena;
    lev.d_pd.adopt(o.d_pd, A);
    lev.fill.adopt(o.fill, A);
    lev.fill_by_patch = o.fill_by_patch;
    lev.fill_src.adopt(o.fill_src, A);
    lev.fill_img.adopt(o.fill_img, A);
    lev.pcell.adopt(o.pcell, A);
    lev.pcell_by_patch = o.pcell_by_patch;
    lev.lagw = o.lagw;
    lev.band.adopt(o.band, A);
    lev.band_by_patch = o.band_by_patch;
    lev.rst.adopt(o.rst, A);
    lev.rst_by_patch = o.rst_by_patch;
    TileList* mine[5] = {&lev.tiles, &lev.gtiles, &lev.ntiles, &lev.ptiles, &lev.wtiles};
    const TileList* theirs[5] = {&o.tiles, &o.gtiles, &o.ntiles, &o.ptiles, &o.wtiles};
    for (int i = 0; i < 5; ++i) {
        for (int d = 0; d < 3; ++d) mine[i]->tdim[d] = theirs[i]->tdim[d];
        mine[i]->by_patch = theirs[i]->by_patch;
        mine[i]->count = theirs[i]->count;
        mine[i]->order = theirs[i]->order;
        mine[i]->dev.adopt(theirs[i]->dev, A);
    }
    lev.wofs.adopt(o.wofs, A);
    lev.wsize = o.wsize;
    if (l == 0 && ps->open) {
        ps->rad_pts.adopt(prev->rad_pts, A);
        ps->rad = prev->rad;
    }
}

// number of leading levels of prev that ps can take over: same system and
// boundary, and levels 0..l with the same ratios and boxes (in order)
int same_levels(const mol_patchset* ps, const mol_patchset* prev)
{
    if (!prev || prev->sp.system != ps->sp.system || prev->open != ps->open) return 0;
    for (int d = 0; d < 3; ++d)
        if (prev->N0[d] != ps->N0[d]) return 0;
    int n = 0;
    for (; n < std::min(ps->nlev, prev->nlev); ++n) {
        const Level& a = ps->L[n];
        const Level& b = prev->L[n];
        if (a.ratio != b.ratio || a.boxes.size() != b.boxes.size() || a.nelems != b.nelems) break;
        bool same = true;
        for (size_t q = 0; q < a.boxes.size() && same; ++q)
            for (int d = 0; d < 3; ++d)
                if (a.boxes[q].lo[d] != b.boxes[q].lo[d] || a.boxes[q].hi[d] != b.boxes[q].hi[d]) same = false;
        if (!same) break;
    }
    return n;
}

int build(mol_patchset* ps, const mol_hierarchy_desc* h, const mol_patchset* prev = nullptr)
{
    const int* bx = h->boxes;
    for (int l = 0; l < ps->nlev; ++l) {
        Level& lev = ps->L[l];
        lev.ratio = l == 0 ? 1 : h->ratio[l];
        if (l > 0 && (lev.ratio < 2 || lev.ratio > 4))
            return fail(MOL_EINVAL, "level %d: ratio %d not in {2,3,4}", l, lev.ratio);
        for (int d = 0; d < 3; ++d)
            lev.period[d] = l == 0 ? ps->N0[d] : ps->L[l - 1].period[d] * lev.ratio;
        lev.h = l == 0 ? ps->dx0 : ps->L[l - 1].h / lev.ratio;
        int np = h->npatch[l];
        if (np < 1) return fail(MOL_EINVAL, "level %d has no patch", l);
        int64_t vol = 0, off = 0;
        for (int p = 0; p < np; ++p, bx += 6) {
            Box b;
            for (int d = 0; d < 3; ++d) {
                b.lo[d] = bx[d];
                b.hi[d] = bx[3 + d];
                if (b.hi[d] < b.lo[d] || b.lo[d] < 0 || b.hi[d] >= lev.period[d])
                    return fail(MOL_EINVAL, "level %d patch %d: box outside [0, %d) on axis %d",
                                l, p, lev.period[d], d);
            }
            for (const Box& o : lev.boxes)
                if (overlap(o, b)) return fail(MOL_EINVAL, "level %d patch %d overlaps another", l, p);
            lev.boxes.push_back(b);
            vol += (int64_t)b.n(0) * b.n(1) * b.n(2);
            PatchDev pd{};
            for (int d = 0; d < 3; ++d) {
                pd.n[d] = b.n(d);
                pd.lo[d] = b.lo[d];
            }
            // rows padded to 8 doubles and the patch start shifted by 8 - G
            // doubles: interior rows start on 64-byte boundaries.  Rows of
            // at least 256 doubles are padded to 16 and shifted by 16 - G, so
            // that their interior rows start on 128-byte boundaries and touch
            // no more 128-byte lines than they fill (the extra padding is
            // under 6%).  Shorter rows keep the 8-double pitch: a pitch that
            // is a multiple of 16 measured slower there (48^3 adjoint
            // workspace, 16..48-point AMR patches).
            const int align = pd.n[0] + 2 * G >= 256 ? 16 : 8;
            pd.pitch_y = (int)round_up(pd.n[0] + 2 * G, align);
            pd.pitch_z = pd.pitch_y * (pd.n[1] + 2 * G);
            pd.fs = round_up((int64_t)pd.pitch_z * (pd.n[2] + 2 * G), 32);
            pd.off = off + (align - G);
            off += round_up((align - G) + pd.fs * ps->sp.nf, 32);
            lev.pd.push_back(pd);
        }
        lev.nelems = off;
        if (l == 0 && vol != (int64_t)ps->N0[0] * ps->N0[1] * ps->N0[2])
            return fail(MOL_EINVAL, "level 0 boxes must tile the periodic domain exactly");
        if (ps->open && l == 0 && np != 1) return fail(MOL_EINVAL, "an open domain needs one level-0 patch");
        if (ps->open && l == 1)
            for (const Box& b : lev.boxes)
                for (int d = 0; d < 3; ++d)
                    if (floor_div(b.lo[d], lev.ratio) < 6 || floor_div(b.hi[d], lev.ratio) > ps->N0[d] - 7)
                        return fail(MOL_EINVAL, "level 1 patch must keep 6 level-0 points from the open boundary");
    }

    const int nsame = same_levels(ps, prev);
    for (int l = 0; l < ps->nlev; ++l) {
        Level& lev = ps->L[l];
        if (l < nsame) {
            reuse_level(ps, prev, l);
            continue;
        }
        int rc = lev.d_pd.upload(lev.pd, &ps->arena);
        if (rc) return rc;
        // ---- same-level ghost copies and coarse-fine points ----
        auto cand = candidates(lev, G, lev, 1);
        std::vector<GhostCopy> fill;
        std::vector<RadPt> rad;
        std::vector<ProlongPt> pro;
        std::vector<int64_t> pro_by_patch(lev.pd.size() + 1, 0);
        std::vector<ProlongCell> cells;
        lev.fill_by_patch.assign(lev.pd.size() + 1, 0);
        lev.pcell_by_patch.assign(lev.pd.size() + 1, 0);
        const Level* par = l > 0 ? &ps->L[l - 1] : nullptr;
        std::vector<std::vector<int>> pcand;
        std::vector<int> allpar;
        if (par) {
            pcand = candidates(lev, G, *par, lev.ratio);
            for (size_t q = 0; q < par->boxes.size(); ++q) allpar.push_back((int)q);
        }
        const int R = lev.ratio;
        for (size_t p = 0; p < lev.pd.size(); ++p) {
            lev.fill_by_patch[p] = (int64_t)fill.size();
            pro_by_patch[p] = (int64_t)pro.size();
            lev.pcell_by_patch[p] = (int64_t)cells.size();
            const PatchDev& pd = lev.pd[p];
            // parent cells of this patch's coarse-fine ghost points: cell
            // coordinates floor(g / R), owner patch and owned position of i0
            struct CellTmp {
                int key[3], q0, cw[3];
                uint64_t mask;
                int frac;
            };
            std::vector<CellTmp> ct;
            std::map<std::array<int, 3>, size_t> cidx;
            for (int k = -G; k < pd.n[2] + G; ++k)
                for (int j = -G; j < pd.n[1] + G; ++j)
                    for (int i = -G; i < pd.n[0] + G; ++i) {
                        if (i >= 0 && i < pd.n[0] && j >= 0 && j < pd.n[1] && k >= 0 && k < pd.n[2])
                            continue;
                        int g[3] = {pd.lo[0] + i, pd.lo[1] + j, pd.lo[2] + k}, gw[3];
                        int64_t dst = pd.off + local_index(pd, i + G, j + G, k + G);
                        if (l == 0 && ps->open) {  // evolved by the radiative condition
                            rad.push_back(RadPt{{i + G, j + G, k + G, 0}});
                            continue;
                        }
                        int q = find_owner(lev, g, cand[p], gw);
                        if (q >= 0) {
                            const PatchDev& qd = lev.pd[q];
                            int64_t src = qd.off + local_index(qd, gw[0] - qd.lo[0] + G,
                                                               gw[1] - qd.lo[1] + G, gw[2] - qd.lo[2] + G);
                            fill.push_back(GhostCopy{dst, src, pd.fs, qd.fs});
                            continue;
                        }
                        if (!par) return fail(MOL_EINVAL, "level 0 ghost point without a source");
                        // coarse position g/R = i0 + m/R per axis
                        int i0[3], m[3], c0[3], cw[3];
                        for (int d = 0; d < 3; ++d) {
                            gw[d] = wrapi(g[d], lev.period[d]);
                            m[d] = gw[d] % R;
                            i0[d] = gw[d] / R;
                        }
                        int q0 = find_owner(*par, i0, pcand[p], cw);
                        if (q0 < 0) q0 = find_owner(*par, i0, allpar, cw);
                        if (q0 < 0)
                            return fail(MOL_EINVAL, "level %d patch %zu: ghost point has no parent data", l, p);
                        // every stencil node must be interior data of the parent level
                        for (int c = (m[2] ? -2 : 0); c <= (m[2] ? 3 : 0); ++c)
                            for (int b = (m[1] ? -2 : 0); b <= (m[1] ? 3 : 0); ++b)
                                for (int a = (m[0] ? -2 : 0); a <= (m[0] ? 3 : 0); ++a) {
                                    int nd[3] = {i0[0] + a, i0[1] + b, i0[2] + c}, tmp[3];
                                    if (find_owner(*par, nd, pcand[p], tmp) < 0 &&
                                        find_owner(*par, nd, allpar, tmp) < 0)
                                        return fail(MOL_EINVAL,
                                                    "level %d patch %zu: prolongation stencil leaves the "
                                                    "parent level (nest fine levels at least 6 parent points "
                                                    "inside it)", l, p);
                                }
                        const PatchDev& qd = par->pd[q0];
                        for (int d = 0; d < 3; ++d) c0[d] = cw[d] - qd.lo[d] + G - (m[d] ? 2 : 0);
                        ProlongPt e{};
                        e.dst = dst;
                        e.cbase = qd.off + local_index(qd, c0[0], c0[1], c0[2]);
                        e.dfs = pd.fs;
                        e.cfs = qd.fs;
                        e.cpy = qd.pitch_y;
                        e.cpz = qd.pitch_z;
                        for (int d = 0; d < 3; ++d) e.m[d] = (int8_t)m[d];
                        pro.push_back(e);
                        const std::array<int, 3> key = {floor_div(g[0], R), floor_div(g[1], R), floor_div(g[2], R)};
                        auto it = cidx.find(key);
                        if (it == cidx.end()) {
                            it = cidx.emplace(key, ct.size()).first;
                            ct.push_back(CellTmp{{key[0], key[1], key[2]}, q0, {cw[0], cw[1], cw[2]}, 0, 0});
                        }
                        CellTmp& c = ct[it->second];
                        c.mask |= uint64_t(1) << ((m[2] * R + m[1]) * R + m[0]);
                        for (int d = 0; d < 3; ++d)
                            if (m[d]) c.frac |= 1 << d;
                    }
            // cells ordered by their fractional axes (uniform work within a wave)
            std::stable_sort(ct.begin(), ct.end(), [](const CellTmp& a, const CellTmp& b) { return a.frac < b.frac; });
            for (const CellTmp& c : ct) {
                const PatchDev& qd = par->pd[c.q0];
                int c0[3];
                for (int d = 0; d < 3; ++d) c0[d] = c.cw[d] - qd.lo[d] + G - ((c.frac >> d & 1) ? 2 : 0);
                ProlongCell e{};
                e.dbase = pd.off + local_index(pd, R * c.key[0] - pd.lo[0] + G, R * c.key[1] - pd.lo[1] + G,
                                               R * c.key[2] - pd.lo[2] + G);
                e.cbase = qd.off + local_index(qd, c0[0], c0[1], c0[2]);
                e.dfs = pd.fs;
                e.cfs = qd.fs;
                e.dpy = pd.pitch_y;
                e.dpz = pd.pitch_z;
                e.cpy = qd.pitch_y;
                e.cpz = qd.pitch_z;
                e.mask = c.mask;
                e.frac = c.frac;
                cells.push_back(e);
            }
        }
        lev.fill_by_patch[lev.pd.size()] = (int64_t)fill.size();
        pro_by_patch[lev.pd.size()] = (int64_t)pro.size();
        lev.pcell_by_patch[lev.pd.size()] = (int64_t)cells.size();
        if ((rc = lev.fill.upload(fill, &ps->arena))) return rc;
        if (l == 0 && ps->open && (rc = ps->rad_pts.upload(rad, &ps->arena))) return rc;
        if ((rc = lev.pcell.upload(cells, &ps->arena))) return rc;
        if (par) {
            // every parent point that some stencil reads, once, grouped by the
            // fine patch that first needs it (so per-patch launches cover it)
            std::vector<uint8_t> mark((size_t)par->nelems, 0);
            std::vector<GhostCopy> band;
            // parent patch of each band position: patch blocks are contiguous and ordered
            std::vector<int64_t> pstart(par->pd.size());
            for (size_t q = 0; q < par->pd.size(); ++q) pstart[q] = par->pd[q].off;
            std::vector<int> allpar2;
            for (size_t q = 0; q < par->boxes.size(); ++q) allpar2.push_back((int)q);
            lev.band_by_patch.assign(lev.pd.size() + 1, 0);
            std::vector<int64_t> fs_of(par->pd.size());
            for (size_t p = 0; p < lev.pd.size(); ++p) {
                lev.band_by_patch[p] = (int64_t)band.size();
                for (int64_t t = pro_by_patch[p]; t < pro_by_patch[p + 1]; ++t) {
                    const ProlongPt& e = pro[t];
                    for (int c = 0; c < (e.m[2] ? 6 : 1); ++c)
                        for (int b = 0; b < (e.m[1] ? 6 : 1); ++b)
                            for (int a = 0; a < (e.m[0] ? 6 : 1); ++a) {
                                const int64_t o = e.cbase + (int64_t)c * e.cpz + (int64_t)b * e.cpy + a;
                                if (!mark[o]) {
                                    mark[o] = 1;
                                    // global index of this ghosted-box position, and its owner
                                    const size_t q = (size_t)(std::upper_bound(pstart.begin(), pstart.end(), o) -
                                                              pstart.begin()) - 1;
                                    const PatchDev& qd = par->pd[q];
                                    const int64_t loc = o - qd.off;
                                    const int lz = (int)(loc / qd.pitch_z), ly = (int)((loc % qd.pitch_z) / qd.pitch_y),
                                              lx = (int)(loc % qd.pitch_y);
                                    int g[3] = {qd.lo[0] + lx - G, qd.lo[1] + ly - G, qd.lo[2] + lz - G}, gw[3];
                                    const int own = find_owner(*par, g, allpar2, gw);
                                    if (own < 0)
                                        return fail(MOL_EINVAL, "level %d: prolongation stencil leaves the parent level", l);
                                    const PatchDev& od = par->pd[own];
                                    band.push_back(GhostCopy{o,
                                                             od.off + local_index(od, gw[0] - od.lo[0] + G,
                                                                                  gw[1] - od.lo[1] + G, gw[2] - od.lo[2] + G),
                                                             qd.fs, od.fs});
                                }
                            }
                }
            }
            lev.band_by_patch[lev.pd.size()] = (int64_t)band.size();
            if ((rc = lev.band.upload(band, &ps->arena))) return rc;
        }
        // owner-gather form of the fill (for the adjoint)
        {
            std::vector<size_t> idx(fill.size());
            for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](size_t a, size_t b) { return fill[a].src < fill[b].src; });
            std::vector<GhostSource> srcs;
            std::vector<GhostImage> imgs;
            for (size_t t = 0; t < idx.size(); ++t) {
                const GhostCopy& e = fill[idx[t]];
                if (srcs.empty() || srcs.back().src != e.src)
                    srcs.push_back(GhostSource{e.src, e.sfs, (int32_t)imgs.size(), (int32_t)imgs.size()});
                imgs.push_back(GhostImage{e.dst, e.dfs});
                srcs.back().end = (int32_t)imgs.size();
            }
            if ((rc = lev.fill_src.upload(srcs, &ps->arena))) return rc;
            if ((rc = lev.fill_img.upload(imgs, &ps->arena))) return rc;
        }
        if (par) {
            // Lagrange weights at xi = m/R through nodes -2..3 (Sec. III.A)
            // (row m = 0 is (0, 0, 1, 0, 0, 0); the kernel takes that node as is)
            std::vector<double> lw(R * 6, 0.0);
            for (int m = 0; m < R; ++m) {
                double xi = (double)m / R;
                for (int j = 0; j < 6; ++j) {
                    double num = 1.0, den = 1.0;
                    for (int q = 0; q < 6; ++q) {
                        if (q == j) continue;
                        num *= xi - (q - 2);
                        den *= (double)(j - q);
                    }
                    lw[m * 6 + j] = num / den;
                }
            }
            lev.lagw = lw;
            // injection: coarse interior points that coincide with fine interior points
            std::vector<RestrictPt> rst;
            lev.rst_by_patch.assign(lev.pd.size() + 1, 0);
            std::vector<std::vector<RestrictPt>> per(lev.pd.size());
            std::vector<int> allfine;
            for (size_t q = 0; q < lev.boxes.size(); ++q) allfine.push_back((int)q);
            for (size_t q = 0; q < par->pd.size(); ++q) {
                const PatchDev& qd = par->pd[q];
                for (int k = 0; k < qd.n[2]; ++k)
                    for (int j = 0; j < qd.n[1]; ++j)
                        for (int i = 0; i < qd.n[0]; ++i) {
                            int gf[3] = {R * (qd.lo[0] + i), R * (qd.lo[1] + j), R * (qd.lo[2] + k)}, fw[3];
                            int p = find_owner(lev, gf, allfine, fw);
                            if (p < 0) continue;
                            const PatchDev& fd = lev.pd[p];
                            per[p].push_back(RestrictPt{
                                fd.off + local_index(fd, fw[0] - fd.lo[0] + G, fw[1] - fd.lo[1] + G,
                                                     fw[2] - fd.lo[2] + G),
                                qd.off + local_index(qd, i + G, j + G, k + G), fd.fs, qd.fs});
                        }
            }
            for (size_t p = 0; p < lev.pd.size(); ++p) {
                lev.rst_by_patch[p] = (int64_t)rst.size();
                rst.insert(rst.end(), per[p].begin(), per[p].end());
            }
            lev.rst_by_patch[lev.pd.size()] = (int64_t)rst.size();
            if ((rc = lev.rst.upload(rst, &ps->arena))) return rc;
        }
        int td[3];
        int64_t npts = 0;
        for (const PatchDev& pd : lev.pd) npts += (int64_t)pd.n[0] * pd.n[1] * pd.n[2];
        default_tile(ps->sp.system, npts, td);
        build_tiles(lev, td, 0, lev.tiles, &ps->arena);
        int tg[3] = {MOL_ADJ_GTX, MOL_ADJ_GTY, MOL_ADJ_GTZ};
        build_tiles(lev, tg, G, lev.gtiles, &ps->arena);
        if (ps->sp.system == MOL_CCZ4) {
            int tp[3] = {MOL_ADJ_PTX, MOL_ADJ_PTY, MOL_ADJ_PTZ};
            build_tiles(lev, tp, 0, lev.ptiles, &ps->arena);
            int tw[3] = {MOL_ADJ_WTX, MOL_ADJ_WTY, MOL_ADJ_WTZ};
            build_tiles(lev, tw, 0, lev.wtiles, &ps->arena);
        }
        if (ps->sp.system == MOL_CCZ4) {
            std::vector<int64_t> wo(lev.pd.size());
            int64_t w = 0;
            for (size_t p = 0; p < lev.pd.size(); ++p) {
                wo[p] = w;
                w += (int64_t)ccz4_adjoint_slots() * adj_wfs(lev.pd[p].n);
            }
            lev.wsize = w;
            if ((rc = lev.wofs.upload(wo, &ps->arena))) return rc;
        }
        int tn[3] = {32, 4, 2};
        build_tiles(lev, tn, 0, lev.ntiles, &ps->arena);
    }
    // reduction partials: the norms' 5 (8 reserved) or the monitors' per block
    ps->arena.reserve(sizeof(double) * std::max(8, monitor_partials()) * ps->red_blocks,
                      reinterpret_cast<void**>(&ps->scratch));
    int64_t tmax = 0;
    for (int l = 0; l + 1 < ps->nlev; ++l) tmax = std::max(tmax, ps->L[l].nelems);
    if (tmax > 0) ps->arena.reserve(sizeof(double) * tmax, reinterpret_cast<void**>(&ps->tband));
    return ps->arena.commit();
}

int check_level(const mol_patchset* ps, int level)
{
    if (!ps) return fail(MOL_EINVAL, "null patchset");
    if (level < 0 || level >= ps->nlev) return fail(MOL_EINVAL, "level %d out of range", level);
    return MOL_OK;
}

SysParams level_params(const mol_patchset* ps, int level)
{
    SysParams sp = ps->sp;
    sp.h = ps->L[level].h;
    return sp;
}

// BOR weights (App. D, RK4): with theta = r/R and e = 1/R, the fine increments
// in units of the coarse k_j are
//   k1F = e b'(theta), k2F = k1F + e^2 b''/2 + e^3 (b''' - F)/8,
//   k3F = k1F + e^2 b''/2 + e^3 (b''' + F)/8,  F = 4 (delta_j3 - delta_j2),
// and the fine stage states are b(theta) + (0, k1F/2, k2F/2, k3F).
// b_4 = -theta^2/2 + 2 theta^3/3 (the sign for which b(1) = (1,2,2,1)/6).
void bor_weights(int R, int r, int s, double w[4])
{
    const double t = (double)r / R, e = 1.0 / R;
    const double c1[4] = {1.0, 0.0, 0.0, 0.0};
    const double c2[4] = {-1.5, 1.0, 1.0, -0.5};
    const double c3[4] = {2.0 / 3.0, -2.0 / 3.0, -2.0 / 3.0, 2.0 / 3.0};
    for (int j = 0; j < 4; ++j) {
        double b0 = c1[j] * t + c2[j] * t * t + c3[j] * t * t * t;
        double b1 = c1[j] + 2.0 * c2[j] * t + 3.0 * c3[j] * t * t;
        double b2 = 2.0 * c2[j] + 6.0 * c3[j] * t;
        double b3 = 6.0 * c3[j];
        double F = j == 2 ? 4.0 : (j == 1 ? -4.0 : 0.0);
        double k1 = e * b1;
        double k2 = k1 + 0.5 * e * e * b2 + 0.125 * e * e * e * (b3 - F);
        double k3 = k1 + 0.5 * e * e * b2 + 0.125 * e * e * e * (b3 + F);
        w[j] = s == 1 ? b0 : s == 2 ? b0 + 0.5 * k1 : s == 3 ? b0 + 0.5 * k2 : b0 + k3;
    }
}

// Weights w_j of the parent state U^n + sum_j w_j k_j that feeds fine step r,
// stage s, per time-refinement strategy (Sec. III.B): BOR (App. D, above);
// Berger-Oliger with the dense output, b_j(theta) at the stage time
// theta = (r + c_s)/R, c = (0, 1/2, 1/2, 1) (App. C); linear Berger-Oliger,
// theta (1, 2, 2, 1)/6; no sub-cycling (R = 1 in time), the parent's own
// stage states.
void time_weights_rk4(int tmode, int R, int r, int s, double w[4])
{
    static const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    static const double cw[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    static const double c1[4] = {1.0, 0.0, 0.0, 0.0};
    static const double c2[4] = {-1.5, 1.0, 1.0, -0.5};
    static const double c3[4] = {2.0 / 3.0, -2.0 / 3.0, -2.0 / 3.0, 2.0 / 3.0};
    const double th = (r + cs[s - 1]) / R;
    for (int j = 0; j < 4; ++j) {
        switch (tmode) {
        case MOL_TIME_BO: w[j] = c1[j] * th + c2[j] * th * th + c3[j] * th * th * th; break;
        case MOL_TIME_BO1: w[j] = th * cw[j]; break;
        case MOL_TIME_NOSUB: w[j] = (s > 1 && j == s - 2) ? (s == 4 ? 1.0 : 0.5) : 0.0; break;
        default: break;
        }
    }
    if (tmode == MOL_TIME_BOR) bor_weights(R, r, s, w);
}

// The same for SSP-RK3 (App. C dense output b(theta) = (theta - 5/6 theta^2,
// theta^2/6, 4/6 theta^2), stage times c = (0, 1, 1/2), weights (1, 1, 4)/6):
// BOR (App. D) with theta = r/R, fine k_1 = b'/R and k_2 = b'/R + b''/R^2 in
// units of the parent k's, stage states b, b + k_1, b + (k_1 + k_2)/4.
void time_weights_ssp3(int tmode, int R, int r, int s, double w[4])
{
    static const double cs[3] = {0.0, 1.0, 0.5};
    static const double cw[3] = {1.0 / 6.0, 1.0 / 6.0, 4.0 / 6.0};
    w[3] = 0.0;
    if (tmode == MOL_TIME_BOR) {
        const double th = (double)r / R, iR = 1.0 / R;
        const double b[3] = {th - (5.0 / 6.0) * th * th, th * th / 6.0, (4.0 / 6.0) * th * th};
        const double b1[3] = {1.0 - (5.0 / 3.0) * th, th / 3.0, (4.0 / 3.0) * th};
        const double b2[3] = {-5.0 / 3.0, 1.0 / 3.0, 4.0 / 3.0};
        for (int j = 0; j < 3; ++j)
            w[j] = s == 1 ? b[j] : s == 2 ? b[j] + b1[j] * iR : b[j] + 0.5 * b1[j] * iR + 0.25 * b2[j] * iR * iR;
        return;
    }
    const double th = (r + cs[s - 1]) / R;
    for (int j = 0; j < 3; ++j) {
        switch (tmode) {
        case MOL_TIME_BO: w[j] = j == 0 ? th - (5.0 / 6.0) * th * th : j == 1 ? th * th / 6.0 : (4.0 / 6.0) * th * th; break;
        case MOL_TIME_BO1: w[j] = th * cw[j]; break;
        default: w[j] = s == 2 ? (j == 0 ? 1.0 : 0.0) : s == 3 ? (j < 2 ? 0.25 : 0.0) : 0.0; break;
        }
    }
}

// mode bits: MOL_TIME_* (48) and MOL_ADV_SSPRK3
void time_weights(int mode, int R, int r, int s, double w[4])
{
    if (mode & MOL_ADV_SSPRK3)
        time_weights_ssp3(mode & 48, R, r, s, w);
    else
        time_weights_rk4(mode & 48, R, r, s, w);
}

hipStream_t S(void* s) { return (hipStream_t)s; }

// a wave level that is one periodic patch (the whole domain, no finer level,
// at least 4 points per axis): the wave stage kernels read stencil
// neighbours at the periodic images, and the driver skips the ghost fill
bool level_wraps(const mol_patchset* ps, int l)
{
    const auto& lev = ps->L[l];
    return ps->sp.system == MOL_WAVE && l == 0 && ps->nlev == 1 && !ps->open && lev.pd.size() == 1 &&
           lev.pd[0].n[0] >= 4 && lev.pd[0].n[1] >= 4 && lev.pd[0].n[2] >= 4;
}

// a CCZ4 level that is one periodic patch (the whole domain, no finer level,
// at least 2G points per axis): its stage kernel writes the periodic ghost
// images of its output, so the driver fills ghosts only before the first
// stage of a step (the caller's U)
bool level_images(const mol_patchset* ps, int l)
{
    const auto& lev = ps->L[l];
    return ps->sp.system == MOL_CCZ4 && l == 0 && ps->nlev == 1 && !ps->open && lev.pd.size() == 1 &&
           lev.pd[0].n[0] >= 2 * G && lev.pd[0].n[1] >= 2 * G && lev.pd[0].n[2] >= 2 * G;
}

int stage_impl(mol_patchset* ps, int level, int mode, int stage, double dt, const double* Un,
               const double* Us, double* acc, double* out, double* kst, hipStream_t st, int plain,
               bool wrap = false, bool images = false)
{
    Level& lev = ps->L[level];
    SysParams sp = level_params(ps, level);
    StageArgs a{};
    a.patches = lev.d_pd.p;
    a.mode = mode;
    a.stage = stage;
    a.dt = dt;
    a.Un = Un;
    a.Us = Us;
    a.acc = acc;
    a.out = out;
    a.kst = kst;
    a.stream = lev.nelems * (int64_t)sizeof(double) >= (int64_t(128) << 20);
    a.wrap = wrap ? 1 : 0;
    a.images = images ? 1 : 0;
    if (!plain) {
        a.tiles = lev.tiles.dev.p;
        a.ntiles = (int)lev.tiles.dev.n;
        hipError_t e = launch_stage(sp, a, lev.tiles.tdim, st);
        if (e != hipSuccess) return hip_fail(e, "stage launch");
    } else {
        for (size_t p = 0; p < lev.pd.size(); ++p) {
            a.tiles = lev.tiles.dev.p + lev.tiles.by_patch[p];
            a.ntiles = lev.tiles.count[p];
            hipError_t e = launch_stage(sp, a, lev.tiles.tdim, st);
            if (e != hipSuccess) return hip_fail(e, "stage launch");
        }
    }
    if (level == 0 && ps->open) {
        // the outer ghost points evolve in the same stage (they are not filled)
        hipError_t e = launch_radiative(a, lev.pd[0], ps->rad_pts.p, ps->rad_pts.n, ps->sp.nf, ps->rad, ps->xlo,
                                        lev.h, st);
        if (e != hipSuccess) return hip_fail(e, "radiative boundary launch");
    }
    return MOL_OK;
}

int fill_impl(mol_patchset* ps, int level, double* U, int nf, hipStream_t st, int plain)
{
    Level& lev = ps->L[level];
    if (nf <= 0) nf = ps->sp.nf;
    if (!plain) {
        hipError_t e = launch_fill(lev.fill.p, lev.fill.n, nf, U, st);
        return e == hipSuccess ? MOL_OK : hip_fail(e, "fill launch");
    }
    for (size_t p = 0; p < lev.pd.size(); ++p) {
        int64_t b = lev.fill_by_patch[p], n = lev.fill_by_patch[p + 1] - b;
        hipError_t e = launch_fill(lev.fill.p + b, n, nf, U, st);
        if (e != hipSuccess) return hip_fail(e, "fill launch");
    }
    return MOL_OK;
}

int prolong_impl(mol_patchset* ps, int fl, int r, int stage, const double* Unc,
                 const double* const* kc, double* Uf, hipStream_t st, int plain, int tmode = MOL_TIME_BOR)
{
    Level& lev = ps->L[fl];
    double w[4];
    time_weights(tmode, (tmode & 48) == MOL_TIME_NOSUB ? 1 : lev.ratio, r, stage, w);
    const int nf = ps->sp.nf;
    // BOR stage state on the parent band, then Lagrange interpolation from it
    const int nl = plain ? (int)lev.pd.size() : 1;
    for (int p = 0; p < nl; ++p) {
        const int64_t b0 = plain ? lev.band_by_patch[p] : 0;
        const int64_t bn = plain ? lev.band_by_patch[p + 1] - b0 : lev.band.n;
        hipError_t e = launch_bor_band(lev.band.p + b0, bn, nf, w, Unc, kc[0], kc[1], kc[2], kc[3],
                                       ps->tband, st);
        if (e != hipSuccess) return hip_fail(e, "BOR band launch");
    }
    for (int p = 0; p < nl; ++p) {
        const int64_t b0 = plain ? lev.pcell_by_patch[p] : 0;
        const int64_t bn = plain ? lev.pcell_by_patch[p + 1] - b0 : lev.pcell.n;
        hipError_t e = launch_prolong(lev.pcell.p + b0, bn, nf, lev.ratio, lev.lagw.data(), ps->tband, Uf, st);
        if (e != hipSuccess) return hip_fail(e, "prolong launch");
    }
    return MOL_OK;
}

int restrict_impl(mol_patchset* ps, int fl, const double* Uf, double* Uc, hipStream_t st, int plain)
{
    Level& lev = ps->L[fl];
    if (!plain) {
        hipError_t e = launch_restrict(lev.rst.p, lev.rst.n, ps->sp.nf, Uf, Uc, st);
        return e == hipSuccess ? MOL_OK : hip_fail(e, "restrict launch");
    }
    for (size_t p = 0; p < lev.pd.size(); ++p) {
        int64_t b = lev.rst_by_patch[p], n = lev.rst_by_patch[p + 1] - b;
        hipError_t e = launch_restrict(lev.rst.p + b, n, ps->sp.nf, Uf, Uc, st);
        if (e != hipSuccess) return hip_fail(e, "restrict launch");
    }
    return MOL_OK;
}

// Sec. III skeleton with BOR sub-cycling: level l takes one RK4 step of size
// dt; its finer level then takes R steps of dt/R whose coarse-fine ghosts
// come from this step's U^n and k_1..k_4; the fine result is injected.
// tmode: MOL_TIME_* or-ed with MOL_ADV_SSPRK3 for SSP-RK3 steps
// u_filled: the level's U already has its same-level ghosts (a later step
// of a multi-step call: every step leaves U filled)
// last: the last step of the call; on a level whose stages read periodic
// images (wrap) the fill of the new U is needed only for the caller, so the
// earlier steps of a multi-step call skip it
int advance_level(mol_patchset* ps, const mol_level_state* st, int l, int r, double dt,
                  hipStream_t s, int plain, int tmode, bool u_filled = false, bool last = true)
{
    const mol_level_state& X = st[l];
    const bool kids = l + 1 < ps->nlev;
    const int nf = ps->sp.nf;
    const bool ssp = tmode & MOL_ADV_SSPRK3;
    // RK4 (accumulator form) or SSP-RK3 (Shu-Osher form); while the children
    // step, U keeps U^n and the new state waits in S1 (RK4) or S0 (SSP-RK3)
    double* const stage_in[4] = {X.U, X.S0, X.S1, X.S0};
    double* const stage_out[4] = {X.S0, X.S1, ssp ? (kids ? X.S0 : X.U) : X.S0, kids ? X.S1 : X.U};
    double* const next = ssp ? X.S0 : X.S1;
    const int nst = ssp ? 3 : 4;
    // a wave level that is one periodic patch (the whole domain, no finer
    // level, at least 4 points per axis) reads its stencil neighbours at the
    // periodic images: no ghost fill before its stages
    const bool wrap = level_wraps(ps, l);
    // a CCZ4 level that is one periodic patch: every stage writes the ghost
    // images of its output, so only the caller's U is filled (first stage)
    const bool images = level_images(ps, l);
    int rc;
    for (int sidx = 0; sidx < nst; ++sidx) {
        double* Us = stage_in[sidx];
        // U of a later sub-step (r > 0), or of a later step of a multi-step
        // call, was filled at the end of the previous one
        const bool filled = (images && sidx > 0) || (sidx == 0 && (r > 0 || u_filled));
        if (!wrap && !filled && (rc = fill_impl(ps, l, Us, nf, s, plain))) return rc;
        if (l > 0) {
            const mol_level_state& P = st[l - 1];
            const double* kc[4] = {P.k[0], P.k[1], P.k[2], P.k[3]};
            if ((rc = prolong_impl(ps, l, r, sidx + 1, P.U, kc, Us, s, plain, tmode))) return rc;
        }
        if ((rc = stage_impl(ps, l, ssp ? ST_SSP3 : ST_RK4, sidx + 1, dt, X.U, Us, X.acc, stage_out[sidx],
                             kids ? X.k[sidx] : nullptr, s, plain, wrap, images)))
            return rc;
    }
    if (kids) {
        // sub-cycling: R fine steps of dt/R; without it, one step of dt
        const int R = (tmode & 48) == MOL_TIME_NOSUB ? 1 : ps->L[l + 1].ratio;
        for (int rr = 0; rr < R; ++rr)
            if ((rc = advance_level(ps, st, l + 1, rr, dt / R, s, plain, tmode))) return rc;
        if ((rc = restrict_impl(ps, l + 1, st[l + 1].U, next, s, plain))) return rc;
        hipError_t e = hipMemcpyAsync(X.U, next, sizeof(double) * ps->L[l].nelems,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return (images || (wrap && !last)) ? MOL_OK : fill_impl(ps, l, X.U, nf, s, plain);
}

int check_states(const mol_patchset* ps, const mol_level_state* st)
{
    if (!st) return fail(MOL_EINVAL, "null level states");
    for (int l = 0; l < ps->nlev; ++l) {
        const mol_level_state& X = st[l];
        if (!X.U || !X.S0 || !X.S1 || !X.acc) return fail(MOL_EINVAL, "level %d: null buffer", l);
        if (X.U == X.S0 || X.U == X.S1 || X.S0 == X.S1)
            return fail(MOL_EINVAL, "level %d: state buffers must be distinct", l);
        if (l + 1 < ps->nlev)
            for (int j = 0; j < 4; ++j)
                if (!X.k[j]) return fail(MOL_EINVAL, "level %d: k buffers required (has a finer level)", l);
    }
    return MOL_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

const char* mol_last_error(void) { return g_err.c_str(); }

namespace {
int create_impl(const mol_hierarchy_desc* h, const mol_system_desc* s, const mol_patchset* prev, mol_patchset** out)
{
    if (!h || !s || !out) return fail(MOL_EINVAL, "null argument");
    *out = nullptr;
    if (h->nlevels < 1 || h->nlevels > MOL_MAX_LEVELS)
        return fail(MOL_EINVAL, "nlevels %d not in [1, %d]", h->nlevels, MOL_MAX_LEVELS);
    if (!h->npatch || !h->boxes || (h->nlevels > 1 && !h->ratio))
        return fail(MOL_EINVAL, "null hierarchy arrays");
    if (!(h->dx0 > 0.0)) return fail(MOL_EINVAL, "dx0 must be positive");
    for (int d = 0; d < 3; ++d)
        if (h->N0[d] < 1) return fail(MOL_EINVAL, "N0[%d] must be >= 1", d);
    if (s->system != MOL_WAVE && s->system != MOL_MHD && s->system != MOL_CCZ4 && s->system != MOL_MHD_GLM)
        return fail(MOL_EINVAL, "unknown system %d", s->system);
    const bool mhd = s->system == MOL_MHD || s->system == MOL_MHD_GLM;
    mol_patchset* ps = new (std::nothrow) mol_patchset();
    if (!ps) return fail(MOL_ENOMEM, "host allocation failed");
    ps->sp.system = s->system;
    ps->sp.nf = s->system == MOL_WAVE ? 2 : s->system == MOL_MHD ? 8 : s->system == MOL_MHD_GLM ? 9 : 25;
    ps->sp.upwind = s->upwind;
    ps->sp.sigma = s->sigma;
    ps->sp.gamma_ad = s->gamma_ad;
    ps->sp.weno_eps = s->weno_eps;
    ps->sp.weno_q = s->weno_q;
    ps->sp.kappa_z = s->kappa_z;
    ps->sp.kappa_c = s->kappa_c;
    ps->sp.bm_f0 = s->bm_f0;
    ps->sp.bm_f1 = s->bm_f1;
    ps->sp.gd_g = s->gd_g;
    ps->sp.gd_eta = s->gd_eta;
    ps->sp.mhd_recon = s->mhd_recon;
    ps->sp.mhd_flux = s->mhd_flux;
    ps->sp.mhd_ch = s->mhd_ch;
    ps->sp.mhd_kpsi = s->mhd_kpsi;
    if (s->system == MOL_MHD_GLM && !(s->mhd_ch >= 0.0 && s->mhd_kpsi >= 0.0)) {
        delete ps;
        return fail(MOL_EINVAL, "c_h and kappa_psi must be non-negative");
    }
    if (mhd && !(s->gamma_ad > 1.0)) {
        delete ps;
        return fail(MOL_EINVAL, "gamma_ad must exceed 1");
    }
    if (mhd && (s->mhd_recon < MOL_RECON_WENO5Z || s->mhd_recon > MOL_RECON_WENO3 ||
                                 (s->mhd_flux != MOL_FLUX_LLF && s->mhd_flux != MOL_FLUX_HLL &&
                                  s->mhd_flux != MOL_FLUX_SPLIT))) {
        delete ps;
        return fail(MOL_EINVAL, "unknown MHD reconstruction %d or flux %d", s->mhd_recon, s->mhd_flux);
    }
    ps->nlev = h->nlevels;
    ps->open = h->open ? 1 : 0;
    for (int f = 0; f < 32; ++f) {
        ps->rad.v[f] = 1.0;
        ps->rad.uinf[f] = 0.0;
    }
    for (int d = 0; d < 3; ++d) {
        ps->N0[d] = h->N0[d];
        ps->xlo[d] = h->xlo[d];
    }
    ps->dx0 = h->dx0;
    int rc = build(ps, h, prev);
    if (rc) {
        delete ps;
        return rc;
    }
    *out = ps;
    return MOL_OK;
}
}  // namespace

int mol_create_patchset(const mol_hierarchy_desc* h, const mol_system_desc* s, mol_patchset** out)
{
    return create_impl(h, s, nullptr, out);
}

int mol_create_patchset_from(const mol_hierarchy_desc* h, const mol_system_desc* s, const mol_patchset* prev,
                             mol_patchset** out)
{
    if (!prev) return fail(MOL_EINVAL, "null previous patchset");
    return create_impl(h, s, prev, out);
}

void mol_destroy_patchset(mol_patchset* ps)
{
    if (!ps) return;
    (void)hipDeviceSynchronize();  // device work may still read the schedules
    delete ps;
}

int mol_nfields(const mol_patchset* ps) { return ps ? ps->sp.nf : fail(MOL_EINVAL, "null patchset"); }

int mol_level_npatch(const mol_patchset* ps, int level)
{
    int rc = check_level(ps, level);
    return rc ? rc : (int)ps->L[level].pd.size();
}

int mol_level_layout(const mol_patchset* ps, int level, int64_t* nelems, int64_t* offs,
                     int32_t* dims, int64_t* fstrides, int32_t* row_pitch)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    const Level& lev = ps->L[level];
    if (nelems) *nelems = lev.nelems;
    for (size_t p = 0; p < lev.pd.size(); ++p) {
        if (offs) offs[p] = lev.pd[p].off;
        if (dims)
            for (int d = 0; d < 3; ++d) dims[3 * p + d] = lev.pd[p].n[d];
        if (fstrides) fstrides[p] = lev.pd[p].fs;
        if (row_pitch) row_pitch[p] = lev.pd[p].pitch_y;
    }
    return MOL_OK;
}

int mol_fill_ghosts(mol_patchset* ps, int level, double* U, int nf, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!U) return fail(MOL_EINVAL, "null buffer");
    if (nf > ps->sp.nf) return fail(MOL_EINVAL, "nf %d exceeds the system's %d fields", nf, ps->sp.nf);
    return fill_impl(ps, level, U, nf, S(stream), 0);
}

int mol_rhs(mol_patchset* ps, int level, const double* U, double* dUdt, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!U || !dUdt) return fail(MOL_EINVAL, "null buffer");
    if (U == dUdt) return fail(MOL_EINVAL, "U and dUdt must not alias");
    return stage_impl(ps, level, ST_RHS, 0, 1.0, U, U, nullptr, dUdt, nullptr, S(stream), 0);
}

int mol_rk_stage(mol_patchset* ps, int level, int scheme, int stage, double dt, const double* Un,
                 const double* Us, double* Acc, double* Uout, double* k_store, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!Un || !Us || !Uout) return fail(MOL_EINVAL, "null buffer");
    if (!std::isfinite(dt) || dt <= 0.0) return fail(MOL_EINVAL, "dt must be positive and finite");
    if ((const double*)Uout == Us) return fail(MOL_EINVAL, "Uout must not alias Us");
    if (scheme == MOL_RK4) {
        if (stage < 1 || stage > 4) return fail(MOL_EINVAL, "RK4 stage %d not in 1..4", stage);
        if (!Acc) return fail(MOL_EINVAL, "RK4 needs the accumulator");
        if ((const double*)Uout == Un && stage != 4)
            return fail(MOL_EINVAL, "Uout may alias Un only at the last stage");
        return stage_impl(ps, level, ST_RK4, stage, dt, Un, Us, Acc, Uout, k_store, S(stream), 0, false,
                          level_images(ps, level));
    }
    if (scheme == MOL_SSPRK3) {
        if (stage < 1 || stage > 3) return fail(MOL_EINVAL, "SSP-RK3 stage %d not in 1..3", stage);
        if ((const double*)Uout == Un && stage != 3)
            return fail(MOL_EINVAL, "Uout may alias Un only at the last stage");
        return stage_impl(ps, level, ST_SSP3, stage, dt, Un, Us, Acc, Uout, k_store, S(stream), 0, false,
                          level_images(ps, level));
    }
    return fail(MOL_EINVAL, "unknown scheme %d", scheme);
}

int mol_bor_weights(int R, int r, int stage, double w[4])
{
    if (R < 1 || r < 0 || r >= R || stage < 1 || stage > 4 || !w)
        return fail(MOL_EINVAL, "bad BOR arguments");
    bor_weights(R, r, stage, w);
    return MOL_OK;
}

int mol_time_weights(int tmode, int R, int r, int stage, double w[4])
{
    if (tmode & ~(48 | MOL_ADV_SSPRK3)) return fail(MOL_EINVAL, "unknown time-refinement strategy %d", tmode);
    const int nst = (tmode & MOL_ADV_SSPRK3) ? 3 : 4;
    if (R < 1 || r < 0 || r >= R || stage < 1 || stage > nst || !w || ((tmode & 48) == MOL_TIME_NOSUB && R != 1))
        return fail(MOL_EINVAL, "bad time-weight arguments");
    time_weights(tmode, R, r, stage, w);
    return MOL_OK;
}

int mol_set_radiative(mol_patchset* ps, const double* v, const double* uinf)
{
    if (!ps || !v || !uinf) return fail(MOL_EINVAL, "null argument");
    if (!ps->open) return fail(MOL_EUNSUPPORTED, "the patchset has a periodic domain");
    for (int f = 0; f < ps->sp.nf; ++f) {
        if (!std::isfinite(v[f]) || !(v[f] >= 0.0) || !std::isfinite(uinf[f]))
            return fail(MOL_EINVAL, "field %d: radiative speed must be finite and >= 0", f);
        ps->rad.v[f] = v[f];
        ps->rad.uinf[f] = uinf[f];
    }
    return MOL_OK;
}

int mol_prolong(mol_patchset* ps, int fine_level, int r, int stage, const double* Un_c,
                const double* const* k_c, double* U_f, void* stream)
{
    int rc = check_level(ps, fine_level);
    if (rc) return rc;
    if (fine_level < 1) return fail(MOL_EINVAL, "level 0 has no parent");
    const int R = ps->L[fine_level].ratio;
    if (r < 0 || r >= R) return fail(MOL_EINVAL, "fine step %d not in [0, %d)", r, R);
    if (stage < 1 || stage > 4) return fail(MOL_EINVAL, "stage %d not in 1..4", stage);
    if (!Un_c || !k_c || !U_f) return fail(MOL_EINVAL, "null buffer");
    for (int j = 0; j < 4; ++j)
        if (!k_c[j]) return fail(MOL_EINVAL, "null k buffer");
    return prolong_impl(ps, fine_level, r, stage, Un_c, k_c, U_f, S(stream), 0);
}

int mol_restrict(mol_patchset* ps, int fine_level, const double* U_f, double* U_c, void* stream)
{
    int rc = check_level(ps, fine_level);
    if (rc) return rc;
    if (fine_level < 1) return fail(MOL_EINVAL, "level 0 has no parent");
    if (!U_f || !U_c) return fail(MOL_EINVAL, "null buffer");
    return restrict_impl(ps, fine_level, U_f, U_c, S(stream), 0);
}

int mol_rhs_adjoint(mol_patchset* ps, int level, const double* U, const double* lam, double* lamU,
                    double* work, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (ps->open) return fail(MOL_EUNSUPPORTED, "the adjoint needs a periodic domain");
    if (ps->sp.system != MOL_WAVE && ps->sp.system != MOL_CCZ4)
        return fail(MOL_EUNSUPPORTED, "the right-hand-side adjoint exists for the wave and CCZ4 systems");
    if (!lam || !lamU) return fail(MOL_EINVAL, "null buffer");
    if (lam == lamU) return fail(MOL_EINVAL, "lam and lamU must not alias");
    Level& lev = ps->L[level];
    SysParams sp = level_params(ps, level);
    hipError_t e;
    if (ps->sp.system == MOL_WAVE) {
        // the wave operator is linear: its transpose does not depend on U
        e = launch_wave_adjoint(sp, lev.d_pd.p, lev.gtiles.dev.p, (int)lev.gtiles.dev.n, lev.gtiles.tdim, lam, lamU,
                                S(stream));
    } else {
        if (!U || !work) return fail(MOL_EINVAL, "the CCZ4 adjoint needs U and the workspace");
        if (U == lamU || work == lamU || work == U || work == lam)
            return fail(MOL_EINVAL, "U, lamU and work must not alias");
        e = launch_ccz4_adjoint(sp, lev.d_pd.p, lev.ptiles.dev.p, (int)lev.ptiles.dev.n, lev.ptiles.tdim,
                                lev.gtiles.dev.p, (int)lev.gtiles.dev.n, lev.gtiles.tdim, U, lam, work, lev.wofs.p,
                                lamU, S(stream));
    }
    return e == hipSuccess ? MOL_OK : hip_fail(e, "adjoint launch");
}

// Workspace of mol_rhs_adjoint_noalloc: one file-scope device array per GPU.
// In host code `scratch` is a host-side stand-in, not a device address; the
// device address of the current device's copy comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch_dev.
static __device__ __align__(256) double scratch[MOL_ADJOINT_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::array<double*, kMaxDevices> g_scratch_dev{};

int scratch_address(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MOL_EUNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(MOL_EHIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return MOL_OK;
}
}  // namespace

int mol_rhs_adjoint_noalloc(mol_patchset* ps, int level, const double* U, const double* lam, double* lamU,
                            void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    const int64_t need = ps->L[level].wsize;
    const int64_t have = MOL_ADJOINT_SCRATCH_BYTES / (int64_t)sizeof(double);
    if (need > have)
        return fail(MOL_EINVAL,
                    "level %d needs %lld doubles of adjoint workspace (%.1f MiB); the static scratch holds %lld "
                    "(%lld MiB): use mol_rhs_adjoint with a workspace",
                    level, (long long)need, need * 8.0 / (1 << 20), (long long)have,
                    (long long)(MOL_ADJOINT_SCRATCH_BYTES >> 20));
    double* w = nullptr;
    if (need > 0 && (rc = scratch_address(&w))) return rc;
    return mol_rhs_adjoint(ps, level, U, lam, lamU, w, stream);
}

int64_t mol_adjoint_workspace(const mol_patchset* ps, int level)
{
    if (!ps) return fail(MOL_EINVAL, "null patchset");
    if (level < 0 || level >= ps->nlev) return fail(MOL_EINVAL, "level %d out of range", level);
    return ps->L[level].wsize;
}

int mol_fill_ghosts_adjoint(mol_patchset* ps, int level, double* lamU, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (ps->open) return fail(MOL_EUNSUPPORTED, "the adjoint needs a periodic domain");
    if (!lamU) return fail(MOL_EINVAL, "null buffer");
    Level& lev = ps->L[level];
    hipError_t e = launch_fill_adjoint(lev.fill_src.p, lev.fill_src.n, lev.fill_img.p, ps->sp.nf,
                                       lamU, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "fill adjoint launch");
}

namespace {
// Reverse of U' = U + sum_s c_s k_s, k_s = dt L(U_s), U_s = U + b_s k_{s-1}:
//   lk_s = c_s lam + b_{s+1} m_{s+1};  m_s = fill^T(L'(U_s)^T (dt lk_s));
//   lam  <- lam + m_1 + m_2 + m_3 + m_4.
// Ust: the stage states U_1 = U^n .. U_4 (ghosts filled; unused by the
// wave).  w0 = dt lk; w1 and w2 hold the current m and the running sum of the
// m's (the buffer that receives m_4 becomes the sum).
int rk4_adjoint_core(mol_patchset* ps, int level, double dt, const double* const Ust[4], double* lam, double* w0,
                     double* w1, double* w2, double* work, void* stream)
{
    const int64_t n = ps->L[level].nelems;
    hipStream_t s = S(stream);
    static const double cw[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    static const double bsub[4] = {0.0, 0.5, 0.5, 1.0};
    hipError_t e = hipSuccess;
    int rc;
    double* wk = w0;
    double* wm = w1;
    double* wsum = w2;
    const Level& lev = ps->L[level];
    if (ps->sp.system == MOL_CCZ4 && lev.pd.size() == 1 && lev.pd[0].n[0] >= 7 && lev.pd[0].n[1] >= 7 &&
        lev.pd[0].n[2] >= 7) {
        // one periodic patch: each stage's gather takes its stencil points at
        // their periodic images (no ghost entries, no fill transpose) and
        // forms wsum and the next stage's input (or the new lam) itself
        const SysParams sp = level_params(ps, level);
        double* win = w0;
        double* wnext = w1;
        e = launch_axpby(n, dt * cw[3], lam, 0.0, lam, win, s);
        if (e != hipSuccess) return hip_fail(e, "axpby");
        for (int st = 3; st >= 0; --st) {
            const double a = st > 0 ? dt * cw[st - 1] : 0.0, b = st > 0 ? dt * bsub[st] : 0.0;
            e = launch_ccz4_adjoint_stage(sp, lev.d_pd.p, lev.ptiles.dev.p, (int)lev.ptiles.dev.n, lev.ptiles.tdim,
                                          lev.wtiles.dev.p, (int)lev.wtiles.dev.n, lev.wtiles.tdim, Ust[st], win,
                                          work, lev.wofs.p, lam, lam, w2, st > 0 ? wnext : nullptr, a, b, st == 3,
                                          st == 0, s);
            if (e != hipSuccess) return hip_fail(e, "adjoint stage launch");
            std::swap(win, wnext);
        }
        return MOL_OK;
    }
    const double* prev = nullptr;  // m_{s+1}
    for (int st = 3; st >= 0; --st) {
        if (st == 3)
            e = launch_axpby(n, dt * cw[3], lam, 0.0, lam, wk, s);
        else
            e = launch_axpby(n, dt * cw[st], lam, dt * bsub[st + 1], prev, wk, s);
        if (e != hipSuccess) return hip_fail(e, "axpby");
        if ((rc = mol_rhs_adjoint(ps, level, Ust[st], wk, wm, work, stream))) return rc;
        if ((rc = mol_fill_ghosts_adjoint(ps, level, wm, stream))) return rc;
        if (st == 3) {
            std::swap(wm, wsum);
            prev = wsum;
        } else {
            e = launch_axpby(n, 1.0, wsum, 1.0, wm, wsum, s);
            if (e != hipSuccess) return hip_fail(e, "axpby");
            prev = wm;
        }
    }
    e = launch_axpby(n, 1.0, lam, 1.0, wsum, lam, s);
    return e == hipSuccess ? MOL_OK : hip_fail(e, "axpby");
}

int rk4_adjoint_check(mol_patchset* ps, int level, double dt)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (ps->open) return fail(MOL_EUNSUPPORTED, "the adjoint needs a periodic domain");
    if (ps->sp.system != MOL_WAVE && ps->sp.system != MOL_CCZ4)
        return fail(MOL_EUNSUPPORTED, "the RK4 adjoint exists for the wave and CCZ4 systems");
    if (ps->nlev != 1) return fail(MOL_EUNSUPPORTED, "the RK4 adjoint handles one periodic level");
    if (!std::isfinite(dt) || dt <= 0.0) return fail(MOL_EINVAL, "dt must be positive and finite");
    return MOL_OK;
}
}  // namespace

int mol_rk4_adjoint_step(mol_patchset* ps, int level, double dt, const double* Un, double* lam,
                         double* const w[6], double* work, void* stream)
{
    int rc = rk4_adjoint_check(ps, level, dt);
    if (rc) return rc;
    const bool nl = ps->sp.system == MOL_CCZ4;
    if (!lam || !w || !w[0] || !w[1] || !w[2]) return fail(MOL_EINVAL, "null buffer");
    if (nl && (!Un || !w[3] || !w[4] || !w[5] || !work))
        return fail(MOL_EINVAL, "the CCZ4 RK4 adjoint needs U^n, six work buffers and the workspace");
    hipStream_t s = S(stream);
    // for a nonlinear system w3..w5 hold the stage states U_2..U_4,
    // recomputed from U^n with the forward stage kernel (w2 serves as its
    // accumulator)
    const double* Ust[4] = {Un, nullptr, nullptr, nullptr};
    if (nl) {
        const double* in[3] = {Un, w[3], w[4]};
        for (int st = 0; st < 3; ++st) {
            if ((rc = stage_impl(ps, level, ST_RK4, st + 1, dt, Un, in[st], w[2], w[3 + st], nullptr, s, 0))) return rc;
            if ((rc = fill_impl(ps, level, w[3 + st], ps->sp.nf, s, 0))) return rc;
            Ust[st + 1] = w[3 + st];
        }
    }
    return rk4_adjoint_core(ps, level, dt, Ust, lam, w[0], w[1], w[2], work, stream);
}

int mol_rk4_adjoint_step_stages(mol_patchset* ps, int level, double dt, const double* const Ust[4], double* lam,
                                double* const w[3], double* work, void* stream)
{
    int rc = rk4_adjoint_check(ps, level, dt);
    if (rc) return rc;
    const bool nl = ps->sp.system == MOL_CCZ4;
    if (!lam || !w || !w[0] || !w[1] || !w[2]) return fail(MOL_EINVAL, "null buffer");
    if (nl && (!Ust || !Ust[0] || !Ust[1] || !Ust[2] || !Ust[3] || !work))
        return fail(MOL_EINVAL, "the CCZ4 RK4 adjoint needs the four stage states and the workspace");
    const double* none[4] = {nullptr, nullptr, nullptr, nullptr};
    const double* const* st = Ust ? Ust : none;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 3; ++j)
            if (st[i] && (st[i] == lam || st[i] == w[j] || st[i] == work))
                return fail(MOL_EINVAL, "a stage state aliases lam, a work buffer or the workspace");
    const double* U4[4] = {st[0], st[1], st[2], st[3]};
    return rk4_adjoint_core(ps, level, dt, U4, lam, w[0], w[1], w[2], work, stream);
}

namespace {
int norms_impl(mol_patchset* ps, int level, const double* U, int field, double shift, double radius,
               const CoordBox& box, double* out_dev, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!U || !out_dev) return fail(MOL_EINVAL, "null buffer");
    if (field < 0 || field >= ps->sp.nf) return fail(MOL_EINVAL, "field %d out of range", field);
    Level& lev = ps->L[level];
    hipError_t e = launch_norms(lev.d_pd.p, lev.ntiles.dev.p, (int)lev.ntiles.dev.n, lev.ntiles.tdim, U,
                                field, shift, radius, lev.h, ps->xlo, box, ps->scratch, ps->red_blocks,
                                out_dev, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "norms launch");
}
}  // namespace

int mol_norms(mol_patchset* ps, int level, const double* U, int field, double shift, double radius,
              double* out_dev, void* stream)
{
    const double inf = std::numeric_limits<double>::infinity();
    const CoordBox all = {{-inf, -inf, -inf}, {inf, inf, inf}};
    return norms_impl(ps, level, U, field, shift, radius, all, out_dev, stream);
}

int mol_box_norms(mol_patchset* ps, int level, const double* U, int field, double shift, const double lo[3],
                  const double hi[3], double* out_dev, void* stream)
{
    if (!lo || !hi) return fail(MOL_EINVAL, "null box");
    CoordBox b;
    for (int d = 0; d < 3; ++d) {
        if (std::isnan(lo[d]) || std::isnan(hi[d])) return fail(MOL_EINVAL, "box bound is NaN");
        b.lo[d] = lo[d];
        b.hi[d] = hi[d];
    }
    const double inf = std::numeric_limits<double>::infinity();
    return norms_impl(ps, level, U, field, shift, inf, b, out_dev, stream);
}

int mol_monitor(mol_patchset* ps, int level, const double* U, uint32_t which, double* pointwise, double* out_dev,
                void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!U || !out_dev) return fail(MOL_EINVAL, "null buffer");
    if (which == 0 || (which & ~MOL_MON_ALL)) return fail(MOL_EINVAL, "monitor mask 0x%x is empty or unknown", which);
    const bool ccz4 = ps->sp.system == MOL_CCZ4;
    if (!ccz4 && (which & ~MOL_MON_KO))
        return fail(MOL_EUNSUPPORTED, "only MOL_MON_KO exists for this system (the others are CCZ4 monitors)");
    if (pointwise && (pointwise == U)) return fail(MOL_EINVAL, "pointwise must not alias U");
    Level& lev = ps->L[level];
    SysParams sp = level_params(ps, level);
    hipError_t e = launch_monitor(lev.d_pd.p, lev.ntiles.dev.p, (int)lev.ntiles.dev.n, lev.ntiles.tdim, ps->sp.nf,
                                  ccz4 ? 1 : 0, which, lev.h, sp.sigma, U, pointwise, ps->scratch, ps->red_blocks,
                                  out_dev, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "monitor launch");
}

int mol_ccz4_puncture(mol_patchset* ps, int level, int nholes, const double* holes, int whole, double* U,
                      void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (ps->sp.system != MOL_CCZ4) return fail(MOL_EUNSUPPORTED, "CCZ4 system only");
    if (!holes || !U) return fail(MOL_EINVAL, "null argument");
    if (nholes < 1 || nholes > MOL_MAX_HOLES) return fail(MOL_EINVAL, "nholes %d not in [1, %d]", nholes, MOL_MAX_HOLES);
    if (whole != 0 && whole != 1) return fail(MOL_EINVAL, "whole must be 0 or 1");
    for (int a = 0; a < nholes; ++a) {
        if (!(holes[10 * a] > 0.0)) return fail(MOL_EINVAL, "hole %d: mass must be positive", a);
        for (int q = 0; q < 10; ++q)
            if (!std::isfinite(holes[10 * a + q])) return fail(MOL_EINVAL, "hole %d: non-finite parameter", a);
    }
    Level& lev = ps->L[level];
    const TileList& tl = whole ? lev.gtiles : lev.ntiles;
    hipError_t e = launch_puncture(lev.d_pd.p, tl.dev.p, (int)tl.dev.n, tl.tdim, nholes, holes, lev.h, ps->xlo, whole,
                                   U, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "puncture launch");
}

int mol_sphere_adjoint(mol_patchset* ps, int level, int field, double radius, double scale, double* lam,
                       void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!lam) return fail(MOL_EINVAL, "null buffer");
    if (field < 0 || field >= ps->sp.nf) return fail(MOL_EINVAL, "field %d out of range", field);
    Level& lev = ps->L[level];
    hipError_t e = launch_sphere_adjoint(lev.d_pd.p, lev.ntiles.dev.p, (int)lev.ntiles.dev.n, lev.ntiles.tdim,
                                         ps->sp.nf, field, radius, scale, lev.h, ps->xlo, lam, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "sphere adjoint launch");
}

namespace {
// Gaussian initial data of the system: the wave's phi (Pi = 0), or the CCZ4
// lapse pulse on flat data (chi = 1, gt = identity, alpha = 1 + pulse, the
// rest 0); U written when lam is null, else the VJP into grad_dev
int gaussian_impl(mol_patchset* ps, int level, int system, const double prm[5], double* U, const double* lam,
                  double* grad_dev, void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (ps->sp.system != system)
        return fail(MOL_EUNSUPPORTED, system == MOL_WAVE ? "wave system only" : "CCZ4 system only");
    if (!prm || (!U && !lam) || (lam && !grad_dev)) return fail(MOL_EINVAL, "null argument");
    if (!(prm[1] > 0.0)) return fail(MOL_EINVAL, "width must be positive");
    Level& lev = ps->L[level];
    double per[3];
    for (int d = 0; d < 3; ++d) per[d] = lev.period[d] * lev.h;
    const int fg = system == MOL_WAVE ? 0 : 18;  // phi, or alpha
    const unsigned ones = system == MOL_WAVE ? 0u : (1u << 0 | 1u << 1 | 1u << 4 | 1u << 6 | 1u << 18);
    hipError_t e = launch_gaussian(lev.d_pd.p, lev.ntiles.dev.p, (int)lev.ntiles.dev.n, lev.ntiles.tdim, prm, lev.h,
                                   ps->xlo, per, ps->sp.nf, fg, ones, U, lam, lam ? ps->scratch : nullptr,
                                   lam ? ps->red_blocks : 0, grad_dev, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "gaussian launch");
}
}  // namespace

int mol_wave_gaussian(mol_patchset* ps, int level, const double prm[5], double* U, void* stream)
{
    if (!U) return fail(MOL_EINVAL, "null argument");
    return gaussian_impl(ps, level, MOL_WAVE, prm, U, nullptr, nullptr, stream);
}

int mol_wave_gaussian_vjp(mol_patchset* ps, int level, const double prm[5], const double* lam,
                          double* grad_dev, void* stream)
{
    if (!lam) return fail(MOL_EINVAL, "null argument");
    return gaussian_impl(ps, level, MOL_WAVE, prm, nullptr, lam, grad_dev, stream);
}

int mol_ccz4_lapse_pulse(mol_patchset* ps, int level, const double prm[5], double* U, void* stream)
{
    if (!U) return fail(MOL_EINVAL, "null argument");
    return gaussian_impl(ps, level, MOL_CCZ4, prm, U, nullptr, nullptr, stream);
}

int mol_ccz4_lapse_pulse_vjp(mol_patchset* ps, int level, const double prm[5], const double* lam,
                             double* grad_dev, void* stream)
{
    if (!lam) return fail(MOL_EINVAL, "null argument");
    return gaussian_impl(ps, level, MOL_CCZ4, prm, nullptr, lam, grad_dev, stream);
}

int mol_advance(mol_patchset* ps, const mol_level_state* states, double dt0, int mode, void* stream)
{
    return mol_advance_steps(ps, states, dt0, 1, mode, stream);
}

int mol_advance_steps(mol_patchset* ps, const mol_level_state* states, double dt0, int nsteps, int mode,
                      void* stream)
{
    if (!ps) return fail(MOL_EINVAL, "null patchset");
    if (nsteps < 1) return fail(MOL_EINVAL, "nsteps must be at least 1");
    if (ps->sp.system != MOL_WAVE && ps->sp.system != MOL_CCZ4 && ps->sp.system != MOL_MHD &&
        ps->sp.system != MOL_MHD_GLM)
        return fail(MOL_EINVAL, "unknown system");
    if (!std::isfinite(dt0) || dt0 <= 0.0) return fail(MOL_EINVAL, "dt must be positive and finite");
    const int launch = mode & 15, tmode = mode & ~15;
    if ((launch != MOL_BATCHED && launch != MOL_PLAIN) || (tmode & ~(48 | MOL_ADV_SSPRK3)))
        return fail(MOL_EINVAL, "unknown mode %d", mode);
    int rc = check_states(ps, states);
    if (rc) return rc;
    for (int k = 0; k < nsteps; ++k)
        if ((rc = advance_level(ps, states, 0, 0, dt0, S(stream), launch == MOL_PLAIN, tmode, k > 0, k + 1 == nsteps)))
            return rc;
    return MOL_OK;
}

int mol_tag(mol_patchset* ps, int level, const double* U, int field, double threshold, uint8_t* flags_dev,
            void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!U || !flags_dev) return fail(MOL_EINVAL, "null buffer");
    if (field < 0 || field >= ps->sp.nf) return fail(MOL_EINVAL, "field %d out of range", field);
    Level& lev = ps->L[level];
    hipError_t e = launch_tag(lev.d_pd.p, lev.ntiles.dev.p, (int)lev.ntiles.dev.n, lev.ntiles.tdim, U, field,
                              threshold, lev.period, flags_dev, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "tag launch");
}

int mol_cluster(const uint8_t* flags, const int dims[3], int buffer, int max_boxes, int* boxes_out, int* nboxes)
{
    if (!flags || !dims || !nboxes || (max_boxes > 0 && !boxes_out)) return fail(MOL_EINVAL, "null argument");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || buffer < 0) return fail(MOL_EINVAL, "bad dimensions");
    const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
    auto at = [&](int i, int j, int k) { return ((int64_t)k * dims[1] + j) * dims[0] + i; };
    // dilation by `buffer` along each axis in turn (periodic)
    std::vector<uint8_t> a(flags, flags + n), b(n);
    for (int d = 0; d < 3; ++d) {
        std::fill(b.begin(), b.end(), 0);
        for (int k = 0; k < dims[2]; ++k)
            for (int j = 0; j < dims[1]; ++j)
                for (int i = 0; i < dims[0]; ++i) {
                    if (!a[at(i, j, k)]) continue;
                    const int reach = std::min(buffer, dims[d] - 1);
                    for (int o = -reach; o <= reach; ++o) {
                        int c[3] = {i, j, k};
                        c[d] = wrapi(c[d] + o, dims[d]);
                        b[at(c[0], c[1], c[2])] = 1;
                    }
                }
        a.swap(b);
    }
    // face-connected components (no wrap), bounding boxes
    std::vector<int> comp(n, -1);
    std::vector<std::array<int, 6>> bb;
    std::vector<int64_t> stack;
    for (int64_t s0 = 0; s0 < n; ++s0) {
        if (!a[s0] || comp[s0] >= 0) continue;
        const int id = (int)bb.size();
        std::array<int, 6> box = {dims[0], dims[1], dims[2], -1, -1, -1};
        comp[s0] = id;
        stack.assign(1, s0);
        while (!stack.empty()) {
            const int64_t q = stack.back();
            stack.pop_back();
            const int c[3] = {(int)(q % dims[0]), (int)((q / dims[0]) % dims[1]), (int)(q / ((int64_t)dims[0] * dims[1]))};
            for (int d = 0; d < 3; ++d) {
                box[d] = std::min(box[d], c[d]);
                box[3 + d] = std::max(box[3 + d], c[d]);
            }
            for (int d = 0; d < 3; ++d)
                for (int o = -1; o <= 1; o += 2) {
                    int e[3] = {c[0], c[1], c[2]};
                    e[d] += o;
                    if (e[d] < 0 || e[d] >= dims[d]) continue;
                    const int64_t r = at(e[0], e[1], e[2]);
                    if (a[r] && comp[r] < 0) {
                        comp[r] = id;
                        stack.push_back(r);
                    }
                }
        }
        bb.push_back(box);
    }
    // merge overlapping boxes until none overlap
    for (bool merged = true; merged;) {
        merged = false;
        for (size_t i = 0; i < bb.size() && !merged; ++i)
            for (size_t j = i + 1; j < bb.size() && !merged; ++j) {
                bool ov = true;
                for (int d = 0; d < 3; ++d)
                    if (bb[i][3 + d] < bb[j][d] || bb[j][3 + d] < bb[i][d]) ov = false;
                if (ov) {
                    for (int d = 0; d < 3; ++d) {
                        bb[i][d] = std::min(bb[i][d], bb[j][d]);
                        bb[i][3 + d] = std::max(bb[i][3 + d], bb[j][3 + d]);
                    }
                    bb.erase(bb.begin() + (std::ptrdiff_t)j);
                    merged = true;
                }
            }
    }
    *nboxes = (int)bb.size();
    if ((int)bb.size() > max_boxes) return fail(MOL_EINVAL, "%zu boxes needed, room for %d", bb.size(), max_boxes);
    // deterministic order: by lower corner (z, y, x)
    std::sort(bb.begin(), bb.end(), [](const std::array<int, 6>& x, const std::array<int, 6>& y) {
        return std::make_tuple(x[2], x[1], x[0]) < std::make_tuple(y[2], y[1], y[0]);
    });
    for (size_t i = 0; i < bb.size(); ++i)
        for (int q = 0; q < 6; ++q) boxes_out[6 * i + q] = bb[i][q];
    return MOL_OK;
}

int mol_regrid_create(mol_patchset* pn, const mol_patchset* po, mol_regrid** out)
{
    if (!pn || !po || !out) return fail(MOL_EINVAL, "null argument");
    *out = nullptr;
    if (pn->sp.system != po->sp.system || pn->nlev != po->nlev || pn->open != po->open)
        return fail(MOL_EINVAL, "the patchsets differ in system, level count or boundary");
    for (int l = 0; l < pn->nlev; ++l)
        if (pn->L[l].ratio != po->L[l].ratio) return fail(MOL_EINVAL, "level %d: ratios differ", l);
    const Level& n0 = pn->L[0];
    const Level& o0 = po->L[0];
    if (n0.boxes.size() != o0.boxes.size() || n0.nelems != o0.nelems)
        return fail(MOL_EINVAL, "level 0 differs");
    for (size_t q = 0; q < n0.boxes.size(); ++q)
        for (int d = 0; d < 3; ++d)
            if (n0.boxes[q].lo[d] != o0.boxes[q].lo[d] || n0.boxes[q].hi[d] != o0.boxes[q].hi[d])
                return fail(MOL_EINVAL, "level 0 boxes differ");
    mol_regrid* r = new (std::nothrow) mol_regrid();
    if (!r) return fail(MOL_ENOMEM, "host allocation failed");
    r->pn = pn;
    r->po = po;
    for (int l = 1; l < pn->nlev; ++l) {
        const Level& lev = pn->L[l];
        const Level& old = po->L[l];
        const Level& par = pn->L[l - 1];
        const int R = lev.ratio;
        std::vector<int> allold, allpar;
        for (size_t q = 0; q < old.boxes.size(); ++q) allold.push_back((int)q);
        for (size_t q = 0; q < par.boxes.size(); ++q) allpar.push_back((int)q);
        std::vector<GhostCopy> copy;
        std::vector<ProlongCell> cells;
        for (size_t p = 0; p < lev.pd.size(); ++p) {
            const PatchDev& pd = lev.pd[p];
            struct CellTmp {
                int key[3], q0, cw[3];
                uint64_t mask;
                int frac;
            };
            std::vector<CellTmp> ct;
            std::map<std::array<int, 3>, size_t> cidx;
            for (int k = 0; k < pd.n[2]; ++k)
                for (int j = 0; j < pd.n[1]; ++j)
                    for (int i = 0; i < pd.n[0]; ++i) {
                        int g[3] = {pd.lo[0] + i, pd.lo[1] + j, pd.lo[2] + k}, gw[3];
                        const int64_t dst = pd.off + local_index(pd, i + G, j + G, k + G);
                        const int q = find_owner(old, g, allold, gw);
                        if (q >= 0) {
                            const PatchDev& qd = old.pd[q];
                            const int64_t src = qd.off + local_index(qd, gw[0] - qd.lo[0] + G, gw[1] - qd.lo[1] + G,
                                                                     gw[2] - qd.lo[2] + G);
                            copy.push_back(GhostCopy{dst, src, pd.fs, qd.fs});
                            continue;
                        }
                        int i0[3], m[3], cw[3];
                        for (int d = 0; d < 3; ++d) {
                            gw[d] = wrapi(g[d], lev.period[d]);
                            m[d] = gw[d] % R;
                            i0[d] = gw[d] / R;
                        }
                        const int q0 = find_owner(par, i0, allpar, cw);
                        if (q0 < 0) {
                            delete r;
                            return fail(MOL_EINVAL, "level %d: new point outside the new parent level", l);
                        }
                        for (int c = (m[2] ? -2 : 0); c <= (m[2] ? 3 : 0); ++c)
                            for (int b = (m[1] ? -2 : 0); b <= (m[1] ? 3 : 0); ++b)
                                for (int a = (m[0] ? -2 : 0); a <= (m[0] ? 3 : 0); ++a) {
                                    int nd[3] = {i0[0] + a, i0[1] + b, i0[2] + c}, tmp[3];
                                    if (find_owner(par, nd, allpar, tmp) < 0) {
                                        delete r;
                                        return fail(MOL_EINVAL, "level %d: interpolation stencil leaves the new "
                                                    "parent level", l);
                                    }
                                }
                        const std::array<int, 3> key = {floor_div(g[0], R), floor_div(g[1], R), floor_div(g[2], R)};
                        auto it = cidx.find(key);
                        if (it == cidx.end()) {
                            it = cidx.emplace(key, ct.size()).first;
                            ct.push_back(CellTmp{{key[0], key[1], key[2]}, q0, {cw[0], cw[1], cw[2]}, 0, 0});
                        }
                        CellTmp& c = ct[it->second];
                        c.mask |= uint64_t(1) << ((m[2] * R + m[1]) * R + m[0]);
                        for (int d = 0; d < 3; ++d)
                            if (m[d]) c.frac |= 1 << d;
                    }
            std::stable_sort(ct.begin(), ct.end(), [](const CellTmp& a, const CellTmp& b) { return a.frac < b.frac; });
            for (const CellTmp& c : ct) {
                const PatchDev& qd = par.pd[c.q0];
                int c0[3];
                for (int d = 0; d < 3; ++d) c0[d] = c.cw[d] - qd.lo[d] + G - ((c.frac >> d & 1) ? 2 : 0);
                ProlongCell e{};
                e.dbase = pd.off + local_index(pd, R * c.key[0] - pd.lo[0] + G, R * c.key[1] - pd.lo[1] + G,
                                               R * c.key[2] - pd.lo[2] + G);
                e.cbase = qd.off + local_index(qd, c0[0], c0[1], c0[2]);
                e.dfs = pd.fs;
                e.cfs = qd.fs;
                e.dpy = pd.pitch_y;
                e.dpz = pd.pitch_z;
                e.cpy = qd.pitch_y;
                e.cpz = qd.pitch_z;
                e.mask = c.mask;
                e.frac = c.frac;
                cells.push_back(e);
            }
        }
        int rc;
        if ((rc = r->copy[l].upload(copy)) || (rc = r->cells[l].upload(cells))) {
            delete r;
            return rc;
        }
    }
    *out = r;
    return MOL_OK;
}

int mol_regrid_apply(mol_regrid* r, const double* const* U_old, double* const* U_new, void* stream)
{
    if (!r || !U_old || !U_new) return fail(MOL_EINVAL, "null argument");
    mol_patchset* pn = r->pn;
    for (int l = 0; l < pn->nlev; ++l)
        if (!U_old[l] || !U_new[l]) return fail(MOL_EINVAL, "level %d: null buffer", l);
    hipStream_t s = S(stream);
    hipError_t e = hipMemcpyAsync(U_new[0], U_old[0], sizeof(double) * pn->L[0].nelems, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    const int nf = pn->sp.nf;
    for (int l = 1; l < pn->nlev; ++l) {
        int rc = fill_impl(pn, l - 1, U_new[l - 1], nf, s, 0);
        if (rc) return rc;
        if ((e = launch_copy2(r->copy[l].p, r->copy[l].n, nf, U_old[l], U_new[l], s)) != hipSuccess)
            return hip_fail(e, "regrid copy launch");
        if ((e = launch_prolong(r->cells[l].p, r->cells[l].n, nf, pn->L[l].ratio, pn->L[l].lagw.data(), U_new[l - 1],
                                U_new[l], s)) != hipSuccess)
            return hip_fail(e, "regrid interpolation launch");
    }
    return MOL_OK;
}

void mol_regrid_destroy(mol_regrid* r)
{
    if (!r) return;
    (void)hipDeviceSynchronize();  // device work may still read the plan's lists
    delete r;
}

extern "C++" {  // helpers below are C++ (they return std::vector)
namespace {
// launch shapes of a level's stage kernel worth timing: the z-chunk length of
// the z-marching kernels, the thread tile of the point-wise wave kernel
std::vector<std::array<int, 3>> tiling_candidates(int system)
{
    std::vector<std::array<int, 3>> c;
    switch (system) {
    case MOL_WAVE:
        for (int z : {4, 8, 16, 32, 64, 128, 256, 512}) c.push_back({MOL_WAVE_WX, MOL_WAVE_WY, z});
        c.push_back({32, 4, 2});
        c.push_back({64, 4, 1});
        c.push_back({16, 8, 2});
        c.push_back({16, 4, 4});
        c.push_back({8, 8, 4});
        break;
    case MOL_MHD:
    case MOL_MHD_GLM:
        for (int z : {4, 8, 16, 32}) c.push_back({15, 15, z});
        break;
    default:
        c.push_back({MOL_CCZ4_TX, MOL_CCZ4_TY, MOL_CCZ4_TZ});
        c.push_back({8, 8, 8});
        c.push_back({8, 4, 8});
        break;
    }
    return c;
}

bool tiling_valid(int system, const int td[3])
{
    if (td[0] < 1 || td[1] < 1 || td[2] < 1) return false;
    switch (system) {
    case MOL_WAVE:
        if (td[0] == MOL_WAVE_WX && td[1] == MOL_WAVE_WY) return td[2] > 1 && td[2] <= 1024;  // z-marching
        return td[0] * td[1] * td[2] <= 256;                                                 // point-wise
    case MOL_MHD:
    case MOL_MHD_GLM: return td[0] == 15 && td[1] == 15 && td[2] <= 1024;
    default:
        return (td[0] == MOL_CCZ4_TX && td[1] == MOL_CCZ4_TY && td[2] == MOL_CCZ4_TZ) ||
               (td[0] == 8 && td[1] == 8 && td[2] == 8) || (td[0] == 8 && td[1] == 4 && td[2] == 8);
    }
}

// replace the level's stage tile list (the old one is kept until the
// patchset is destroyed: graphs captured earlier still read it)
int set_tiles(mol_patchset* ps, int level, const int td[3], int order)
{
    Level& lev = ps->L[level];
    TileList tl;
    int rc = build_tiles(lev, td, 0, tl, nullptr, order);
    if (rc) {
        tl.dev.release();
        return rc;
    }
    ps->retired.push_back(lev.tiles.dev);
    lev.tiles = tl;
    return MOL_OK;
}
}  // namespace
}  // extern "C++"

int mol_set_tiling(mol_patchset* ps, int level, const mol_tiling* t)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!t) return fail(MOL_EINVAL, "null tiling");
    if (t->order < 0 || t->order > 3) return fail(MOL_EINVAL, "tile order %d not in 0..3", t->order);
    if (!tiling_valid(ps->sp.system, t->tdim))
        return fail(MOL_EINVAL, "tile %d x %d x %d is not a launch shape of this system's stage kernel", t->tdim[0],
                    t->tdim[1], t->tdim[2]);
    return set_tiles(ps, level, t->tdim, t->order);
}

int mol_autotune(mol_patchset* ps, int level, const mol_level_state* st, double dt, int reps, mol_tiling* best,
                 void* stream)
{
    int rc = check_level(ps, level);
    if (rc) return rc;
    if (!st || !st->U || !st->S0 || !st->S1 || !st->acc) return fail(MOL_EINVAL, "null state buffer");
    if (!std::isfinite(dt) || dt <= 0.0) return fail(MOL_EINVAL, "dt must be positive and finite");
    if (reps < 1 || reps > 1000) return fail(MOL_EINVAL, "reps %d not in [1, 1000]", reps);
    Level& lev = ps->L[level];
    hipStream_t s = S(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    mol_tiling win{};
    win.ms = -1.0;
    const TileList keep = lev.tiles;
    rc = MOL_OK;
    // the kernel variant the driver launches on this level
    const bool wrap = level_wraps(ps, level), images = level_images(ps, level);
    // tile orders: patches as listed or largest first; for CCZ4 also the
    // column orders (the wave and MHD kernels march along z already)
    const int last_order = ps->sp.system == MOL_CCZ4 ? 3 : 1;
    for (const auto& td : tiling_candidates(ps->sp.system)) {
        for (int order = 0; order <= last_order && rc == MOL_OK; ++order) {
            TileList tl;
            if ((rc = build_tiles(lev, td.data(), 0, tl, nullptr, order))) break;
            lev.tiles = tl;
            // RK4 stage 2: reads U, S0 and acc, writes acc and S1
            rc = stage_impl(ps, level, ST_RK4, 2, dt, st->U, st->S0, st->acc, st->S1, nullptr, s, 0, wrap, images);
            if (rc == MOL_OK && (e = hipEventRecord(e0, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
            for (int r = 0; r < reps && rc == MOL_OK; ++r)
                rc = stage_impl(ps, level, ST_RK4, 2, dt, st->U, st->S0, st->acc, st->S1, nullptr, s, 0, wrap,
                                images);
            float ms = 0.0f;
            if (rc == MOL_OK && (e = hipEventRecord(e1, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
            if (rc == MOL_OK && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
            if (rc == MOL_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
                rc = hip_fail(e, "hipEventElapsedTime");
            lev.tiles = keep;
            tl.dev.release();
            if (rc) break;
            const double per = ms / reps;
            if (win.ms < 0.0 || per < win.ms) {
                for (int d = 0; d < 3; ++d) win.tdim[d] = td[d];
                win.order = order;
                win.ms = per;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = set_tiles(ps, level, win.tdim, win.order))) return rc;
    if (best) *best = win;
    return MOL_OK;
}

int mol_graph_create(mol_patchset* ps, const mol_level_state* states, double dt0, mol_graph** out)
{
    return mol_graph_create_steps(ps, states, dt0, 1, out);
}

int mol_graph_create_steps(mol_patchset* ps, const mol_level_state* states, double dt0, int nsteps,
                           mol_graph** out)
{
    if (!ps || !out) return fail(MOL_EINVAL, "null argument");
    *out = nullptr;
    if (nsteps < 1) return fail(MOL_EINVAL, "nsteps must be at least 1");
    if (!std::isfinite(dt0) || dt0 <= 0.0) return fail(MOL_EINVAL, "dt must be positive and finite");
    int rc = check_states(ps, states);
    if (rc) return rc;
    hipError_t e;
    if (!ps->capture_stream) {
        e = hipStreamCreateWithFlags(&ps->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    }
    mol_graph* g = new (std::nothrow) mol_graph();
    if (!g) return fail(MOL_ENOMEM, "host allocation failed");
    e = hipStreamBeginCapture(ps->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    for (int k = 0; k < nsteps && !rc; ++k)
        rc = advance_level(ps, states, 0, 0, dt0, ps->capture_stream, 0, MOL_TIME_BOR, k > 0, k + 1 == nsteps);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ps->capture_stream, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        return rc ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = g;
    return MOL_OK;
}

int mol_graph_launch(mol_graph* g, void* stream)
{
    if (!g || !g->exec) return fail(MOL_EINVAL, "null graph");
    hipError_t e = hipGraphLaunch(g->exec, S(stream));
    return e == hipSuccess ? MOL_OK : hip_fail(e, "hipGraphLaunch");
}

void mol_graph_destroy(mol_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
