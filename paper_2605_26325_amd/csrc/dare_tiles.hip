// Directionality-aware reslice at interpolation radius 1 (Sec. 2.1 "Reslicing", Eq. 1, Eq. 2,
// Fig. 2): the trilinear cell of every pixel, each cell voxel blended over the direction bins
// that pass the angular gates.
//
// The per-request part runs on the device in FP64 (`request_setup`, one wave): the slice pose
// T = P.C, Eq. 1 for every bin, the two gates and Eq. 2 for the survivors, the plane frame in
// voxel units, and the choice of tile edge.  A request is then cut into square tiles of output
// pixels, each with a record of its voxel box (`compute_tile`).  One workgroup takes one
// (request, tile) unit and runs three phases out of LDS:
//   slots   the brick-table entries of every surviving bin over the bricks of the tile's voxel
//           box (one table read per (bin, brick), not per voxel), issued first so that their
//           latency overlaps the next phase;
//   voxels  every voxel within the trilinear support of the tile's piece of plane, enumerated
//           as short runs along the plane normal's dominant axis (one thread per column of the
//           other two axes), tested and listed; then every listed voxel gathers its surviving
//           bins' pairs and blends them into V_v = sum_b w_b c_vb a_vb / sum_b w_b c_vb, kept in
//           LDS as one float, NaN when no surviving bin holds a sample (or the voxel lies
//           outside the grid);
//   pixels  FP64 position, the 8 cell values from LDS, tent weights, num / den or NaN.
// Where all 8 corners are valid the tent weights sum to 1 and the blend is the trilinear
// interpolation (nested lerps); a NaN corner sends the pixel to the sums over its valid corners.
//
// A single reslice launches one workgroup per 16 x 16 tile; each workgroup evaluates the
// request setup and its tile's record itself, since no other memory holds them: the bins on one
// wave and the plane and tile geometry on another, at the same time.  A batch
// runs the request setup once per request and the tile records once per tile (`k_tiles_setup`:
// one workgroup per request, one thread per tile; it also appends the units to a list), then one
// persistent kernel over all staged units (`k_tiles`), which reads both records through scalar
// loads, with tiles of 32 x 32 pixels wherever their voxel box fits the LDS budget.  The
// per-voxel and per-pixel arithmetic does not depend on the tile, so a request gives the same
// bits alone and in a batch.  Requests whose pixels are too coarse for staging to pay (a 16 x 16
// tile's box beyond the budget) gather per pixel.
#include <algorithm>

#include "dare_batch.h"
#include "dare_reslice_dev.h"

namespace dare {

namespace {

constexpr int kItemsMax = 2048;      // staged voxels (box columns x run depth) per tile
constexpr int kColsMax = 1024;       // box columns per tile
constexpr int kSlotsMax = 1280;      // (box brick, bin) table entries per tile
constexpr int kRunSpan = 127;        // box voxels along the dominant axis, less one, at most
constexpr int kThreadsBatch = 256;   // threads of a batch workgroup
constexpr int kSetupThreads = 256;   // threads of a batch setup workgroup (one request at a time)
constexpr int kTileBig = 32;         // batched tile edge where the box fits
constexpr int kFillRun = 4096;       // pixels per unit of a batched request that is all NaN

// Listed voxels per thread per gather round, and surviving bins whose pair loads a thread issues
// together for all of them.
template <int DT>
constexpr int items_per_round() { return 2; }
template <int DT>
constexpr int bins_per_round() { return DT == DARE_FP8_E4M3 ? 4 : 8; }
// The same for the persistent batch kernel, whose register budget is held to 7 workgroups per CU:
// 2-byte halves (BF16, FP16) take 4 voxels of 4 bins (16 pairs, one register each, a quarter
// fewer gather rounds than 2 x 8); FP32 pairs (two registers) and FP8 (the scales besides) stay
// at 2 voxels, as 4 would spill.
template <int DT>
constexpr int batch_items_per_round() { return DT == DARE_BF16 || DT == DARE_F16 ? 4 : 2; }
template <int DT>
constexpr int batch_bins_per_round() { return DT == DARE_F32 ? 8 : 4; }

// LDS of a workgroup working on one staged tile.
template <int DT>
struct TileLds {
    alignas(16) int slot[kSlotsMax];                      // [box brick][bin], rows of kactp
    float2 scale[DT == DARE_FP8_E4M3 ? kSlotsMax : 1];    // FP8 value and count scales per slot
    signed char rs[kColsMax];                             // first voxel of each column's run, less lo_d
    alignas(16) float V[kItemsMax];                       // V_v, or NaN where not valid, [column][run]
    int list[kItemsMax];                                  // voxels to gather: e | local << 11 | brick << 20
    int nlist;
};

// Pointers in the global address space, so that loads and stores through them are global (not
// flat) operations, whose waits do not wait for LDS and vice versa.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> global(T* p) {
    return (gptr<T>)(p);
}

// Workgroup-uniform values, moved to scalar registers.
__device__ __forceinline__ int ui(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uf(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ double ud(double x) { return uniform_f64(x); }
__device__ __forceinline__ SmallDiv usd(uint32_t m, int d) { return SmallDiv{(uint32_t)ui((int)m), ui(d)}; }

// Upper bound of a tile's box edge along one axis (T pixels per side): the corner cells'
// floors differ by at most ceil of the tile's extent, and the box adds one voxel below and two
// above (the upper cell voxel and a margin for rounding).
__device__ __forceinline__ int box_edge_bound(int T, double ex, double ey) {
    const double ext = (double)(T - 1) * (fabs(ex) + fabs(ey));
    return (int)floor(ext * (1.0 + 1e-9) + 1e-6) + 5;
}

// Entry i of a 3-vector held in registers, without indexing it (which would put it in memory).
template <class T>
__device__ __forceinline__ T pick3(const T (&v)[3], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}

// What a tile record needs of its request, held in registers by the thread that writes it.
struct Plane {
    double c00[3], ex[3], ey[3];          // voxel coordinates of pixel (i, j): c00 + i ex + j ey
    SliceFrame f;
    int n[3];
    int W, H, tile, tiles_x, depth, kact;
    float slop, half;
};

// The plane from a request record.
__device__ __forceinline__ Plane plane_of(const SliceRec& rec) {
    Plane pl;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pl.c00[a] = rec.c00[a];
        pl.ex[a] = rec.ex[a];
        pl.ey[a] = rec.ey[a];
        pl.f.fm[a] = rec.fm[a];
        pl.f.fu[a] = rec.fu[a];
        pl.f.fw[a] = rec.fw[a];
        pl.n[a] = rec.vol.n[a];
    }
    pl.f.lu = rec.lu;
    pl.f.lw = rec.lw;
    pl.f.dax = rec.dax;
    pl.W = rec.W;
    pl.H = rec.H;
    pl.tile = rec.tile;
    pl.tiles_x = rec.tiles_x;
    pl.depth = rec.depth;
    pl.kact = rec.kact;
    pl.slop = rec.slop;
    pl.half = rec.half;
    return pl;
}

// Does a T x T tile of this request fit the LDS budget wherever it falls?
__device__ __forceinline__ bool tile_fits(const Plane& pl, int T) {
    const int dax = pl.f.dax, pax = dax == 0 ? 1 : 0, qax = dax == 2 ? 1 : 2;
    int e[3];
    int64_t nbb = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        e[a] = box_edge_bound(T, pl.ex[a], pl.ey[a]);
        nbb *= e[a] / 8 + 2;
    }
    const int64_t cols = (int64_t)pick3(e, pax) * pick3(e, qax);
    const int kactp = (pl.kact + 7) & ~7;
    return cols <= kColsMax && cols * pl.depth <= kItemsMax && nbb * kactp <= kSlotsMax && pick3(e, dax) <= kRunSpan &&
           pl.depth <= kRunSpan;
}

// One lane: the request's plane in voxel coordinates (FP64), its frame, volume view and output,
// and the slab of a tile: voxels with |m.(v - c0)| < |m|_1 (plus slop for FP32 rounding of
// coordinates up to the grid's size) form runs of at most ceil(2 half) voxels along dax.  Stored
// in `rec` and returned (tile edge and surviving bins not yet set).
__device__ __forceinline__ Plane request_frame(const VolDev* __restrict__ vd, const SliceArgs& s, const double T[12],
                                               SliceRec& rec) {
    Plane pl;
    pl.f = frame_of(vd, s, T);
    store_frame(pl.f, rec);
    const double inv_h = vd->inv_h;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pl.c00[a] = (T[a * 4 + 3] - vd->origin[a]) * inv_h;
        pl.ex[a] = (s.sx * T[a * 4 + 0]) * inv_h;
        pl.ey[a] = (s.sy * T[a * 4 + 1]) * inv_h;
        rec.c00[a] = pl.c00[a];
        rec.ex[a] = pl.ex[a];
        rec.ey[a] = pl.ey[a];
    }
    const VolView vv = view_of(vd);
    rec.vol = vv;
    rec.out = s.out;
    rec.W = pl.W = s.W;
    rec.H = pl.H = s.H;
#pragma unroll
    for (int a = 0; a < 3; ++a) pl.n[a] = vv.n[a];
    const int nmax = max(vv.n[0], max(vv.n[1], vv.n[2]));
    pl.slop = 2e-3f + 1e-6f * (float)(nmax + 64);
    const float l1m = fabsf(pl.f.fm[0]) + fabsf(pl.f.fm[1]) + fabsf(pl.f.fm[2]);
    pl.half = (l1m + pl.slop) * fabsf(1.0f / pick3(pl.f.fm, pl.f.dax));
    pl.depth = (int)ceilf(2.0f * pl.half);
    rec.slop = pl.slop;
    rec.half = pl.half;
    rec.depth = pl.depth;
    pl.tile = 16;
    pl.tiles_x = (s.W + 15) / 16;
    pl.kact = 0;
    return pl;
}

// One lane, once the frame and the surviving bins are known: the mode and the tile edge.
__device__ __forceinline__ int request_mode(Plane& pl, SliceRec& rec, int max_tile) {
    const int kact = pl.kact;
    int mode = kact > 0 ? 2 : 0, tile = 16;
    if (kact > 0) {
        if (max_tile >= kTileBig && tile_fits(pl, kTileBig)) {
            mode = 1;
            tile = kTileBig;
        } else if (tile_fits(pl, 16)) {
            mode = 1;
        }
    }
    pl.tile = tile;
    pl.tiles_x = (pl.W + tile - 1) / tile;
    rec.mode = mode;
    rec.tile = tile;
    rec.tiles_x = pl.tiles_x;
    rec.ntiles = pl.tiles_x * ((pl.H + tile - 1) / tile);
    return mode;
}

// Bins past the survivors: no slots, zero weight (one wave, lane b for bin b).
__device__ __forceinline__ void pad_bins(SliceRec& rec, int kact) {
    const int lane = threadIdx.x & 63;
    if (lane >= kact) {
        rec.act_bin[lane] = 0;
        rec.act_w[lane] = 0.0f;
    }
}

// One wave: the per-request setup of a radius-1 reslice, in FP64 on the device, into `rec`.
// Lane 0 returns the number of work units (tiles) of the request and its mode in *mode_out.
__device__ int request_setup(const VolDev* __restrict__ vd, const SliceArgs& s, SliceRec& rec, int max_tile,
                             int* mode_out) {
    double T[12];
    const int kact = slice_gates(vd, s, rec, T);
    pad_bins(rec, kact);
    if ((threadIdx.x & 63) != 0) return 0;
    Plane pl = request_frame(vd, s, T, rec);
    pl.kact = kact;
    *mode_out = request_mode(pl, rec, max_tile);
    return rec.ntiles;
}

// One thread: the part of tile t's record that needs only the plane's position in voxel units
// (c00 + i ex + j ey, FP64) and the grid: its pixels, and its voxel box, the four corner pixels'
// cells with one voxel of margin below and two above (positions are affine in (i, j), so the
// corners' cells bound every pixel's cell; the margin absorbs rounding), clipped to [-1, n], and
// the box's bricks.  `mode` is left 1, or 0 when no in-grid voxel is in reach.
__device__ __forceinline__ void tile_box(const double (&c00)[3], const double (&ex)[3], const double (&ey)[3],
                                         const int (&n)[3], int T, int W, int H, int tiles_x, int r, int t,
                                         TileRec& tr) {
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int i0 = tx * T, j0 = ty * T;
    const int i1 = min(i0 + T - 1, W - 1), j1 = min(j0 + T - 1, H - 1);
    bool empty = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int mn = 0, mx = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double ci = (double)((k & 1) ? i1 : i0), cj = (double)((k & 2) ? j1 : j0);
            const double c = fma(cj, ey[a], fma(ci, ex[a], c00[a]));
            const int f = (int)fmin(fmax(floor(c), -1048576.0), 1048576.0);
            mn = k == 0 ? f : min(mn, f);
            mx = k == 0 ? f : max(mx, f);
            if (k == 0) tr.c0[a] = (float)c;
        }
        const int lo = max(mn - 1, -1), hi = min(mx + 2, n[a]);
        tr.lo[a] = lo;
        tr.hi[a] = hi;
        tr.blo[a] = max(lo, 0) >> 3;
        tr.bdim[a] = (min(hi, n[a] - 1) >> 3) - tr.blo[a] + 1;
        // no in-grid voxel in reach: every pixel of the tile is unassigned
        empty = empty || max(lo, 0) > min(hi, n[a] - 1);
    }
    tr.r = r;
    tr.mode = empty ? 0 : 1;
    tr.i0 = i0;
    tr.j0 = j0;
    tr.ni = i1 - i0 + 1;
    tr.nj = j1 - j0 + 1;
    tr.nbb = tr.bdim[0] * tr.bdim[1] * tr.bdim[2];
    tr.m_bdx = small_div(max(tr.bdim[0], 1)).m;
    tr.m_bdy = small_div(max(tr.bdim[1], 1)).m;
}

// One thread, after `tile_box`: the part of the record that needs the plane's frame (the box's
// columns along the dominant axis, whether they fit the LDS budget, the slab and lateral
// thresholds), all but what depends on the number of surviving bins (`tile_bins`).
__device__ __forceinline__ void tile_frame(const Plane& pl, TileRec& tr) {
    const int dax = pl.f.dax, pax = dax == 0 ? 1 : 0, qax = dax == 2 ? 1 : 2;
    const int lo[3] = {tr.lo[0], tr.lo[1], tr.lo[2]}, hi[3] = {tr.hi[0], tr.hi[1], tr.hi[2]};
    const int bp = pick3(hi, pax) - pick3(lo, pax) + 1, bq = pick3(hi, qax) - pick3(lo, qax) + 1;
    const int depth = pl.depth;
    // the request's bound makes every staged tile fit; a tile beyond it would be left NaN, so the
    // check only keeps the LDS accesses in bounds
    const bool fits = bp >= 2 && bq >= 2 && depth >= 2 && depth <= kRunSpan && bp * bq <= kColsMax &&
                      bp * bq * depth <= kItemsMax && pick3(hi, dax) - pick3(lo, dax) <= kRunSpan;
    tr.mode = (tr.mode == 1 && fits) ? 1 : 0;
    float l1u = 0.0f, l1w = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        l1u += fabsf(pl.f.fu[a]);
        l1w += fabsf(pl.f.fw[a]);
    }
    tr.bp = bp;
    tr.bq = bq;
    tr.ncols = bp * bq;
    tr.depth = depth;
    tr.m_bp = small_div(max(bp, 1)).m;
    // every voxel with weight for a pixel of the tile lies within |m.(v - c0)| < |m|_1 and,
    // along the in-plane axes, within the tile's extent widened by |u|_1, |w|_1 (the margins
    // cover FP32 rounding and the pose rigidity tolerance)
    const float slop = pl.slop;
    tr.thr_n = fabsf(pl.f.fm[0]) + fabsf(pl.f.fm[1]) + fabsf(pl.f.fm[2]) + slop;
    tr.thr_u = l1u + 0.02f + slop;
    tr.thr_v = l1w + 0.02f + slop;
    tr.hi_u = (float)(tr.ni - 1) * pl.f.lu + tr.thr_u;
    tr.hi_v = (float)(tr.nj - 1) * pl.f.lw + tr.thr_v;
    tr.inv_md = 1.0f / pick3(pl.f.fm, dax);
    tr.half = pl.half;
}

// One thread: the parts of a tile record that depend on the number of surviving bins.
__device__ __forceinline__ void tile_bins(int kact, TileRec& tr) {
    const int kactp = (kact + 7) & ~7;
    tr.kactp = kactp;
    tr.m_kactp = small_div(max(kactp, 1)).m;
    if (tr.nbb * kactp > kSlotsMax) tr.mode = 0;
}

__device__ __forceinline__ void compute_tile(const Plane& pl, int r, int t, TileRec& tr) {
    tile_box(pl.c00, pl.ex, pl.ey, pl.n, pl.tile, pl.W, pl.H, pl.tiles_x, r, t, tr);
    tile_frame(pl, tr);
    tile_bins(pl.kact, tr);
}

// Slots phase: the table entry of every (box brick, bin) pair, -1 past the surviving bins.  The
// table reads are issued first (`load_slots`, into registers) and written to LDS after the
// classification (`store_slots`), so that their latency overlaps that ALU work.
template <int NT>
constexpr int slots_per_thread() { return (kSlotsMax + NT - 1) / NT; }

template <int NT>
__device__ __forceinline__ void load_slots(const SliceRec& rec, const TileRec& tr, int (&sl)[slots_per_thread<NT>()]) {
    const int kact = ui(rec.kact), kactp = ui(tr.kactp), n = ui(tr.nbb) * kactp;
    const int bdx = ui(tr.bdim[0]), bdy = ui(tr.bdim[1]);
    const int bx0 = ui(tr.blo[0]), by0 = ui(tr.blo[1]), bz0 = ui(tr.blo[2]);
    const SmallDiv dk = usd(tr.m_kactp, kactp), dx = usd(tr.m_bdx, bdx), dy = usd(tr.m_bdy, bdy);
    const gptr<const int32_t> table = global(rec.vol.table);
    const int64_t nbricks = rec.vol.nbricks;
    const int nbx = ui(rec.vol.nbx), nby = ui(rec.vol.nby);
    // below 2^24 bricks per bin (grids up to 2048^3) every index product fits 24 x 24 -> 32 bits
    const bool small = nbricks < (int64_t)1 << 24;
    const uint32_t nb32 = (uint32_t)ui((int)(nbricks & 0xFFFFFF));
#pragma unroll
    for (int i = 0; i < slots_per_thread<NT>(); ++i) {
        const int e = (int)threadIdx.x + NT * i;
        const int bb = sdiv(e, dk), k = e - (int)__umul24((uint32_t)bb, (uint32_t)kactp);
        sl[i] = -1;
        if (e < n && k < kact) {
            const int byz = sdiv(bb, dx), bx = bb - (int)__umul24((uint32_t)byz, (uint32_t)bdx);
            const int bz = sdiv(byz, dy), by = byz - (int)__umul24((uint32_t)bz, (uint32_t)bdy);
            const int bin = rec.act_bin[k];
            if (small) {
                const uint32_t brick =
                    __umul24(__umul24((uint32_t)(bz0 + bz), (uint32_t)nby) + (uint32_t)(by0 + by), (uint32_t)nbx) +
                    (uint32_t)(bx0 + bx);
                sl[i] = table[__umul24((uint32_t)bin, nb32) + brick];
            } else {
                const int64_t brick = ((int64_t)(bz0 + bz) * nby + (by0 + by)) * nbx + (bx0 + bx);
                sl[i] = table[(int64_t)bin * nbricks + brick];
            }
        }
    }
}

template <int DT, int NT>
__device__ __forceinline__ void store_slots(const SliceRec& rec, const TileRec& tr, TileLds<DT>& tl,
                                            const int (&sl)[slots_per_thread<NT>()]) {
    constexpr int SP = slots_per_thread<NT>();
    const int n = ui(tr.nbb) * ui(tr.kactp);
    float2 sc[SP];
    if constexpr (DT == DARE_FP8_E4M3) {
        const gptr<const float2> scales = global(rec.vol.scales);
#pragma unroll
        for (int i = 0; i < SP; ++i) {
            sc[i] = make_float2(0.0f, 0.0f);
            if (sl[i] >= 0) sc[i] = *(const float2*)&scales[sl[i]];
        }
    }
#pragma unroll
    for (int i = 0; i < SP; ++i) {
        const int e = (int)threadIdx.x + NT * i;
        if (e < n) {
            tl.slot[e] = sl[i];
            if constexpr (DT == DARE_FP8_E4M3) tl.scale[e] = sc[i];
        }
    }
}

// A stored pair read in the folded form of its storage: the blend runs on the coded value and
// the affine map of the storage is applied once to the blended value (the blend is a convex
// combination, so this is the blend of the decoded values).
template <int DT>
__device__ __forceinline__ void folded(typename Pair<DT>::T p, float2 sc, float& v, float& c) {
    if constexpr (DT == DARE_F32) {
        v = p.x;
        c = p.y;
    } else if constexpr (DT == DARE_BF16) {
        v = __uint_as_float(p << 16);
        c = __uint_as_float(p & 0xFFFF0000u);
    } else if constexpr (DT == DARE_F16) {
        v = f16_to_f32(p & 0xFFFFu);
        c = f16_to_f32(p >> 16);
    } else {
        v = e4m3_to_f32(p & 0xFFu) * sc.x;
        c = e4m3_to_f32(p >> 8) * sc.y;
    }
}

template <int DT>
__device__ __forceinline__ float unfold(float q) {
    if constexpr (DT == DARE_F32) return q;
    else if constexpr (DT == DARE_FP8_E4M3) return q + 127.5f;
    else return q * 127.5f + 127.5f;
}

// First voxel of the run of column (vp, vq): the first whole voxel above centre - half, where
// centre is the plane's coordinate along DAX at the column (FP32 about the tile's origin c0).
// The column's voxels with |m.(v - c0)| < thr_n are among the depth voxels from there.
template <int DAX>
__device__ __forceinline__ int run_start(const float (&c0)[3], const float (&m)[3], float inv_md, float half, int vp,
                                         int vq) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    const float centre = c0[DAX] - (m[PAX] * ((float)vp - c0[PAX]) + m[QAX] * ((float)vq - c0[QAX])) * inv_md;
    return (int)floorf(centre - half) + 1;
}

// The bits that voxel coordinate v along axis A contributes to its brick-local index: the index
// interleaves the coordinates' bits, so it is the sum (an OR of disjoint fields) of one part per
// axis, and a list entry can add the dominant axis's part to a per-column remainder.
template <int A>
__host__ __device__ constexpr int local_part(int v) {
    return A == 0 ? ((v & 6) << 6) | (v & 1) : (A == 1 ? ((v & 6) << 4) | ((v & 1) << 1) : (v & 7) << 2);
}
constexpr bool local_parts_match() {
    for (int x = 0; x < 8; ++x)
        for (int y = 0; y < 8; ++y)
            for (int z = 0; z < 8; ++z)
                if (brick_local(x, y, z) != (local_part<0>(x) | local_part<1>(y) | local_part<2>(z))) return false;
    return true;
}
static_assert(local_parts_match(), "the brick-local index is the sum of its per-axis parts");

// Voxels phase, first part: one thread per box column (p, q) walks the column's run along the
// dominant axis; each voxel is tested against the tile's slab and lateral extent (the test terms
// of the column computed once, the axis term added per voxel).  The voxels that pass are appended
// to the gather list; the others keep the NaN that the run's entries of V start from.
template <int DT, int DAX, int NT>
__device__ __forceinline__ void classify_voxels(const SliceRec& rec, const TileRec& tr, TileLds<DT>& tl) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    const int ncols = ui(tr.ncols), depth = ui(tr.depth), bp = ui(tr.bp);
    const SmallDiv dbp = usd(tr.m_bp, bp);
    const int lo_p = ui(tr.lo[PAX]), lo_q = ui(tr.lo[QAX]), lo_d = ui(tr.lo[DAX]), hi_d = ui(tr.hi[DAX]);
    const int n[3] = {ui(rec.vol.n[0]), ui(rec.vol.n[1]), ui(rec.vol.n[2])};
    const int blo[3] = {ui(tr.blo[0]), ui(tr.blo[1]), ui(tr.blo[2])};
    const int bdx = ui(tr.bdim[0]), bdy = ui(tr.bdim[1]);
    // box brick index = sum over axes of (v_a / 8 - blo_a) * stride_a
    const int bstride[3] = {1, bdx, bdx * bdy};
    float m[3], fu[3], fw[3], c0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m[a] = uf(rec.fm[a]);
        fu[a] = uf(rec.fu[a]);
        fw[a] = uf(rec.fw[a]);
        c0[a] = uf(tr.c0[a]);
    }
    const float thr_n = uf(tr.thr_n), thr_u = uf(tr.thr_u), thr_v = uf(tr.thr_v), hi_u = uf(tr.hi_u), hi_v = uf(tr.hi_v);
    const float inv_md = uf(tr.inv_md), half = uf(tr.half);
    // voxels along the dominant axis that may pass: inside the box and the grid
    const int vlo = max(lo_d, 0), vhi = min(hi_d, n[DAX] - 1);
    for (int cb = 0; cb < ncols; cb += NT) {
        const int col = cb + (int)threadIdx.x;
        const bool live = col < ncols;
        const int cq = sdiv(col, dbp), cp = col - (int)__umul24((uint32_t)cq, (uint32_t)bp);
        const int vp = lo_p + cp, vq = lo_q + cq;
        const int rs = run_start<DAX>(c0, m, inv_md, half, vp, vq);
        // a column that a pixel's cell uses has its run start within [lo_d - depth, lo_d + kRunSpan]
        if (live) tl.rs[col] = (signed char)min(max(rs - lo_d, -128), 127);
        const bool col_in = live && (unsigned)vp < (unsigned)n[PAX] && (unsigned)vq < (unsigned)n[QAX];
        const int chi = col_in ? vhi : -1;
        const float dp = (float)vp - c0[PAX], dq = (float)vq - c0[QAX];
        const float bn = m[PAX] * dp + m[QAX] * dq;
        const float bu = fu[PAX] * dp + fu[QAX] * dq;
        const float bw = fw[PAX] * dp + fw[QAX] * dq;
        // the column's part of a list entry (wrapping arithmetic: only passing voxels, whose
        // coordinates lie in the grid, use it, and their entry is in range)
        const uint32_t ent0 =
            (uint32_t)__umul24((uint32_t)col, (uint32_t)depth) +
            ((uint32_t)(local_part<PAX>(vp) | local_part<QAX>(vq)) << 11) +
            ((uint32_t)(((vp >> 3) - blo[PAX]) * bstride[PAX] + ((vq >> 3) - blo[QAX]) * bstride[QAX] -
                        blo[DAX] * bstride[DAX])
             << 20);
        for (int k = 0; k < depth; ++k) {
            const int vd = rs + k;
            const float dd = (float)vd - c0[DAX];
            const float dn = bn + m[DAX] * dd, du = bu + fu[DAX] * dd, dv = bw + fw[DAX] * dd;
            const bool pass = vd >= vlo && vd <= chi && fabsf(dn) < thr_n && du > -thr_u && du < hi_u &&
                              dv > -thr_v && dv < hi_v;
            if (pass) {
                const int pos = atomicAdd(&tl.nlist, 1);
                const uint32_t ent = ent0 + (uint32_t)k + ((uint32_t)local_part<DAX>(vd) << 11) +
                                     ((uint32_t)__umul24((uint32_t)vd >> 3, (uint32_t)bstride[DAX]) << 20);
                tl.list[pos] = (int)ent;
            }
        }
    }
}

// Pairs of every surviving bin for U listed voxels of a thread: the slot rows of NB bins are
// read from LDS 4 at a time, then the NB x U pair loads are issued before any is used.  A pair
// that is not loaded (no slot: -1, or anything outside the pool) stays zero and adds nothing.  A thread past the end of the list
// reads the last entry's row (its result is not stored).  NARROW: the pool spans less than 4 GiB,
// so a pair's byte offset from the pool's base fits 32 bits.
template <int DT, int U, int NB, bool NARROW>
__device__ __forceinline__ void gather(const SliceRec& rec, const TileLds<DT>& tl, const int (&row)[U],
                                       const int (&loc)[U], float (&A)[U], float (&B)[U]) {
    using PT = Pair<DT>;
    using T = typename PT::T;
    static_assert(NB % 4 == 0 && 8 % NB == 0, "slot rows (kactp entries, a multiple of 8) are read 4 at a time");
    constexpr int LG = sizeof(T) == 8 ? 3 : (sizeof(T) == 4 ? 2 : 1);
    static_assert(sizeof(T) == (1u << LG), "pair size");
    const gptr<const T> data = global((const T*)rec.vol.data);
    const gptr<const char> bytes = global((const char*)rec.vol.data);
    const int kact = ui(rec.kact);
    const uint32_t cap = (uint32_t)ui((int)rec.vol.cap);
#pragma unroll
    for (int u = 0; u < U; ++u) A[u] = B[u] = 0.0f;
    for (int k0 = 0; k0 < kact; k0 += NB) {
        int sl[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int g = 0; g < NB; g += 4) {
                const int4 s4 = *reinterpret_cast<const int4*>(&tl.slot[row[u] + k0 + g]);
                sl[u][g] = s4.x;
                sl[u][g + 1] = s4.y;
                sl[u][g + 2] = s4.z;
                sl[u][g + 3] = s4.w;
            }
        T pr[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int g = 0; g < NB; ++g) {
                pr[u][g] = T{};
                if ((uint32_t)sl[u][g] < cap) {   // a slot of the pool (-1: none)
                    if constexpr (NARROW)
                        pr[u][g] = *(const T*)&bytes[((uint32_t)sl[u][g] << (9 + LG)) | (uint32_t)loc[u]];
                    else
                        pr[u][g] = *(const T*)&data[(((size_t)sl[u][g] << 9) | (uint32_t)loc[u]) ];
                }
            }
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const float w = uf(rec.act_w[k0 + g]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float2 sc = make_float2(0.0f, 0.0f);
                if constexpr (DT == DARE_FP8_E4M3) sc = tl.scale[row[u] + k0 + g];
                float v, c;
                folded<DT>(pr[u][g], sc, v, c);
                const float wc = w * c;
                A[u] = __builtin_fmaf(wc, v, A[u]);
                B[u] = B[u] + wc;
            }
        }
    }
}

// Voxels phase, second part: every listed voxel's surviving bins gathered and blended into V_v,
// NaN when none holds a sample.
template <int DT, int NT, int U, int NB, bool NARROW>
__device__ __forceinline__ void gather_list(const SliceRec& rec, const TileRec& tr, TileLds<DT>& tl, int nlist) {
    using T = typename Pair<DT>::T;
    constexpr int LG = sizeof(T) == 8 ? 3 : (sizeof(T) == 4 ? 2 : 1);
    const int kactp = ui(tr.kactp);
    for (int base = 0; base < nlist; base += U * NT) {
        bool ok[U];
        int row[U], loc[U], ent[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * NT + (int)threadIdx.x;
            ok[u] = i < nlist;
            ent[u] = tl.list[min(i, nlist - 1)];
            row[u] = (int)__umul24((uint32_t)ent[u] >> 20, (uint32_t)kactp);
            // the pair's index in its brick, or its byte offset there where offsets are 32-bit
            loc[u] = ((ent[u] >> 11) & 511) << (NARROW ? LG : 0);
        }
        float A[U], B[U];
        gather<DT, U, NB, NARROW>(rec, tl, row, loc, A, B);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const bool valid = B[u] > 0.0f;
            tl.V[ent[u] & 2047] = valid ? unfold<DT>(A[u] * __builtin_amdgcn_rcpf(B[u])) : __builtin_nanf("");
        }
    }
}

template <int DT, int NT, int U, int NB>
__device__ __forceinline__ void gather_voxels(const SliceRec& rec, const TileRec& tr, TileLds<DT>& tl) {
    using T = typename Pair<DT>::T;
    const int nlist = ui(tl.nlist);
    if (nlist == 0) return;
    const uint64_t pool_bytes = (uint64_t)(uint32_t)ui((int)rec.vol.cap) * kBrickVox * sizeof(T);
    if (pool_bytes <= 0xFFFFFFFFull)
        gather_list<DT, NT, U, NB, true>(rec, tr, tl, nlist);
    else
        gather_list<DT, NT, U, NB, false>(rec, tr, tl, nlist);
}

// Pixels phase of a staged tile: FP64 position, the cell's 8 values from LDS (two adjacent run
// entries per cell column), then the tent blend.  With all 8 corners valid the weights sum to 1
// and the blend is the trilinear interpolation, taken as nested lerps; a NaN corner makes that
// NaN, and the pixel takes sum w V / sum w over its valid corners instead.
template <int DT, int DAX, int NT>
__device__ __forceinline__ void stage_pixels(const SliceRec& rec, const TileRec& tr, const TileLds<DT>& tl) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    const int T = ui(rec.tile), W = ui(rec.W);
    const int i0 = ui(tr.i0), j0 = ui(tr.j0), ni = ui(tr.ni), nj = ui(tr.nj);
    const int lo_p = ui(tr.lo[PAX]), lo_q = ui(tr.lo[QAX]), lo_d = ui(tr.lo[DAX]);
    const int bp = ui(tr.bp), bq = ui(tr.bq), depth = ui(tr.depth);
    const int n[3] = {ui(rec.vol.n[0]), ui(rec.vol.n[1]), ui(rec.vol.n[2])};
    double c00[3], ex[3], ey[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c00[a] = ud(rec.c00[a]);
        ex[a] = ud(rec.ex[a]);
        ey[a] = ud(rec.ey[a]);
    }
    const int shift = T == kTileBig ? 5 : 4, rstep = NT >> shift;
    // a thread keeps its column (NT is a multiple of the tile edge): the column's part of the
    // position is computed once, and its output pointer steps by whole rows
    static_assert(NT % kTileBig == 0, "threads of a workgroup cover whole tile rows");
    const int li = (int)threadIdx.x & (T - 1), i = i0 + li;
    if (li >= ni) return;
    double ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ci[a] = fma((double)i, ex[a], c00[a]);
    // run entries of the cell's four columns relative to column (cp, cq)
    const int dcol[4] = {0, depth, bp * depth, (bp + 1) * depth};
    int lj = (int)threadIdx.x >> shift;
    gptr<float> out = global(rec.out) + ((size_t)(j0 + lj) * W + i);
    const size_t ostep = (size_t)rstep * W;
    for (; lj < nj; lj += rstep, out += ostep) {
        const double dj = (double)(j0 + lj);
        double c[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] = fma(dj, ey[a], ci[a]);
        int b[3];
        float fr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double f = floor(c[a]);
            b[a] = (int)f;
            fr[a] = (float)(c[a] - f);
        }
        // inside [-1, n) on every axis: the cell floor in [-1, n - 1]
        if (!((uint32_t)b[0] + 1u < (uint32_t)n[0] + 1u && (uint32_t)b[1] + 1u < (uint32_t)n[1] + 1u &&
              (uint32_t)b[2] + 1u < (uint32_t)n[2] + 1u)) {
            *out = __builtin_nanf("");
            continue;
        }
        // the cell's columns lie in the box and its two layers in each column's run; the clamps
        // only keep the LDS reads in bounds
        const int cp = min(max(b[PAX] - lo_p, 0), bp - 2), cq = min(max(b[QAX] - lo_q, 0), bq - 2);
        const int col0 = (int)__umul24((uint32_t)cq, (uint32_t)bp) + cp;
        const int e0 = (int)__umul24((uint32_t)col0, (uint32_t)depth), kd = b[DAX] - lo_d;
        const int cols[4] = {col0, col0 + 1, col0 + bp, col0 + bp + 1};
        float lov[4], hiv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = min(max(kd - (int)tl.rs[cols[q]], 0), depth - 2);
            const int e = e0 + dcol[q] + k;
            lov[q] = tl.V[e];
            hiv[q] = tl.V[e + 1];
        }
        float lq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) lq[q] = __builtin_fmaf(fr[DAX], hiv[q] - lov[q], lov[q]);
        const float l0 = __builtin_fmaf(fr[PAX], lq[1] - lq[0], lq[0]);
        const float l1 = __builtin_fmaf(fr[PAX], lq[3] - lq[2], lq[2]);
        float val = __builtin_fmaf(fr[QAX], l1 - l0, l0);
        if (__builtin_isnan(val)) {
            // the low voxel's weight from FP64 (tent_weight at R = 1)
            float gr[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gr[a] = (float)((double)b[a] + 1.0 - c[a]);
            const float wp[2] = {gr[PAX], fr[PAX]}, wq[2] = {gr[QAX], fr[QAX]};
            const float wd[2] = {gr[DAX], fr[DAX]};
            float num = 0.0f, den = 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float wpq = wp[q & 1] * wq[q >> 1];
                const float t0 = wpq * wd[0], t1 = wpq * wd[1];
                const bool v0 = !__builtin_isnan(lov[q]), v1 = !__builtin_isnan(hiv[q]);
                num = __builtin_fmaf(t0, v0 ? lov[q] : 0.0f, num);
                den = __builtin_fmaf(t0, v0 ? 1.0f : 0.0f, den);
                num = __builtin_fmaf(t1, v1 ? hiv[q] : 0.0f, num);
                den = __builtin_fmaf(t1, v1 ? 1.0f : 0.0f, den);
            }
            val = den > 0.0f ? num * __builtin_amdgcn_rcpf(den) : __builtin_nanf("");
        }
        *out = val;
    }
}

// A 16 x 16 tile of a request that gathers per pixel (mode 2) or has no surviving bin (mode 0):
// one pixel per thread.
template <int DT>
__device__ __forceinline__ void direct_tile(const SliceRec& rec, int t) {
    const int tiles_x = ui(rec.tiles_x);
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int i = tx * 16 + ((int)threadIdx.x & 15), j = ty * 16 + ((int)threadIdx.x >> 4);
    if (i >= rec.W || j >= rec.H) return;
    const gptr<float> out = global(rec.out) + (size_t)j * rec.W + i;
    const int n[3] = {rec.vol.n[0], rec.vol.n[1], rec.vol.n[2]};
    double c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = fma((double)j, rec.ey[a], fma((double)i, rec.ex[a], rec.c00[a]));
    if (rec.mode == 0 || !(c[0] >= -1.0 && c[0] < (double)n[0] && c[1] >= -1.0 && c[1] < (double)n[1] &&
                           c[2] >= -1.0 && c[2] < (double)n[2])) {
        *out = __builtin_nanf("");
        return;
    }
    *out = pixel_direct<DT, 1>(rec.vol, rec, rec.kact, c);
}

// Every pixel of a staged tile that has nothing in reach: NaN.
template <int NT>
__device__ __forceinline__ void nan_tile(const SliceRec& rec, const TileRec& tr) {
    const int T = ui(rec.tile), shift = T == kTileBig ? 5 : 4;
    const int i0 = ui(tr.i0), j0 = ui(tr.j0), ni = ui(tr.ni), nj = ui(tr.nj), W = ui(rec.W);
    const gptr<float> out = global(rec.out);
    for (int idx = (int)threadIdx.x; idx < T * T; idx += NT) {
        const int li = idx & (T - 1), lj = idx >> shift;
        if (li < ni && lj < nj) out[(size_t)(j0 + lj) * W + (i0 + li)] = __builtin_nanf("");
    }
}

// The voxels phase of a staged tile whose slot-table entries `sl` are loaded (or in flight);
// `rec` and `tr` are the request's and the tile's records (LDS or global).  U listed voxels per
// thread and NB bins per round in the gather.  `last` runs before the barrier that ends the phase.
template <int DT, int NT, int U, int NB, class Last>
__device__ __forceinline__ void stage_voxels(const SliceRec& rec, const TileRec& tr, TileLds<DT>& tl,
                                             const int (&sl)[slots_per_thread<NT>()], Last&& last) {
    {   // every run entry starts NaN; the gather overwrites the listed voxels'
        const int nitems = (int)__umul24((uint32_t)ui(tr.ncols), (uint32_t)ui(tr.depth));
        const float4 nan4 = make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
        for (int i = 4 * (int)threadIdx.x; i < nitems; i += 4 * NT) *reinterpret_cast<float4*>(&tl.V[i]) = nan4;
    }
    if (threadIdx.x == 0) tl.nlist = 0;
    __syncthreads();
    switch (ui(rec.dax)) {
        case 0: classify_voxels<DT, 0, NT>(rec, tr, tl); break;
        case 1: classify_voxels<DT, 1, NT>(rec, tr, tl); break;
        default: classify_voxels<DT, 2, NT>(rec, tr, tl); break;
    }
    store_slots<DT, NT>(rec, tr, tl, sl);
    __syncthreads();
    gather_voxels<DT, NT, U, NB>(rec, tr, tl);
    last();
    __syncthreads();
}

// The pixels phase of a staged tile whose voxels phase is done.
template <int DT, int NT>
__device__ __forceinline__ void stage_tile_pixels(const SliceRec& rec, const TileRec& tr, const TileLds<DT>& tl) {
    switch (ui(rec.dax)) {
        case 0: stage_pixels<DT, 0, NT>(rec, tr, tl); break;
        case 1: stage_pixels<DT, 1, NT>(rec, tr, tl); break;
        default: stage_pixels<DT, 2, NT>(rec, tr, tl); break;
    }
}

// One tile, start to end.
template <int DT, int NT, int U, int NB>
__device__ __forceinline__ void run_tile(const SliceRec& rec, const TileRec& tr, TileLds<DT>& tl) {
    if (ui(tr.mode) != 1) {
        nan_tile<NT>(rec, tr);
        return;
    }
    int sl[slots_per_thread<NT>()];
    load_slots<NT>(rec, tr, sl);
    stage_voxels<DT, NT, U, NB>(rec, tr, tl, sl, [] {});
    stage_tile_pixels<DT, NT>(rec, tr, tl);
}

// Single reslice: one workgroup per 16 x 16 tile; wave 0 evaluates the request setup, then lane
// 0 the tile's record.
template <int DT>
__global__ void __launch_bounds__(256) k_reslice_tile(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ TileLds<DT> tl;
    __shared__ SliceRec rec;
    __shared__ TileRec tr;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    // the request setup on three waves at once: wave 0 the bins (Eq. 1, gates, Eq. 2), wave 1 the
    // plane and its frame, wave 2 this tile's pixels and voxel box (16 x 16 tiles); then the
    // parts that need them together
    double T[12];
    if (threadIdx.x < 64) {
        pad_bins(rec, slice_gates(vd, s, rec, T));
    } else if (threadIdx.x < 192) {
        slice_pose(vd, s, T);
        if (threadIdx.x == 64) {
            request_frame(vd, s, T, rec);
        } else if (threadIdx.x == 128) {
            // the plane's position in voxel units, as request_frame computes it
            const double inv_h = vd->inv_h;
            double c00[3], ex[3], ey[3];
            const int n[3] = {vd->nx, vd->ny, vd->nz};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                c00[a] = (T[a * 4 + 3] - vd->origin[a]) * inv_h;
                ex[a] = (s.sx * T[a * 4 + 0]) * inv_h;
                ey[a] = (s.sy * T[a * 4 + 1]) * inv_h;
            }
            tile_box(c00, ex, ey, n, 16, s.W, s.H, (s.W + 15) / 16, 0, t, tr);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Plane pl = plane_of(rec);
        if (request_mode(pl, rec, 16) == 1) {
            tile_frame(pl, tr);
            tile_bins(pl.kact, tr);
        }
    }
    __syncthreads();
    if (ui(rec.mode) == 1) run_tile<DT, 256, items_per_round<DT>(), bins_per_round<DT>()>(rec, tr, tl);
    else direct_tile<DT>(rec, t);
}

// Batch setup: one workgroup per request.  Its first wave writes the request record, then every
// thread writes the records of tiles (one at a time) when it stages them; the units are appended: staged tiles' records from the front
// of `tiles` (counts[0]), the other requests' units (request, tile) from the back of `units`
// (counts[2]: entry k at cap - 1 - k), so that each kind runs in a kernel of its own.
__global__ void __launch_bounds__(kSetupThreads) k_tiles_setup(const BatchReq* __restrict__ reqs,
                                                               SliceRec* __restrict__ recs, int2* __restrict__ units,
                                                               TileRec* __restrict__ tiles, int* __restrict__ counts,
                                                               int cap) {
    __shared__ SliceRec rec;
    __shared__ int sh[3];                 // units, mode, first entry of the request's units
    const int nreq = counts[1];
    for (int r = blockIdx.x; r < nreq; r += gridDim.x) {
        if (threadIdx.x < 64) {
            int mode = 0;
            int nt = request_setup(reqs[r].vol, reqs[r].s, rec, kTileBig, &mode);
            if (threadIdx.x == 0) {
                // a request with no surviving bin is filled with NaN in flat runs of kFillRun
                // pixels (fewer units than its tiles), marked by a negative tile index
                if (mode == 0) nt = (int)(((int64_t)reqs[r].s.W * reqs[r].s.H + kFillRun - 1) / kFillRun);
                sh[0] = nt;
                sh[1] = mode;
                sh[2] = atomicAdd(counts + (mode == 1 ? 0 : 2), nt);
            }
        }
        __syncthreads();
        const int nt = sh[0], mode = sh[1], base = sh[2];
        {   // the record to global memory (the tile kernels read it)
            const int* src = reinterpret_cast<const int*>(&rec);
            int* dst = reinterpret_cast<int*>(recs + r);
            for (int w = threadIdx.x; w < (int)(sizeof(SliceRec) / sizeof(int)); w += kSetupThreads) dst[w] = src[w];
        }
        if (mode == 1) {
            const Plane pl = plane_of(rec);
            for (int k = threadIdx.x; k < nt; k += kSetupThreads) compute_tile(pl, r, k, tiles[base + k]);
        } else {
            for (int k = threadIdx.x; k < nt; k += kSetupThreads)
                units[cap - 1 - (base + k)] = make_int2(r, mode == 0 ? ~k : k);
        }
        __syncthreads();
    }
}

// Waves per SIMD that the LDS of a batch tile workgroup allows (the register budget is held to it).
template <int DT>
constexpr int tiles_waves_per_eu() {
    return (160 * 1024 / (int)sizeof(TileLds<DT>)) * (kThreadsBatch / 64) / 4;
}

// The k-th tile of XCD x: the XCDs take blocks of kTileBlock consecutive tiles of the list in
// turn.  Neighbouring tiles of a request, which share the voxels along their edges, mostly fall
// in one block and so are read through one L2, while the blocks spread each request's cost (its
// surviving bins, how much of it leaves the grid) over all XCDs.
constexpr int kTileBlock = 32;
__device__ __forceinline__ int xcd_tile(int x, int k) {
    return ((k / kTileBlock) * 8 + x) * kTileBlock + (k % kTileBlock);
}

// Batch tiles: a persistent grid over the staged tiles.  Workgroups are dealt to the 8 XCDs
// round-robin; XCD x's workgroups claim its tiles one at a time from its counter in the batch
// header, so that a workgroup that drew cheap tiles (few surviving bins, pixels outside the grid)
// takes more.  A workgroup's first claim is implicit (k = its rank in the XCD); the others come
// from the counter, offset by the number of workgroups per XCD, and each is issued at the start
// of the tile before it, so that its latency overlaps that tile's voxels phase.  Claims grow with
// k and so do their tiles: a workgroup stops at its first claim past the list.  Both records are
// read through scalar loads.
template <int DT>
__global__ void __launch_bounds__(kThreadsBatch) __attribute__((amdgpu_waves_per_eu(tiles_waves_per_eu<DT>())))
k_tiles(const SliceRec* __restrict__ recs, const TileRec* __restrict__ tiles, int* __restrict__ counts) {
    constexpr int NT = kThreadsBatch;
    __shared__ TileLds<DT> tl;
    __shared__ int take;
    const int n = counts[0];
    const int x = blockIdx.x & 7, per = gridDim.x >> 3;
    int* claims = counts + kClaimStride * (1 + x);
    // the slot-table entries of the next staged tile are read before the pixels phase of the
    // current one, so that their latency overlaps it
    int sl[slots_per_thread<NT>()];
    int u = xcd_tile(x, (int)(blockIdx.x >> 3));
    if (u < n && ui(tiles[u].mode) == 1) load_slots<NT>(recs[ui(tiles[u].r)], tiles[u], sl);
    while (u < n) {
        int k = 0;
        if (threadIdx.x == 0) k = per + atomicAdd(claims, 1);
        const TileRec& tr = tiles[u];
        const SliceRec& rec = recs[ui(tr.r)];
        const bool staged = ui(tr.mode) == 1;
        auto next = [&] {
            if (threadIdx.x == 0) take = xcd_tile(x, k);
        };
        if (staged) {
            stage_voxels<DT, NT, batch_items_per_round<DT>(), batch_bins_per_round<DT>()>(rec, tr, tl, sl, next);
        } else {
            next();
            __syncthreads();
        }
        const int un = ui(take);
        if (un < n && ui(tiles[un].mode) == 1) load_slots<NT>(recs[ui(tiles[un].r)], tiles[un], sl);
        if (staged) stage_tile_pixels<DT, NT>(rec, tr, tl);
        else nan_tile<NT>(rec, tr);
        __syncthreads();
        u = un;
    }
}

// Batch units of requests that gather per pixel (16 x 16 tiles) or have no surviving bin (runs of
// kFillRun pixels, negative tile index): the back of the unit list.
template <int DT>
__global__ void __launch_bounds__(256) k_tiles_direct(const SliceRec* __restrict__ recs,
                                                      const int2* __restrict__ units, const int* __restrict__ counts,
                                                      int cap) {
    const int n = counts[2];
    for (int u = blockIdx.x; u < n; u += gridDim.x) {
        const int2 un = units[cap - 1 - u];
        const int r = ui(un.x), t = ui(un.y);
        const SliceRec& rec = recs[r];
        if (t < 0) {
            const int64_t npx = (int64_t)rec.W * rec.H, p0 = (int64_t)(~t) * kFillRun;
            const int64_t p1 = p0 + kFillRun < npx ? p0 + kFillRun : npx;
            const gptr<float> out = global(rec.out);
            for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) out[p] = __builtin_nanf("");
        } else {
            direct_tile<DT>(rec, t);
        }
    }
}

// Workgroups of the persistent tile kernel: as many as the device holds at once (a static
// share of the units per workgroup), rounded down to whole rounds over the 8 XCDs.
template <int DT>
int tiles_grid() {
    static int grid[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (grid[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tiles<DT>, kThreadsBatch, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 8;
        grid[dev] = std::max(8, per_cu * cus / 8 * 8);
    }
    return grid[dev];
}

}  // namespace

static_assert(sizeof(SliceRec) % sizeof(int) == 0, "the record is copied in 4-byte words");

hipError_t launch_reslice_tile(const VolDev* vd, int dtype, const SliceArgs& s, hipStream_t stream) {
    const int64_t units = (int64_t)((s.W + 15) / 16) * ((s.H + 15) / 16);
    if (units > INT32_MAX) return hipErrorInvalidValue;
#define L(D) hipLaunchKernelGGL(k_reslice_tile<D>, dim3((unsigned)units), dim3(256), 0, stream, vd, s)
    DARE_DISPATCH_DT(dtype, L)
#undef L
    return hipGetLastError();
}

hipError_t launch_tiles_batch(int dtype, const BatchReq* reqs, SliceRec* recs, int2* units, TileRec* tiles,
                              int* counts, int nreq_max, int cap, hipStream_t stream) {
    const int sgrid = nreq_max < 1024 ? (nreq_max > 0 ? nreq_max : 1) : 1024;
    hipLaunchKernelGGL(k_tiles_setup, dim3(sgrid), dim3(kSetupThreads), 0, stream, reqs, recs, units, tiles, counts,
                       cap);
#define L(D)                                                                                                   \
    hipLaunchKernelGGL(k_tiles<D>, dim3(tiles_grid<D>()), dim3(kThreadsBatch), 0, stream, recs, tiles, counts); \
    hipLaunchKernelGGL(k_tiles_direct<D>, dim3(1024), dim3(256), 0, stream, recs, units, counts, cap)
    DARE_DISPATCH_DT(dtype, L)
#undef L
    return hipGetLastError();
}

int64_t tile_units_max(int W, int H) { return (int64_t)((W + 15) / 16) * ((H + 15) / 16); }

}  // namespace dare
