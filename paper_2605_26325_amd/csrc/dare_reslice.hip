// Directionality-aware reslice kernels (Sec. 2.1 "Reslicing", Eq. 1, Eq. 2, Fig. 2).
//
// One workgroup reslices one unit of one request: a 16x16 pixel tile when the
// interpolation radius is one voxel, otherwise a run of pixels that G lanes
// share (each lane takes some rows of the (2R)^3 neighbourhood and the lanes'
// partial sums are combined with wavefront shuffles).
//
// Per workgroup, wave 0 composes the slice pose with the calibration (FP64),
// evaluates Eq. 1 for every direction bin, drops the bins beyond either
// angular threshold and evaluates Eq. 2 for the rest, compacting the
// survivors into a small LDS table.  Then every lane computes its pixel's
// FP64 position, gathers the neighbourhood voxels of each surviving bin from
// the bin-major brick pool, blends each voxel over directions
// (V = sum w c a / sum w c), and blends voxels with tent weights, skipping
// voxels with no surviving sample.  A pixel with nothing left is NaN.
#include "dare_reslice_dev.h"

namespace dare {

namespace {

// ---------------------------------------------------------------- radius 1: trilinear cell
//
// The per-voxel direction blend V_v = sum_b w_b c_vb a_vb / sum_b w_b c_vb does
// not depend on the pixel, so a workgroup blends every voxel its 16x16 tile
// touches once and keeps the result in LDS (NaN = no surviving sample); each
// pixel then blends the 8 values of its cell with tent weights.
//
// The voxels a tile touches lie within |m.(v - c)| < |m|_1 of the slice plane
// (m its unit normal, in voxel units) and within the tile's lateral extent
// widened by the same support.  They are enumerated as short runs along the
// normal's dominant axis, one run per column of the other two axes, so the
// staging work follows the footprint rather than the tile's bounding box.
// All surviving bins of a voxel are loaded before any is accumulated, to keep
// several gathers in flight.  Tiles whose bounding box exceeds the LDS budget
// (coarse output pitch, where neighbouring pixels share few voxels) gather per
// pixel instead.
constexpr int kBoxMax = 3072;        // LDS values per tile (its clamped voxel box)
constexpr int kBoxEdgeMax = 17;      // voxels per axis: the box spans at most 3 bricks
constexpr int kSlotMax = 1024;       // (surviving bin, box brick) slots resolved per tile

// Box sizes that the staging phases divide by: bricks of the box, bricks along x and y, run
// depth, columns along p, voxels along x and y.
enum { kDivNbb, kDivBdx, kDivBdy, kDivDepth, kDivDp, kDivDx, kDivDy };

template <int DT>
struct TileLds {
    int mode;                        // 0: nothing in reach, 1: staged, 2: per-pixel gather
    int lo[3], dim[3];
    int blo[3], bdim[3], nbb;
    int dax, pax, qax;               // dominant normal axis, the other two
    int depth, ncols;
    // divisions by the box's sizes (dividends below kBoxMax), indexed by the kDiv* names
    SmallDiv div[7];
    float m[3], c0[3], ua[3], va[3];
    float thr_n, thr_u, thr_v, len_u, len_v, inv_md, half;
    int nlist;                       // staged voxels (compacted)
    int slot[kSlotMax];
    float2 scale[DT == DARE_FP8_E4M3 ? kSlotMax : 1];
    float V[kBoxMax];
    unsigned short list[kBoxMax];    // box index of each voxel to stage
};

// Wave 0: the tile's voxel box and work decomposition.  Lanes 0..3 place the
// tile's four corner pixels (FP64); positions are affine in (i, j), so their
// cells bound every pixel's cell (one voxel of margin per side absorbs
// rounding).  Lane 0 derives the footprint tests from the slice's plane frame.
template <int DT>
__device__ __forceinline__ void tile_setup(const VolView& vd, const SliceArgs& s, const double T[12],
                                           const SetupLds& sh, int kact, int i0, int j0, TileLds<DT>& tl) {
    const int lane = threadIdx.x;
    const int i1 = min(i0 + kTile - 1, s.W - 1), j1 = min(j0 + kTile - 1, s.H - 1);
    SlicePos q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = T[a * 4 + 3];
        q.e0[a] = T[a * 4 + 0];
        q.e1[a] = T[a * 4 + 1];
        q.o[a] = vd.origin[a];
    }
    q.inv_h = vd.inv_h;
    q.sx = s.sx;
    q.sy = s.sy;
    const int n[3] = {vd.n[0], vd.n[1], vd.n[2]};
    const int k = lane & 3;
    double c[3];
    pixel_coords(q, (k & 1) ? i1 : i0, (k & 2) ? j1 : j0, c);
    int lo[3], hi[3];
    float c0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int f = (int)fmin(fmax(floor(c[a]), -1048576.0), 1048576.0);
        // every lane of a group of 4 takes all four corners, so every lane holds the box
        int mn = __shfl(f, 0, 4), mx = mn;
#pragma unroll
        for (int o = 1; o < 4; ++o) {
            const int g = __shfl(f, o, 4);
            mn = min(mn, g);
            mx = max(mx, g);
        }
        lo[a] = max(mn - 1, 0);
        hi[a] = min(mx + 2, n[a] - 1);
        c0[a] = (float)__shfl(c[a], 0, 4);
    }
    // lanes 0..6 set up one division each, in parallel
    const int dax = sh.dax;
    float l1m = 0.0f;
    int dd[3], bd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        l1m += fabsf(sh.fm[a]);
        dd[a] = max(hi[a] - lo[a] + 1, 0);
        bd[a] = dd[a] > 0 ? (hi[a] >> 3) - (lo[a] >> 3) + 1 : 0;
    }
    // a column's voxels within the slab are the integers in (centre - half, centre + half), at
    // most ceil(2 half) of them; half carries the slop that covers the FP32 rounding of centre
    const float half = (l1m + 2e-3f) * fabsf(1.0f / sh.fm[dax]);
    const int depth = (int)ceilf(2.0f * half);
    if (lane < 7) {
        const int dv = lane == kDivNbb ? bd[0] * bd[1] * bd[2] : lane == kDivBdx ? bd[0] : lane == kDivBdy ? bd[1]
                     : lane == kDivDepth ? depth : lane == kDivDp ? dd[dax == 0 ? 1 : 0]
                     : lane == kDivDx ? dd[0] : dd[1];
        tl.div[lane] = small_div(dv);
    }
    if (lane != 0) return;
    int mode = kact > 0 ? 1 : 0;
    int nvox = 1, nbb = 1;
    float l1u = 0.0f, l1w = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (lo[a] > hi[a]) mode = 0;
        const int d = hi[a] - lo[a] + 1;
        tl.lo[a] = lo[a];
        tl.dim[a] = d > 0 ? d : 0;
        if (d > kBoxEdgeMax) mode = mode ? 2 : 0;
        nvox *= tl.dim[a];
        tl.blo[a] = lo[a] >> 3;
        tl.bdim[a] = d > 0 ? (hi[a] >> 3) - (lo[a] >> 3) + 1 : 0;
        nbb *= tl.bdim[a];
        tl.m[a] = sh.fm[a];
        tl.ua[a] = sh.fu[a];
        tl.va[a] = sh.fw[a];
        tl.c0[a] = c0[a];
        l1u += fabsf(sh.fu[a]);
        l1w += fabsf(sh.fw[a]);
    }
    if (mode == 1 && (nvox > kBoxMax || kact * nbb > kSlotMax)) mode = 2;
    tl.mode = mode;
    tl.nbb = nbb;
    // every voxel with non-zero weight for a pixel of the tile satisfies, for c0 the
    // tile's first pixel: |m.(v - c0)| < |m|_1, and ua.(v - c0), va.(v - c0) within the
    // tile's extent widened by |ua|_1, |va|_1 (margins cover FP32 rounding and the
    // pose rigidity tolerance)
    tl.thr_n = l1m + 2e-3f;
    tl.thr_u = l1u + 0.02f;
    tl.thr_v = l1w + 0.02f;
    tl.len_u = (float)(i1 - i0) * sh.lu;
    tl.len_v = (float)(j1 - j0) * sh.lw;
    tl.dax = dax;
    tl.pax = dax == 0 ? 1 : 0;
    tl.qax = dax == 2 ? 1 : 2;
    tl.inv_md = 1.0f / sh.fm[dax];
    tl.half = half;
    tl.depth = mode == 1 ? depth : 0;
    tl.ncols = mode == 1 ? tl.dim[tl.pax] * tl.dim[tl.qax] : 0;
    tl.nlist = 0;
}

// Blend one staged voxel over the surviving bins; NaN when none holds a sample.
template <int DT>
__device__ __forceinline__ float blend_voxel(const typename Pair<DT>::T* __restrict__ data, const SetupLds& sh,
                                             const TileLds<DT>& tl, int kact, int bb, int local) {
    using PT = Pair<DT>;
    const int nbb = tl.nbb;
    if (kact == 1) {
        const int slot = tl.slot[bb];
        if (slot < 0) return __builtin_nanf("");
        float2 sc = make_float2(0.0f, 0.0f);
        if constexpr (DT == DARE_FP8_E4M3) sc = tl.scale[bb];
        float a, cnt;
        PT::decode(data[(size_t)slot * kBrickVox + local], sc, a, cnt);
        return cnt > 0.0f ? a : __builtin_nanf("");
    }
    float A = 0.0f, B = 0.0f;
    for (int k0 = 0; k0 < kact; k0 += kBinChunk) {
        int sl[kBinChunk];
        typename PT::T p[kBinChunk];
#pragma unroll
        for (int u = 0; u < kBinChunk; ++u) sl[u] = (k0 + u < kact) ? tl.slot[(k0 + u) * nbb + bb] : -1;
#pragma unroll
        for (int u = 0; u < kBinChunk; ++u)
            if (sl[u] >= 0) p[u] = data[(size_t)sl[u] * kBrickVox + local];
#pragma unroll
        for (int u = 0; u < kBinChunk; ++u) {
            if (sl[u] < 0) continue;
            float2 sc = make_float2(0.0f, 0.0f);
            if constexpr (DT == DARE_FP8_E4M3) sc = tl.scale[(k0 + u) * nbb + bb];
            float a, cnt;
            PT::decode(p[u], sc, a, cnt);
            const float wc = sh.act_w[k0 + u] * cnt;
            A = __builtin_fmaf(wc, a, A);
            B = B + wc;
        }
    }
    return B > 0.0f ? A / B : __builtin_nanf("");
}

// Two staged voxels at once (a tile listing more voxels than threads): the pair loads of both
// are issued before either is accumulated, so the pair costs one memory round trip per chunk
// of kPairChunk bins instead of one per voxel.  Per voxel the arithmetic and its order are
// blend_voxel's.
constexpr int kPairChunk = 8;

template <int DT>
__device__ __forceinline__ void blend_voxel_pair(const typename Pair<DT>::T* __restrict__ data, const SetupLds& sh,
                                                 const TileLds<DT>& tl, int kact, int bbA, int locA, int bbB,
                                                 int locB, bool two, float& VA, float& VB) {
    using PT = Pair<DT>;
    const int nbb = tl.nbb;
    if (kact == 1) {
        const int sA = tl.slot[bbA], sB = two ? tl.slot[bbB] : -1;
        typename PT::T pA, pB;
        if (sA >= 0) pA = data[(size_t)sA * kBrickVox + locA];
        if (sB >= 0) pB = data[(size_t)sB * kBrickVox + locB];
        float2 scA = make_float2(0.0f, 0.0f), scB = make_float2(0.0f, 0.0f);
        if constexpr (DT == DARE_FP8_E4M3) {
            scA = tl.scale[bbA];
            if (two) scB = tl.scale[bbB];
        }
        float a, cnt;
        VA = __builtin_nanf("");
        VB = __builtin_nanf("");
        if (sA >= 0) {
            PT::decode(pA, scA, a, cnt);
            VA = cnt > 0.0f ? a : __builtin_nanf("");
        }
        if (sB >= 0) {
            PT::decode(pB, scB, a, cnt);
            VB = cnt > 0.0f ? a : __builtin_nanf("");
        }
        return;
    }
    float A0 = 0.0f, B0 = 0.0f, A1 = 0.0f, B1 = 0.0f;
    for (int k0 = 0; k0 < kact; k0 += kPairChunk) {
        int slA[kPairChunk], slB[kPairChunk];
        typename PT::T pA[kPairChunk], pB[kPairChunk];
#pragma unroll
        for (int u = 0; u < kPairChunk; ++u) {
            slA[u] = (k0 + u < kact) ? tl.slot[(k0 + u) * nbb + bbA] : -1;
            slB[u] = (two && k0 + u < kact) ? tl.slot[(k0 + u) * nbb + bbB] : -1;
        }
#pragma unroll
        for (int u = 0; u < kPairChunk; ++u) {
            if (slA[u] >= 0) pA[u] = data[(size_t)slA[u] * kBrickVox + locA];
            if (slB[u] >= 0) pB[u] = data[(size_t)slB[u] * kBrickVox + locB];
        }
#pragma unroll
        for (int u = 0; u < kPairChunk; ++u) {
            const float w = sh.act_w[k0 + u < kact ? k0 + u : 0];
            if (slA[u] >= 0) {
                float2 sc = make_float2(0.0f, 0.0f);
                if constexpr (DT == DARE_FP8_E4M3) sc = tl.scale[(k0 + u) * nbb + bbA];
                float a, cnt;
                PT::decode(pA[u], sc, a, cnt);
                const float wc = w * cnt;
                A0 = __builtin_fmaf(wc, a, A0);
                B0 = B0 + wc;
            }
            if (slB[u] >= 0) {
                float2 sc = make_float2(0.0f, 0.0f);
                if constexpr (DT == DARE_FP8_E4M3) sc = tl.scale[(k0 + u) * nbb + bbB];
                float a, cnt;
                PT::decode(pB[u], sc, a, cnt);
                const float wc = w * cnt;
                A1 = __builtin_fmaf(wc, a, A1);
                B1 = B1 + wc;
            }
        }
    }
    VA = B0 > 0.0f ? A0 / B0 : __builtin_nanf("");
    VB = B1 > 0.0f ? A1 / B1 : __builtin_nanf("");
}

// Phase (b) of a staged tile whose normal's dominant axis is DAX: the box voxels within the
// slab and lateral extent of the tile's pixels, enumerated as runs along DAX (one per column
// of the other two axes) and appended to the tile's list.
template <int DT, int DAX>
__device__ __forceinline__ void list_footprint(TileLds<DT>& tl) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    const int depth = tl.depth;
    const int nwork = tl.ncols * depth;
    const int lo[3] = {tl.lo[0], tl.lo[1], tl.lo[2]}, dim[3] = {tl.dim[0], tl.dim[1], tl.dim[2]};
    const float m[3] = {tl.m[0], tl.m[1], tl.m[2]}, c0[3] = {tl.c0[0], tl.c0[1], tl.c0[2]};
    const float ua[3] = {tl.ua[0], tl.ua[1], tl.ua[2]}, va[3] = {tl.va[0], tl.va[1], tl.va[2]};
    const float thr_n = tl.thr_n, thr_u = tl.thr_u, thr_v = tl.thr_v, len_u = tl.len_u, len_v = tl.len_v;
    const float inv_md = tl.inv_md, half = tl.half;
    const SmallDiv div_depth = tl.div[kDivDepth], div_dp = tl.div[kDivDp];
    for (int e = threadIdx.x; e < nwork; e += blockDim.x) {
        const int col = sdiv(e, div_depth), k = e - col * depth;
        const int cq = sdiv(col, div_dp);
        const int vp = lo[PAX] + (col - cq * div_dp.d), vq = lo[QAX] + cq;
        const float centre = c0[DAX] - (m[PAX] * ((float)vp - c0[PAX]) + m[QAX] * ((float)vq - c0[QAX])) * inv_md;
        // runs start at the first whole voxel above centre - half (or at the box floor)
        const int vdd = max((int)floorf(centre - half) + 1, lo[DAX]) + k;
        if (vdd >= lo[DAX] + dim[DAX]) continue;
        int v[3];
        v[DAX] = vdd;
        v[PAX] = vp;
        v[QAX] = vq;
        const float d0 = (float)v[0] - c0[0], d1 = (float)v[1] - c0[1], d2 = (float)v[2] - c0[2];
        const float dn = m[0] * d0 + m[1] * d1 + m[2] * d2;
        const float du = ua[0] * d0 + ua[1] * d1 + ua[2] * d2;
        const float dv = va[0] * d0 + va[1] * d1 + va[2] * d2;
        if (!(fabsf(dn) < thr_n && du > -thr_u && du < len_u + thr_u && dv > -thr_v && dv < len_v + thr_v))
            continue;
        const int idx = atomicAdd(&tl.nlist, 1);
        tl.list[idx] = (unsigned short)(((v[2] - lo[2]) * dim[1] + (v[1] - lo[1])) * dim[0] + (v[0] - lo[0]));
    }
}

// One 16x16 tile; the slice's setup (pose, surviving bins and weights, plane frame) is in `sh`.
template <int DT>
__device__ __forceinline__ void reslice_tile_r1(const VolView& vd, const SliceArgs& s, int unit, SetupLds& sh,
                                                TileLds<DT>& tl) {
    const int tx = unit % s.tiles_x, ty = unit / s.tiles_x;
    const int i0 = tx * kTile, j0 = ty * kTile;
    if (threadIdx.x < 64) {
        double T[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) T[k] = sh.T[k];
        tile_setup<DT>(vd, s, T, sh, sh.kact, i0, j0, tl);
    }
    __syncthreads();
    const int kact = uniform_i32(sh.kact);
    const int mode = uniform_i32(tl.mode);
    if (mode == 1) {
        // (a) brick slots (and FP8 scales) of every surviving bin over the box's bricks
        const int nbb = tl.nbb;
        const int64_t nbricks = vd.nbricks;
        const SmallDiv div_nbb = tl.div[kDivNbb], div_bdx = tl.div[kDivBdx], div_bdy = tl.div[kDivBdy];
        for (int e = threadIdx.x; e < kact * nbb; e += blockDim.x) {
            const int k = sdiv(e, div_nbb), r = e - k * nbb;
            const int byz = sdiv(r, div_bdx), bxx = r - byz * div_bdx.d;
            const int bzz = sdiv(byz, div_bdy), byy = byz - bzz * div_bdy.d;
            const int64_t brick = ((int64_t)(tl.blo[2] + bzz) * vd.nby + (tl.blo[1] + byy)) * vd.nbx + (tl.blo[0] + bxx);
            const int slot = vd.table[(int64_t)sh.act_bin[k] * nbricks + brick];
            tl.slot[e] = slot;
            if constexpr (DT == DARE_FP8_E4M3) tl.scale[e] = slot >= 0 ? vd.scales[slot] : make_float2(0.0f, 0.0f);
        }
        // (b) the voxels the tile touches, compacted into a list (ALU work only)
        switch (uniform_i32(tl.dax)) {
            case 0: list_footprint<DT, 0>(tl); break;
            case 1: list_footprint<DT, 1>(tl); break;
            default: list_footprint<DT, 2>(tl); break;
        }
        __syncthreads();
        // (c) one thread per listed voxel (two when the list is longer than the workgroup): all
        // bins' gathers in flight at once, then the blend
        const typename Pair<DT>::T* __restrict__ data = (const typename Pair<DT>::T*)vd.data;
        const int nlist = uniform_i32(tl.nlist);
        const int dxb = tl.dim[0], dyb = tl.dim[1];
        const int lox = tl.lo[0], loy = tl.lo[1], loz = tl.lo[2];
        const int bx0 = tl.blo[0], by0 = tl.blo[1], bz0 = tl.blo[2], bdx = tl.bdim[0], bdy = tl.bdim[1];
        const SmallDiv div_dx = tl.div[kDivDx], div_dy = tl.div[kDivDy];
        auto locate = [&](int bi, int& bb, int& local) {
            const int eyz = sdiv(bi, div_dx), ex = bi - eyz * dxb;
            const int ez = sdiv(eyz, div_dy), ey = eyz - ez * dyb;
            const int vx = lox + ex, vy = loy + ey, vz = loz + ez;
            bb = (((vz >> 3) - bz0) * bdy + ((vy >> 3) - by0)) * bdx + ((vx >> 3) - bx0);
            local = brick_local(vx, vy, vz);
        };
        if (nlist <= (int)blockDim.x) {
            for (int e = threadIdx.x; e < nlist; e += blockDim.x) {
                const int bi = tl.list[e];
                int bb, local;
                locate(bi, bb, local);
                tl.V[bi] = blend_voxel<DT>(data, sh, tl, kact, bb, local);
            }
        } else {
            for (int e = threadIdx.x; e < nlist; e += 2 * blockDim.x) {
                const int e2 = e + blockDim.x;
                const bool two = e2 < nlist;
                const int biA = tl.list[e], biB = two ? tl.list[e2] : biA;
                int bbA, locA, bbB, locB;
                locate(biA, bbA, locA);
                locate(biB, bbB, locB);
                float VA, VB;
                blend_voxel_pair<DT>(data, sh, tl, kact, bbA, locA, bbB, locB, two, VA, VB);
                tl.V[biA] = VA;
                if (two) tl.V[biB] = VB;
            }
        }
        __syncthreads();
    }
    const int i = i0 + (threadIdx.x & (kTile - 1));
    const int j = j0 + (threadIdx.x >> 4);
    if (i >= s.W || j >= s.H) return;
    float* out = s.out + (size_t)j * s.W + i;
    if (mode == 0) {
        *out = __builtin_nanf("");
        return;
    }
    SlicePos q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = uniform_f64(sh.T[a * 4 + 3]);
        q.e0[a] = uniform_f64(sh.T[a * 4 + 0]);
        q.e1[a] = uniform_f64(sh.T[a * 4 + 1]);
        q.o[a] = vd.origin[a];
    }
    q.inv_h = vd.inv_h;
    q.sx = s.sx;
    q.sy = s.sy;
    const int nx = vd.n[0], ny = vd.n[1], nz = vd.n[2];
    double c[3];
    pixel_coords(q, i, j, c);
    if (!(c[0] >= -1.0 && c[0] < (double)nx && c[1] >= -1.0 && c[1] < (double)ny && c[2] >= -1.0 &&
          c[2] < (double)nz)) {
        *out = __builtin_nanf("");
        return;
    }
    if (mode == 2) {
        *out = pixel_direct<DT, 2>(vd, sh, kact, c);
        return;
    }
    const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
    const int x0 = (int)f0, y0 = (int)f1, z0 = (int)f2;
    const float fx = (float)(c[0] - f0), fy = (float)(c[1] - f1), fz = (float)(c[2] - f2);
    // per-axis tent weights of the cell's two voxels, 0 for a voxel outside the box (the box lies
    // inside the grid and holds every in-grid cell voxel of the tile); clamped box coordinates keep
    // every LDS read in bounds, and corners of weight 0 are skipped (only voxels with weight were
    // staged)
    const int e0[3] = {x0 - tl.lo[0], y0 - tl.lo[1], z0 - tl.lo[2]};
    const int dm[3] = {tl.dim[0], tl.dim[1], tl.dim[2]};
    const float fr[3] = {fx, fy, fz};
    float w[3][2];
    int cc[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w[a][0] = (unsigned)e0[a] < (unsigned)dm[a] ? 1.0f - fr[a] : 0.0f;
        w[a][1] = (unsigned)(e0[a] + 1) < (unsigned)dm[a] ? fr[a] : 0.0f;
        cc[a][0] = min(max(e0[a], 0), dm[a] - 1);
        cc[a][1] = min(max(e0[a] + 1, 0), dm[a] - 1);
    }
    float tw[8], Vc[8];
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) {                 // c8 = (dz << 2) | (dy << 1) | dx
        const int ddx = c8 & 1, ddy = (c8 >> 1) & 1, ddz = c8 >> 2;
        tw[c8] = (w[0][ddx] * w[1][ddy]) * w[2][ddz];
        Vc[c8] = tl.V[(cc[2][ddz] * dm[1] + cc[1][ddy]) * dm[0] + cc[0][ddx]];
    }
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) {
        if (tw[c8] > 0.0f && Vc[c8] == Vc[c8]) {
            num = __builtin_fmaf(tw[c8], Vc[c8], num);
            den = den + tw[c8];
        }
    }
    *out = den > 0.0f ? num / den : __builtin_nanf("");
}

}  // namespace


// The per-slice setup (FP64 pose, Eq. 1 gates and Eq. 2 weights, plane frame) is computed once on
// the host and arrives with the launch, with the volume's geometry and pointers; wave 0 copies the
// setup to LDS.
template <int DT>
__global__ void __launch_bounds__(256) k_reslice_r1(SliceArgs s, SliceCore core, VolView vd) {
    __shared__ SetupLds sh;
    __shared__ TileLds<DT> tl;
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        sh.act_bin[l] = core.act_bin[l];
        sh.act_w[l] = core.act_w[l];
        if (l < 12) sh.T[l] = core.T[l];
        if (l < 3) {
            sh.fm[l] = core.fm[l];
            sh.fu[l] = core.fu[l];
            sh.fw[l] = core.fw[l];
        }
        if (l == 0) {
            sh.lu = core.lu;
            sh.lw = core.lw;
            sh.dax = core.dax;
            sh.kact = core.kact;
        }
    }
    __syncthreads();
    reslice_tile_r1<DT>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh, tl);
}

// FP8 storage: the scale loads lift the register count just past the 128 that keeps four waves
// per SIMD (every tile of a 512^2 slice resident at once); capping it there, at the price of a few
// spilled registers, takes a launch from 17.4 to 12.4 us.  The other storage forms fit already,
// and the cap changes their schedule for the worse, so only this copy of the kernel carries it.
template <int DT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_reslice_r1_w4(SliceArgs s, SliceCore core, VolView vd) {
    __shared__ SetupLds sh;
    __shared__ TileLds<DT> tl;
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        sh.act_bin[l] = core.act_bin[l];
        sh.act_w[l] = core.act_w[l];
        if (l < 12) sh.T[l] = core.T[l];
        if (l < 3) {
            sh.fm[l] = core.fm[l];
            sh.fu[l] = core.fu[l];
            sh.fw[l] = core.fw[l];
        }
        if (l == 0) {
            sh.lu = core.lu;
            sh.lw = core.lw;
            sh.dax = core.dax;
            sh.kact = core.kact;
        }
    }
    __syncthreads();
    reslice_tile_r1<DT>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh, tl);
}

template <int DT, int G>
__global__ void __launch_bounds__(256) k_reslice_rn(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ SetupLds sh;
    reslice_unit_rn<DT, G>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// ---------------------------------------------------------------------------- launchers

int reslice_lanes(int radius) { return radius <= 1 ? 1 : (radius <= 2 ? 16 : 64); }

int64_t reslice_units(int radius, int W, int H) {
    if (radius <= 1) return (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    const int ppw = 256 / reslice_lanes(radius);
    return ((int64_t)W * H + ppw - 1) / ppw;
}

hipError_t launch_reslice(const VolDev* vd, int dtype, int radius, const SliceArgs& s, const SliceCore& core,
                          const VolView& view, hipStream_t stream) {
    const int64_t units = reslice_units(radius, s.W, s.H);
    const dim3 grid((unsigned)units), block(256);
    const int G = reslice_lanes(radius);
#define L1(D)                                                                                  \
    if constexpr (D == DARE_FP8_E4M3)                                                          \
        hipLaunchKernelGGL(k_reslice_r1_w4<D>, grid, block, 0, stream, s, core, view);         \
    else                                                                                       \
        hipLaunchKernelGGL(k_reslice_r1<D>, grid, block, 0, stream, s, core, view)
#define L16(D) hipLaunchKernelGGL((k_reslice_rn<D, 16>), grid, block, 0, stream, vd, s)
#define L64(D) hipLaunchKernelGGL((k_reslice_rn<D, 64>), grid, block, 0, stream, vd, s)
    if (G == 1) {
        DARE_DISPATCH_DT(dtype, L1)
    } else if (G == 16) {
        DARE_DISPATCH_DT(dtype, L16)
    } else {
        DARE_DISPATCH_DT(dtype, L64)
    }
#undef L1
#undef L16
#undef L64
    return hipGetLastError();
}

}  // namespace dare
