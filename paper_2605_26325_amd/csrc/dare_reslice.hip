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
#include <math.h>

#include "dare_codec.h"
#include "dare_internal.h"

#pragma clang fp contract(off)

namespace dare {

namespace {

using SetupLds = SliceSetup;

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ __forceinline__ double uniform_f64(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int uniform_i32(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Wave 0 only: slice pose, Eq. 1 / thresholds / Eq. 2 per bin, survivors compacted.
// Returns the number of surviving bins; T receives the composed pose (rows 0..2).
__device__ __forceinline__ int slice_setup(const VolDev* __restrict__ vd, const SliceArgs& s, SetupLds& sh,
                                           double T[12]) {
    const int lane = threadIdx.x;
    const double* P = s.P;
    const double* C = vd->calib;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = P[r * 4 + 0] * C[0 * 4 + c];
            acc = acc + P[r * 4 + 1] * C[1 * 4 + c];
            acc = acc + P[r * 4 + 2] * C[2 * 4 + c];
            acc = acc + P[r * 4 + 3] * C[3 * 4 + c];
            T[r * 4 + c] = acc;
        }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) sh.T[k] = T[k];
    }
    // every lane reads its representative unconditionally: one memory round trip, not two
    const int K = vd->st.K;
    double rn[3], rx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rn[a] = vd->rep_n[lane][a];
        rx[a] = vd->rep_x[lane][a];
    }
    const int ax = vd->normal_axis;
    const double e0[3] = {T[0], T[4], T[8]};
    const double en[3] = {T[ax], T[4 + ax], T[8 + ax]};
    const double l0 = sqrt(dot3(e0, e0));
    const double ln = sqrt(dot3(en, en));
    const double xr[3] = {e0[0] / l0, e0[1] / l0, e0[2] / l0};
    const double nr[3] = {en[0] / ln, en[1] / ln, en[2] / ln};
    bool keep = false;
    double w = 0.0;
    if (lane < K) {
        const double dn = dot3(rn, nr);
        const double di = fabs(dot3(rx, xr));
        keep = dn >= vd->cos_normal && di >= vd->cos_inplane;
        if (keep) w = exp(vd->k_normal * (dn - 1.0) + vd->k_inplane * (di - 1.0));
    }
    const unsigned long long m = __ballot(keep);
    if (keep) {
        const int idx = __popcll(m & ((1ull << lane) - 1ull));
        sh.act_bin[idx] = lane;
        sh.act_w[idx] = (float)w;
    }
    // plane frame in voxel units; it only drives conservative footprint tests, so FP32
    const double inv_h = vd->inv_h;
    float u[3], v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = (float)(T[a * 4 + 0] * s.sx * inv_h);
        v[a] = (float)(T[a * 4 + 1] * s.sy * inv_h);
    }
    const float lu = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const float lv = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    float nm[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    const float rm = 1.0f / sqrtf(nm[0] * nm[0] + nm[1] * nm[1] + nm[2] * nm[2]);
    int dax = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) nm[a] *= rm;
    if (fabsf(nm[1]) > fabsf(nm[dax])) dax = 1;
    if (fabsf(nm[2]) > fabsf(nm[dax])) dax = 2;
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sh.fm[a] = nm[a];
            sh.fu[a] = u[a] / lu;
            sh.fw[a] = v[a] / lv;
        }
        sh.lu = lu;
        sh.lw = lv;
        sh.dax = dax;
        sh.kact = __popcll(m);
    }
    return __popcll(m);
}

struct SlicePos {            // per-workgroup uniform position terms
    double t[3], e0[3], e1[3], o[3], inv_h, sx, sy;
};

__device__ __forceinline__ void load_pos(const VolDev* __restrict__ vd, const SetupLds& sh, const SliceArgs& s,
                                         SlicePos& q) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = uniform_f64(sh.T[a * 4 + 3]);
        q.e0[a] = uniform_f64(sh.T[a * 4 + 0]);
        q.e1[a] = uniform_f64(sh.T[a * 4 + 1]);
        q.o[a] = vd->origin[a];
    }
    q.inv_h = vd->inv_h;
    q.sx = s.sx;
    q.sy = s.sy;
}

// Continuous voxel coordinates of output pixel (i, j): c = (p - o) / h, p = (t + (i sx) e0) + (j sy) e1.
__device__ __forceinline__ void pixel_coords(const SlicePos& q, int i, int j, double c[3]) {
    const double is = (double)i * q.sx;
    const double js = (double)j * q.sy;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double p = (q.t[a] + is * q.e0[a]) + js * q.e1[a];
        c[a] = (p - q.o[a]) * q.inv_h;
    }
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    // consecutive units (neighbouring tiles of one slice) go to the same XCD's L2:
    // the dispatcher deals workgroups round-robin over the 8 XCDs.
    if ((nblocks & 7) != 0) return bid;
    return (bid & 7) * (nblocks >> 3) + (bid >> 3);
}

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
constexpr int kBinChunk = 16;        // gathers issued together per voxel

template <int DT>
struct TileLds {
    int mode;                        // 0: nothing in reach, 1: staged, 2: per-pixel gather
    int lo[3], dim[3];
    int blo[3], bdim[3], nbb;
    int dax, pax, qax;               // dominant normal axis, the other two
    int depth, ncols;
    float m[3], c0[3], ua[3], va[3];
    float thr_n, thr_u, thr_v, len_u, len_v, inv_md;
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
__device__ __forceinline__ void tile_setup(const VolDev* __restrict__ vd, const SliceArgs& s, const double T[12],
                                           const SetupLds& sh, int kact, int i0, int j0, TileLds<DT>& tl) {
    const int lane = threadIdx.x;
    const int i1 = min(i0 + kTile - 1, s.W - 1), j1 = min(j0 + kTile - 1, s.H - 1);
    SlicePos q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = T[a * 4 + 3];
        q.e0[a] = T[a * 4 + 0];
        q.e1[a] = T[a * 4 + 1];
        q.o[a] = vd->origin[a];
    }
    q.inv_h = vd->inv_h;
    q.sx = s.sx;
    q.sy = s.sy;
    const int n[3] = {vd->nx, vd->ny, vd->nz};
    const int k = lane & 3;
    double c[3];
    pixel_coords(q, (k & 1) ? i1 : i0, (k & 2) ? j1 : j0, c);
    int lo[3], hi[3];
    float c0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int f = (int)fmin(fmax(floor(c[a]), -1048576.0), 1048576.0);
        int mn = f, mx = f;
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
    if (lane != 0) return;
    int mode = kact > 0 ? 1 : 0;
    int nvox = 1, nbb = 1;
    float l1m = 0.0f, l1u = 0.0f, l1w = 0.0f;
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
        l1m += fabsf(sh.fm[a]);
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
    const int dax = sh.dax;
    tl.thr_n = l1m + 2e-3f;
    tl.thr_u = l1u + 0.02f;
    tl.thr_v = l1w + 0.02f;
    tl.len_u = (float)(i1 - i0) * sh.lu;
    tl.len_v = (float)(j1 - j0) * sh.lw;
    tl.dax = dax;
    tl.pax = dax == 0 ? 1 : 0;
    tl.qax = dax == 2 ? 1 : 2;
    tl.inv_md = 1.0f / sh.fm[dax];
    tl.depth = mode == 1 ? (int)ceilf(2.0f * (l1m + 2e-3f) / fabsf(sh.fm[dax])) + 2 : 0;
    tl.ncols = mode == 1 ? tl.dim[tl.pax] * tl.dim[tl.qax] : 0;
    tl.nlist = 0;
}

__device__ __forceinline__ VolView view_of(const VolDev* __restrict__ vd) {
    VolView v;
    v.table = vd->table;
    v.data = vd->data;
    v.scales = vd->scales;
    v.nbricks = vd->nbricks;
    v.n[0] = vd->nx;
    v.n[1] = vd->ny;
    v.n[2] = vd->nz;
    v.nbx = vd->nbx;
    v.nby = vd->nby;
#pragma unroll
    for (int a = 0; a < 3; ++a) v.origin[a] = vd->origin[a];
    v.inv_h = vd->inv_h;
    return v;
}

// Per-pixel gather of the 8 cell voxels over the surviving bins (no staging).  The whole
// workgroup works on one request: bin ids and weights are broadcast as scalars.  All loads of
// NB bins are issued before any is used (indices of absent voxels point at entry 0, which
// exists, and their values are discarded), so NB bins cost two memory round trips.
template <int DT, int NB>
__device__ __forceinline__ float pixel_direct(const VolView& vv, const SetupLds& sh, int kact, const double c[3]) {
    using PT = Pair<DT>;
    const int nx = vv.n[0], ny = vv.n[1], nz = vv.n[2];
    const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
    const int x0 = (int)f0, y0 = (int)f1, z0 = (int)f2;
    const float fx = (float)(c[0] - f0), fy = (float)(c[1] - f1), fz = (float)(c[2] - f2);
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
    const int nbx = vv.nbx, nby = vv.nby;
    int tix[8], lix[8];
    bool in[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {                  // v = (dz << 2) | (dy << 1) | dx
        const int vx = x0 + (v & 1), vy = y0 + ((v >> 1) & 1), vz = z0 + (v >> 2);
        in[v] = (unsigned)vx < (unsigned)nx && (unsigned)vy < (unsigned)ny && (unsigned)vz < (unsigned)nz;
        tix[v] = in[v] ? ((vz >> 3) * nby + (vy >> 3)) * nbx + (vx >> 3) : 0;
        lix[v] = (((vz & 7) << 3) | (vy & 7)) << 3 | (vx & 7);
    }
    const typename PT::T* __restrict__ data = (const typename PT::T*)vv.data;
    const int64_t nbricks = vv.nbricks;
    float A[8], B[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) { A[v] = 0.0f; B[v] = 0.0f; }
    for (int k0 = 0; k0 < kact; k0 += NB) {
        int sl[NB][8];
        typename PT::T pr[NB][8];
        float2 sc[NB][8];
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            const int b = uniform_i32(sh.act_bin[k0 + h < kact ? k0 + h : k0]);
            const int32_t* __restrict__ tab = vv.table + (int64_t)b * nbricks;
#pragma unroll
            for (int v = 0; v < 8; ++v) sl[h][v] = tab[tix[v]];
        }
#pragma unroll
        for (int h = 0; h < NB; ++h)
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int s0 = sl[h][v] >= 0 ? sl[h][v] : 0;
                pr[h][v] = data[(size_t)s0 * kBrickVox + lix[v]];
                sc[h][v] = make_float2(0.0f, 0.0f);
                if constexpr (DT == DARE_FP8_E4M3) sc[h][v] = vv.scales[s0];
            }
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            if (k0 + h >= kact) break;
            const float wgt = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sh.act_w[k0 + h])));
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                if (!in[v] || sl[h][v] < 0) continue;
                float a, cnt;
                PT::decode(pr[h][v], sc[h][v], a, cnt);
                if (kact == 1) {              // a single direction: its weight cancels, V = a
                    A[v] = a;
                    B[v] = cnt;
                } else {
                    const float wc = wgt * cnt;
                    A[v] = __builtin_fmaf(wc, a, A[v]);
                    B[v] = B[v] + wc;
                }
            }
        }
    }
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int v = (dz << 2) | (dy << 1) | dx;
                const float t = (wx[dx] * wy[dy]) * wz[dz];
                if (B[v] > 0.0f && t > 0.0f) {
                    num = __builtin_fmaf(t, kact == 1 ? A[v] : A[v] / B[v], num);
                    den = den + t;
                }
            }
    return den > 0.0f ? num / den : __builtin_nanf("");
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

// One 16x16 tile.  With have_setup the slice setup is already in `sh` (batched
// requests share one record computed by a pre-pass); otherwise wave 0 computes it.
template <int DT>
__device__ __forceinline__ void reslice_tile_r1(const VolDev* __restrict__ vd, const SliceArgs& s, int unit,
                                                SetupLds& sh, TileLds<DT>& tl, bool have_setup) {
    const int tx = unit % s.tiles_x, ty = unit / s.tiles_x;
    const int i0 = tx * kTile, j0 = ty * kTile;
    if (threadIdx.x < 64) {
        double T[12];
        int ka;
        if (have_setup) {
#pragma unroll
            for (int k = 0; k < 12; ++k) T[k] = sh.T[k];
            ka = sh.kact;
        } else {
            ka = slice_setup(vd, s, sh, T);
        }
        tile_setup<DT>(vd, s, T, sh, ka, i0, j0, tl);
    }
    __syncthreads();
    const int kact = uniform_i32(sh.kact);
    const int mode = uniform_i32(tl.mode);
    if (mode == 1) {
        // (a) brick slots (and FP8 scales) of every surviving bin over the box's bricks
        const int nbb = tl.nbb;
        const int64_t nbricks = vd->nbricks;
        for (int e = threadIdx.x; e < kact * nbb; e += blockDim.x) {
            const int k = e / nbb, r = e - k * nbb;
            const int bxx = r % tl.bdim[0], byz = r / tl.bdim[0];
            const int byy = byz % tl.bdim[1], bzz = byz / tl.bdim[1];
            const int64_t brick = ((int64_t)(tl.blo[2] + bzz) * vd->nby + (tl.blo[1] + byy)) * vd->nbx + (tl.blo[0] + bxx);
            const int slot = vd->table[(int64_t)sh.act_bin[k] * nbricks + brick];
            tl.slot[e] = slot;
            if constexpr (DT == DARE_FP8_E4M3) tl.scale[e] = slot >= 0 ? vd->scales[slot] : make_float2(0.0f, 0.0f);
        }
        // (b) the voxels the tile touches, compacted into a list (ALU work only)
        {
            const int dax = tl.dax, pax = tl.pax, qax = tl.qax, depth = tl.depth;
            const int nwork = tl.ncols * depth;
            const int lo[3] = {tl.lo[0], tl.lo[1], tl.lo[2]}, dim[3] = {tl.dim[0], tl.dim[1], tl.dim[2]};
            const float m[3] = {tl.m[0], tl.m[1], tl.m[2]}, c0[3] = {tl.c0[0], tl.c0[1], tl.c0[2]};
            const float ua[3] = {tl.ua[0], tl.ua[1], tl.ua[2]}, va[3] = {tl.va[0], tl.va[1], tl.va[2]};
            const float thr_n = tl.thr_n, thr_u = tl.thr_u, thr_v = tl.thr_v, len_u = tl.len_u, len_v = tl.len_v;
            const float inv_md = tl.inv_md, half = thr_n * fabsf(inv_md);
            for (int e = threadIdx.x; e < nwork; e += blockDim.x) {
                const int col = e / depth, k = e - col * depth;
                const int vp = lo[pax] + col % dim[pax], vq = lo[qax] + col / dim[pax];
                const float centre = c0[dax] - (m[pax] * ((float)vp - c0[pax]) + m[qax] * ((float)vq - c0[qax])) * inv_md;
                // runs start one below the slab (or at the box floor): depth covers the whole slab
                const int vdd = max((int)floorf(centre - half), lo[dax]) + k;
                if (vdd >= lo[dax] + dim[dax]) continue;
                const int vx = dax == 0 ? vdd : (pax == 0 ? vp : vq);
                const int vy = dax == 1 ? vdd : (pax == 1 ? vp : vq);
                const int vz = dax == 2 ? vdd : (pax == 2 ? vp : vq);
                const float d0 = (float)vx - c0[0], d1 = (float)vy - c0[1], d2 = (float)vz - c0[2];
                const float dn = m[0] * d0 + m[1] * d1 + m[2] * d2;
                const float du = ua[0] * d0 + ua[1] * d1 + ua[2] * d2;
                const float dv = va[0] * d0 + va[1] * d1 + va[2] * d2;
                if (!(fabsf(dn) < thr_n && du > -thr_u && du < len_u + thr_u && dv > -thr_v && dv < len_v + thr_v))
                    continue;
                const int idx = atomicAdd(&tl.nlist, 1);
                tl.list[idx] = (unsigned short)(((vz - lo[2]) * dim[1] + (vy - lo[1])) * dim[0] + (vx - lo[0]));
            }
        }
        __syncthreads();
        // (c) one thread per listed voxel: all its bins' gathers in flight at once, then the blend
        const typename Pair<DT>::T* __restrict__ data = (const typename Pair<DT>::T*)vd->data;
        const int nlist = tl.nlist;
        const int dxb = tl.dim[0], dyb = tl.dim[1];
        const int lox = tl.lo[0], loy = tl.lo[1], loz = tl.lo[2];
        const int bx0 = tl.blo[0], by0 = tl.blo[1], bz0 = tl.blo[2], bdx = tl.bdim[0], bdy = tl.bdim[1];
        for (int e = threadIdx.x; e < nlist; e += blockDim.x) {
            const int bi = tl.list[e];
            const int ex = bi % dxb, eyz = bi / dxb;
            const int vx = lox + ex, vy = loy + eyz % dyb, vz = loz + eyz / dyb;
            const int bb = (((vz >> 3) - bz0) * bdy + ((vy >> 3) - by0)) * bdx + ((vx >> 3) - bx0);
            const int local = (((vz & 7) << 3) | (vy & 7)) << 3 | (vx & 7);
            tl.V[bi] = blend_voxel<DT>(data, sh, tl, kact, bb, local);
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
    load_pos(vd, sh, s, q);
    const int nx = vd->nx, ny = vd->ny, nz = vd->nz;
    double c[3];
    pixel_coords(q, i, j, c);
    if (!(c[0] >= -1.0 && c[0] < (double)nx && c[1] >= -1.0 && c[1] < (double)ny && c[2] >= -1.0 &&
          c[2] < (double)nz)) {
        *out = __builtin_nanf("");
        return;
    }
    if (mode == 2) {
        *out = pixel_direct<DT, 2>(view_of(vd), sh, kact, c);
        return;
    }
    const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
    const int x0 = (int)f0, y0 = (int)f1, z0 = (int)f2;
    const float fx = (float)(c[0] - f0), fy = (float)(c[1] - f1), fz = (float)(c[2] - f2);
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
    const int lox = tl.lo[0], loy = tl.lo[1], loz = tl.lo[2], dx = tl.dim[0], dy = tl.dim[1], dz = tl.dim[2];
    // indices first, then all 8 LDS reads at once (absent corners read entry 0 and are discarded)
    float tw[8], Vc[8];
    int ix[8];
    bool ok[8];
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) {                 // c8 = (dz << 2) | (dy << 1) | dx
        const int ddx = c8 & 1, ddy = (c8 >> 1) & 1, ddz = c8 >> 2;
        tw[c8] = (wx[ddx] * wy[ddy]) * wz[ddz];      // only voxels with weight were staged
        const int vx = x0 + ddx, vy = y0 + ddy, vz = z0 + ddz;
        const int ex = vx - lox, ey = vy - loy, ez = vz - loz;
        // the box holds every in-grid cell voxel of the tile: its test only bounds the index
        ok[c8] = tw[c8] > 0.0f && (unsigned)vx < (unsigned)nx && (unsigned)vy < (unsigned)ny &&
                 (unsigned)vz < (unsigned)nz && (unsigned)ex < (unsigned)dx && (unsigned)ey < (unsigned)dy &&
                 (unsigned)ez < (unsigned)dz;
        ix[c8] = ok[c8] ? (ez * dy + ey) * dx + ex : 0;
    }
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) Vc[c8] = tl.V[ix[c8]];
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) {
        if (ok[c8] && Vc[c8] == Vc[c8]) {
            num = __builtin_fmaf(tw[c8], Vc[c8], num);
            den = den + tw[c8];
        }
    }
    *out = den > 0.0f ? num / den : __builtin_nanf("");
}

// ---------------------------------------------------------------- radius R >= 2: lane-split neighbourhood
template <int DT, int G>
__device__ __forceinline__ void reslice_unit_rn(const VolDev* __restrict__ vd, const SliceArgs& s, int unit,
                                                SetupLds& sh) {
    using PT = Pair<DT>;
    constexpr int PPW = 256 / G;   // pixels per workgroup
    if (threadIdx.x < 64) {
        double T[12];
        slice_setup(vd, s, sh, T);
    }
    __syncthreads();
    SlicePos q;
    load_pos(vd, sh, s, q);
    const int kact = uniform_i32(sh.kact);
    const int R = vd->radius;
    const float invR = 1.0f / (float)R;
    const int g = threadIdx.x % G;
    const int64_t pix = (int64_t)unit * PPW + threadIdx.x / G;
    const bool live = pix < (int64_t)s.W * s.H;
    const int i = live ? (int)(pix % s.W) : 0;
    const int j = live ? (int)(pix / s.W) : 0;
    const int nx = vd->nx, ny = vd->ny, nz = vd->nz;
    double c[3];
    pixel_coords(q, i, j, c);
    const bool near = live && kact > 0 && c[0] > -(double)R && c[0] < (double)(nx - 1 + R) && c[1] > -(double)R &&
                      c[1] < (double)(ny - 1 + R) && c[2] > -(double)R && c[2] < (double)(nz - 1 + R);
    float num = 0.0f, den = 0.0f;
    if (near) {
        const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
        const int x0 = (int)f0, y0 = (int)f1, z0 = (int)f2;
        const float fr[3] = {(float)(c[0] - f0), (float)(c[1] - f1), (float)(c[2] - f2)};
        const int span = 2 * R;
        const int nbx = vd->nbx, nby = vd->nby;
        const typename PT::T* __restrict__ data = (const typename PT::T*)vd->data;
        const int64_t nbricks = vd->nbricks;
        for (int r = g; r < span * span; r += G) {
            const int oz = r / span - R + 1, oy = r % span - R + 1;
            const int vz = z0 + oz, vy = y0 + oy;
            if ((unsigned)vz >= (unsigned)nz || (unsigned)vy >= (unsigned)ny) continue;
            const float tz = fmaxf(0.0f, 1.0f - fabsf((float)oz - fr[2]) * invR);
            const float ty = fmaxf(0.0f, 1.0f - fabsf((float)oy - fr[1]) * invR);
            const float tyz = ty * tz;
            if (!(tyz > 0.0f)) continue;
            const int rb = ((vz >> 3) * nby + (vy >> 3)) * nbx;
            const int rl = ((vz & 7) << 6) | ((vy & 7) << 3);
            for (int ox = -R + 1; ox <= R; ++ox) {
                const int vx = x0 + ox;
                if ((unsigned)vx >= (unsigned)nx) continue;
                const float tx = fmaxf(0.0f, 1.0f - fabsf((float)ox - fr[0]) * invR);
                const float t = tx * tyz;
                if (!(t > 0.0f)) continue;
                float A = 0.0f, B = 0.0f;
                for (int k = 0; k < kact; ++k) {
                    const int b = uniform_i32(sh.act_bin[k]);
                    const int slot = vd->table[(int64_t)b * nbricks + rb + (vx >> 3)];
                    if (slot < 0) continue;
                    float2 sc = make_float2(0.0f, 0.0f);
                    if constexpr (DT == DARE_FP8_E4M3) sc = vd->scales[slot];
                    float a, cnt;
                    PT::decode(data[(size_t)slot * kBrickVox + (rl | (vx & 7))], sc, a, cnt);
                    const float wc = sh.act_w[k] * cnt;
                    A = __builtin_fmaf(wc, a, A);
                    B = B + wc;
                }
                if (B > 0.0f) {
                    num = __builtin_fmaf(t, A / B, num);
                    den = den + t;
                }
            }
        }
    }
    // combine the G lanes of this pixel
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
        num += __shfl_xor(num, off, G);
        den += __shfl_xor(den, off, G);
    }
    if (live && g == 0) s.out[(size_t)j * s.W + i] = den > 0.0f ? num / den : __builtin_nanf("");
}

}  // namespace

template <int DT>
__global__ void __launch_bounds__(256) k_reslice_r1(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ SetupLds sh;
    __shared__ TileLds<DT> tl;
    reslice_tile_r1<DT>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh, tl, false);
}

template <int DT, int G>
__global__ void __launch_bounds__(256) k_reslice_rn(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ SetupLds sh;
    reslice_unit_rn<DT, G>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// ---------------------------------------------------------------- batched passes (radius 1)
//
// A batch runs as three flat passes with no workgroup barriers:
//   setup  one wave per request: pose, Eq. 1 / gates / Eq. 2, plane frame and the
//          slab of the slice (the voxels within the trilinear support of the plane
//          over the slice's bounding box, as runs along the normal's dominant axis);
//   voxel  one thread per slab candidate: all surviving bins gathered at once and
//          blended into V_v, written to the request's slab in the workspace;
//   pixel  one thread per output pixel: FP64 position, the 8 cell values from the
//          slab (mostly L2 hits), tent blend.
// The per-voxel and per-pixel arithmetic and its order are those of the fused
// kernel, so a batched request equals the same request resliced alone.

// First voxel of the slab run of column (vp, vq): one below the slab or the grid floor.
__device__ __forceinline__ int run_start(const SliceSetup& su, int vp, int vq) {
    const float centre = su.c0[su.dax] - (su.fm[su.pax] * ((float)vp - su.c0[su.pax]) +
                                          su.fm[su.qax] * ((float)vq - su.c0[su.qax])) * su.inv_md;
    return max((int)floorf(centre - su.half), 0);
}

// Wave 0: the slab of the whole slice.  Lanes 0..3 place its corner pixels.
__device__ __forceinline__ void slab_setup(const VolDev* __restrict__ vd, const SliceArgs& s, const double T[12],
                                           int kact, int64_t v_cap, SliceSetup& su) {
    const int lane = threadIdx.x;
    SlicePos q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = T[a * 4 + 3];
        q.e0[a] = T[a * 4 + 0];
        q.e1[a] = T[a * 4 + 1];
        q.o[a] = vd->origin[a];
    }
    q.inv_h = vd->inv_h;
    q.sx = s.sx;
    q.sy = s.sy;
    const int k = lane & 3;
    double c[3];
    pixel_coords(q, (k & 1) ? s.W - 1 : 0, (k & 2) ? s.H - 1 : 0, c);
    int lo[3], hi[3];
    const int n[3] = {vd->nx, vd->ny, vd->nz};
    float c0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int f = (int)fmin(fmax(floor(c[a]), -1048576.0), 1048576.0);
        int mn = f, mx = f;
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
    if (lane != 0) return;
    float l1m = 0.0f, l1u = 0.0f, l1w = 0.0f;
    bool empty = false;
    for (int a = 0; a < 3; ++a) {
        empty = empty || lo[a] > hi[a];
        l1m += fabsf(su.fm[a]);
        l1u += fabsf(su.fu[a]);
        l1w += fabsf(su.fw[a]);
        su.c0[a] = c0[a];
    }
    const int dax = su.dax, pax = dax == 0 ? 1 : 0, qax = dax == 2 ? 1 : 2;
    su.pax = pax;
    su.qax = qax;
    su.lo_p = lo[pax];
    su.lo_q = lo[qax];
    su.dim_p = empty ? 0 : hi[pax] - lo[pax] + 1;
    su.dim_q = empty ? 0 : hi[qax] - lo[qax] + 1;
    su.len_u = (float)(s.W - 1) * su.lu;
    su.len_v = (float)(s.H - 1) * su.lw;
    // FP32 rounding of the tests grows with the coordinates' magnitude
    const float span = fmaxf(fmaxf(fabsf(c0[0]), fabsf(c0[1])), fabsf(c0[2])) + su.len_u + su.len_v;
    const float slop = 2e-3f + 1e-6f * span;
    su.thr_n = l1m + slop;
    su.thr_u = l1u + 0.02f + slop;
    su.thr_v = l1w + 0.02f + slop;
    su.inv_md = 1.0f / su.fm[dax];
    su.half = su.thr_n * fabsf(su.inv_md);
    const float dep = ceilf(2.0f * su.half) + 2.0f;
    su.depth = dep <= (float)kSlabDepthMax ? (int)dep : kSlabDepthMax + 1;
    const int64_t ncand = (int64_t)su.dim_p * su.dim_q * su.depth;
    su.staged = (su.depth <= kSlabDepthMax && ncand <= v_cap) ? 1 : 0;
    su.ncand = (kact > 0 && su.staged) ? (int)ncand : 0;
}

__global__ void __launch_bounds__(64) k_batch_setup(const BatchReq* __restrict__ reqs, SliceSetup* __restrict__ setups,
                                                     const int* __restrict__ counts) {
    const int nreq = counts[1];
    for (int r = blockIdx.x; r < nreq; r += gridDim.x) {
        const VolDev* vd = reqs[r].vol;
        const SliceArgs& s = reqs[r].s;
        SliceSetup& su = setups[r];
        double T[12];
        const int ka = slice_setup(vd, s, su, T);
        slab_setup(vd, s, T, ka, reqs[r].v_cap, su);
        if (threadIdx.x == 0) {
            su.vol = view_of(vd);
            su.sx = s.sx;
            su.sy = s.sy;
            su.W = s.W;
            su.H = s.H;
            su.out = s.out;
            su.v_off = reqs[r].v_off;
        }
    }
}

// V_v of voxel (vx, vy, vz) over the surviving bins, straight from the brick pool.
template <int DT>
__device__ __forceinline__ float blend_at(const SliceSetup& su, int kact, int vx, int vy, int vz) {
    using PT = Pair<DT>;
    const VolView& vv = su.vol;
    const typename PT::T* __restrict__ data = (const typename PT::T*)vv.data;
    const int64_t nbricks = vv.nbricks;
    const int64_t brick = ((int64_t)(vz >> 3) * vv.nby + (vy >> 3)) * vv.nbx + (vx >> 3);
    const int local = (((vz & 7) << 3) | (vy & 7)) << 3 | (vx & 7);
    if (kact == 1) {
        const int slot = vv.table[(int64_t)su.act_bin[0] * nbricks + brick];
        if (slot < 0) return __builtin_nanf("");
        float2 sc = make_float2(0.0f, 0.0f);
        if constexpr (DT == DARE_FP8_E4M3) sc = vv.scales[slot];
        float a, cnt;
        PT::decode(data[(size_t)slot * kBrickVox + local], sc, a, cnt);
        return cnt > 0.0f ? a : __builtin_nanf("");
    }
    float A = 0.0f, B = 0.0f;
    for (int k0 = 0; k0 < kact; k0 += kBinChunk) {
        int sl[kBinChunk];
        typename PT::T pr[kBinChunk];
#pragma unroll
        for (int u = 0; u < kBinChunk; ++u)
            sl[u] = (k0 + u < kact) ? vv.table[(int64_t)su.act_bin[k0 + u] * nbricks + brick] : -1;
#pragma unroll
        for (int u = 0; u < kBinChunk; ++u)
            if (sl[u] >= 0) pr[u] = data[(size_t)sl[u] * kBrickVox + local];
#pragma unroll
        for (int u = 0; u < kBinChunk; ++u) {
            if (sl[u] < 0) continue;
            float2 sc = make_float2(0.0f, 0.0f);
            if constexpr (DT == DARE_FP8_E4M3) sc = vv.scales[sl[u]];
            float a, cnt;
            PT::decode(pr[u], sc, a, cnt);
            const float wc = su.act_w[k0 + u] * cnt;
            A = __builtin_fmaf(wc, a, A);
            B = B + wc;
        }
    }
    return B > 0.0f ? A / B : __builtin_nanf("");
}

// The passes run over flat index spaces in blocks of 256: each request's range starts on a
// block boundary, so a workgroup iteration belongs to one request and everything it reads of
// that request (setup record, volume view) is uniform.  Each workgroup first copies the
// requests' first blocks into LDS; the request of block b is then the last r with
// first(r) <= b, found by a binary search in LDS.
template <bool VOX>
__device__ __forceinline__ int load_begins(const BatchReq* __restrict__ reqs, const int* __restrict__ counts,
                                           int* s_beg) {
    const int nreq = counts[1];
    for (int i = threadIdx.x; i < nreq; i += blockDim.x)
        s_beg[i] = (int)((VOX ? reqs[i].v_beg : reqs[i].p_beg) >> 8);
    __syncthreads();
    return nreq;
}

__device__ __forceinline__ int find_req(const int* s_beg, int nreq, int blk) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_beg[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return uniform_i32(lo);
}

template <int DT>
__global__ void __launch_bounds__(256) k_voxel_pass(const BatchReq* __restrict__ reqs,
                                                    const SliceSetup* __restrict__ setups, float* __restrict__ scratch,
                                                    const int* __restrict__ counts) {
    extern __shared__ int s_beg[];
    const int nreq = load_begins<true>(reqs, counts, s_beg);
    const int nblk = (int)(reinterpret_cast<const int64_t*>(counts + 4)[0] >> 8);
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int r = find_req(s_beg, nreq, blk);
        const SliceSetup& su = setups[r];
        const int e = ((blk - s_beg[r]) << 8) + (int)threadIdx.x;
        if (e >= su.ncand) continue;
        const int dax = su.dax, pax = su.pax;
        const int dim_p = su.dim_p, ncols = su.dim_p * su.dim_q;
        const int nd = su.vol.n[dax];
        const int col = e % ncols, k = e / ncols;
        const int vp = su.lo_p + col % dim_p, vq = su.lo_q + col / dim_p;
        const int vdd = run_start(su, vp, vq) + k;
        float V = __builtin_nanf("");
        if (vdd < nd) {
            const int vx = dax == 0 ? vdd : (pax == 0 ? vp : vq);
            const int vy = dax == 1 ? vdd : (pax == 1 ? vp : vq);
            const int vz = dax == 2 ? vdd : (pax == 2 ? vp : vq);
            const float d0 = (float)vx - su.c0[0], d1 = (float)vy - su.c0[1], d2 = (float)vz - su.c0[2];
            const float dn = su.fm[0] * d0 + su.fm[1] * d1 + su.fm[2] * d2;
            const float du = su.fu[0] * d0 + su.fu[1] * d1 + su.fu[2] * d2;
            const float dv = su.fw[0] * d0 + su.fw[1] * d1 + su.fw[2] * d2;
            if (fabsf(dn) < su.thr_n && du > -su.thr_u && du < su.len_u + su.thr_u && dv > -su.thr_v &&
                dv < su.len_v + su.thr_v)
                V = blend_at<DT>(su, su.kact, vx, vy, vz);
        }
        scratch[su.v_off + e] = V;
    }
}

// Pixels of staged requests (STAGED) or of requests that gather per pixel (!STAGED): two
// kernels, so that the staged one keeps the register budget of its 8 slab reads.  A kernel
// skips the other kind's requests one whole range at a time.
template <int DT, bool STAGED>
__global__ void __launch_bounds__(256) k_pixel_pass(const BatchReq* __restrict__ reqs,
                                                    const SliceSetup* __restrict__ setups,
                                                    const float* __restrict__ scratch, const int* __restrict__ counts) {
    extern __shared__ int s_beg[];
    const int nreq = load_begins<false>(reqs, counts, s_beg);
    const int nblk = (int)(reinterpret_cast<const int64_t*>(counts + 4)[1] >> 8);
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int r = find_req(s_beg, nreq, blk);
        const SliceSetup& su = setups[r];
        if ((su.staged != 0) != STAGED) {
            if (r + 1 >= nreq) break;
            const int next = s_beg[r + 1];            // first block of the next request
            blk += (next - blk + (int)gridDim.x - 1) / (int)gridDim.x * (int)gridDim.x - (int)gridDim.x;
            continue;
        }
        const int W = su.W;
        const int p = ((blk - s_beg[r]) << 8) + (int)threadIdx.x;
        if (p >= W * su.H) continue;
        const int j = p / W, i = p - j * W;
        float* out = su.out + p;
        const int kact = su.kact;
        SlicePos q;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q.t[a] = su.T[a * 4 + 3];
            q.e0[a] = su.T[a * 4 + 0];
            q.e1[a] = su.T[a * 4 + 1];
            q.o[a] = su.vol.origin[a];
        }
        q.inv_h = su.vol.inv_h;
        q.sx = su.sx;
        q.sy = su.sy;
        const int n[3] = {su.vol.n[0], su.vol.n[1], su.vol.n[2]};
        double c[3];
        pixel_coords(q, i, j, c);
        if (kact == 0 || !(c[0] >= -1.0 && c[0] < (double)n[0] && c[1] >= -1.0 && c[1] < (double)n[1] &&
                           c[2] >= -1.0 && c[2] < (double)n[2])) {
            *out = __builtin_nanf("");
            continue;
        }
        if constexpr (!STAGED) {
            *out = pixel_direct<DT, 2>(su.vol, su, kact, c);
            continue;
        } else {
        const float* __restrict__ slab = scratch + su.v_off;
        const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
        const int b0[3] = {(int)f0, (int)f1, (int)f2};
        const float fx = (float)(c[0] - f0), fy = (float)(c[1] - f1), fz = (float)(c[2] - f2);
        const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
        const int pax = su.pax, qax = su.qax, dax = su.dax;
        const int dim_p = su.dim_p, dim_q = su.dim_q, depth = su.depth, ncols = dim_p * dim_q;
        // indices first, then all 8 loads at once (absent corners read entry 0 and are discarded)
        float tw[8], Vc[8];
        int ix[8];
        bool ok[8];
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) {                 // c8 = (dz << 2) | (dy << 1) | dx
            const int ddx = c8 & 1, ddy = (c8 >> 1) & 1, ddz = c8 >> 2;
            tw[c8] = (wx[ddx] * wy[ddy]) * wz[ddz];
            const int v[3] = {b0[0] + ddx, b0[1] + ddy, b0[2] + ddz};
            const int vp = v[pax], vq = v[qax];
            const int cp = vp - su.lo_p, cq = vq - su.lo_q;
            const int kk = v[dax] - run_start(su, vp, vq);
            // a cell voxel with weight inside the grid always lies in the slab; the slab test
            // only keeps the index in bounds
            ok[c8] = tw[c8] > 0.0f && (unsigned)v[0] < (unsigned)n[0] && (unsigned)v[1] < (unsigned)n[1] &&
                     (unsigned)v[2] < (unsigned)n[2] && (unsigned)cp < (unsigned)dim_p &&
                     (unsigned)cq < (unsigned)dim_q && (unsigned)kk < (unsigned)depth;
            ix[c8] = ok[c8] ? kk * ncols + cq * dim_p + cp : 0;
        }
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) Vc[c8] = slab[ix[c8]];
        float num = 0.0f, den = 0.0f;
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) {
            if (ok[c8] && Vc[c8] == Vc[c8]) {
                num = __builtin_fmaf(tw[c8], Vc[c8], num);
                den = den + tw[c8];
            }
        }
        *out = den > 0.0f ? num / den : __builtin_nanf("");
        }
    }
}

template <int DT, int G>
__global__ void __launch_bounds__(256) k_reslice_rn_batch(const BatchReq* __restrict__ reqs,
                                                          const int2* __restrict__ units,
                                                          const int* __restrict__ counts) {
    __shared__ SetupLds sh;
    const int n = counts[0];
    for (int u = blockIdx.x; u < n; u += gridDim.x) {
        const int r = __builtin_amdgcn_readfirstlane(units[u].x);
        const int t = __builtin_amdgcn_readfirstlane(units[u].y);
        const BatchReq& rq = reqs[r];
        reslice_unit_rn<DT, G>(rq.vol, rq.s, t, sh);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------- launchers

int reslice_lanes(int radius) { return radius <= 1 ? 1 : (radius <= 2 ? 16 : 64); }

int64_t reslice_units(int radius, int W, int H) {
    if (radius <= 1) return (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    const int ppw = 256 / reslice_lanes(radius);
    return ((int64_t)W * H + ppw - 1) / ppw;
}

#define DARE_DISPATCH_DT(dtype, MACRO) \
    switch (dtype) {                   \
        case DARE_F32: MACRO(DARE_F32); break; \
        case DARE_BF16: MACRO(DARE_BF16); break; \
        case DARE_F16: MACRO(DARE_F16); break; \
        case DARE_FP8_E4M3: MACRO(DARE_FP8_E4M3); break; \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_reslice(const VolDev* vd, int dtype, int radius, const SliceArgs& s, hipStream_t stream) {
    const int64_t units = reslice_units(radius, s.W, s.H);
    const dim3 grid((unsigned)units), block(256);
    const int G = reslice_lanes(radius);
#define L1(D) hipLaunchKernelGGL(k_reslice_r1<D>, grid, block, 0, stream, vd, s)
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

hipError_t launch_reslice_batch(int dtype, int radius, const BatchReq* reqs, SliceSetup* setups, const int2* units,
                                const int* counts, float* scratch, int nreq_max, int grid, hipStream_t stream) {
    const int G = reslice_lanes(radius);
    const int nreq_grid = nreq_max < 1024 ? nreq_max : 1024;
    const size_t lds = (size_t)nreq_max * sizeof(int);
#define V1(D) hipLaunchKernelGGL(k_voxel_pass<D>, dim3(grid), dim3(256), lds, stream, reqs, setups, scratch, counts)
#define P1(D)                                                                                                  \
    hipLaunchKernelGGL((k_pixel_pass<D, true>), dim3(grid), dim3(256), lds, stream, reqs, setups, scratch, counts); \
    hipLaunchKernelGGL((k_pixel_pass<D, false>), dim3(grid), dim3(256), lds, stream, reqs, setups, scratch, counts)
#define B16(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 16>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
#define B64(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 64>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
    if (G == 1) {
        hipLaunchKernelGGL(k_batch_setup, dim3(nreq_grid), dim3(64), 0, stream, reqs, setups, counts);
        DARE_DISPATCH_DT(dtype, V1)
        DARE_DISPATCH_DT(dtype, P1)
    } else if (G == 16) {
        DARE_DISPATCH_DT(dtype, B16)
    } else {
        DARE_DISPATCH_DT(dtype, B64)
    }
#undef V1
#undef P1
#undef B16
#undef B64
    return hipGetLastError();
}

}  // namespace dare
