// Directionality-aware reslice at interpolation radius R = 2..4 voxels (Sec. 2.1 "Reslicing",
// Eq. 1, Eq. 2, Fig. 2; the paper times radii of 0.125, 0.25 and 0.5 mm).
//
// Every pixel blends the voxels within L-infinity distance R of its position with tent weights
// prod_a max(0, 1 - |c_a - v_a| / R), (2R)^3 voxels per pixel, each voxel's value being its
// direction blend V_v = sum_b w_b c_vb a_vb / sum_b w_b c_vb over the surviving bins.  V_v does
// not depend on the pixel, and at these radii neighbouring pixels share almost all of their
// voxels, so one workgroup per 16x16 tile blends every voxel the tile reaches once into LDS
// (the radius-1 scheme with the reach widened by R), then each pixel sums its (2R)^3 values
// from LDS.  Tiles whose voxel box exceeds the LDS budget (coarse output pitch) gather per pixel.
#include "dare_reslice_dev.h"
#include "dare_staged.h"

namespace dare {

namespace {

template <int R>
struct RsLimits {
    static constexpr int kEdge = 13 + 2 * R;                    // box voxels per axis at 0.5-voxel pitch
    static constexpr int kBoxMax = kEdge * kEdge * kEdge;       // LDS values per tile
    static constexpr int kSlotMax = 2048;                       // (surviving bin, box brick) slots
};

template <int DT, int R>
struct TileLdsR {
    int mode;                        // 0: nothing in reach, 1: staged, 2: per-pixel gather
    int lo[3], dim[3];
    int blo[3], bdim[3], nbb;
    int dax, pax, qax;
    int depth, ncols;
    float m[3], c0[3], ua[3], va[3];
    float thr_n, thr_u, thr_v, len_u, len_v, inv_md;
    int nlist;
    int slot[RsLimits<R>::kSlotMax];
    float2 scale[DT == DARE_FP8_E4M3 ? RsLimits<R>::kSlotMax : 1];
    float V[RsLimits<R>::kBoxMax];
    unsigned short list[RsLimits<R>::kBoxMax];
};

// Wave 0: the tile's voxel box (its corner pixels' cells widened by R, one voxel of margin)
// and the footprint tests scaled by R.
template <int DT, int R>
__device__ __forceinline__ void tile_setup_r(const VolDev* __restrict__ vd, const SliceArgs& s, const double T[12],
                                             const SetupLds& sh, int kact, int i0, int j0, TileLdsR<DT, R>& tl) {
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
        lo[a] = max(mn - R, 0);
        hi[a] = min(mx + R + 1, n[a] - 1);
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
    if (mode == 1 && (nvox > RsLimits<R>::kBoxMax || kact * nbb > RsLimits<R>::kSlotMax)) mode = 2;
    tl.mode = mode;
    tl.nbb = nbb;
    // a voxel within L-infinity distance R of a pixel p of the tile satisfies |m.(v - p)| < R |m|_1,
    // and its lateral offsets exceed the tile's extent by less than R |ua|_1, R |va|_1
    const int dax = sh.dax;
    tl.thr_n = (float)R * l1m + 2e-3f;
    tl.thr_u = (float)R * l1u + 0.02f;
    tl.thr_v = (float)R * l1w + 0.02f;
    tl.len_u = (float)(i1 - i0) * sh.lu;
    tl.len_v = (float)(j1 - j0) * sh.lw;
    tl.dax = dax;
    tl.pax = dax == 0 ? 1 : 0;
    tl.qax = dax == 2 ? 1 : 2;
    tl.inv_md = 1.0f / sh.fm[dax];
    // a column's voxels in reach are the integers in (centre - half, centre + half), half =
    // thr_n / |m[dax]|: at most ceil(2 half) of them, the first one above centre - half
    tl.depth = mode == 1 ? (int)ceilf(2.0f * (tl.thr_n * fabsf(tl.inv_md))) : 0;
    tl.ncols = mode == 1 ? tl.dim[tl.pax] * tl.dim[tl.qax] : 0;
    tl.nlist = 0;
}

// V_v of one voxel from the staged brick slots; NaN when no surviving bin holds a sample.
template <int DT, int R>
__device__ __forceinline__ float blend_voxel_r(const typename Pair<DT>::T* __restrict__ data, const SetupLds& sh,
                                               const TileLdsR<DT, R>& tl, int kact, int bb, int local) {
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

// The same V_v read straight from the volume (tiles that gather per pixel): the arithmetic and
// its order are blend_voxel_r's.
template <int DT>
__device__ __forceinline__ float voxel_value(const VolDev* __restrict__ vd, const SetupLds& sh, int kact, int vx,
                                             int vy, int vz) {
    using PT = Pair<DT>;
    const typename PT::T* __restrict__ data = (const typename PT::T*)vd->data;
    const int64_t nbricks = vd->nbricks;
    const int64_t brick = ((int64_t)(vz >> 3) * vd->nby + (vy >> 3)) * vd->nbx + (vx >> 3);
    const int local = brick_local(vx, vy, vz);
    if (kact == 1) {
        const int slot = vd->table[(int64_t)sh.act_bin[0] * nbricks + brick];
        if (slot < 0) return __builtin_nanf("");
        float2 sc = make_float2(0.0f, 0.0f);
        if constexpr (DT == DARE_FP8_E4M3) sc = vd->scales[slot];
        float a, cnt;
        PT::decode(data[(size_t)slot * kBrickVox + local], sc, a, cnt);
        return cnt > 0.0f ? a : __builtin_nanf("");
    }
    float A = 0.0f, B = 0.0f;
    for (int k = 0; k < kact; ++k) {
        const int slot = vd->table[(int64_t)sh.act_bin[k] * nbricks + brick];
        if (slot < 0) continue;
        float2 sc = make_float2(0.0f, 0.0f);
        if constexpr (DT == DARE_FP8_E4M3) sc = vd->scales[slot];
        float a, cnt;
        PT::decode(data[(size_t)slot * kBrickVox + local], sc, a, cnt);
        const float wc = sh.act_w[k] * cnt;
        A = __builtin_fmaf(wc, a, A);
        B = B + wc;
    }
    return B > 0.0f ? A / B : __builtin_nanf("");
}

// One 16x16 tile at radius R.
template <int DT, int R>
__device__ __forceinline__ void reslice_tile_rs(const VolDev* __restrict__ vd, const SliceArgs& s, int unit,
                                                SetupLds& sh, TileLdsR<DT, R>& tl) {
    const int tx = unit % s.tiles_x, ty = unit / s.tiles_x;
    const int i0 = tx * kTile, j0 = ty * kTile;
    if (threadIdx.x < 64) {
        double T[12];
        const int ka = slice_setup(vd, s, sh, T);
        tile_setup_r<DT, R>(vd, s, T, sh, ka, i0, j0, tl);
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
        // (b) the voxels in reach, as runs along the normal's dominant axis, compacted into a list
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
                const int vdd = max((int)floorf(centre - half) + 1, lo[dax]) + k;
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
        // (c) one thread per listed voxel: its direction blend into LDS
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
            const int local = brick_local(vx, vy, vz);
            tl.V[bi] = blend_voxel_r<DT, R>(data, sh, tl, kact, bb, local);
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
    const int n[3] = {vd->nx, vd->ny, vd->nz};
    double c[3];
    pixel_coords(q, i, j, c);
    if (!(c[0] > -(double)R && c[0] < (double)(n[0] - 1 + R) && c[1] > -(double)R && c[1] < (double)(n[1] - 1 + R) &&
          c[2] > -(double)R && c[2] < (double)(n[2] - 1 + R))) {
        *out = __builtin_nanf("");
        return;
    }
    const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
    const int b0[3] = {(int)f0, (int)f1, (int)f2};
    const float fr[3] = {(float)(c[0] - f0), (float)(c[1] - f1), (float)(c[2] - f2)};
    const float gr[3] = {(float)(f0 + 1.0 - c[0]), (float)(f1 + 1.0 - c[1]), (float)(f2 + 1.0 - c[2])};
    const float invR = 1.0f / (float)R;
    // tent weights per axis for offsets -R+1 .. R
    float tw[3][2 * R];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 0; o < 2 * R; ++o) tw[a][o] = tent_weight(o - R + 1, fr[a], gr[a], R, invR);
    float num = 0.0f, den = 0.0f;
    if (mode == 2) {
        for (int oz = 0; oz < 2 * R; ++oz)
            for (int oy = 0; oy < 2 * R; ++oy)
#pragma unroll
                for (int ox = 0; ox < 2 * R; ++ox) {
                    const int vx = b0[0] + ox - R + 1, vy = b0[1] + oy - R + 1, vz = b0[2] + oz - R + 1;
                    const float t = (tw[0][ox] * tw[1][oy]) * tw[2][oz];
                    if (!(t > 0.0f) || (unsigned)vx >= (unsigned)n[0] || (unsigned)vy >= (unsigned)n[1] ||
                        (unsigned)vz >= (unsigned)n[2])
                        continue;
                    const float V = voxel_value<DT>(vd, sh, kact, vx, vy, vz);
                    if (V == V) {
                        num = __builtin_fmaf(t, V, num);
                        den = den + t;
                    }
                }
    } else {
        // every in-grid voxel with weight was staged; voxels outside the box are outside the grid
        const int dx = tl.dim[0], dy = tl.dim[1], dz = tl.dim[2];
        const int ex0 = b0[0] - R + 1 - tl.lo[0], ey0 = b0[1] - R + 1 - tl.lo[1], ez0 = b0[2] - R + 1 - tl.lo[2];
        for (int oz = 0; oz < 2 * R; ++oz) {
            const int ez = ez0 + oz;
            for (int oy = 0; oy < 2 * R; ++oy) {
                const int ey = ey0 + oy;
                const bool row_in = (unsigned)ez < (unsigned)dz && (unsigned)ey < (unsigned)dy;
                const float tyz = tw[1][oy] * tw[2][oz];
                const int rowb = (ez * dy + ey) * dx;
#pragma unroll
                for (int ox = 0; ox < 2 * R; ++ox) {
                    const int ex = ex0 + ox;
                    const float t = tw[0][ox] * tyz;
                    const bool ok = row_in && (unsigned)ex < (unsigned)dx && t > 0.0f;
                    const float V = tl.V[ok ? rowb + ex : 0];
                    if (ok && V == V) {
                        num = __builtin_fmaf(t, V, num);
                        den = den + t;
                    }
                }
            }
        }
    }
    *out = den > 0.0f ? num / den : __builtin_nanf("");
}

}  // namespace

template <int DT, int R>
__global__ void __launch_bounds__(256) k_reslice_rs(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ SetupLds sh;
    __shared__ TileLdsR<DT, R> tl;
    reslice_tile_rs<DT, R>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh, tl);
}

// Batched form: (request, tile) units, grid-stride; every tile computes its own setup, so a
// request's result is the one it gets alone.
template <int DT, int R>
__global__ void __launch_bounds__(256) k_reslice_rs_batch(const BatchReq* __restrict__ reqs,
                                                          const int2* __restrict__ units,
                                                          const int* __restrict__ counts) {
    __shared__ SetupLds sh;
    __shared__ TileLdsR<DT, R> tl;
    const int nunits = counts[0];
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const int r = __builtin_amdgcn_readfirstlane(units[u].x);
        const int t = __builtin_amdgcn_readfirstlane(units[u].y);
        reslice_tile_rs<DT, R>(reqs[r].vol, reqs[r].s, t, sh, tl);
        __syncthreads();
    }
}

int64_t staged_tiles(int W, int H) { return (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile); }

hipError_t launch_reslice_staged(const VolDev* vd, int dtype, int radius, const SliceArgs& s, hipStream_t stream) {
    const dim3 grid((unsigned)staged_tiles(s.W, s.H)), block(256);
#define S2(D) hipLaunchKernelGGL((k_reslice_rs<D, 2>), grid, block, 0, stream, vd, s)
#define S3(D) hipLaunchKernelGGL((k_reslice_rs<D, 3>), grid, block, 0, stream, vd, s)
#define S4(D) hipLaunchKernelGGL((k_reslice_rs<D, 4>), grid, block, 0, stream, vd, s)
    switch (radius) {
        case 2: DARE_DISPATCH_DT(dtype, S2) break;
        case 3: DARE_DISPATCH_DT(dtype, S3) break;
        case 4: DARE_DISPATCH_DT(dtype, S4) break;
        default: return hipErrorInvalidValue;
    }
#undef S2
#undef S3
#undef S4
    return hipGetLastError();
}

hipError_t launch_reslice_staged_batch(int dtype, int radius, const BatchReq* reqs, const int2* units,
                                       const int* counts, int grid, hipStream_t stream) {
#define B2(D) hipLaunchKernelGGL((k_reslice_rs_batch<D, 2>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
#define B3(D) hipLaunchKernelGGL((k_reslice_rs_batch<D, 3>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
#define B4(D) hipLaunchKernelGGL((k_reslice_rs_batch<D, 4>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
    switch (radius) {
        case 2: DARE_DISPATCH_DT(dtype, B2) break;
        case 3: DARE_DISPATCH_DT(dtype, B3) break;
        case 4: DARE_DISPATCH_DT(dtype, B4) break;
        default: return hipErrorInvalidValue;
    }
#undef B2
#undef B3
#undef B4
    return hipGetLastError();
}

int64_t batch_units(int radius, int W, int H) {
    return staged_radius(radius) ? staged_tiles(W, H) : reslice_units(radius, W, H);
}

}  // namespace dare
