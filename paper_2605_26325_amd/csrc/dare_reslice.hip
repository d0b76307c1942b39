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

struct SetupLds {
    double T[12];
    int kact;
    int act_bin[kMaxBins];
    float act_w[kMaxBins];
};

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
__device__ __forceinline__ void slice_setup(const VolDev* __restrict__ vd, const double* __restrict__ P,
                                            SetupLds& sh) {
    const int lane = threadIdx.x;
    const double* C = vd->calib;
    double T[12];
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
    const int K = vd->st.K;
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
        const double dn = dot3(vd->rep_n[lane], nr);
        const double di = fabs(dot3(vd->rep_x[lane], xr));
        keep = dn >= vd->cos_normal && di >= vd->cos_inplane;
        if (keep) w = exp(vd->k_normal * (dn - 1.0) + vd->k_inplane * (di - 1.0));
    }
    const unsigned long long m = __ballot(keep);
    if (keep) {
        const int idx = __popcll(m & ((1ull << lane) - 1ull));
        sh.act_bin[idx] = lane;
        sh.act_w[idx] = (float)w;
    }
    if (lane == 0) sh.kact = __popcll(m);
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
template <int DT>
__device__ __forceinline__ void reslice_tile_r1(const VolDev* __restrict__ vd, const SliceArgs& s, int unit,
                                                SetupLds& sh) {
    using PT = Pair<DT>;
    if (threadIdx.x < 64) slice_setup(vd, s.P, sh);
    __syncthreads();
    SlicePos q;
    load_pos(vd, sh, s, q);
    const int kact = uniform_i32(sh.kact);
    const int tx = unit % s.tiles_x, ty = unit / s.tiles_x;
    const int i = tx * kTile + (threadIdx.x & (kTile - 1));
    const int j = ty * kTile + (threadIdx.x >> 4);
    if (i >= s.W || j >= s.H) return;
    float* out = s.out + (size_t)j * s.W + i;
    const int nx = vd->nx, ny = vd->ny, nz = vd->nz;
    double c[3];
    pixel_coords(q, i, j, c);
    if (kact == 0 || !(c[0] >= -1.0 && c[0] < (double)nx && c[1] >= -1.0 && c[1] < (double)ny && c[2] >= -1.0 &&
                       c[2] < (double)nz)) {
        *out = __builtin_nanf("");
        return;
    }
    const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
    const int x0 = (int)f0, y0 = (int)f1, z0 = (int)f2;
    const float fx = (float)(c[0] - f0), fy = (float)(c[1] - f1), fz = (float)(c[2] - f2);
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
    // brick coordinates, in-brick offsets and in-grid flags of the two voxels per axis
    const int nbx = vd->nbx, nby = vd->nby;
    int bx[2], lx[2], rowb[2][2], rowl[2][2];
    bool inx[2], inyz[2][2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int v = x0 + d;
        inx[d] = (unsigned)v < (unsigned)nx;
        bx[d] = v >> 3;
        lx[d] = v & 7;
    }
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int vy = y0 + dy, vz = z0 + dz;
            inyz[dz][dy] = (unsigned)vy < (unsigned)ny && (unsigned)vz < (unsigned)nz;
            rowb[dz][dy] = ((vz >> 3) * nby + (vy >> 3)) * nbx;
            rowl[dz][dy] = ((vz & 7) << 6) | ((vy & 7) << 3);
        }
    const typename PT::T* __restrict__ data = (const typename PT::T*)vd->data;
    const int64_t nbricks = vd->nbricks;
    float num = 0.0f, den = 0.0f;
    if (kact == 1) {
        // one surviving direction: its weight cancels within each voxel
        const int32_t* __restrict__ tab = vd->table + (int64_t)uniform_i32(sh.act_bin[0]) * nbricks;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    if (!(inx[dx] && inyz[dz][dy])) continue;
                    const int slot = tab[rowb[dz][dy] + bx[dx]];
                    if (slot < 0) continue;
                    float2 sc = make_float2(0.0f, 0.0f);
                    if constexpr (DT == DARE_FP8_E4M3) sc = vd->scales[slot];
                    float a, cnt;
                    PT::decode(data[(size_t)slot * kBrickVox + (rowl[dz][dy] | lx[dx])], sc, a, cnt);
                    if (cnt > 0.0f) {
                        const float t = (wx[dx] * wy[dy]) * wz[dz];
                        num = __builtin_fmaf(t, a, num);
                        den = den + t;
                    }
                }
    } else {
        float A[8], B[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) { A[k] = 0.0f; B[k] = 0.0f; }
        for (int k = 0; k < kact; ++k) {
            const int b = uniform_i32(sh.act_bin[k]);
            const float wgt = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sh.act_w[k])));
            const int32_t* __restrict__ tab = vd->table + (int64_t)b * nbricks;
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        if (!(inx[dx] && inyz[dz][dy])) continue;
                        const int slot = tab[rowb[dz][dy] + bx[dx]];
                        if (slot < 0) continue;
                        float2 sc = make_float2(0.0f, 0.0f);
                        if constexpr (DT == DARE_FP8_E4M3) sc = vd->scales[slot];
                        float a, cnt;
                        PT::decode(data[(size_t)slot * kBrickVox + (rowl[dz][dy] | lx[dx])], sc, a, cnt);
                        const float wc = wgt * cnt;
                        const int v = (dz << 2) | (dy << 1) | dx;
                        A[v] = __builtin_fmaf(wc, a, A[v]);
                        B[v] = B[v] + wc;
                    }
        }
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const int v = (dz << 2) | (dy << 1) | dx;
                    if (B[v] > 0.0f) {
                        const float t = (wx[dx] * wy[dy]) * wz[dz];
                        num = __builtin_fmaf(t, A[v] / B[v], num);
                        den = den + t;
                    }
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
    if (threadIdx.x < 64) slice_setup(vd, s.P, sh);
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
    reslice_tile_r1<DT>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh);
}

template <int DT, int G>
__global__ void __launch_bounds__(256) k_reslice_rn(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ SetupLds sh;
    reslice_unit_rn<DT, G>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// Batched form: a table of (request, unit) pairs; each workgroup walks units
// blockIdx.x, blockIdx.x + gridDim.x, ... up to the device-side count, so the
// grid can stay fixed while the work varies (graph replay).
template <int DT>
__global__ void __launch_bounds__(256) k_reslice_r1_batch(const BatchReq* __restrict__ reqs,
                                                          const int2* __restrict__ units,
                                                          const int* __restrict__ nunits) {
    __shared__ SetupLds sh;
    const int n = *nunits;
    for (int u = blockIdx.x; u < n; u += gridDim.x) {
        const int2 ru = units[u];
        const BatchReq& rq = reqs[ru.x];
        reslice_tile_r1<DT>(rq.vol, rq.s, ru.y, sh);
        __syncthreads();
    }
}

template <int DT, int G>
__global__ void __launch_bounds__(256) k_reslice_rn_batch(const BatchReq* __restrict__ reqs,
                                                          const int2* __restrict__ units,
                                                          const int* __restrict__ nunits) {
    __shared__ SetupLds sh;
    const int n = *nunits;
    for (int u = blockIdx.x; u < n; u += gridDim.x) {
        const int2 ru = units[u];
        const BatchReq& rq = reqs[ru.x];
        reslice_unit_rn<DT, G>(rq.vol, rq.s, ru.y, sh);
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

hipError_t launch_reslice_batch(int dtype, int radius, const BatchReq* reqs, const int2* units, const int* nunits,
                                int grid, hipStream_t stream) {
    const int G = reslice_lanes(radius);
#define B1(D) hipLaunchKernelGGL(k_reslice_r1_batch<D>, dim3(grid), dim3(256), 0, stream, reqs, units, nunits)
#define B16(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 16>), dim3(grid), dim3(256), 0, stream, reqs, units, nunits)
#define B64(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 64>), dim3(grid), dim3(256), 0, stream, reqs, units, nunits)
    if (G == 1) {
        DARE_DISPATCH_DT(dtype, B1)
    } else if (G == 16) {
        DARE_DISPATCH_DT(dtype, B16)
    } else {
        DARE_DISPATCH_DT(dtype, B64)
    }
#undef B1
#undef B16
#undef B64
    return hipGetLastError();
}

}  // namespace dare
