// Device helpers shared by the single-request reslice kernels and the batched passes:
// slice setup (FP64 pose composition, Eq. 1 gates and Eq. 2 weights), FP64 pixel
// positions, the per-pixel gather of a trilinear cell, and the radius >= 2 unit.
#pragma once

#include <math.h>

#include "dare_codec.h"
#include "dare_internal.h"

#pragma clang fp contract(off)

namespace dare {

namespace {


using SetupLds = SliceCore;

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

// The slice pose T = P.C, rows 0..2 (every lane the same).
__device__ __forceinline__ void slice_pose(const VolDev* __restrict__ vd, const SliceArgs& s, double T[12]) {
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
}

// One wave: the slice pose, and Eq. 1 / thresholds / Eq. 2 per bin (lane b takes bin b), the
// survivors compacted into act_bin / act_w.  Returns the number of surviving bins (every lane);
// lane 0 stores T and kact.
__device__ __forceinline__ int slice_gates(const VolDev* __restrict__ vd, const SliceArgs& s, SetupLds& sh,
                                           double T[12]) {
    const int lane = threadIdx.x & 63;
    slice_pose(vd, s, T);
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
    // cosines against the slice's unit in-plane axis and normal: the dot products with the raw
    // columns divided by the columns' lengths
    const double l0 = sqrt(dot3(e0, e0));
    const double ln = sqrt(dot3(en, en));
    bool keep = false;
    float w = 0.0f;
    if (lane < K) {
        const double dn = dot3(rn, en) / ln;
        const double di = fabs(dot3(rx, e0)) / l0;
        keep = dn >= vd->cos_normal && di >= vd->cos_inplane;
        // Eq. 2's exponent in FP64, the weight itself in FP32 (it is stored in FP32)
        if (keep) w = expf((float)(vd->k_normal * (dn - 1.0) + vd->k_inplane * (di - 1.0)));
    }
    const unsigned long long m = __ballot(keep);
    if (keep) {
        const int idx = __popcll(m & ((1ull << lane) - 1ull));
        sh.act_bin[idx] = lane;
        sh.act_w[idx] = w;
    }
    if (lane == 0) sh.kact = __popcll(m);
    return __popcll(m);
}

// The plane frame in voxel units (it only drives conservative footprint tests, so FP32): unit
// in-plane axes fu, fw, their pixel lengths lu, lw, unit normal fm and its dominant axis dax.
struct SliceFrame {
    float fm[3], fu[3], fw[3], lu, lw;
    int dax;
};

__device__ __forceinline__ SliceFrame frame_of(const VolDev* __restrict__ vd, const SliceArgs& s,
                                               const double T[12]) {
    const double inv_h = vd->inv_h;
    float u[3], v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = (float)(T[a * 4 + 0] * s.sx * inv_h);
        v[a] = (float)(T[a * 4 + 1] * s.sy * inv_h);
    }
    SliceFrame f;
    f.lu = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    f.lw = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    float nm[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    const float rm = 1.0f / sqrtf(nm[0] * nm[0] + nm[1] * nm[1] + nm[2] * nm[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) nm[a] *= rm;
    int dax = 0;
    if (fabsf(nm[1]) > fabsf(nm[dax])) dax = 1;
    if (fabsf(nm[2]) > fabsf(nm[dax])) dax = 2;
    const float ilu = 1.0f / f.lu, ilv = 1.0f / f.lw;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f.fm[a] = nm[a];
        f.fu[a] = u[a] * ilu;
        f.fw[a] = v[a] * ilv;
    }
    f.dax = dax;
    return f;
}

__device__ __forceinline__ void store_frame(const SliceFrame& f, SetupLds& sh) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        sh.fm[a] = f.fm[a];
        sh.fu[a] = f.fu[a];
        sh.fw[a] = f.fw[a];
    }
    sh.lu = f.lu;
    sh.lw = f.lw;
    sh.dax = f.dax;
}

// One lane: the plane frame into the setup record.
__device__ __forceinline__ void slice_frame(const VolDev* __restrict__ vd, const SliceArgs& s, const double T[12],
                                            SetupLds& sh) {
    store_frame(frame_of(vd, s, T), sh);
}

// Wave 0 only: slice pose, Eq. 1 / thresholds / Eq. 2 per bin, survivors compacted, and the
// plane frame (lane 0).  Returns the number of surviving bins; T receives the composed pose.
__device__ __forceinline__ int slice_setup(const VolDev* __restrict__ vd, const SliceArgs& s, SetupLds& sh,
                                           double T[12]) {
    const int kact = slice_gates(vd, s, sh, T);
    if ((threadIdx.x & 63) == 0) slice_frame(vd, s, T, sh);
    return kact;
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

constexpr int kBinChunk = 16;        // gathers issued together per voxel

// Division by a divisor shared by a workgroup, for small dividends: x / d = the high word of
// x * m with m = ceil(2^32 / d), exact for 0 <= x < 2^16 and 2 <= d < 2^16 (m exceeds 2^32 / d
// by less than 1, which moves x * m / 2^32 by less than 2^-16, less than the 1/d gap between
// x / d and the next integer).  d = 1 passes x through.  m is set from a correctly rounded FP64
// integer quotient: with 2^32 = q d + r, floor((2^32 - 1) / d) is q - 1 when r = 0 and q
// otherwise, so one more is ceil(2^32 / d) in both cases.
struct SmallDiv {
    uint32_t m;
    int d;
};

__device__ __forceinline__ SmallDiv small_div(int d) {
    SmallDiv s;
    s.d = d;
    s.m = d > 1 ? 0xFFFFFFFFu / (uint32_t)d + 1u : 0u;
    return s;
}

__device__ __forceinline__ int sdiv(int x, SmallDiv s) {
    return s.d == 1 ? x : (int)__umulhi((uint32_t)x, s.m);
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
    v.cap = vd->cap;
#pragma unroll
    for (int a = 0; a < 3; ++a) v.origin[a] = vd->origin[a];
    v.inv_h = vd->inv_h;
    return v;
}

// Tent weight 1 - |o - f| / R of the voxel at integer offset o (-R < o <= R) from the cell floor
// along one axis, for a sample at fraction f of its cell, with g = 1 - f.  Both come from the
// FP64 position (f = c - floor(c), g = floor(c) + 1 - c), and the low side (o <= 0) is written
// through g: as f nears 1 it rounds to 1 in FP32 while g stays positive, so a voxel whose FP64
// weight is positive keeps a positive weight (and a pixel whose only valid voxels lie there stays
// assigned, as in FP64).
__device__ __forceinline__ float tent_weight(int o, float f, float g, int R, float invR) {
    return o <= 0 ? fmaxf(0.0f, ((float)(R - 1 + o) + g) * invR) : fmaxf(0.0f, ((float)(R - o) + f) * invR);
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
    // the low voxel's weight from FP64 (tent_weight at R = 1)
    const float gx = (float)(f0 + 1.0 - c[0]), gy = (float)(f1 + 1.0 - c[1]), gz = (float)(f2 + 1.0 - c[2]);
    const float wx[2] = {gx, fx}, wy[2] = {gy, fy}, wz[2] = {gz, fz};
    const int nbx = vv.nbx, nby = vv.nby;
    int tix[8], lix[8];
    bool in[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {                  // v = (dz << 2) | (dy << 1) | dx
        const int vx = x0 + (v & 1), vy = y0 + ((v >> 1) & 1), vz = z0 + (v >> 2);
        in[v] = (unsigned)vx < (unsigned)nx && (unsigned)vy < (unsigned)ny && (unsigned)vz < (unsigned)nz;
        tix[v] = in[v] ? ((vz >> 3) * nby + (vy >> 3)) * nbx + (vx >> 3) : 0;
        lix[v] = brick_local(vx, vy, vz);
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
        const float gr[3] = {(float)(f0 + 1.0 - c[0]), (float)(f1 + 1.0 - c[1]), (float)(f2 + 1.0 - c[2])};
        const int span = 2 * R;
        const int nbx = vd->nbx, nby = vd->nby;
        const typename PT::T* __restrict__ data = (const typename PT::T*)vd->data;
        const int64_t nbricks = vd->nbricks;
        for (int r = g; r < span * span; r += G) {
            const int oz = r / span - R + 1, oy = r % span - R + 1;
            const int vz = z0 + oz, vy = y0 + oy;
            if ((unsigned)vz >= (unsigned)nz || (unsigned)vy >= (unsigned)ny) continue;
            const float tz = tent_weight(oz, fr[2], gr[2], R, invR);
            const float ty = tent_weight(oy, fr[1], gr[1], R, invR);
            const float tyz = ty * tz;
            if (!(tyz > 0.0f)) continue;
            const int rb = ((vz >> 3) * nby + (vy >> 3)) * nbx;
            for (int ox = -R + 1; ox <= R; ++ox) {
                const int vx = x0 + ox;
                if ((unsigned)vx >= (unsigned)nx) continue;
                const float tx = tent_weight(ox, fr[0], gr[0], R, invR);
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
                    PT::decode(data[(size_t)slot * kBrickVox + brick_local(vx, vy, vz)], sc, a, cnt);
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

#define DARE_DISPATCH_DT(dtype, MACRO)                       \
    switch (dtype) {                                         \
        case DARE_F32: MACRO(DARE_F32); break;               \
        case DARE_BF16: MACRO(DARE_BF16); break;             \
        case DARE_F16: MACRO(DARE_F16); break;               \
        case DARE_FP8_E4M3: MACRO(DARE_FP8_E4M3); break;     \
        default: return hipErrorInvalidValue;                \
    }

}  // namespace dare
