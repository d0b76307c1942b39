// Volume reconstruction kernels (Sec. 2.1 "Volume reconstruction", Fig. 1):
// frame pose composition, direction-bin assignment, brick occupancy and
// allocation, nearest-voxel accumulation and finalisation into the stored
// precision.  Positions are FP64 with no contraction so that every
// nearest-voxel decision is reproducible; sums and counts are exact integers
// accumulated with 64-bit atomics, so the result is independent of order.
#include <math.h>

#include <algorithm>

#include "dare_codec.h"
#include "dare_frames.h"
#include "dare_internal.h"

#pragma clang fp contract(off)

namespace dare {

namespace {

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// Pointers by address space: constant (what a whole workgroup reads and no running kernel
// writes: scalar loads) and global (per-lane accesses and atomics: global, not flat, operations).
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
using gptr = __attribute__((address_space(1))) T*;

// What the per-pixel kernels read of the volume header, through scalar loads.
struct PixelView {
    double origin[3], inv_h;
    int nx, ny, nz, nbx, nby;
    int64_t nbricks;
    const FrameDesc* frames;
    const int32_t* frame_bin;
    int32_t* table;
};

__device__ __forceinline__ PixelView pixel_view(const VolDev* vd) {
    const cptr<VolDev> c = (cptr<VolDev>)vd;
    PixelView v;
#pragma unroll
    for (int a = 0; a < 3; ++a) v.origin[a] = c->origin[a];
    v.inv_h = c->inv_h;
    v.nx = c->nx;
    v.ny = c->ny;
    v.nz = c->nz;
    v.nbx = c->nbx;
    v.nby = c->nby;
    v.nbricks = c->nbricks;
    v.frames = c->frames;
    v.frame_bin = c->frame_bin;
    v.table = c->table;
    return v;
}

// Frame f's placement (translation and raw columns; the unit axes are not needed here), through
// scalar loads: a workgroup works on one frame.
__device__ __forceinline__ FrameDesc frame_uniform(const PixelView& v, int f) {
    const cptr<FrameDesc> p = (cptr<FrameDesc>)v.frames + f;
    FrameDesc d;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.t[a] = p->t[a];
        d.e0[a] = p->e0[a];
        d.e1[a] = p->e1[a];
        d.xh[a] = 0.0;
        d.nh[a] = 0.0;
    }
    d.pad = 0.0;
    return d;
}

__device__ __forceinline__ int64_t brick_entry(const PixelView& v, int b, int vx, int vy, int vz) {
    return (int64_t)b * v.nbricks + ((int64_t)(vz >> 3) * v.nby + (vy >> 3)) * v.nbx + (vx >> 3);
}

__device__ __forceinline__ int64_t brick_entry(const VolDev* vd, int b, int vx, int vy, int vz) {
    return (int64_t)b * vd->nbricks + ((int64_t)(vz >> 3) * vd->nby + (vy >> 3)) * vd->nbx + (vx >> 3);
}

// Pixel block and frame of this workgroup in a flat grid of nbx blocks per frame.  Workgroups
// are dealt to the 8 XCDs round-robin; when nbx is a multiple of 8, XCD x takes the x-th eighth
// of every frame's pixel blocks (a band of image rows).  Frames of a sweep are near-parallel, so
// a band of rows falls on the same part of the volume frame after frame, and each XCD's L2 keeps
// the accumulators of its own part instead of all eight sharing every line.
// The launch covers frames f0, f0 + 1, ...
__device__ __forceinline__ void frame_block(int nbx, int f0, int& bx, int& f) {
    const int g = blockIdx.x;
    if ((nbx & 7) == 0) {
        const int per = nbx >> 3, k = g >> 3;
        f = k / per;
        bx = (g & 7) * per + (k - f * per);
    } else {
        f = g / nbx;
        bx = g - f * nbx;
    }
    f += f0;
}

}  // namespace

// K1: T = P . C per frame (row-major, summed left to right), rigidity check of P.
__global__ void k_compose_frames(VolDev* vd, const float* __restrict__ poses, int n) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    FrameDesc d;
    if (!compose_frame(poses + (size_t)f * 16, vd->calib, vd->normal_axis, d)) atomicOr(&vd->st.bad_pose, 1);
    vd->frames[f] = d;
}

// K2: leader clustering of frame orientations, frames in order, by one workgroup.  The
// sequential rule (an entry joins its best qualifying bin, else opens a new one, else, with the
// codebook full, joins its best bin overall) only changes the codebook when an entry opens a bin,
// so chunks of 256 consecutive entries are tested in parallel against the current codebook:
// every entry before the chunk's first opener is final as tested, the opener takes the next bin,
// and the scan resumes after it.  Identical results in at most n / 256 + max_bins steps.
__global__ void __launch_bounds__(256) k_assign_bins(VolDev* vd, int n, int K0) {
    __shared__ double rep[kMaxBins][6];   // per bin: representative normal, then in-plane axis
    __shared__ int s_first, s_sat;
    const int tid = threadIdx.x;
    if (tid < K0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            rep[tid][a] = vd->rep_n[tid][a];
            rep[tid][3 + a] = vd->rep_x[tid][a];
        }
    }
    if (tid == 0) {
        s_first = 256;
        s_sat = vd->st.saturated;
    }
    int K = K0;
    const double ct = vd->cos_tol;
    const int kmax = vd->max_bins;
    for (int base = 0; base < n;) {
        __syncthreads();
        const int f = base + tid;
        double nf[3] = {0, 0, 0}, xf[3] = {0, 0, 0};
        int best = -1, any = -1;
        if (f < n) {
            const FrameDesc* fd = vd->frames + f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nf[a] = fd->nh[a];
                xf[a] = fd->xh[a];
            }
            double best_s = -INFINITY, any_s = -INFINITY;
            for (int b = 0; b < K; ++b) {   // strict > keeps the lowest index on ties
                const double rn[3] = {rep[b][0], rep[b][1], rep[b][2]};
                const double rx[3] = {rep[b][3], rep[b][4], rep[b][5]};
                const double dn = dot3(nf, rn);
                const double di = fabs(dot3(xf, rx));
                const double sc = dn + di;
                if (sc > any_s) {
                    any_s = sc;
                    any = b;
                }
                if (dn >= ct && di >= ct && sc > best_s) {
                    best_s = sc;
                    best = b;
                }
            }
            if (best < 0 && K < kmax) atomicMin(&s_first, tid);
        }
        __syncthreads();
        const int p = s_first;
        if (f < n && tid < p) {
            vd->frame_bin[f] = best >= 0 ? best : any;
            if (best < 0) s_sat = 1;   // only with the codebook full
        }
        if (tid == p) {
            vd->frame_bin[f] = K;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                rep[K][a] = nf[a];
                rep[K][3 + a] = xf[a];
            }
        }
        __syncthreads();
        if (tid == 0) s_first = 256;
        if (p < 256) {
            ++K;
            base += p + 1;
        } else {
            base += 256;
        }
    }
    __syncthreads();
    if (tid >= K0 && tid < K) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            vd->rep_n[tid][a] = rep[tid][a];
            vd->rep_x[tid][a] = rep[tid][3 + a];
        }
    }
    if (tid == 0) {
        vd->st.K = K;
        vd->st.saturated = s_sat;
    }
}

__device__ __forceinline__ void mark_entry(VolDev* vd, int64_t e) {
    const gptr<int32_t> te = (gptr<int32_t>)vd->table + e;
    const int cur = __hip_atomic_load(te, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == -1) {
        int expected = -1;
        if (__hip_atomic_compare_exchange_strong(te, &expected, -2, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            const uint32_t k = atomicAdd(&vd->st.new_count, 1u);
            if (k < vd->cap) ((gptr<int32_t>)vd->new_list)[k] = (int32_t)e;
        }
    } else if (cur >= 0) {
        const gptr<uint32_t> fl = (gptr<uint32_t>)vd->dirty_flags + cur;
        if (__hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
            __hip_atomic_exchange(fl, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            const uint32_t d = atomicAdd(&vd->st.dirty_count, 1u);
            ((gptr<int32_t>)vd->dirty_list)[d] = cur;
        }
    }
}

// Marks the entry of each lane that has one, except where the lane before it in the wave holds
// the same entry (neighbouring pixels mostly land in one brick): that lane marks it, which is
// all a mark needs.  Every lane of the wave must call this.
__device__ __forceinline__ void mark_wave(VolDev* vd, int64_t e) {
    const int64_t prev = __shfl_up(e, 1);
    if (e >= 0 && ((threadIdx.x & 63) == 0 || prev != e)) mark_entry(vd, e);
}

// K3a: mark every (bin, brick) that a pixel of the batch lands in.
__global__ void __launch_bounds__(256) k_mark_pixels(VolDev* vd, int w, int h, double sx, double sy, int f0) {
    int bx, f;
    frame_block((w * h + 255) >> 8, f0, bx, f);
    const PixelView v = pixel_view(vd);
    const FrameDesc fd = frame_uniform(v, f);
    const int bin = *((cptr<int32_t>)v.frame_bin + f);
    const int pix = bx * 256 + threadIdx.x;
    int64_t e = -1;
    int vx, vy, vz;
    if (pix < w * h && frame_voxel(&fd, v.origin, v.inv_h, v.nx, v.ny, v.nz, pix % w, pix / w, sx, sy, vx, vy, vz))
        e = brick_entry(v, bin, vx, vy, vz);
    mark_wave(vd, e);
}

// Fan probes: one frame descriptor per (frame, sector), each with the frame's pose and the
// sector's in-plane direction, so that the bin assignment runs over them as over frames.
__global__ void k_compose_fan(VolDev* vd, const float* __restrict__ poses, int n, FanArgs fan, int width) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * fan.sectors) return;
    const int f = k / fan.sectors;
    FrameDesc d;
    if (!compose_frame(poses + (size_t)f * 16, vd->calib, 2, d)) atomicOr(&vd->st.bad_pose, 1);
    fan_sector_axis(d, fan, width, k - f * fan.sectors);
    vd->frames[k] = d;
}

// K3a for fan frames: the pixel's (frame, sector) descriptor gives its pose and bin.
__global__ void __launch_bounds__(256) k_mark_fan(VolDev* vd, int w, int h, FanArgs fan, int f0) {
    int bx, f;
    frame_block((w * h + 255) >> 8, f0, bx, f);
    const int pix = bx * 256 + threadIdx.x;
    int64_t entry = -1;
    if (pix < w * h) {
        const int i = pix % w, j = pix / w;
        const int e = f * fan.sectors + i * fan.sectors / w;
        int vx, vy, vz;
        if (fan_voxel(vd->frames + e, vd->origin, vd->inv_h, vd->nx, vd->ny, vd->nz, fan, i, j, vx, vy, vz))
            entry = brick_entry(vd, vd->frame_bin[e], vx, vy, vz);
    }
    mark_wave(vd, entry);
}

// Undo the marks of a rejected batch and restore the codebook size.
__global__ void k_rollback(VolDev* vd, uint32_t new_count, uint32_t dirty_count, int K0, int sat0) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < new_count && k < vd->cap) vd->table[vd->new_list[k]] = -1;
    if (k < dirty_count) vd->dirty_flags[vd->dirty_list[k]] = 0u;
    if (k == 0) {
        vd->st.new_count = 0u;
        vd->st.dirty_count = 0u;
        vd->st.K = K0;
        vd->st.saturated = sat0;
        vd->st.bad_pose = 0;
    }
}

// K3b: give each marked entry the next pool slot, zero its accumulators and
// queue it for finalisation.
__global__ void __launch_bounds__(256) k_alloc(VolDev* vd, uint32_t new_count, uint32_t used,
                                               uint32_t dirty_count) {
    const uint32_t k = blockIdx.x;
    const uint32_t slot = used + k;
    unsigned long long* acc = vd->acc + (size_t)slot * kBrickVox;
    acc[threadIdx.x] = 0ull;
    acc[threadIdx.x + 256] = 0ull;
    if (threadIdx.x == 0) {
        vd->table[vd->new_list[k]] = (int32_t)slot;
        vd->dirty_flags[slot] = 1u;
        vd->dirty_list[dirty_count + k] = (int32_t)slot;
        if (k == 0) {
            vd->st.used = used + new_count;
            vd->st.dirty_count = dirty_count + new_count;
            vd->st.new_count = 0u;
        }
    }
}

// K4: add each pixel's intensity and a count to its (bin, voxel).
__global__ void __launch_bounds__(256) k_accumulate(const VolDev* __restrict__ vd, const uint8_t* __restrict__ frames,
                                                    int w, int h, double sx, double sy, int f0) {
    int bx, f;
    frame_block((w * h + 255) >> 8, f0, bx, f);
    const PixelView v = pixel_view(vd);
    const FrameDesc fd = frame_uniform(v, f);
    const int bin = *((cptr<int32_t>)v.frame_bin + f);
    const gptr<unsigned long long> acc = (gptr<unsigned long long>)((cptr<VolDev>)vd)->acc;
    const int pix = bx * 256 + threadIdx.x;
    int vx = 0, vy = 0, vz = 0;
    const bool ok =
        pix < w * h && frame_voxel(&fd, v.origin, v.inv_h, v.nx, v.ny, v.nz, pix % w, pix / w, sx, sy, vx, vy, vz);
    // the pixel and its table entry, both loads in flight together (lanes without a voxel read
    // entry 0 of each, and drop what they read)
    const unsigned long long inten = ((gptr<const uint8_t>)frames)[ok ? (size_t)f * w * h + pix : 0];
    const int slot = ((gptr<const int32_t>)v.table)[ok ? brick_entry(v, bin, vx, vy, vz) : 0];
    asm volatile("" ::"v"(inten), "v"(slot));
    if (!ok || slot < 0) return;   // slot < 0 is unreachable: every entry hit was marked and allocated
    __hip_atomic_fetch_add(acc + (size_t)slot * kBrickVox + brick_local(vx, vy, vz), (inten << 32) | 1ull,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// K4 for fan frames.
__global__ void __launch_bounds__(256) k_accumulate_fan(const VolDev* __restrict__ vd,
                                                        const uint8_t* __restrict__ frames, int w, int h, FanArgs fan,
                                                        int f0) {
    int bx, f;
    frame_block((w * h + 255) >> 8, f0, bx, f);
    const int pix = bx * 256 + threadIdx.x;
    if (pix >= w * h) return;
    const int i = pix % w, j = pix / w;
    const int e = f * fan.sectors + i * fan.sectors / w;
    int vx, vy, vz;
    if (!fan_voxel(vd->frames + e, vd->origin, vd->inv_h, vd->nx, vd->ny, vd->nz, fan, i, j, vx, vy, vz)) return;
    const int slot = vd->table[brick_entry(vd, vd->frame_bin[e], vx, vy, vz)];
    if (slot < 0) return;   // unreachable: every entry hit here was marked and allocated
    const unsigned long long inten = frames[(size_t)f * w * h + pix];
    atomicAdd(vd->acc + (size_t)slot * kBrickVox + brick_local(vx, vy, vz), (inten << 32) | 1ull);
}

// K5: exact sums -> stored (value, count) pairs of every dirty slot.
template <int DT>
__global__ void __launch_bounds__(256) k_finalize(VolDev* vd) {
    __shared__ float red[2][4];
    const int slot = vd->dirty_list[blockIdx.x];
    const unsigned long long* acc = vd->acc + (size_t)slot * kBrickVox;
    float a[2], c[2];
    uint32_t C[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const unsigned long long u = acc[threadIdx.x + 256 * k];
        C[k] = (uint32_t)(u & 0xFFFFFFFFull);
        const uint32_t S = (uint32_t)(u >> 32);
        c[k] = (float)C[k];
        a[k] = C[k] ? (float)S / c[k] : 0.0f;
    }
    const size_t base = (size_t)slot * kBrickVox;
    const float inv = 1.0f / 127.5f;
    if constexpr (DT == DARE_F32) {
        float2* d = (float2*)vd->data + base;
#pragma unroll
        for (int k = 0; k < 2; ++k) d[threadIdx.x + 256 * k] = make_float2(a[k], c[k]);
    } else if constexpr (DT == DARE_BF16 || DT == DARE_F16) {
        uint32_t* d = (uint32_t*)vd->data + base;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            uint32_t q = 0u, qc = 0u;
            if (C[k]) {
                const float x = (a[k] - 127.5f) * inv;
                if constexpr (DT == DARE_BF16) {
                    q = f32_to_bf16_rne(x);
                    qc = f32_to_bf16_rne(c[k]);
                } else {
                    q = f32_to_f16_rne(x);
                    qc = f32_to_f16_rne(fminf(c[k], 65504.0f));
                }
            }
            d[threadIdx.x + 256 * k] = q | (qc << 16);
        }
    } else {
        // per-brick scales: largest |a - 127.5| and largest count over occupied voxels
        float m = 0.0f, cm = 0.0f;
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (C[k]) {
                m = fmaxf(m, fabsf(a[k] - 127.5f));
                cm = fmaxf(cm, c[k]);
            }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            m = fmaxf(m, __shfl_xor(m, off));
            cm = fmaxf(cm, __shfl_xor(cm, off));
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = m;
            red[1][threadIdx.x >> 6] = cm;
        }
        __syncthreads();
        m = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
        cm = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
        const float s = fmaxf(m / 448.0f, 9.5367431640625e-07f);   // floor 2^-20
        const float t = cm > 0.0f ? cm / 448.0f : 1.0f;
        uint16_t* d = (uint16_t*)vd->data + base;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            uint32_t q = 0u, qc = 0u;
            if (C[k]) {
                q = f32_to_e4m3_rne((a[k] - 127.5f) / s);
                qc = f32_to_e4m3_rne(c[k] / t);
            }
            d[threadIdx.x + 256 * k] = (uint16_t)(q | (qc << 8));
        }
        if (threadIdx.x == 0) vd->scales[slot] = make_float2(s, t);
    }
    if (threadIdx.x == 0) {
        vd->dirty_flags[slot] = 0u;
        if (blockIdx.x == 0) vd->st.dirty_count = 0u;
    }
}

// Marks (-2) of a rejected batch that did not fit the new-entry list.
__global__ void k_clear_marks(int32_t* t, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        if (t[k] == -2) t[k] = -1;
}

__global__ void k_table_fill(int32_t* t, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        t[k] = -1;
}

// Test hooks: dense (bin, z, y, x) arrays <-> the bricked pool.
__global__ void k_dense_mark(VolDev* vd, const uint32_t* __restrict__ C, int K) {
    const int64_t nvox = (int64_t)vd->nx * vd->ny * vd->nz;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nvox * K;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (C[k] == 0u) continue;
        const int b = (int)(k / nvox);
        int64_t r = k - b * nvox;
        const int vx = (int)(r % vd->nx);
        r /= vd->nx;
        const int vy = (int)(r % vd->ny);
        const int vz = (int)(r / vd->ny);
        mark_entry(vd, brick_entry(vd, b, vx, vy, vz));
    }
}

__global__ void k_dense_scatter(const VolDev* vd, const uint32_t* __restrict__ S, const uint32_t* __restrict__ C,
                                int K) {
    const int64_t nvox = (int64_t)vd->nx * vd->ny * vd->nz;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nvox * K;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (C[k] == 0u) continue;
        const int b = (int)(k / nvox);
        int64_t r = k - b * nvox;
        const int vx = (int)(r % vd->nx);
        r /= vd->nx;
        const int vy = (int)(r % vd->ny);
        const int vz = (int)(r / vd->ny);
        const int slot = vd->table[brick_entry(vd, b, vx, vy, vz)];
        vd->acc[(size_t)slot * kBrickVox + brick_local(vx, vy, vz)] =
            ((unsigned long long)S[k] << 32) | (unsigned long long)C[k];
    }
}

__global__ void k_download_sums(const VolDev* vd, uint32_t* __restrict__ S, uint32_t* __restrict__ C, int K) {
    const int64_t nvox = (int64_t)vd->nx * vd->ny * vd->nz;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nvox * K;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(k / nvox);
        int64_t r = k - b * nvox;
        const int vx = (int)(r % vd->nx);
        r /= vd->nx;
        const int vy = (int)(r % vd->ny);
        const int vz = (int)(r / vd->ny);
        const int slot = vd->table[brick_entry(vd, b, vx, vy, vz)];
        unsigned long long u = 0ull;
        if (slot >= 0) u = vd->acc[(size_t)slot * kBrickVox + brick_local(vx, vy, vz)];
        S[k] = (uint32_t)(u >> 32);
        C[k] = (uint32_t)(u & 0xFFFFFFFFull);
    }
}

template <int DT>
__global__ void k_download_storage(const VolDev* vd, float* __restrict__ A, float* __restrict__ Cout, int K) {
    using P = Pair<DT>;
    const int64_t nvox = (int64_t)vd->nx * vd->ny * vd->nz;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nvox * K;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(k / nvox);
        int64_t r = k - b * nvox;
        const int vx = (int)(r % vd->nx);
        r /= vd->nx;
        const int vy = (int)(r % vd->ny);
        const int vz = (int)(r / vd->ny);
        const int slot = vd->table[brick_entry(vd, b, vx, vy, vz)];
        float a = 0.0f, c = 0.0f;
        if (slot >= 0) {
            const typename P::T p = ((const typename P::T*)vd->data)[(size_t)slot * kBrickVox + brick_local(vx, vy, vz)];
            const float2 s = DT == DARE_FP8_E4M3 ? vd->scales[slot] : make_float2(0.0f, 0.0f);
            P::decode(p, s, a, c);
            if (!(c > 0.0f)) { a = 0.0f; c = 0.0f; }
        }
        A[k] = a;
        Cout[k] = c;
    }
}

__global__ void k_copy_probe(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// ---------------------------------------------------------------------------- launchers

static inline int grid_for(int64_t n, int block, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

// Frames per launch of the per-pixel passes (flat grids of pixel blocks x frames), so that a
// grid stays below 2^24 workgroups.
int frames_per_launch(int n, int w, int h) {
    const int64_t nbx = ((int64_t)w * h + 255) / 256;
    const int64_t fc = ((int64_t)1 << 24) / nbx;
    return (int)std::max<int64_t>(1, std::min<int64_t>(n, fc));
}

hipError_t launch_compose_frames(const VolDev* vd, const float* poses, int n, hipStream_t stream) {
    hipLaunchKernelGGL(k_compose_frames, dim3((n + 63) / 64), dim3(64), 0, stream, const_cast<VolDev*>(vd), poses, n);
    return hipGetLastError();
}

hipError_t launch_assign_bins(VolDev* vd, int n, int K0, hipStream_t stream) {
    hipLaunchKernelGGL(k_assign_bins, dim3(1), dim3(256), 0, stream, vd, n, K0);
    return hipGetLastError();
}

hipError_t launch_mark_pixels(const VolDev* vd, int n, int w, int h, double sx, double sy, hipStream_t stream) {
    const int nbx = (w * h + 255) / 256, fc = frames_per_launch(n, w, h);
    for (int f0 = 0; f0 < n; f0 += fc)
        hipLaunchKernelGGL(k_mark_pixels, dim3(nbx * std::min(fc, n - f0)), dim3(256), 0, stream,
                           const_cast<VolDev*>(vd), w, h, sx, sy, f0);
    return hipGetLastError();
}

hipError_t launch_compose_fan(const VolDev* vd, const float* poses, int n, const FanArgs& fan, int width,
                              hipStream_t stream) {
    const int m = n * fan.sectors;
    hipLaunchKernelGGL(k_compose_fan, dim3((m + 63) / 64), dim3(64), 0, stream, const_cast<VolDev*>(vd), poses, n, fan,
                       width);
    return hipGetLastError();
}

hipError_t launch_mark_fan(const VolDev* vd, int n, int w, int h, const FanArgs& fan, hipStream_t stream) {
    const int nbx = (w * h + 255) / 256, fc = frames_per_launch(n, w, h);
    for (int f0 = 0; f0 < n; f0 += fc)
        hipLaunchKernelGGL(k_mark_fan, dim3(nbx * std::min(fc, n - f0)), dim3(256), 0, stream,
                           const_cast<VolDev*>(vd), w, h, fan, f0);
    return hipGetLastError();
}

hipError_t launch_accumulate_fan(const VolDev* vd, const uint8_t* frames, int n, int w, int h, const FanArgs& fan,
                                 hipStream_t stream) {
    const int nbx = (w * h + 255) / 256, fc = frames_per_launch(n, w, h);
    for (int f0 = 0; f0 < n; f0 += fc)
        hipLaunchKernelGGL(k_accumulate_fan, dim3(nbx * std::min(fc, n - f0)), dim3(256), 0, stream, vd, frames, w, h,
                           fan, f0);
    return hipGetLastError();
}

hipError_t launch_rollback(VolDev* vd, uint32_t new_count, uint32_t dirty_count, int K0, int sat0,
                           hipStream_t stream) {
    const uint32_t m = new_count > dirty_count ? new_count : dirty_count;
    hipLaunchKernelGGL(k_rollback, dim3(grid_for(m ? m : 1, 256)), dim3(256), 0, stream, vd, new_count,
                       dirty_count, K0, sat0);
    return hipGetLastError();
}

hipError_t launch_alloc(VolDev* vd, uint32_t new_count, uint32_t used, uint32_t dirty_count, hipStream_t stream) {
    if (new_count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_alloc, dim3(new_count), dim3(256), 0, stream, vd, new_count, used, dirty_count);
    return hipGetLastError();
}

hipError_t launch_accumulate(const VolDev* vd, const uint8_t* frames, int n, int w, int h, double sx, double sy,
                             hipStream_t stream) {
    const int nbx = (w * h + 255) / 256, fc = frames_per_launch(n, w, h);
    for (int f0 = 0; f0 < n; f0 += fc)
        hipLaunchKernelGGL(k_accumulate, dim3(nbx * std::min(fc, n - f0)), dim3(256), 0, stream, vd, frames, w, h, sx,
                           sy, f0);
    return hipGetLastError();
}

hipError_t launch_finalize(VolDev* vd, int dtype, uint32_t dirty_count, hipStream_t stream) {
    if (dirty_count == 0) return hipSuccess;
    switch (dtype) {
        case DARE_F32: hipLaunchKernelGGL(k_finalize<DARE_F32>, dim3(dirty_count), dim3(256), 0, stream, vd); break;
        case DARE_BF16: hipLaunchKernelGGL(k_finalize<DARE_BF16>, dim3(dirty_count), dim3(256), 0, stream, vd); break;
        case DARE_F16: hipLaunchKernelGGL(k_finalize<DARE_F16>, dim3(dirty_count), dim3(256), 0, stream, vd); break;
        case DARE_FP8_E4M3:
            hipLaunchKernelGGL(k_finalize<DARE_FP8_E4M3>, dim3(dirty_count), dim3(256), 0, stream, vd);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_clear_marks(int32_t* table, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_clear_marks, dim3(grid_for(n, 256, 4096)), dim3(256), 0, stream, table, n);
    return hipGetLastError();
}

hipError_t launch_table_fill(int32_t* table, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_table_fill, dim3(grid_for(n, 256, 4096)), dim3(256), 0, stream, table, n);
    return hipGetLastError();
}

hipError_t launch_dense_mark(const VolDev* vd, const uint32_t* C, int K, hipStream_t stream) {
    hipLaunchKernelGGL(k_dense_mark, dim3(4096), dim3(256), 0, stream, const_cast<VolDev*>(vd), C, K);
    return hipGetLastError();
}

hipError_t launch_dense_scatter(const VolDev* vd, const uint32_t* S, const uint32_t* C, int K, hipStream_t stream) {
    hipLaunchKernelGGL(k_dense_scatter, dim3(4096), dim3(256), 0, stream, vd, S, C, K);
    return hipGetLastError();
}

hipError_t launch_download_sums(const VolDev* vd, uint32_t* S, uint32_t* C, int K, int, int, int,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_download_sums, dim3(4096), dim3(256), 0, stream, vd, S, C, K);
    return hipGetLastError();
}

hipError_t launch_download_storage(const VolDev* vd, int dtype, float* A, float* C, int K, int, int, int,
                                   hipStream_t stream) {
    switch (dtype) {
        case DARE_F32: hipLaunchKernelGGL(k_download_storage<DARE_F32>, dim3(4096), dim3(256), 0, stream, vd, A, C, K); break;
        case DARE_BF16: hipLaunchKernelGGL(k_download_storage<DARE_BF16>, dim3(4096), dim3(256), 0, stream, vd, A, C, K); break;
        case DARE_F16: hipLaunchKernelGGL(k_download_storage<DARE_F16>, dim3(4096), dim3(256), 0, stream, vd, A, C, K); break;
        case DARE_FP8_E4M3:
            hipLaunchKernelGGL(k_download_storage<DARE_FP8_E4M3>, dim3(4096), dim3(256), 0, stream, vd, A, C, K);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, uint64_t n, hipStream_t stream) {
    const uint64_t n16 = n / 16;
    hipLaunchKernelGGL(k_copy_probe, dim3(grid_for((int64_t)n16, 256, 256 * 64)), dim3(256), 0, stream,
                       (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

}  // namespace dare
