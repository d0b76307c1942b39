// Per-sample store and its reslice: Sec. 2.1 ("Volume reconstruction", Fig. 1; "Reslicing",
// Eq. 1, Eq. 2) read literally.  Every in-grid pixel of every frame is kept as one sample
// (intensity, frame) in a flat store indexed by voxel, and a reslice weighs every sample by the
// orientation of its own frame; nothing is grouped into direction bins.  This is the reference
// formulation the binned grid approximates (with a bin tolerance of 0 the two coincide), kept at
// GPU speed so that the approximation can be measured on real sizes.
//
// Build (one call, replacing the store's content): compose the frames' poses; count the samples
// of every voxel with 32-bit atomics; an exclusive scan of the counts gives each voxel's first
// sample (CSR row offsets, voxels x fastest); a second pass writes every sample at its voxel's
// next free position.  The order of the samples inside a voxel depends on thread timing, and
// nothing depends on it: a reslice sums FP32 weights and weight x intensity products in FP64,
// where every term is a multiple of 2^-26 below 2^8, so the sums are exact in any order.
//
// Reslice: a small kernel evaluates Eq. 1, the two thresholds and Eq. 2 for every frame (the
// per-slice weight table); the reslice kernel keeps the table in LDS, takes 16 x 16 output pixels
// per workgroup, sums every voxel the tile reaches once (into LDS), and gives each pixel (FP64
// position) its neighbourhood's blend in one of two readings:
//   box   the (2R+1)^3 voxels around the nearest voxel, one weighted average over all their
//         samples: sum w I / sum w;
//   tent  the voxels with |c - v|_inf < R, each blended over its samples first, then averaged
//         with tent weights prod(1 - |c_a - v_a| / R) (the reading the binned grid uses).
#include <math.h>
#include <string.h>

#include <climits>
#include <cmath>

#include "dare_frames.h"
#include "dare_host.h"

#pragma clang fp contract(off)

using namespace dare;

namespace {

constexpr int kScanBlock = 1024;          // counts scanned per workgroup (4 per thread)
constexpr int kLutLds = 8192;             // frames whose weights a reslice workgroup keeps in LDS
constexpr int kTileBox = 1536;            // voxels whose sums a tiled reslice workgroup keeps in LDS
constexpr int32_t kMaxFrames = 1 << 24;   // frame index bits of a packed sample
constexpr uint64_t kAlignBytes = 256;

struct SampleDev {                        // device view of a store, passed by value
    int32_t n[3];
    int32_t n_frames;
    double origin[3];
    double inv_h;
    double calib[16];
    int64_t nvox;
    uint32_t* offsets;                    // nvox + 1: first sample of each voxel, then the total
    uint32_t* cursor;                     // nvox: per-voxel counts, then fill cursors (build)
    uint32_t* samples;                    // intensity | frame << 8
    FrameDesc* frames;
    float* lut;                           // per-frame weights of the reslice in flight
    unsigned long long* block_sums;       // scan scratch: one per kScanBlock counts, then the total
    int32_t* bad_pose;
};

struct LitSlice {                         // one reslice request, by value
    double t[3], e0[3], e1[3];            // rows 0..2 of T = P . C: translation, columns 0 and 1
    double sx, sy;
    int32_t W, H;
    int32_t mode;                         // 0: box, 1: tent
    int32_t R;
    float* out;
};

struct LutArgs {
    double xr[3], nr[3];                  // the slice's unit in-plane axis and normal
    double cos_n, cos_i, k_n, k_i;
};

uint64_t align_up(uint64_t x) { return (x + kAlignBytes - 1) / kAlignBytes * kAlignBytes; }

struct StoreLayout {
    uint64_t o_offsets, o_cursor, o_samples, o_frames, o_lut, o_sums, o_bad, total;
};

StoreLayout store_layout(const dare_geometry* g, int64_t max_samples, int32_t max_frames) {
    const uint64_t nvox = (uint64_t)g->dims[0] * (uint64_t)g->dims[1] * (uint64_t)g->dims[2];
    const uint64_t nblk = (nvox + kScanBlock - 1) / kScanBlock;
    StoreLayout L;
    uint64_t off = 0;
    L.o_offsets = off;
    off = align_up(off + (nvox + 1) * sizeof(uint32_t));
    L.o_cursor = off;
    off = align_up(off + nvox * sizeof(uint32_t));
    L.o_samples = off;
    off = align_up(off + (uint64_t)max_samples * sizeof(uint32_t));
    L.o_frames = off;
    off = align_up(off + (uint64_t)max_frames * sizeof(FrameDesc));
    L.o_lut = off;
    off = align_up(off + (uint64_t)max_frames * sizeof(float));
    L.o_sums = off;
    off = align_up(off + (nblk + 1) * sizeof(unsigned long long));
    L.o_bad = off;
    off = align_up(off + sizeof(int32_t));
    L.total = off;
    return L;
}

__device__ __forceinline__ int64_t voxel_index(const SampleDev& d, int vx, int vy, int vz) {
    return ((int64_t)vz * d.n[1] + vy) * d.n[0] + vx;
}

// Frame f's pose: T = P . C, unit in-plane axis and acquisition normal.
__global__ void k_lit_compose(SampleDev d, const float* __restrict__ poses, int n, int normal_axis) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    FrameDesc fr;
    if (!compose_frame(poses + (size_t)f * 16, d.calib, normal_axis, fr)) atomicOr(d.bad_pose, 1);
    d.frames[f] = fr;
}

// Pass 1 (count) or 2 (place) over every pixel of frames [f0, f0 + gridDim.y).
template <bool PLACE>
__global__ void __launch_bounds__(256) k_lit_pixels(SampleDev d, const uint8_t* __restrict__ frames, int w, int h,
                                                    double sx, double sy, int f0) {
    const int f = f0 + (int)blockIdx.y;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= w * h) return;
    int vx, vy, vz;
    if (!frame_voxel(d.frames + f, d.origin, d.inv_h, d.n[0], d.n[1], d.n[2], pix % w, pix / w, sx, sy, vx, vy, vz))
        return;
    const int64_t v = voxel_index(d, vx, vy, vz);
    const uint32_t k = atomicAdd(d.cursor + v, 1u);
    if constexpr (PLACE)
        d.samples[(size_t)d.offsets[v] + k] = (uint32_t)frames[(size_t)f * w * h + pix] | ((uint32_t)f << 8);
}

// Sum of the workgroup's 256 per-thread values (LDS tree).
__device__ __forceinline__ unsigned long long block_sum(unsigned long long x, unsigned long long* red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const unsigned long long r = red[0];
    __syncthreads();
    return r;
}

// Scan step 1: the sum of every block of kScanBlock counts.
__global__ void __launch_bounds__(256) k_lit_block_sums(SampleDev d) {
    __shared__ unsigned long long red[256];
    const int64_t b = blockIdx.x;
    const int64_t base = b * kScanBlock + (int64_t)threadIdx.x * 4;
    unsigned long long x = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < d.nvox) x += d.cursor[base + k];
    const unsigned long long s = block_sum(x, red);
    if (threadIdx.x == 0) d.block_sums[b] = s;
}

// Inclusive scan of the workgroup's 256 values (Hillis-Steele in LDS).
__device__ __forceinline__ unsigned long long block_scan(unsigned long long x, unsigned long long* buf) {
    buf[threadIdx.x] = x;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
        const unsigned long long y = (int)threadIdx.x >= s ? buf[threadIdx.x - s] : 0ull;
        __syncthreads();
        buf[threadIdx.x] += y;
        __syncthreads();
    }
    const unsigned long long r = buf[threadIdx.x];
    __syncthreads();
    return r;
}

// Scan step 2 (one workgroup): block sums -> their exclusive prefixes, the total after them.
__global__ void __launch_bounds__(256) k_lit_scan_sums(SampleDev d, int64_t nblk) {
    __shared__ unsigned long long buf[256];
    __shared__ unsigned long long last;
    unsigned long long carry = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const unsigned long long x = b < nblk ? d.block_sums[b] : 0ull;
        const unsigned long long inc = block_scan(x, buf);
        if (b < nblk) d.block_sums[b] = carry + inc - x;
        if (threadIdx.x == 255) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    if (threadIdx.x == 0) d.block_sums[nblk] = carry;
}

// Scan step 3: every voxel's first sample = its block's prefix + the counts before it in the block.
__global__ void __launch_bounds__(256) k_lit_scan_apply(SampleDev d, int64_t nblk) {
    __shared__ unsigned long long buf[256];
    const int64_t b = blockIdx.x;
    const int64_t base = b * kScanBlock + (int64_t)threadIdx.x * 4;
    uint32_t c[4];
    unsigned long long x = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = base + k < d.nvox ? d.cursor[base + k] : 0u;
        x += c[k];
    }
    unsigned long long run = d.block_sums[b] + block_scan(x, buf) - x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < d.nvox) d.offsets[base + k] = (uint32_t)run;
        run += c[k];
    }
    if (b == nblk - 1 && threadIdx.x == 0) d.offsets[d.nvox] = (uint32_t)d.block_sums[nblk];
}

// The slice's weight of every frame: Eq. 1 (signed normal term, absolute in-plane term), the two
// thresholds (kept on equality) and Eq. 2, in FP64, stored as FP32.
__global__ void __launch_bounds__(256) k_lit_lut(SampleDev d, LutArgs a) {
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= d.n_frames) return;
    const FrameDesc& fr = d.frames[f];
    const double dn = frame_dot3(fr.nh, a.nr);
    const double di = fabs(frame_dot3(fr.xh, a.xr));
    float w = 0.0f;
    if (dn >= a.cos_n && di >= a.cos_i) w = (float)exp(a.k_n * (dn - 1.0) + a.k_i * (di - 1.0));
    d.lut[f] = w;
}

// Pixel (i, j) of the slice: FP64 sample position c in voxel units and the voxel range of its
// reading (box: the (2R+1)^3 voxels around the nearest one; tent: |c - v|_inf < R), clipped to
// the grid.  False when no voxel is within reach (the pixel stays unassigned).
__device__ inline bool pixel_range(const SampleDev& d, const LitSlice& s, int i, int j, double c[3], int lo[3],
                                   int hi[3]) {
    const double is = (double)i * s.sx, js = (double)j * s.sy;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double q = (s.t[a] + is * s.e0[a]) + js * s.e1[a];
        c[a] = (q - d.origin[a]) * d.inv_h;
    }
    const double R = (double)s.R;
    // nothing within reach: also keeps the integer conversions below in range
    if (!(c[0] > -R - 1.0 && c[0] < d.n[0] + R && c[1] > -R - 1.0 && c[1] < d.n[1] + R && c[2] > -R - 1.0 &&
          c[2] < d.n[2] + R))
        return false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (s.mode == 0) {
            const int ctr = (int)floor(c[a] + 0.5);
            lo[a] = ctr - s.R;
            hi[a] = ctr + s.R;
        } else {
            lo[a] = (int)floor(c[a] - R) + 1;
            hi[a] = (int)ceil(c[a] + R) - 1;
        }
        lo[a] = max(lo[a], 0);
        hi[a] = min(hi[a], d.n[a] - 1);
    }
    return true;
}

// Sum of the weights and of weight x intensity over one voxel's samples, in store order (the
// sums are exact, so any order gives the same result).
__device__ inline void voxel_sums(const SampleDev& d, const float* __restrict__ lut, int64_t v, double& sw,
                                  double& swi) {
    const uint32_t o0 = d.offsets[v], o1 = d.offsets[v + 1];
    sw = 0.0;
    swi = 0.0;
    for (uint32_t k = o0; k < o1; ++k) {
        const uint32_t u = d.samples[k];
        const double w = (double)lut[u >> 8];
        sw += w;
        swi += w * (double)(u & 0xFFu);
    }
}

// The pixel's value from the per-voxel sums that `get(vx, vy, vz, sw, swi)` provides, voxels
// visited z, y, x: box, one average over all samples; tent, voxel averages blended with tent
// weights.  NaN when nothing contributes.
template <class Get>
__device__ inline float blend_range(const LitSlice& s, const double c[3], const int lo[3], const int hi[3], Get get) {
    const double R = (double)s.R;
    double num = 0.0, den = 0.0;
    for (int vz = lo[2]; vz <= hi[2]; ++vz)
        for (int vy = lo[1]; vy <= hi[1]; ++vy)
            for (int vx = lo[0]; vx <= hi[0]; ++vx) {
                double t = 1.0;
                if (s.mode != 0) {
                    const int v[3] = {vx, vy, vz};
#pragma unroll
                    for (int a = 0; a < 3; ++a) t *= fmax(0.0, 1.0 - fabs(c[a] - (double)v[a]) / R);
                    if (!(t > 0.0)) continue;
                }
                double sw, swi;
                get(vx, vy, vz, sw, swi);
                if (s.mode == 0) {
                    num += swi;
                    den += sw;
                } else if (sw > 0.0) {
                    num += t * (swi / sw);
                    den += t;
                }
            }
    return den > 0.0 ? (float)(num / den) : __builtin_nanf("");
}

// One workgroup per 16 x 16 tile of output pixels.  The pixels' voxel ranges are marked in a
// byte map over the tile's bounding box of voxels; each marked voxel's sums are computed once, by
// one thread, into LDS; every pixel then blends from LDS in the same voxel order as above, so
// the result is the same as summing per pixel.  A tile whose box exceeds kTileBox voxels (coarse
// output pitch, large radius) does sum per pixel.
__global__ void __launch_bounds__(256) k_lit_reslice_tiled(SampleDev d, LitSlice s, int tiles_x) {
    extern __shared__ float lut_s[];
    __shared__ double2 sums[kTileBox];
    __shared__ uint8_t mark[kTileBox];
    __shared__ int box[6];
    const int tid = threadIdx.x;
    const int F = d.n_frames;
    const bool in_lds = F <= kLutLds;
    if (in_lds)
        for (int k = tid; k < F; k += 256) lut_s[k] = d.lut[k];
    for (int k = tid; k < kTileBox; k += 256) mark[k] = 0;
    if (tid < 3) {
        box[tid] = INT_MAX;
        box[3 + tid] = INT_MIN;
    }
    __syncthreads();
    const float* __restrict__ lut = in_lds ? lut_s : d.lut;
    const int ty = (int)blockIdx.x / tiles_x, tx = (int)blockIdx.x - ty * tiles_x;
    const int i = tx * 16 + (tid & 15), j = ty * 16 + (tid >> 4);
    const bool inside = i < s.W && j < s.H;
    double c[3];
    int lo[3], hi[3];
    const bool reach = inside && pixel_range(d, s, i, j, c, lo, hi) && lo[0] <= hi[0] && lo[1] <= hi[1] &&
                       lo[2] <= hi[2];
    if (reach) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(&box[a], lo[a]);
            atomicMax(&box[3 + a], hi[a]);
        }
    }
    __syncthreads();
    const int b0[3] = {box[0], box[1], box[2]};
    const int64_t bd[3] = {(int64_t)box[3] - b0[0] + 1, (int64_t)box[4] - b0[1] + 1, (int64_t)box[5] - b0[2] + 1};
    const int64_t nbox = (bd[0] > 0 && bd[1] > 0 && bd[2] > 0) ? bd[0] * bd[1] * bd[2] : 0;
    const int64_t p = (int64_t)j * s.W + i;
    if (nbox > kTileBox) {   // uniform over the workgroup
        if (inside)
            s.out[p] = !reach ? __builtin_nanf("")
                              : blend_range(s, c, lo, hi, [&](int vx, int vy, int vz, double& sw, double& swi) {
                                    voxel_sums(d, lut, voxel_index(d, vx, vy, vz), sw, swi);
                                });
        return;
    }
    const int nx = (int)bd[0], ny = (int)bd[1];
    if (reach)   // every writer stores the same byte
        for (int vz = lo[2]; vz <= hi[2]; ++vz)
            for (int vy = lo[1]; vy <= hi[1]; ++vy)
                for (int vx = lo[0]; vx <= hi[0]; ++vx) mark[((vz - b0[2]) * ny + (vy - b0[1])) * nx + (vx - b0[0])] = 1;
    __syncthreads();
    // a thread's (up to kTileBox / 256) voxels: all row offsets loaded before any sample
    constexpr int kPer = kTileBox / 256;
    uint32_t o0[kPer], o1[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int k = tid + 256 * q;
        o0[q] = o1[q] = 0u;
        if (k < (int)nbox && mark[k]) {
            const int lx = k % nx, r = k / nx, ly = r % ny, lz = r / ny;
            const int64_t v = voxel_index(d, b0[0] + lx, b0[1] + ly, b0[2] + lz);
            o0[q] = d.offsets[v];
            o1[q] = d.offsets[v + 1];
        }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int k = tid + 256 * q;
        if (k < (int)nbox && mark[k]) {
            double sw = 0.0, swi = 0.0;
#pragma unroll 4
            for (uint32_t e = o0[q]; e < o1[q]; ++e) {
                const uint32_t u = d.samples[e];
                const double w = (double)lut[u >> 8];
                sw += w;
                swi += w * (double)(u & 0xFFu);
            }
            sums[k] = make_double2(sw, swi);
        }
    }
    __syncthreads();
    if (!inside) return;
    s.out[p] = !reach ? __builtin_nanf("")
                      : blend_range(s, c, lo, hi, [&](int vx, int vy, int vz, double& sw, double& swi) {
                            const double2 q = sums[((vz - b0[2]) * ny + (vy - b0[1])) * nx + (vx - b0[0])];
                            sw = q.x;
                            swi = q.y;
                        });
}

// Empty store: every voxel's range is [0, 0).
dare_status clear_store(dare_samples* st, hipStream_t stream);

}  // namespace

struct dare_samples {
    int device = 0;
    dare_geometry g{};
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    int64_t max_samples = 0;
    int32_t max_frames = 0;
    int32_t normal_axis = 2;
    int64_t n_samples = 0;
    SampleDev d{};
    unsigned long long* pinned = nullptr;   // readback: scan total, pose flag
};

namespace {

dare_status clear_store(dare_samples* st, hipStream_t stream) {
    HIP_TRY(hipMemsetAsync(st->d.offsets, 0, (size_t)(st->d.nvox + 1) * sizeof(uint32_t), stream));
    st->d.n_frames = 0;
    st->n_samples = 0;
    return DARE_OK;
}

}  // namespace

extern "C" {

uint64_t dare_samples_arena_bytes(const dare_geometry* g, int64_t max_samples, int32_t max_frames) {
    if (check_volume_geometry(g) != DARE_OK || max_samples < 0 || max_frames < 1 || max_frames > kMaxFrames)
        return 0;
    return store_layout(g, max_samples, max_frames).total;
}

dare_status dare_samples_create(const dare_geometry* g, int64_t max_samples, int32_t max_frames, void* arena_dev,
                                uint64_t arena_bytes, dare_samples** out) {
    if (!out) return DARE_ERR_INVALID_ARG;
    *out = nullptr;
    const dare_status gs = check_volume_geometry(g);
    if (gs != DARE_OK) return gs;
    if (!arena_dev || ((uintptr_t)arena_dev % kAlignBytes) != 0) return DARE_ERR_INVALID_ARG;
    if (max_samples < 0 || max_samples > (int64_t)UINT32_MAX || max_frames < 1 || max_frames > kMaxFrames)
        return DARE_ERR_INVALID_ARG;
    const StoreLayout L = store_layout(g, max_samples, max_frames);
    if (arena_bytes < L.total) return DARE_ERR_INVALID_ARG;
    dare_samples* st = new dare_samples();
    if (hipGetDevice(&st->device) != hipSuccess) {
        delete st;
        return DARE_ERR_HIP;
    }
    st->g = *g;
    st->arena = (char*)arena_dev;
    st->arena_bytes = arena_bytes;
    st->max_samples = max_samples;
    st->max_frames = max_frames;
    SampleDev& d = st->d;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = g->dims[a];
        d.origin[a] = g->origin_mm[a];
    }
    d.inv_h = 1.0 / g->spacing_mm;
    memcpy(d.calib, g->calib, sizeof(d.calib));
    d.nvox = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
    d.offsets = (uint32_t*)(st->arena + L.o_offsets);
    d.cursor = (uint32_t*)(st->arena + L.o_cursor);
    d.samples = (uint32_t*)(st->arena + L.o_samples);
    d.frames = (FrameDesc*)(st->arena + L.o_frames);
    d.lut = (float*)(st->arena + L.o_lut);
    d.block_sums = (unsigned long long*)(st->arena + L.o_sums);
    d.bad_pose = (int32_t*)(st->arena + L.o_bad);
    if (hipHostMalloc((void**)&st->pinned, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        delete st;
        return DARE_ERR_HIP;
    }
    if (clear_store(st, nullptr) != DARE_OK || hipDeviceSynchronize() != hipSuccess) {
        (void)hipHostFree(st->pinned);
        delete st;
        return DARE_ERR_HIP;
    }
    *out = st;
    return DARE_OK;
}

dare_status dare_samples_destroy(dare_samples* st) {
    if (!st) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(st->device);
    const hipError_t e = hipDeviceSynchronize();
    if (st->pinned) (void)hipHostFree(st->pinned);
    delete st;
    return hip_status(e);
}

dare_status dare_samples_build(dare_samples* st, const uint8_t* frames_dev, int32_t n, int32_t w, int32_t h,
                               const double pitch_mm[2], const float* probe_poses_dev, int32_t normal_axis,
                               void* stream_) {
    if (!st || !frames_dev || !probe_poses_dev || !pitch_mm || n <= 0 || w <= 0 || h <= 0) return DARE_ERR_INVALID_ARG;
    if (n > st->max_frames || (int64_t)w * h > (int64_t)1 << 30) return DARE_ERR_INVALID_ARG;
    if (!(pitch_mm[0] > 0.0) || !(pitch_mm[1] > 0.0) || !std::isfinite(pitch_mm[0]) || !std::isfinite(pitch_mm[1]))
        return DARE_ERR_INVALID_ARG;
    if (normal_axis != 1 && normal_axis != 2) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(st->device);
    hipStream_t stream = (hipStream_t)stream_;
    SampleDev& d = st->d;
    const int64_t nblk = (d.nvox + kScanBlock - 1) / kScanBlock;
    if (nblk > (int64_t)INT32_MAX) return DARE_ERR_INVALID_ARG;
    {
        const dare_status cs = clear_store(st, stream);
        if (cs != DARE_OK) return cs;
    }
    // poses
    HIP_TRY(hipMemsetAsync(d.bad_pose, 0, sizeof(int32_t), stream));
    hipLaunchKernelGGL(k_lit_compose, dim3((n + 255) / 256), dim3(256), 0, stream, d, probe_poses_dev, n,
                       normal_axis);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(st->pinned + 1, d.bad_pose, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (*(const int32_t*)(st->pinned + 1) != 0) return DARE_ERR_BAD_POSE;
    // counts, then their exclusive scan
    const dim3 pgrid((unsigned)((w * h + 255) / 256));
    HIP_TRY(hipMemsetAsync(d.cursor, 0, (size_t)d.nvox * sizeof(uint32_t), stream));
    for (int f0 = 0; f0 < n; f0 += 65535) {
        const int nf = n - f0 < 65535 ? n - f0 : 65535;
        hipLaunchKernelGGL(k_lit_pixels<false>, dim3(pgrid.x, nf), dim3(256), 0, stream, d, frames_dev, w, h,
                           pitch_mm[0], pitch_mm[1], f0);
    }
    hipLaunchKernelGGL(k_lit_block_sums, dim3((unsigned)nblk), dim3(256), 0, stream, d);
    hipLaunchKernelGGL(k_lit_scan_sums, dim3(1), dim3(256), 0, stream, d, nblk);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(st->pinned, d.block_sums + nblk, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const unsigned long long total = st->pinned[0];
    if (total > (unsigned long long)st->max_samples) return DARE_ERR_BUDGET;   // the store stays empty
    hipLaunchKernelGGL(k_lit_scan_apply, dim3((unsigned)nblk), dim3(256), 0, stream, d, nblk);
    // samples at their voxels' positions
    HIP_TRY(hipMemsetAsync(d.cursor, 0, (size_t)d.nvox * sizeof(uint32_t), stream));
    for (int f0 = 0; f0 < n; f0 += 65535) {
        const int nf = n - f0 < 65535 ? n - f0 : 65535;
        hipLaunchKernelGGL(k_lit_pixels<true>, dim3(pgrid.x, nf), dim3(256), 0, stream, d, frames_dev, w, h,
                           pitch_mm[0], pitch_mm[1], f0);
    }
    HIP_TRY(hipGetLastError());
    d.n_frames = n;
    st->normal_axis = normal_axis;
    st->n_samples = (int64_t)total;
    return DARE_OK;
}

dare_status dare_samples_count(const dare_samples* st, int64_t* n_samples, int32_t* n_frames) {
    if (!st || !n_samples || !n_frames) return DARE_ERR_INVALID_ARG;
    *n_samples = st->n_samples;
    *n_frames = st->d.n_frames;
    return DARE_OK;
}

dare_status dare_samples_reslice(const dare_samples* st, const dare_params* p, const dare_slice_spec* spec,
                                 int32_t mode, float* out_dev, void* stream_) {
    if (!st || !out_dev || (mode != DARE_LITERAL_BOX && mode != DARE_LITERAL_TENT)) return DARE_ERR_INVALID_ARG;
    const dare_status ps = check_method_params(p);
    if (ps != DARE_OK) return ps;
    if (st->d.n_frames > 0 && p->normal_axis != st->normal_axis) return DARE_ERR_INVALID_ARG;
    const dare_status ss = check_slice_spec(spec);
    if (ss != DARE_OK) return ss;
    DeviceGuard dg(st->device);
    hipStream_t stream = (hipStream_t)stream_;
    double T[16];
    compose_pose(spec->probe_pose, st->g.calib, T);
    LitSlice s{};
    for (int a = 0; a < 3; ++a) {
        s.t[a] = T[a * 4 + 3];
        s.e0[a] = T[a * 4 + 0];
        s.e1[a] = T[a * 4 + 1];
    }
    s.sx = spec->pitch_mm[0];
    s.sy = spec->pitch_mm[1];
    s.W = spec->width;
    s.H = spec->height;
    s.mode = mode;
    s.R = (int32_t)p->radius_vox;
    s.out = out_dev;
    if (st->d.n_frames > 0) {
        LutArgs la{};
        const int ax = p->normal_axis;
        const double e0[3] = {T[0], T[4], T[8]}, en[3] = {T[ax], T[4 + ax], T[8 + ax]};
        const double l0 = sqrt((e0[0] * e0[0] + e0[1] * e0[1]) + e0[2] * e0[2]);
        const double ln = sqrt((en[0] * en[0] + en[1] * en[1]) + en[2] * en[2]);
        for (int a = 0; a < 3; ++a) {
            la.xr[a] = e0[a] / l0;
            la.nr[a] = en[a] / ln;
        }
        const double kPi = 3.14159265358979323846;
        la.cos_n = cos(p->thr_normal_deg * kPi / 180.0);
        la.cos_i = cos(p->thr_inplane_deg * kPi / 180.0);
        la.k_n = p->k_normal;
        la.k_i = p->k_inplane;
        hipLaunchKernelGGL(k_lit_lut, dim3((st->d.n_frames + 255) / 256), dim3(256), 0, stream, st->d, la);
    }
    const size_t lds = st->d.n_frames <= kLutLds ? (size_t)st->d.n_frames * sizeof(float) : 0;
    const int tiles_x = (s.W + 15) / 16;
    const int64_t tiles = (int64_t)tiles_x * ((s.H + 15) / 16);
    hipLaunchKernelGGL(k_lit_reslice_tiled, dim3((unsigned)tiles), dim3(256), lds, stream, st->d, s, tiles_x);
    return hip_status(hipGetLastError());
}

}  // extern "C"
