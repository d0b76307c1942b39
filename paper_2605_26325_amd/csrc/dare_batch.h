// Batched reslice: request table, device setup records and work units, shared by the batch
// kernels and the host planners (the C ABI's batch call and the server).
#pragma once

#include <cstddef>

#include "dare_internal.h"

namespace dare {

// One request as the host uploads it: the volume's device header and the slice.
struct BatchReq {
    const VolDev* vol;
    SliceArgs s;
};

// Batch header at the start of a workspace: int32 counts {units, requests, units at the list's
// back, 0}, then the radius-1 tile kernel's claim counter of each of the 8 XCDs, each on a
// 256-byte line of its own (claims[x][0]: counters that share a line serialise each other's
// atomics).  At radius 1 the units are appended on the device, so counts[0] and counts[2] must be
// uploaded as 0, and so must the claims; at other radii the host uploads the unit list and its
// length in counts[0].  The kernels address the header as int32 words from counts.
constexpr int kClaimStride = 64;          // int32 words between two XCDs' claim counters
struct BatchHeader {
    int32_t counts[4];
    int32_t pad[kClaimStride - 4];
    int32_t claims[8][kClaimStride];
};
static_assert(offsetof(BatchHeader, claims) == kClaimStride * sizeof(int32_t), "claims follow one line of counts");

constexpr int kBatchMaxReq = 4096;        // requests per launch group (grid of the setup pass)

// Per-request record of a radius-1 reslice, written on the device by the request setup (FP64
// pose, Eq. 1 gates and Eq. 2 weights in the SliceCore part).
struct SliceRec : SliceCore {
    double c00[3], ex[3], ey[3];          // voxel coordinates of pixel (i, j): c00 + i ex + j ey
    VolView vol;
    float* out;
    int32_t W, H;
    int32_t mode;                         // 0: every pixel NaN, 1: staged tiles, 2: per-pixel gather
    int32_t tile;                         // tile edge in pixels (16 unless staged in 32 x 32 tiles)
    int32_t tiles_x, ntiles;
    float half, slop;                     // slab half-depth along the dominant axis; FP32 test slop
    int32_t depth;                        // voxels per slab run
    int32_t pad;
};

// Per-tile record of a staged radius-1 request, written by the batch setup pass (one lane per
// tile): the tile's pixels, its voxel box and run geometry, and the divisions the staging phases
// need (multiplier m and divisor d of an exact small-integer division).
struct TileRec {
    int32_t r;                            // request
    int32_t mode;                         // 0: every pixel NaN, 1: staged
    int32_t i0, j0, ni, nj;               // first pixel and pixel counts
    int32_t lo[3], hi[3];                 // voxel box, clipped to [-1, n]
    int32_t bp, bq, ncols, depth;         // box columns along p and q, their number, run depth
    int32_t blo[3], bdim[3], nbb, kactp;  // in-grid bricks of the box; bins per slot row
    uint32_t m_bp, m_kactp, m_bdx, m_bdy; // division multipliers for bp, kactp, bdim[0], bdim[1]
    float c0[3];                          // voxel coordinates of the tile's first pixel
    float thr_n, thr_u, thr_v, hi_u, hi_v, inv_md, half;
};

// Radius 1, one request: one workgroup per 16 x 16 tile, each evaluating the request setup.
hipError_t launch_reslice_tile(const VolDev* vd, int dtype, const SliceArgs& s, hipStream_t stream);
// Radius 1, a batch: setup pass (one workgroup per request: the request record, then one tile
// record per thread) + persistent tile kernel + the per-pixel kernel for requests too coarse to stage.
// `counts[0]`, `counts[2]` and the claims must hold 0 and `counts[1]` the number of requests when the stream
// reaches the launch; `units` and `tiles` hold `cap` entries, at least tile_units_max() per
// request in all.
hipError_t launch_tiles_batch(int dtype, const BatchReq* reqs, SliceRec* recs, int2* units, TileRec* tiles,
                              int* counts, int nreq_max, int cap, hipStream_t stream);
// Largest number of units of a W x H radius-1 request (16 x 16 tiles).
int64_t tile_units_max(int W, int H);

// Any radius: radius 1 runs the setup pass and the tile kernels over device-built units and tile
// records (`cap` entries of `units` and `tiles`; grids sized to the device, `grid` unused); other
// radii run the host-built (request, unit) table (`counts[0]` units) over `grid` workgroups.  nreq_max bounds the
// requests of any batch launched with these arguments (the counts are read on the device, so a
// captured graph can be replayed with fewer).
hipError_t launch_reslice_batch(int dtype, int radius, const BatchReq* reqs, SliceRec* recs, int2* units,
                                TileRec* tiles, int* counts, int nreq_max, int cap, int grid, hipStream_t stream);

}  // namespace dare
