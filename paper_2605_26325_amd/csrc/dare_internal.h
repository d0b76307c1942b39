// Internal layout shared by the library's HIP sources (not part of the ABI).
//
// A volume lives entirely in one caller-supplied device arena:
//
//   VolDev        geometry, parameters, codebook and counters        (1 per volume)
//   table         int32 [max_bins][nbz][nby][nbx]: pool slot of each (bin, 8^3 brick), -1 = empty
//   frame scratch FrameDesc [FRAME_CHUNK] + bin index per frame of the current batch
//   new_list      int32 [cap]: table entries marked by the current batch
//   dirty_list    int32 [cap]: slots touched by the current batch
//   dirty_flags   uint32 [cap]
//   acc           uint64 [cap][512]: (sum << 32) | count per voxel, exact integers
//   data          [cap][512] stored (value, count) pairs in the volume's dtype
//   scales        float2 [cap]: FP8 value and count scales per slot
//
// Inside a brick, voxel (lx, ly, lz) is at (lz * 8 + ly) * 8 + lx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dare.h"

namespace dare {

constexpr int kBrick = 8;
constexpr int kBrickVox = 512;

// Position of voxel (vx, vy, vz) inside its 8^3 brick.  The brick is 64 cubes of 2 x 2 x 2
// voxels (x fastest inside a cube), the cubes ordered z fastest, then y, then x: a 128-byte line
// of FP32 pairs holds a 2 x 2 x 4 block (BF16: 2 x 2 x 8), so the 2-3 voxel thick slab of a
// slice whose normal is near x or y (freehand sweeps image near-vertical planes) uses most of
// every line it touches, where x-fastest rows of 8 would be used for 2-3 voxels of 8 when the
// normal is near x.  Every kernel that reads or writes brick storage (accumulators, stored
// pairs) takes positions from here.
__host__ __device__ constexpr int brick_local(int vx, int vy, int vz) {
    return ((vx & 6) << 6) | ((vy & 6) << 4) | ((vz & 6) << 2) | ((vz & 1) << 2) | ((vy & 1) << 1) | (vx & 1);
}
constexpr int kMaxBins = 64;
constexpr int kFrameChunk = 4096;
constexpr int kTile = 16;                 // reslice output tile edge (pixels)

struct VolState {                         // read back by the host at sync points
    int32_t K;
    int32_t saturated;
    int32_t bad_pose;
    uint32_t used;                        // allocated slots
    uint32_t new_count;                   // entries marked by the current batch
    uint32_t dirty_count;                 // slots to finalize
    uint32_t pad[2];
};

struct VolDev {
    VolState st;
    // geometry
    double origin[3];
    double h, inv_h;
    int32_t nx, ny, nz;
    int32_t nbx, nby, nbz;
    int64_t nbricks;                      // bricks per bin
    double calib[16];
    // parameters
    double k_normal, k_inplane;
    double cos_normal, cos_inplane;       // cos of the thresholds (host libm)
    double cos_tol;                       // cos of the bin tolerance
    int32_t radius;                       // R in voxels
    int32_t max_bins;
    int32_t normal_axis;
    int32_t dtype;
    uint32_t cap;                         // slots in the pool
    uint32_t pad0;
    // arena pointers
    int32_t* table;
    struct FrameDesc* frames;
    int32_t* frame_bin;
    int32_t* new_list;
    int32_t* dirty_list;
    uint32_t* dirty_flags;
    unsigned long long* acc;
    void* data;
    float2* scales;
    // codebook: representative acquisition normal and in-plane axis per bin
    double rep_n[kMaxBins][3];
    double rep_x[kMaxBins][3];
};

struct FrameDesc {                        // one composed frame pose
    double t[3], e0[3], e1[3];            // translation and raw columns 0, 1 of T = P.C
    double xh[3], nh[3];                  // unit in-plane axis and acquisition normal
    double pad;
};

struct SliceArgs {                        // one reslice request, by value
    double P[16];                         // probe pose, row-major
    double sx, sy;
    int32_t W, H;
    int32_t tiles_x, tiles;               // 16x16 tiles along x, total tiles
    float* out;
};

// What the reslice passes read of a volume header, copied next to the request's
// setup so that a workgroup fetches everything it needs in one burst of loads.
struct VolView {
    const int32_t* table;
    const void* data;
    const float2* scales;
    int64_t nbricks;
    int32_t n[3];
    int32_t nbx, nby;
    uint32_t cap;                         // slots in the pool
    double origin[3];
    double inv_h;
};

// Per-slice reslice setup: composed pose, surviving bins and their Eq. 2 weights, and the
// plane frame used by the footprint tests.
struct SliceCore {
    double T[12];                         // rows 0..2 of the image pose T = P . C
    float fm[3], fu[3], fw[3];            // unit normal and in-plane unit axes, voxel units
    float lu, lw;                         // voxels per pixel step along the two in-plane axes
    int dax;                              // dominant axis of the normal
    int kact;                             // surviving bins
    int act_bin[kMaxBins];
    float act_w[kMaxBins];
};

inline int pair_bytes(int dtype) {
    switch (dtype) {
        case DARE_F32: return 8;
        case DARE_BF16: return 4;
        case DARE_F16: return 4;
        case DARE_FP8_E4M3: return 2;
    }
    return 0;
}

// Host launchers (defined in the .hip files), all asynchronous on `stream`.
hipError_t launch_compose_frames(const VolDev* vd, const float* poses, int n, hipStream_t stream);
hipError_t launch_assign_bins(VolDev* vd, int n, int K0, hipStream_t stream);
hipError_t launch_mark_pixels(const VolDev* vd, int n, int w, int h, double sx, double sy,
                              hipStream_t stream);
hipError_t launch_rollback(VolDev* vd, uint32_t new_count, uint32_t dirty_count, int K0, int sat0,
                           hipStream_t stream);
hipError_t launch_alloc(VolDev* vd, uint32_t new_count, uint32_t used, uint32_t dirty_count,
                        hipStream_t stream);
hipError_t launch_accumulate(const VolDev* vd, const uint8_t* frames, int n, int w, int h, double sx,
                             double sy, hipStream_t stream);
hipError_t launch_finalize(VolDev* vd, int dtype, uint32_t dirty_count, hipStream_t stream);
hipError_t launch_table_fill(int32_t* table, int64_t n, hipStream_t stream);
hipError_t launch_clear_marks(int32_t* table, int64_t n, hipStream_t stream);
hipError_t launch_dense_mark(const VolDev* vd, const uint32_t* C, int K, hipStream_t stream);
hipError_t launch_dense_scatter(const VolDev* vd, const uint32_t* S, const uint32_t* C, int K,
                                hipStream_t stream);
hipError_t launch_download_sums(const VolDev* vd, uint32_t* S, uint32_t* C, int K, int nx, int ny, int nz,
                                hipStream_t stream);
hipError_t launch_download_storage(const VolDev* vd, int dtype, float* A, float* C, int K, int nx, int ny,
                                   int nz, hipStream_t stream);
// One request at radius 1 or above 4; every kernel reads the volume header `vd` and evaluates
// the slice setup on the device.
hipError_t launch_reslice(const VolDev* vd, int dtype, int radius, const SliceArgs& s, hipStream_t stream);
hipError_t launch_copy_probe(const void* src, void* dst, uint64_t n, hipStream_t stream);

// Reslice work decomposition: lanes per output pixel (1 for radius 1) and the
// number of workgroup units of a W x H request.
int reslice_lanes(int radius);
int64_t reslice_units(int radius, int W, int H);

}  // namespace dare
