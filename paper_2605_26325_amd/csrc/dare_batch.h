// Batched reslice: request table, device setup records and their flat index spaces, shared by
// the batch kernels and the host planners (the C ABI's batch call and the server).
#pragma once

#include "dare_internal.h"

namespace dare {

struct BatchReq {
    const VolDev* vol;
    SliceArgs s;
    SliceCore core;                       // radius 1: the per-slice setup, computed on the host
    // Radius-1 passes run over two flat index spaces: the requests' slabs back to back
    // (v_beg: first index of this request's slab) and their pixels (p_beg), each request's
    // range padded to whole blocks of kFlatBlock.  The slab itself lives at float offset v_off
    // of the scratch; v_cap floats (a multiple of kFlatBlock), 0 for none.
    int64_t v_beg, v_off, v_cap;
    int64_t p_beg;
};

// Batch header at the start of a workspace: int32 {units, requests, 0, 0}, then int64
// {slab index total, pixel index total}, both multiples of kFlatBlock.  counts[2] must be uploaded
// as 0: the setup pass counts there the requests that gather per pixel.
struct BatchHeader {
    int32_t counts[4];
    int64_t totals[2];
};

constexpr int kFlatShift = 10;            // batched passes: elements per workgroup iteration ...
constexpr int kFlatBlock = 1 << kFlatShift;   // ... (4 per thread)
constexpr int kBatchMaxReq = 4096;        // requests per launch group (LDS request tables of the passes)
constexpr int kSlabDepthMax = 10;         // deepest slab run (a plane tilted 45 deg in both axes needs 9)
constexpr int kSlabTileP = 8;             // slab column tile: 8 along p (a brick row when p is x) ...
constexpr int kSlabTileQ = 4;             // ... by 4 along q
constexpr int kSlabPerPixel = 12;         // slab floats per output pixel beyond which pixels gather directly

// Per-request setup record written by the batch setup pass.
struct SliceSetup : SliceCore {
    // slab of the whole slice: voxels within the trilinear support of the slice
    // plane, enumerated as runs of `depth` voxels along the dominant axis, one run per column
    // of the other two axes (pax fastest) over the slice's bounding box
    int pax, qax;
    int lo_p, lo_q, dim_p, dim_q;
    int depth;
    int ntp;                              // column tiles along p
    int ncand;                            // tiles * depth * tile columns, 0 when nothing to stage
    int staged;                           // 1: slab staged; 0: gather per pixel
    float c0[3];                          // voxel coordinates of pixel (0, 0)
    float thr_n, thr_u, thr_v, len_u, len_v, inv_md, half;
    // copies of the request and its volume (batched passes)
    int64_t act_off[kMaxBins];            // act_bin[k] * bricks per bin: table offset of bin k
    double inv_depth, inv_ntp;            // FP64 reciprocals for exact index division
    VolView vol;
    double sx, sy;
    int32_t W, H;
    float* out;
    int64_t v_off;
};

// nreq_max bounds the requests of any batch launched with these arguments (the count itself is
// read from `counts` on the device, so a captured graph can be replayed with fewer).
hipError_t launch_reslice_batch(int dtype, int radius, const BatchReq* reqs, SliceSetup* setups, const int2* units,
                                const int* counts, float* scratch, int nreq_max, int grid, hipStream_t stream);
// Slab floats to reserve for a radius-1 request (0 when its pixels should gather directly):
// the slice's voxel bounding box, two voxels of margin, padded to whole column tiles, over
// the largest pair of axes, times the deepest run, capped at kSlabPerPixel per pixel.
// Defined with the C ABI.
int64_t slab_floats(const dare_volume* v, const dare_slice_spec* spec);
// The per-slice setup of a radius-1 reslice (pose, surviving bins and weights, plane frame),
// computed on the host from its copy of the volume's codebook.  Defined with the C ABI.
void host_core(const dare_volume* v, const dare_slice_spec* spec, SliceCore* core);

}  // namespace dare
