// Reslice at interpolation radius 2..4 with per-tile LDS staging of the voxel direction
// blends (dare_reslice_rs.hip).  Other radii use the per-pixel kernels of dare_reslice.hip.
#pragma once

#include "dare_batch.h"

namespace dare {

inline bool staged_radius(int radius) { return radius >= 2 && radius <= 4; }

hipError_t launch_reslice_staged(const VolDev* vd, int dtype, int radius, const SliceArgs& s, hipStream_t stream);
// Batched form over (request, tile) units; counts[0] holds the number of units.
hipError_t launch_reslice_staged_batch(int dtype, int radius, const BatchReq* reqs, const int2* units,
                                       const int* counts, int grid, hipStream_t stream);
// Work units of a W x H request at this radius for the batched kernels (tiles when staged).
int64_t batch_units(int radius, int W, int H);

}  // namespace dare
