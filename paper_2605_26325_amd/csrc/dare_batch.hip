// Batched reslice: many requests (volumes, poses, sizes) in a fixed set of launches whose
// counts are read from device memory, so that a captured graph can replay any batch.
// Radius 1 runs the request setup pass and the persistent tile kernel (dare_tiles.hip); radii
// 2..4 run the staged (request, tile) kernel (dare_reslice_rs.hip); larger radii run the
// (request, unit) table through the lane-split neighbourhood kernel below.
#include "dare_staged.h"
#include "dare_reslice_dev.h"

namespace dare {

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

hipError_t launch_reslice_batch(int dtype, int radius, const BatchReq* reqs, SliceRec* recs, int2* units,
                                TileRec* tiles, int* counts, int nreq_max, int cap, int grid, hipStream_t stream) {
    if (radius <= 1) return launch_tiles_batch(dtype, reqs, recs, units, tiles, counts, nreq_max, cap, stream);
    const int G = reslice_lanes(radius);
#define B16(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 16>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
#define B64(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 64>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
    if (staged_radius(radius)) {
        return launch_reslice_staged_batch(dtype, radius, reqs, units, counts, grid, stream);
    } else if (G == 16) {
        DARE_DISPATCH_DT(dtype, B16)
    } else {
        DARE_DISPATCH_DT(dtype, B64)
    }
#undef B16
#undef B64
    return hipGetLastError();
}

}  // namespace dare
