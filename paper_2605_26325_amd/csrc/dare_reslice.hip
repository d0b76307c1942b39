// Directionality-aware reslice at interpolation radius R > 4 (Sec. 2.1 "Reslicing", Eq. 1,
// Eq. 2, Fig. 2), and the single-request launcher for every radius.
//
// At these radii a pixel's (2R)^3 neighbourhood is larger than the workgroup, so 64 lanes share
// one pixel: each lane takes some rows of the neighbourhood, and the lanes' partial numerators
// and denominators are combined with wavefront shuffles.  Per workgroup, wave 0 composes the
// slice pose with the calibration (FP64), evaluates Eq. 1 for every direction bin, drops the
// bins beyond either angular threshold and evaluates Eq. 2 for the rest.  Radius 1 runs the
// tile kernel of dare_tiles.hip, radii 2..4 the staged kernel of dare_reslice_rs.hip.
#include "dare_batch.h"
#include "dare_reslice_dev.h"

namespace dare {

template <int DT, int G>
__global__ void __launch_bounds__(256) k_reslice_rn(const VolDev* __restrict__ vd, SliceArgs s) {
    __shared__ SetupLds sh;
    reslice_unit_rn<DT, G>(vd, s, xcd_remap(blockIdx.x, gridDim.x), sh);
}

// ---------------------------------------------------------------------------- launchers

int reslice_lanes(int radius) { return radius <= 1 ? 1 : (radius <= 2 ? 16 : 64); }

int64_t reslice_units(int radius, int W, int H) {
    if (radius <= 1) return (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    const int ppw = 256 / reslice_lanes(radius);
    return ((int64_t)W * H + ppw - 1) / ppw;
}

hipError_t launch_reslice(const VolDev* vd, int dtype, int radius, const SliceArgs& s, hipStream_t stream) {
    if (radius <= 1) return launch_reslice_tile(vd, dtype, s, stream);
    const int64_t units = reslice_units(radius, s.W, s.H);
    if (units > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)units), block(256);
    const int G = reslice_lanes(radius);
#define L16(D) hipLaunchKernelGGL((k_reslice_rn<D, 16>), grid, block, 0, stream, vd, s)
#define L64(D) hipLaunchKernelGGL((k_reslice_rn<D, 64>), grid, block, 0, stream, vd, s)
    if (G == 16) {
        DARE_DISPATCH_DT(dtype, L16)
    } else {
        DARE_DISPATCH_DT(dtype, L64)
    }
#undef L16
#undef L64
    return hipGetLastError();
}

}  // namespace dare
