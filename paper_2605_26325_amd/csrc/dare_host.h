// Host-side helpers shared by the C ABI's translation units (defined in dare_capi.hip): device
// selection for a call, status conversion, and the pose and argument checks every entry point
// applies.
#pragma once

#include <vector>

#include "dare_frames.h"
#include "dare_held.h"
#include "dare_internal.h"


// A volume handle: the host's view of a volume whose device state lives in the caller's arena.
struct dare_volume {
    int device = 0;
    dare_geometry g{};
    dare_params p{};
    dare_dtype dtype = DARE_F32;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    dare::VolDev host{};              // host mirror of the device header (pointers, geometry, codebook)
    dare::VolDev* dev = nullptr;      // device header at the start of the arena
    dare::VolDev* hdr_pinned = nullptr;   // pinned copy of the device header, read at sync points
    int K = 0;
    int saturated = 0;
    uint32_t used = 0;
    // Out-of-core state.  `held` keeps the exact accumulators of bricks moved to host memory,
    // by table entry (bin * bricks per bin + brick).  With `spill` set, a frame batch whose new
    // bricks do not fit moves the least recently touched bricks there; `stamp` holds, per pool
    // slot, the batch counter `clock` at the slot's last touch (kept in spill mode only).
    bool spill = false;
    uint64_t clock = 0;
    std::vector<uint64_t> stamp;
    dare::HeldStore held;
};

namespace dare {

// Makes `dev` current for the lifetime of the guard, then restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline dare_status hip_status(hipError_t e) { return e == hipSuccess ? DARE_OK : DARE_ERR_HIP; }

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return DARE_ERR_HIP;    \
    } while (0)

// Rigid 4x4 row-major transform: finite, |R^T R - I|_inf <= 1e-4, last row (0, 0, 0, 1).
bool rigid_pose(const double* M);
// T = P . C for row-major 4x4 matrices, each entry summed left to right in FP64.
void compose_pose(const double* P, const double* C, double* T);
dare_status check_method_params(const dare_params* p);
dare_status check_volume_geometry(const dare_geometry* g);
dare_status check_slice_spec(const dare_slice_spec* s);

// Fan-probe compounding launchers (dare_compound.hip): descriptors per (frame, sector), then
// the marking and accumulation passes over fan pixels.  Asynchronous on `stream`.
hipError_t launch_compose_fan(const VolDev* vd, const float* poses, int n, const FanArgs& fan, int width,
                              hipStream_t stream);
hipError_t launch_mark_fan(const VolDev* vd, int n, int w, int h, const FanArgs& fan, hipStream_t stream);
hipError_t launch_accumulate_fan(const VolDev* vd, const uint8_t* frames, int n, int w, int h, const FanArgs& fan,
                                 hipStream_t stream);

// Out-of-core moves (dare_spill.hip).  Both synchronise `stream`.
// Move the accumulators of the given pool slots to host memory, free the slots and compact the
// pool so that the remaining slots are 0 .. used - 1 again.
dare_status spill_slots(dare_volume* v, const std::vector<uint32_t>& victims, hipStream_t stream);
// Spill mode, after a batch was rolled back for lack of room: free at least `need` slots (and
// up to an eighth of the pool more), least recently touched first, none of `keep`.
dare_status spill_for_batch(dare_volume* v, const std::vector<int32_t>& keep, uint64_t need, hipStream_t stream);

}  // namespace dare
