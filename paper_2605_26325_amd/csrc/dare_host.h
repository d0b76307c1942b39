// Host-side helpers shared by the C ABI's translation units (defined in dare_capi.hip): device
// selection for a call, status conversion, and the pose and argument checks every entry point
// applies.
#pragma once

#include "dare_internal.h"

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

}  // namespace dare
