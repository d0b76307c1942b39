// Frame placement on the device (Sec. 2.1 "Volume reconstruction": every frame is placed at its
// tracked pose, every pixel voxelized to its nearest voxel), shared by the directional grid's
// compounding and the per-sample store.  FP64 with no contraction, fixed summation order, so
// that every nearest-voxel decision is reproducible bit for bit.
#pragma once

#include <math.h>

#include "dare_internal.h"

#pragma clang fp contract(off)

namespace dare {

__device__ inline double frame_dot3(const double* a, const double* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// T = P . C (P: the frame's FP32 probe pose, row-major; C: the calibration), each entry summed
// left to right, into d: translation, raw columns 0 and 1, unit in-plane axis and unit
// acquisition normal (column `normal_axis` of T).  Returns whether P is rigid (finite,
// |R^T R - I|_inf <= 1e-4, last row (0, 0, 0, 1)).
__device__ inline bool compose_frame(const float* __restrict__ pose, const double* __restrict__ C, int normal_axis,
                                     FrameDesc& d) {
    double P[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) P[k] = (double)pose[k];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 16; ++k) ok = ok && isfinite(P[k]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double g = (P[a] * P[b] + P[4 + a] * P[4 + b]) + P[8 + a] * P[8 + b];
            ok = ok && fabs(g - (a == b ? 1.0 : 0.0)) <= 1e-4;
        }
    ok = ok && fabs(P[12]) <= 1e-4 && fabs(P[13]) <= 1e-4 && fabs(P[14]) <= 1e-4 && fabs(P[15] - 1.0) <= 1e-4;
    double T[12];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = P[r * 4 + 0] * C[0 * 4 + c];
            acc = acc + P[r * 4 + 1] * C[1 * 4 + c];
            acc = acc + P[r * 4 + 2] * C[2 * 4 + c];
            acc = acc + P[r * 4 + 3] * C[3 * 4 + c];
            T[r * 4 + c] = acc;
        }
    double e2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.t[a] = T[a * 4 + 3];
        d.e0[a] = T[a * 4 + 0];
        d.e1[a] = T[a * 4 + 1];
        e2[a] = T[a * 4 + 2];
    }
    const double l0 = sqrt(frame_dot3(d.e0, d.e0));
    const double* en = normal_axis == 1 ? d.e1 : e2;
    const double ln = sqrt(frame_dot3(en, en));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.xh[a] = d.e0[a] / l0;
        d.nh[a] = en[a] / ln;
    }
    d.pad = 0.0;
    return ok;
}

// Nearest voxel floor(c + 0.5) of frame pixel (i, j), c = (p - o) / h with
// p = (t + (i sx) e0) + (j sy) e1; false when it lies outside the grid.
__device__ inline bool frame_voxel(const FrameDesc* __restrict__ fd, const double* __restrict__ origin, double inv_h,
                                   int nx, int ny, int nz, int i, int j, double sx, double sy, int& vx, int& vy,
                                   int& vz) {
    const double is = (double)i * sx;
    const double js = (double)j * sy;
    double c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = (fd->t[a] + is * fd->e0[a]) + js * fd->e1[a];
        c[a] = floor((p - origin[a]) * inv_h + 0.5);
    }
    if (!(c[0] >= 0.0 && c[0] < (double)nx && c[1] >= 0.0 && c[1] < (double)ny && c[2] >= 0.0 && c[2] < (double)nz))
        return false;
    vx = (int)c[0];
    vy = (int)c[1];
    vz = (int)c[2];
    return true;
}

}  // namespace dare
