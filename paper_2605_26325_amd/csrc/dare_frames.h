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

// Nearest voxel floor(c + 0.5) of the image-plane point (u, v) millimetres, c = (p - o) / h with
// p = (t + u e0) + v e1; false when it lies outside the grid.
__device__ inline bool plane_voxel(const FrameDesc* __restrict__ fd, const double* __restrict__ origin, double inv_h,
                                   int nx, int ny, int nz, double is, double js, int& vx, int& vy, int& vz) {
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

// Nearest voxel of linear-array pixel (i, j), at image millimetres (i sx, j sy).
__device__ inline bool frame_voxel(const FrameDesc* __restrict__ fd, const double* __restrict__ origin, double inv_h,
                                   int nx, int ny, int nz, int i, int j, double sx, double sy, int& vx, int& vy,
                                   int& vz) {
    return plane_voxel(fd, origin, inv_h, nx, ny, nz, (double)i * sx, (double)j * sy, vx, vy, vz);
}

// A fan probe (curvilinear, or phased array with r0 = 0): column i's beam leaves the apex with
// unit direction beams[2i], beams[2i + 1] (image mm: lateral, axial), and pixel (i, j) lies on it
// at r0 + j dr from the apex.  Columns are binned in `sectors` equal sectors, column i in sector
// i * sectors / width.
struct FanArgs {
    double apex[2];
    double r0, dr;
    const double* beams;   // device, width x 2
    int sectors;
};

// Nearest voxel of fan pixel (i, j): r = r0 + j dr, (u, v) = (a0 + r b_i0, a1 + r b_i1).
__device__ inline bool fan_voxel(const FrameDesc* __restrict__ fd, const double* __restrict__ origin, double inv_h,
                                 int nx, int ny, int nz, const FanArgs& fan, int i, int j, int& vx, int& vy, int& vz) {
    const double r = fan.r0 + (double)j * fan.dr;
    const double u = fan.apex[0] + r * fan.beams[2 * i];
    const double v = fan.apex[1] + r * fan.beams[2 * i + 1];
    return plane_voxel(fd, origin, inv_h, nx, ny, nz, u, v, vx, vy, vz);
}

// In-plane direction of sector g of a `width`-column fan: across the beam of the sector's middle
// column, x = b1 xhat - b0 yhat with yhat = e1 / |e1| (xhat for a beam along the axial axis).
__device__ inline void fan_sector_axis(FrameDesc& d, const FanArgs& fan, int width, int g) {
    const int G = fan.sectors;
    const int first = (g * width + G - 1) / G;
    const int last = ((g + 1) * width + G - 1) / G - 1;
    const int m = (first + last) / 2;
    const double b0 = fan.beams[2 * m], b1 = fan.beams[2 * m + 1];
    const double ly = sqrt(frame_dot3(d.e1, d.e1));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double yh = d.e1[a] / ly;
        d.xh[a] = b1 * d.xh[a] - b0 * yh;
    }
}

}  // namespace dare
