// Image similarity of a reslice against the acquired frame at the same pose: the evaluation of
// Sec. 3 ("Quantitative image similarity": normalised cross-correlation and the structural
// similarity index between resliced images and their ground truth).
//
// The paper names the measures only; the readings are the standard ones.  NCC is zero-mean and
// taken over the pixels the reslice assigns (finite); SSIM is Wang et al.'s index with an 11 x 11
// Gaussian window (sigma 1.5, weights summing to 1), K1 = 0.01, K2 = 0.03, L = 255, averaged over
// the pixels whose whole window lies inside the image and is assigned in the reslice.
//
// One pass over the image: every thread takes pixels in a grid-stride loop and accumulates, in
// FP64, the NCC sums of its assigned pixels and the SSIM of its pixels whose window qualifies
// (121 taps, FP64); workgroups reduce their partial sums to a workspace row each, and one
// workgroup adds the rows.  The host finishes NCC from the sums (one pass: FP64 keeps the
// cancellation far below the comparison's tolerance at these sizes).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "dare_host.h"

#pragma clang fp contract(off)

using namespace dare;

namespace {

constexpr int kWin = 11;
constexpr int kHalf = kWin / 2;
constexpr int kSums = 8;                 // n, sum a, sum b, sum a^2, sum b^2, sum ab, sum ssim, n ssim
constexpr int kMaxGroups = 1024;

struct Window {
    double g[kWin * kWin];
};

// Sum over the workgroup's 256 threads of v (LDS tree), returned to every thread.
__device__ __forceinline__ double group_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) k_compare(const float* __restrict__ img, const uint8_t* __restrict__ frm,
                                                 int w, int h, Window win, double* __restrict__ partials) {
    __shared__ double red[256];
    double acc[kSums] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double c1 = (0.01 * 255.0) * (0.01 * 255.0), c2 = (0.03 * 255.0) * (0.03 * 255.0);
    const int64_t npx = (int64_t)w * h;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npx; p += (int64_t)gridDim.x * 256) {
        const float a = img[p];
        if (!isfinite(a)) continue;
        const double da = (double)a, db = (double)frm[p];
        acc[0] += 1.0;
        acc[1] += da;
        acc[2] += db;
        acc[3] += da * da;
        acc[4] += db * db;
        acc[5] += da * db;
        const int j = (int)(p / w), i = (int)(p - (int64_t)j * w);
        if (i < kHalf || i >= w - kHalf || j < kHalf || j >= h - kHalf) continue;
        double ma = 0.0, mb = 0.0, saa = 0.0, sbb = 0.0, sab = 0.0;
        bool ok = true;
        for (int y = 0; y < kWin && ok; ++y) {
            const int64_t row = (int64_t)(j - kHalf + y) * w + (i - kHalf);
            for (int x = 0; x < kWin; ++x) {
                const float va = img[row + x];
                if (!isfinite(va)) {
                    ok = false;
                    break;
                }
                const double g = win.g[y * kWin + x];
                const double xa = (double)va, xb = (double)frm[row + x];
                ma += g * xa;
                mb += g * xb;
                saa += g * xa * xa;
                sbb += g * xb * xb;
                sab += g * xa * xb;
            }
        }
        if (!ok) continue;
        const double va = saa - ma * ma, vb = sbb - mb * mb, cab = sab - ma * mb;
        acc[6] += ((2.0 * ma * mb + c1) * (2.0 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2));
        acc[7] += 1.0;
    }
#pragma unroll
    for (int k = 0; k < kSums; ++k) {
        const double s = group_sum(acc[k], red);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kSums + k] = s;
    }
}

__global__ void __launch_bounds__(256) k_compare_total(double* __restrict__ partials, int groups) {
    __shared__ double red[256];
    for (int k = 0; k < kSums; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < groups; b += 256) v += partials[(size_t)b * kSums + k];
        const double s = group_sum(v, red);
        if (threadIdx.x == 0) partials[(size_t)kMaxGroups * kSums + k] = s;
    }
}

}  // namespace

extern "C" {

uint64_t dare_compare_workspace_bytes(void) { return (uint64_t)(kMaxGroups + 1) * kSums * sizeof(double); }

dare_status dare_compare_to_frame(const float* image_dev, const uint8_t* frame_dev, int32_t w, int32_t h,
                                  void* workspace_dev, uint64_t workspace_bytes, double* out_host, void* stream_) {
    if (!image_dev || !frame_dev || !workspace_dev || !out_host || w <= 0 || h <= 0) return DARE_ERR_INVALID_ARG;
    if ((int64_t)w * h > (int64_t)1 << 30 || workspace_bytes < dare_compare_workspace_bytes())
        return DARE_ERR_INVALID_ARG;
    if (((uintptr_t)workspace_dev % alignof(double)) != 0) return DARE_ERR_INVALID_ARG;
    hipStream_t stream = (hipStream_t)stream_;
    Window win;
    double s = 0.0;
    for (int y = 0; y < kWin; ++y)
        for (int x = 0; x < kWin; ++x) {
            const double dx = x - kHalf, dy = y - kHalf;
            win.g[y * kWin + x] = exp(-(dx * dx + dy * dy) / (2.0 * 1.5 * 1.5));
            s += win.g[y * kWin + x];
        }
    for (int k = 0; k < kWin * kWin; ++k) win.g[k] /= s;
    const int64_t npx = (int64_t)w * h;
    const int groups = (int)std::min<int64_t>((npx + 255) / 256, kMaxGroups);
    double* partials = (double*)workspace_dev;
    hipLaunchKernelGGL(k_compare, dim3(groups), dim3(256), 0, stream, image_dev, frame_dev, w, h, win, partials);
    hipLaunchKernelGGL(k_compare_total, dim3(1), dim3(256), 0, stream, partials, groups);
    HIP_TRY(hipGetLastError());
    double tot[kSums];
    HIP_TRY(hipMemcpyAsync(tot, partials + (size_t)kMaxGroups * kSums, sizeof(tot), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const double n = tot[0];
    double ncc = NAN;
    if (n >= 2.0) {
        const double saa = tot[3] - tot[1] * tot[1] / n, sbb = tot[4] - tot[2] * tot[2] / n;
        const double sab = tot[5] - tot[1] * tot[2] / n;
        if (saa > 0.0 && sbb > 0.0) ncc = sab / sqrt(saa * sbb);
    }
    out_host[0] = ncc;
    out_host[1] = tot[7] > 0.0 ? tot[6] / tot[7] : NAN;
    out_host[2] = n;
    out_host[3] = tot[7];
    return DARE_OK;
}

}  // extern "C"
