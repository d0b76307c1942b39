// Batched reslice: many requests (volumes, poses, sizes) in a fixed set of launches whose
// counts are read from device memory, so that a captured graph can replay any batch.
// Radius 1 runs as three passes (setup, voxel slab, pixel); radius >= 2 runs one
// (request, unit) table through the lane-split neighbourhood kernel.
#include "dare_staged.h"
#include "dare_reslice_dev.h"

namespace dare {

// ---------------------------------------------------------------- batched passes (radius 1)
//
// A batch runs as three flat passes with no workgroup barriers:
//   setup  one wave per request: pose, Eq. 1 / gates / Eq. 2, plane frame and the
//          slab of the slice (the voxels within the trilinear support of the plane
//          over the slice's bounding box, as runs along the normal's dominant axis);
//   voxel  one thread per slab candidate: all surviving bins gathered at once and
//          blended into V_v, written to the request's slab in the workspace;
//   pixel  one thread per output pixel: FP64 position, the 8 cell values from the
//          slab (mostly L2 hits), tent blend.
// The per-voxel and per-pixel arithmetic and its order are those of the fused
// kernel, so a batched request equals the same request resliced alone.

// The fields of a request's setup that place its slab runs, for dominant axis DAX (p and q are
// the other two axes, in the order the setup pass chose them).
struct RunGeom {
    float c0d, c0p, c0q, fmp, fmq, inv_md, half;
};

template <int DAX>
__device__ __forceinline__ RunGeom run_geom(const SliceSetup& su) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    return RunGeom{su.c0[DAX], su.c0[PAX], su.c0[QAX], su.fm[PAX], su.fm[QAX], su.inv_md, su.half};
}

// First voxel of the slab run of column (vp, vq): the first whole voxel above centre - half, or
// the grid floor.  The column's slab voxels are the integers in (centre - half, centre + half), at
// most ceil(2 half) of them (half carries the slop that covers the FP32 rounding of centre).  Both
// passes place runs with this one function, so they agree on every run.
__device__ __forceinline__ int run_start(const RunGeom& g, int vp, int vq) {
    const float centre = g.c0d - (g.fmp * ((float)vp - g.c0p) + g.fmq * ((float)vq - g.c0q)) * g.inv_md;
    return max((int)floorf(centre - g.half) + 1, 0);
}

static_assert(kSlabTileP == 8 && kSlabTileQ == 4, "slab tile indexing uses shifts by 3 and 5");

// Position of slab voxel (cp, cq, kk) in the request's slab (the voxel pass writes in this order).
__device__ __forceinline__ int slab_index(int cp, int cq, int kk, int ntp, int depth) {
    const int tile = (cq >> 2) * ntp + (cp >> 3);
    return ((tile * depth + kk) << 5) + ((cq & 3) << 3) + (cp & 7);
}

// Wave 0: the slab of the whole slice.  Lanes 0..3 place its corner pixels.
__device__ __forceinline__ void slab_setup(const VolDev* __restrict__ vd, const SliceArgs& s, const double T[12],
                                           int kact, int64_t v_cap, SliceSetup& su) {
    const int lane = threadIdx.x;
    SlicePos q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = T[a * 4 + 3];
        q.e0[a] = T[a * 4 + 0];
        q.e1[a] = T[a * 4 + 1];
        q.o[a] = vd->origin[a];
    }
    q.inv_h = vd->inv_h;
    q.sx = s.sx;
    q.sy = s.sy;
    const int k = lane & 3;
    double c[3];
    pixel_coords(q, (k & 1) ? s.W - 1 : 0, (k & 2) ? s.H - 1 : 0, c);
    int lo[3], hi[3];
    const int n[3] = {vd->nx, vd->ny, vd->nz};
    float c0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int f = (int)fmin(fmax(floor(c[a]), -1048576.0), 1048576.0);
        int mn = f, mx = f;
#pragma unroll
        for (int o = 1; o < 4; ++o) {
            const int g = __shfl(f, o, 4);
            mn = min(mn, g);
            mx = max(mx, g);
        }
        lo[a] = max(mn - 1, 0);
        hi[a] = min(mx + 2, n[a] - 1);
        c0[a] = (float)__shfl(c[a], 0, 4);
    }
    if (lane != 0) return;
    float l1m = 0.0f, l1u = 0.0f, l1w = 0.0f;
    bool empty = false;
    for (int a = 0; a < 3; ++a) {
        empty = empty || lo[a] > hi[a];
        l1m += fabsf(su.fm[a]);
        l1u += fabsf(su.fu[a]);
        l1w += fabsf(su.fw[a]);
        su.c0[a] = c0[a];
    }
    const int dax = su.dax, pax = dax == 0 ? 1 : 0, qax = dax == 2 ? 1 : 2;
    su.pax = pax;
    su.qax = qax;
    su.lo_p = lo[pax];
    su.lo_q = lo[qax];
    su.dim_p = empty ? 0 : hi[pax] - lo[pax] + 1;
    su.dim_q = empty ? 0 : hi[qax] - lo[qax] + 1;
    su.len_u = (float)(s.W - 1) * su.lu;
    su.len_v = (float)(s.H - 1) * su.lw;
    // FP32 rounding of the tests grows with the coordinates' magnitude
    const float span = fmaxf(fmaxf(fabsf(c0[0]), fabsf(c0[1])), fabsf(c0[2])) + su.len_u + su.len_v;
    const float slop = 2e-3f + 1e-6f * span;
    su.thr_n = l1m + slop;
    su.thr_u = l1u + 0.02f + slop;
    su.thr_v = l1w + 0.02f + slop;
    su.inv_md = 1.0f / su.fm[dax];
    su.half = su.thr_n * fabsf(su.inv_md);
    const float dep = ceilf(2.0f * su.half);
    su.depth = dep <= (float)kSlabDepthMax ? (int)dep : kSlabDepthMax + 1;
    su.ntp = (su.dim_p + kSlabTileP - 1) / kSlabTileP;
    const int ntq = (su.dim_q + kSlabTileQ - 1) / kSlabTileQ;
    const int64_t ncand = (int64_t)su.ntp * ntq * su.depth * (kSlabTileP * kSlabTileQ);
    su.staged = (su.depth <= kSlabDepthMax && ncand <= v_cap) ? 1 : 0;
    su.ncand = (kact > 0 && su.staged) ? (int)ncand : 0;
}

__global__ void __launch_bounds__(64) k_batch_setup(const BatchReq* __restrict__ reqs, SliceSetup* __restrict__ setups,
                                                     int* __restrict__ counts) {
    const int nreq = counts[1];
    for (int r = blockIdx.x; r < nreq; r += gridDim.x) {
        const VolDev* vd = reqs[r].vol;
        const SliceArgs& s = reqs[r].s;
        const SliceCore& cr = reqs[r].core;      // computed on the host, as for a single reslice
        SliceSetup& su = setups[r];
        const int lane = threadIdx.x;
        su.act_bin[lane] = cr.act_bin[lane];
        su.act_w[lane] = cr.act_w[lane];
        double T[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) T[k] = cr.T[k];
        const int ka = cr.kact;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 12; ++k) su.T[k] = T[k];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                su.fm[a] = cr.fm[a];
                su.fu[a] = cr.fu[a];
                su.fw[a] = cr.fw[a];
            }
            su.lu = cr.lu;
            su.lw = cr.lw;
            su.dax = cr.dax;
            su.kact = ka;
        }
        slab_setup(vd, s, T, ka, reqs[r].v_cap, su);
        // table offset of every bin slot (0 beyond the survivors: read, then ignored); the
        // survivors' ids were written by other lanes of this wave
        __syncthreads();
        su.act_off[threadIdx.x] = threadIdx.x < ka ? (int64_t)su.act_bin[threadIdx.x] * vd->nbricks : 0;
        if (threadIdx.x == 0) {
            su.inv_depth = 1.0 / (double)su.depth;
            su.inv_ntp = 1.0 / (double)(su.ntp > 0 ? su.ntp : 1);
            su.vol = view_of(vd);
            su.sx = s.sx;
            su.sy = s.sy;
            su.W = s.W;
            su.H = s.H;
            su.out = s.out;
            su.v_off = reqs[r].v_off;
            if (!su.staged) atomicAdd(counts + 2, 1);    // requests left to the per-pixel gather kernel
        }
    }
}

// Slab elements per thread in a block of the voxel pass, and surviving bins whose gathers the
// pass issues together for all of them: two for pairs of 4 bytes or less, one for FP32 pairs,
// whose extra registers would cost more occupancy than the added loads in flight gain.
constexpr int kVoxPerThread = kFlatBlock / 256;
static_assert(kFlatBlock % 256 == 0, "a voxel-pass block spreads evenly over 256 threads");
template <int DT>
constexpr int vox_bins() { return sizeof(typename Pair<DT>::T) > 4 ? 1 : 2; }

// V_v of a thread's slab voxels over the surviving bins, straight from the brick pool: the
// table reads of all of them, then their pair loads, are issued before any is used, so the
// thread waits for one memory round trip per group of vox_bins bins instead of one per voxel.
// Per voxel the arithmetic and its order are those of a single-voxel blend over the present
// bins in bin order; a voxel that failed the slab tests (ok false) comes out NaN.
template <int DT>
__device__ __forceinline__ void blend_vox(const SliceSetup& su, const bool (&ok)[kVoxPerThread],
                                          const int64_t (&brick)[kVoxPerThread],
                                          const int (&local)[kVoxPerThread], float (&V)[kVoxPerThread]) {
    using PT = Pair<DT>;
    constexpr int U = kVoxPerThread;
    constexpr int kVoxBins = vox_bins<DT>();
    const VolView& vv = su.vol;
    const typename PT::T* __restrict__ data = (const typename PT::T*)vv.data;
    const int* __restrict__ table = vv.table;
    const int kact = su.kact;
    if (kact == 1) {
        const int64_t off = su.act_off[0];
        int sl[U];
        typename PT::T pr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sl[u] = ok[u] ? table[off + brick[u]] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (sl[u] >= 0) pr[u] = data[(size_t)sl[u] * kBrickVox + local[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            V[u] = __builtin_nanf("");
            if (sl[u] >= 0) {
                float2 sc = make_float2(0.0f, 0.0f);
                if constexpr (DT == DARE_FP8_E4M3) sc = vv.scales[sl[u]];
                float a, cnt;
                PT::decode(pr[u], sc, a, cnt);
                V[u] = cnt > 0.0f ? a : __builtin_nanf("");
            }
        }
        return;
    }
    float A[U], B[U];
#pragma unroll
    for (int u = 0; u < U; ++u) A[u] = B[u] = 0.0f;
    for (int k0 = 0; k0 < kact; k0 += kVoxBins) {
        int sl[kVoxBins][U];
        typename PT::T pr[kVoxBins][U];
#pragma unroll
        for (int g = 0; g < kVoxBins; ++g) {
            if (k0 + g < kact) {
                const int64_t off = su.act_off[k0 + g];
#pragma unroll
                for (int u = 0; u < U; ++u) sl[g][u] = ok[u] ? table[off + brick[u]] : -1;
            }
        }
#pragma unroll
        for (int g = 0; g < kVoxBins; ++g)
            if (k0 + g < kact) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (sl[g][u] >= 0) pr[g][u] = data[(size_t)sl[g][u] * kBrickVox + local[u]];
            }
#pragma unroll
        for (int g = 0; g < kVoxBins; ++g) {
            if (k0 + g < kact) {
                const float w = su.act_w[k0 + g];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (sl[g][u] >= 0) {
                        float2 sc = make_float2(0.0f, 0.0f);
                        if constexpr (DT == DARE_FP8_E4M3) sc = vv.scales[sl[g][u]];
                        float a, cnt;
                        PT::decode(pr[g][u], sc, a, cnt);
                        const float wc = w * cnt;
                        A[u] = __builtin_fmaf(wc, a, A[u]);
                        B[u] = B[u] + wc;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) V[u] = B[u] > 0.0f ? A[u] / B[u] : __builtin_nanf("");
}

// The passes run over flat index spaces in blocks of kFlatBlock: each request's range starts on
// a block boundary, so a workgroup iteration belongs to one request and everything it reads of
// that request (setup record, volume view) is uniform; each thread takes kFlatBlock / 256
// elements of the block, so that this uniform work is shared by as many.  Each workgroup
// first copies the requests' first blocks into LDS; the request of block b is then the last r
// with first(r) <= b, found by a binary search in LDS.
template <bool VOX>
__device__ __forceinline__ int load_begins(const BatchReq* __restrict__ reqs, const int* __restrict__ counts,
                                           int* s_beg) {
    const int nreq = counts[1];
    for (int i = threadIdx.x; i < nreq; i += blockDim.x)
        s_beg[i] = (int)((VOX ? reqs[i].v_beg : reqs[i].p_beg) >> kFlatShift);
    __syncthreads();
    return nreq;
}

__device__ __forceinline__ int find_req(const int* s_beg, int nreq, int blk) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_beg[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return uniform_i32(lo);
}

// x = q d + r for 0 <= x < 2^31 and d >= 1, from an FP64 reciprocal of d: the product is within
// one of the quotient, and one correction step makes it exact.
__device__ __forceinline__ void divmod(int x, int d, double inv_d, int& q, int& r) {
    q = (int)((double)x * inv_d);
    r = x - q * d;
    if (r < 0) {
        q -= 1;
        r += d;
    } else if (r >= d) {
        q += 1;
        r -= d;
    }
}

// One block of a request's slab whose normal's dominant axis is DAX: kVoxPerThread candidates
// per thread (e0 = this thread's first), each placed in the slab order, tested against the
// plane slab and the lateral extent, then blended over the surviving bins.  The request's
// fields are read once per block.
template <int DT, int DAX>
__device__ __forceinline__ void voxel_block(const SliceSetup& su, int e0, float* __restrict__ scratch) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    const RunGeom rg = run_geom<DAX>(su);
    const int ncand = su.ncand, depth = su.depth, ntp = su.ntp, lo_p = su.lo_p, lo_q = su.lo_q;
    const int dim_p = su.dim_p, dim_q = su.dim_q, nd = su.vol.n[DAX], nbx = su.vol.nbx, nby = su.vol.nby;
    const double inv_depth = su.inv_depth, inv_ntp = su.inv_ntp;
    float c0[3], fm[3], fu[3], fw[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c0[a] = su.c0[a];
        fm[a] = su.fm[a];
        fu[a] = su.fu[a];
        fw[a] = su.fw[a];
    }
    const float thr_n = su.thr_n, thr_u = su.thr_u, thr_v = su.thr_v;
    const float hi_u = su.len_u + su.thr_u, hi_v = su.len_v + su.thr_v;
    bool ok[kVoxPerThread];
    int64_t brick[kVoxPerThread];
    int local[kVoxPerThread];
#pragma unroll
    for (int u = 0; u < kVoxPerThread; ++u) {
        const int e = e0 + 256 * u;
        ok[u] = false;
        brick[u] = 0;
        local[u] = 0;
        if (e >= ncand) continue;
        // slab order: column tiles of kSlabTileP x kSlabTileQ (p fastest), each with all its
        // depth layers, so that a workgroup consumes whole brick rows and a pixel's 8 cell
        // values share a few cache lines
        const int w = e & (kSlabTileP * kSlabTileQ - 1), rest = e >> 5;
        int tile, k, tq, tp;
        divmod(rest, depth, inv_depth, tile, k);
        divmod(tile, ntp, inv_ntp, tq, tp);
        const int cp = tp * kSlabTileP + (w & (kSlabTileP - 1));
        const int cq = tq * kSlabTileQ + (w >> 3);
        const int vp = lo_p + cp, vq = lo_q + cq;
        const int vdd = run_start(rg, vp, vq) + k;
        if (cp >= dim_p || cq >= dim_q || vdd >= nd) continue;
        int v[3];
        v[DAX] = vdd;
        v[PAX] = vp;
        v[QAX] = vq;
        const float d0 = (float)v[0] - c0[0], d1 = (float)v[1] - c0[1], d2 = (float)v[2] - c0[2];
        const float dn = fm[0] * d0 + fm[1] * d1 + fm[2] * d2;
        const float du = fu[0] * d0 + fu[1] * d1 + fu[2] * d2;
        const float dv = fw[0] * d0 + fw[1] * d1 + fw[2] * d2;
        if (fabsf(dn) < thr_n && du > -thr_u && du < hi_u && dv > -thr_v && dv < hi_v) {
            brick[u] = ((int64_t)(v[2] >> 3) * nby + (v[1] >> 3)) * nbx + (v[0] >> 3);
            local[u] = brick_local(v[0], v[1], v[2]);
            ok[u] = true;
        }
    }
    float V[kVoxPerThread];
    blend_vox<DT>(su, ok, brick, local, V);
    float* __restrict__ slab = scratch + su.v_off;
#pragma unroll
    for (int u = 0; u < kVoxPerThread; ++u)
        if (e0 + 256 * u < ncand) slab[e0 + 256 * u] = V[u];
}

template <int DT>
__global__ void __launch_bounds__(256) k_voxel_pass(const BatchReq* __restrict__ reqs,
                                                    const SliceSetup* __restrict__ setups, float* __restrict__ scratch,
                                                    const int* __restrict__ counts) {
    extern __shared__ int s_beg[];
    const int nreq = load_begins<true>(reqs, counts, s_beg);
    const int nblk = (int)(reinterpret_cast<const int64_t*>(counts + 4)[0] >> kFlatShift);
    // plain order: requests' candidate counts differ, and interleaving them over the XCDs balances
    // the load better than giving each XCD a contiguous run (which was 3 % slower)
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int r = find_req(s_beg, nreq, blk);
        const SliceSetup& su = setups[r];
        const int e0 = ((blk - s_beg[r]) << kFlatShift) + (int)threadIdx.x;
        switch (uniform_i32(su.dax)) {
            case 0: voxel_block<DT, 0>(su, e0, scratch); break;
            case 1: voxel_block<DT, 1>(su, e0, scratch); break;
            default: voxel_block<DT, 2>(su, e0, scratch); break;
        }
    }
}

// The pixels p0, p0 + 256, ... of one block of a staged request whose normal's dominant axis is
// DAX: FP64 position, the 8 cell values from the slab, tent weights.  The corner-to-slab mapping
// is fixed at compile time per dominant axis.
template <int DAX>
__device__ __forceinline__ void staged_block(const SliceSetup& su, int p0, const float* __restrict__ scratch) {
    constexpr int PAX = DAX == 0 ? 1 : 0, QAX = DAX == 2 ? 1 : 2;
    const int W = su.W, npx = W * su.H;
    SlicePos q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.t[a] = su.T[a * 4 + 3];
        q.e0[a] = su.T[a * 4 + 0];
        q.e1[a] = su.T[a * 4 + 1];
        q.o[a] = su.vol.origin[a];
    }
    q.inv_h = su.vol.inv_h;
    q.sx = su.sx;
    q.sy = su.sy;
    const int n[3] = {su.vol.n[0], su.vol.n[1], su.vol.n[2]};
    const bool live = su.kact > 0 && su.ncand > 0;   // a pixel inside the grid implies a non-empty slab
    const float* __restrict__ slab = scratch + su.v_off;
    const int depth = su.depth, ntp = su.ntp, last = su.ncand - 1, lo_p = su.lo_p, lo_q = su.lo_q;
    const RunGeom rg = run_geom<DAX>(su);
    const int pe = min(p0 - (int)threadIdx.x + kFlatBlock, npx);
    for (int p = p0; p < pe; p += 256) {
        const int j = p / W, i = p - j * W;
        float* out = su.out + p;
        double c[3];
        pixel_coords(q, i, j, c);
        if (!live || !(c[0] >= -1.0 && c[0] < (double)n[0] && c[1] >= -1.0 && c[1] < (double)n[1] &&
                       c[2] >= -1.0 && c[2] < (double)n[2])) {
            *out = __builtin_nanf("");
            continue;
        }
        const double f0 = floor(c[0]), f1 = floor(c[1]), f2 = floor(c[2]);
        const int b0[3] = {(int)f0, (int)f1, (int)f2};
        const float fr[3] = {(float)(c[0] - f0), (float)(c[1] - f1), (float)(c[2] - f2)};
        // per-axis tent weights of the cell's lower and upper voxel, 0 for a voxel outside the
        // grid: a corner's weight is their product, 0 for absent corners, which then add exactly
        // nothing to the sums below (the fused kernel skips them)
        float w[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w[a][0] = (unsigned)b0[a] < (unsigned)n[a] ? 1.0f - fr[a] : 0.0f;
            w[a][1] = (unsigned)(b0[a] + 1) < (unsigned)n[a] ? fr[a] : 0.0f;
        }
        // the cell's 4 columns (offsets along p, q): slab index of layer b0[DAX]; the next layer
        // along the dominant axis is 32 floats further.  A voxel with weight inside the grid
        // always lies in the slab, so only a clamp keeps the other corners' reads in bounds.
        const int bp = b0[PAX], bq = b0[QAX], bd = b0[DAX];
        int base[4];
#pragma unroll
        for (int col = 0; col < 4; ++col) {
            const int vp = bp + (col & 1), vq = bq + (col >> 1);
            base[col] = slab_index(vp - lo_p, vq - lo_q, bd - run_start(rg, vp, vq), ntp, depth);
        }
        float Vc[8];
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) {             // c8 = (dz << 2) | (dy << 1) | dx
            const int od = (c8 >> DAX) & 1, col = ((c8 >> PAX) & 1) | (((c8 >> QAX) & 1) << 1);
            Vc[c8] = slab[min(max(base[col] + (od << 5), 0), last)];
        }
        float num = 0.0f, den = 0.0f;
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) {
            const float tw = (w[0][c8 & 1] * w[1][(c8 >> 1) & 1]) * w[2][c8 >> 2];
            const bool use = Vc[c8] == Vc[c8];
            num = use ? __builtin_fmaf(tw, Vc[c8], num) : num;
            den = use ? den + tw : den;
        }
        *out = den > 0.0f ? num / den : __builtin_nanf("");
    }
}

// Pixels of staged requests (STAGED) or of requests that gather per pixel (!STAGED): two
// kernels, so that the staged one keeps the register budget of its 8 slab reads.  A kernel
// skips the other kind's requests one whole range at a time.
template <int DT, bool STAGED>
__global__ void __launch_bounds__(256) k_pixel_pass(const BatchReq* __restrict__ reqs,
                                                    const SliceSetup* __restrict__ setups,
                                                    const float* __restrict__ scratch, const int* __restrict__ counts) {
    if (!STAGED && counts[2] == 0) return;             // every request of the batch is staged
    extern __shared__ int s_beg[];
    const int nreq = load_begins<false>(reqs, counts, s_beg);
    const int nblk = (int)(reinterpret_cast<const int64_t*>(counts + 4)[1] >> kFlatShift);
    // each XCD sweeps a contiguous run of blocks, so that one request's slab is read through one
    // L2 (fabric reads fall from 5x the slab to about its size)
    for (int blk = xcd_remap(blockIdx.x, gridDim.x); blk < nblk; blk += gridDim.x) {
        const int r = find_req(s_beg, nreq, blk);
        const SliceSetup& su = setups[r];
        if ((su.staged != 0) != STAGED) {
            if (r + 1 >= nreq) break;
            const int next = s_beg[r + 1];            // first block of the next request
            blk += (next - blk + (int)gridDim.x - 1) / (int)gridDim.x * (int)gridDim.x - (int)gridDim.x;
            continue;
        }
        const int p0 = ((blk - s_beg[r]) << kFlatShift) + (int)threadIdx.x;
        if constexpr (STAGED) {
            switch (uniform_i32(su.dax)) {
                case 0: staged_block<0>(su, p0, scratch); break;
                case 1: staged_block<1>(su, p0, scratch); break;
                default: staged_block<2>(su, p0, scratch); break;
            }
        } else {
            const int W = su.W, npx = W * su.H;
            for (int p = p0; p < p0 - (int)threadIdx.x + kFlatBlock && p < npx; p += 256) {
                const int j = p / W, i = p - j * W;
                float* out = su.out + p;
                const int kact = su.kact;
                SlicePos q;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    q.t[a] = su.T[a * 4 + 3];
                    q.e0[a] = su.T[a * 4 + 0];
                    q.e1[a] = su.T[a * 4 + 1];
                    q.o[a] = su.vol.origin[a];
                }
                q.inv_h = su.vol.inv_h;
                q.sx = su.sx;
                q.sy = su.sy;
                const int n[3] = {su.vol.n[0], su.vol.n[1], su.vol.n[2]};
                double c[3];
                pixel_coords(q, i, j, c);
                if (kact == 0 || !(c[0] >= -1.0 && c[0] < (double)n[0] && c[1] >= -1.0 && c[1] < (double)n[1] &&
                                   c[2] >= -1.0 && c[2] < (double)n[2])) {
                    *out = __builtin_nanf("");
                    continue;
                }
                *out = pixel_direct<DT, 2>(su.vol, su, kact, c);
            }
        }
    }
}

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

hipError_t launch_reslice_batch(int dtype, int radius, const BatchReq* reqs, SliceSetup* setups, const int2* units,
                                const int* counts, float* scratch, int nreq_max, int grid, hipStream_t stream) {
    const int G = reslice_lanes(radius);
    const int nreq_grid = nreq_max < 1024 ? nreq_max : 1024;
    const size_t lds = (size_t)nreq_max * sizeof(int);
#define V1(D) hipLaunchKernelGGL(k_voxel_pass<D>, dim3(grid), dim3(256), lds, stream, reqs, setups, scratch, counts)
#define P1(D)                                                                                                  \
    hipLaunchKernelGGL((k_pixel_pass<D, true>), dim3(grid), dim3(256), lds, stream, reqs, setups, scratch, counts); \
    hipLaunchKernelGGL((k_pixel_pass<D, false>), dim3(grid), dim3(256), lds, stream, reqs, setups, scratch, counts)
#define B16(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 16>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
#define B64(D) hipLaunchKernelGGL((k_reslice_rn_batch<D, 64>), dim3(grid), dim3(256), 0, stream, reqs, units, counts)
    if (G == 1) {
        hipLaunchKernelGGL(k_batch_setup, dim3(nreq_grid), dim3(64), 0, stream, reqs, setups, const_cast<int*>(counts));
        DARE_DISPATCH_DT(dtype, V1)
        DARE_DISPATCH_DT(dtype, P1)
    } else if (staged_radius(radius)) {
        return launch_reslice_staged_batch(dtype, radius, reqs, units, counts, grid, stream);
    } else if (G == 16) {
        DARE_DISPATCH_DT(dtype, B16)
    } else {
        DARE_DISPATCH_DT(dtype, B64)
    }
#undef V1
#undef P1
#undef B16
#undef B64
    return hipGetLastError();
}

}  // namespace dare
