// C ABI: argument validation, arena layout, reconstruction orchestration,
// reslice launches and the batched request planner.  Host code only; the
// kernels live in dare_compound.hip and dare_reslice.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dare_host.h"
#include "dare_staged.h"

using namespace dare;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBatchGrid = 2048;   // workgroups of each batched pass (grid-stride)

bool finite_all(const double* v, int n) {
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

// Rigid 4x4 row-major transform: finite, |R^T R - I|_inf <= 1e-4, last row (0,0,0,1).
bool rigid(const double* M) {
    if (!finite_all(M, 16)) return false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double d = (M[a] * M[b] + M[4 + a] * M[4 + b]) + M[8 + a] * M[8 + b];
            if (fabs(d - (a == b ? 1.0 : 0.0)) > 1e-4) return false;
        }
    return fabs(M[12]) <= 1e-4 && fabs(M[13]) <= 1e-4 && fabs(M[14]) <= 1e-4 && fabs(M[15] - 1.0) <= 1e-4;
}

bool valid_dtype(int d) { return d >= DARE_F32 && d <= DARE_FP8_E4M3; }

dare_status check_params(const dare_params* p) {
    if (!p) return DARE_ERR_INVALID_ARG;
    if (!std::isfinite(p->k_normal) || !std::isfinite(p->k_inplane)) return DARE_ERR_INVALID_ARG;
    if (!(p->thr_normal_deg >= 0.0 && p->thr_normal_deg <= 180.0)) return DARE_ERR_INVALID_ARG;
    if (!(p->thr_inplane_deg >= 0.0 && p->thr_inplane_deg <= 180.0)) return DARE_ERR_INVALID_ARG;
    if (!(p->bin_tol_deg >= 0.0 && p->bin_tol_deg <= 180.0)) return DARE_ERR_INVALID_ARG;
    if (!(p->radius_vox >= 1.0 && p->radius_vox <= 8.0) || p->radius_vox != floor(p->radius_vox))
        return DARE_ERR_INVALID_ARG;
    if (p->max_bins < 1 || p->max_bins > kMaxBins) return DARE_ERR_INVALID_ARG;
    if (p->normal_axis != 1 && p->normal_axis != 2) return DARE_ERR_INVALID_ARG;
    return DARE_OK;
}

dare_status check_geometry(const dare_geometry* g) {
    if (!g) return DARE_ERR_INVALID_ARG;
    if (!finite_all(g->origin_mm, 3) || !(g->spacing_mm > 0.0) || !std::isfinite(g->spacing_mm))
        return DARE_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a)
        if (g->dims[a] <= 0 || g->dims[a] > (1 << 16)) return DARE_ERR_INVALID_ARG;
    if (!rigid(g->calib)) return DARE_ERR_BAD_POSE;
    return DARE_OK;
}

dare_status check_spec(const dare_slice_spec* s) {
    if (!s) return DARE_ERR_INVALID_ARG;
    if (s->width <= 0 || s->height <= 0 || (int64_t)s->width * s->height > (int64_t)1 << 30)
        return DARE_ERR_INVALID_ARG;
    if (!(s->pitch_mm[0] > 0.0) || !(s->pitch_mm[1] > 0.0) || !std::isfinite(s->pitch_mm[0]) ||
        !std::isfinite(s->pitch_mm[1]))
        return DARE_ERR_INVALID_ARG;
    if (!rigid(s->probe_pose)) return DARE_ERR_BAD_POSE;
    return DARE_OK;
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int64_t nbx, nby, nbz, nbricks;
    uint64_t off_table, off_frames, off_fbin, off_new, off_dirty, off_flags, off_acc, off_data, off_scales, end;
    uint64_t fixed;
    uint64_t per_slot;
};

Layout layout(const dare_geometry* g, const dare_params* p, int dtype, uint64_t cap) {
    Layout L{};
    L.nbx = (g->dims[0] + kBrick - 1) / kBrick;
    L.nby = (g->dims[1] + kBrick - 1) / kBrick;
    L.nbz = (g->dims[2] + kBrick - 1) / kBrick;
    L.nbricks = L.nbx * L.nby * L.nbz;
    uint64_t off = align_up(sizeof(VolDev));
    L.off_table = off;
    off = align_up(off + (uint64_t)p->max_bins * L.nbricks * sizeof(int32_t));
    L.off_frames = off;
    off = align_up(off + (uint64_t)kFrameChunk * sizeof(FrameDesc));
    L.off_fbin = off;
    off = align_up(off + (uint64_t)kFrameChunk * sizeof(int32_t));
    L.fixed = off + 6 * kAlign;
    L.per_slot = 3 * sizeof(int32_t) + kBrickVox * sizeof(unsigned long long) + kBrickVox * pair_bytes(dtype) +
                 sizeof(float2);
    L.off_new = off;
    off = align_up(off + cap * sizeof(int32_t));
    L.off_dirty = off;
    off = align_up(off + cap * sizeof(int32_t));
    L.off_flags = off;
    off = align_up(off + cap * sizeof(uint32_t));
    L.off_acc = off;
    off = align_up(off + cap * kBrickVox * sizeof(unsigned long long));
    L.off_data = off;
    off = align_up(off + cap * kBrickVox * (uint64_t)pair_bytes(dtype));
    L.off_scales = off;
    off = align_up(off + cap * sizeof(float2));
    L.end = off;
    return L;
}

// Device header at a sync point: the state, and the codebook the host keeps a copy of (for the
// codebook and active-bin queries; reslices read the codebook on the device).
dare_status read_state(dare_volume* v, hipStream_t stream, VolState* out) {
    HIP_TRY(hipMemcpyAsync(v->hdr_pinned, v->dev, sizeof(VolDev), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *out = v->hdr_pinned->st;
    memcpy(v->host.rep_n, v->hdr_pinned->rep_n, sizeof(v->host.rep_n));
    memcpy(v->host.rep_x, v->hdr_pinned->rep_x, sizeof(v->host.rep_x));
    return DARE_OK;
}

void compose_host(const double* P, const double* C, double* T) {
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = P[r * 4 + 0] * C[0 * 4 + c];
            acc = acc + P[r * 4 + 1] * C[1 * 4 + c];
            acc = acc + P[r * 4 + 2] * C[2 * 4 + c];
            acc = acc + P[r * 4 + 3] * C[3 * 4 + c];
            T[r * 4 + c] = acc;
        }
}

// Eq. 1 for every direction bin, the angular gates and Eq. 2 (Sec. 2.1 "Reslicing"), in FP64 on
// the host copy of the codebook: surviving bins in increasing order with their weights.
int gate_bins(const dare_volume* v, const double T[16], int32_t* bins, double* w) {
    const VolDev& h = v->host;
    const int ax = v->p.normal_axis;
    const double e0[3] = {T[0], T[4], T[8]}, en[3] = {T[ax], T[4 + ax], T[8 + ax]};
    const double l0 = sqrt((e0[0] * e0[0] + e0[1] * e0[1]) + e0[2] * e0[2]);
    const double ln = sqrt((en[0] * en[0] + en[1] * en[1]) + en[2] * en[2]);
    const double xr[3] = {e0[0] / l0, e0[1] / l0, e0[2] / l0}, nr[3] = {en[0] / ln, en[1] / ln, en[2] / ln};
    int n = 0;
    for (int b = 0; b < v->K; ++b) {
        const double* rn = h.rep_n[b];
        const double* rx = h.rep_x[b];
        const double dn = (rn[0] * nr[0] + rn[1] * nr[1]) + rn[2] * nr[2];
        const double di = fabs((rx[0] * xr[0] + rx[1] * xr[1]) + rx[2] * xr[2]);
        if (dn >= h.cos_normal && di >= h.cos_inplane) {
            bins[n] = b;
            w[n] = exp(h.k_normal * (dn - 1.0) + h.k_inplane * (di - 1.0));
            ++n;
        }
    }
    return n;
}

SliceArgs make_args(const dare_slice_spec* s, float* out) {
    SliceArgs a{};
    memcpy(a.P, s->probe_pose, sizeof(a.P));
    a.sx = s->pitch_mm[0];
    a.sy = s->pitch_mm[1];
    a.W = s->width;
    a.H = s->height;
    a.tiles_x = (s->width + kTile - 1) / kTile;
    a.tiles = a.tiles_x * ((s->height + kTile - 1) / kTile);
    a.out = out;
    return a;
}

}  // namespace

namespace dare {

}  // namespace dare

namespace dare {
const VolDev* volume_device(const dare_volume* v) { return v->dev; }
int volume_dtype(const dare_volume* v) { return v->dtype; }
int volume_radius(const dare_volume* v) { return (int)v->p.radius_vox; }
int volume_device_id(const dare_volume* v) { return v->device; }
uint64_t volume_arena_size(const dare_volume* v) { return v->arena_bytes; }
dare_status check_slice_spec(const dare_slice_spec* s) { return check_spec(s); }
bool rigid_pose(const double* M) { return rigid(M); }
void compose_pose(const double* P, const double* C, double* T) { compose_host(P, C, T); }
dare_status check_method_params(const dare_params* p) { return check_params(p); }
dare_status check_volume_geometry(const dare_geometry* g) { return check_geometry(g); }
}  // namespace dare

namespace {

struct Group {
    std::vector<BatchReq> reqs;
    std::vector<int2> units;      // radii above 1: built here; radius 1: built on the device
    int64_t nunits = 0;           // units (radius 1: the most the device may append)
};

// Batch workspace of one launch group: [header] [requests] [units] [tile records] [request
// records].  The header and requests are uploaded, and the units when built on the host (radii
// above 1, which have no records); at radius 1 units and records are written on the device.
struct GroupLayout {
    uint64_t o_req, o_units, o_tiles, o_rec, upload, total;
};

GroupLayout group_layout(size_t nreq, size_t nunits, bool host_units) {
    GroupLayout L;
    L.o_req = align_up(sizeof(BatchHeader));
    L.o_units = L.o_req + align_up(nreq * sizeof(BatchReq));
    L.o_tiles = L.o_units + align_up(nunits * sizeof(int2));
    L.o_rec = L.o_tiles + (host_units ? 0 : align_up(nunits * sizeof(TileRec)));
    L.upload = host_units ? L.o_tiles : L.o_units;
    L.total = L.o_rec + (host_units ? 0 : align_up(nreq * sizeof(SliceRec)));
    return L;
}

// Pinned staging for batch request tables.  An upload from pageable memory would make the call
// wait for the stream; from pinned memory it is asynchronous, and a buffer is reused only once
// the event recorded after its copy has completed.  Buffers are kept per device until the
// process ends.
class StagingPool {
public:
    // A pinned buffer of at least `bytes` not read by any pending copy; `release` records the
    // copy that reads it on `stream`.
    struct Lease {
        char* p = nullptr;
        int idx = -1;
    };
    Lease acquire(uint64_t bytes) {
        std::lock_guard<std::mutex> lk(mu_);
        for (;;) {
            int oldest = -1;
            for (int k = 0; k < (int)bufs_.size(); ++k) {
                Buf& b = bufs_[k];
                if (b.leased) continue;
                if (b.pending && hipEventQuery(b.ev) != hipSuccess) {
                    if (oldest < 0 || b.seq < bufs_[oldest].seq) oldest = k;
                    continue;
                }
                b.pending = false;
                if (b.cap < bytes && !grow(b, bytes)) return Lease{};
                b.leased = true;
                return Lease{b.p, k};
            }
            if ((int)bufs_.size() < kMaxBufs) {
                Buf b;
                if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) return Lease{};
                if (!grow(b, bytes)) {
                    (void)hipEventDestroy(b.ev);
                    return Lease{};
                }
                b.leased = true;
                bufs_.push_back(b);
                return Lease{b.p, (int)bufs_.size() - 1};
            }
            if (oldest < 0) return Lease{};                  // every buffer leased by other threads
            if (hipEventSynchronize(bufs_[oldest].ev) != hipSuccess) return Lease{};
            bufs_[oldest].pending = false;
        }
    }
    hipError_t release(const Lease& l, hipStream_t stream) {
        std::lock_guard<std::mutex> lk(mu_);
        Buf& b = bufs_[l.idx];
        b.leased = false;
        b.pending = true;
        b.seq = ++seq_;
        return hipEventRecord(b.ev, stream);
    }

private:
    struct Buf {
        char* p = nullptr;
        uint64_t cap = 0;
        hipEvent_t ev = nullptr;
        bool leased = false, pending = false;
        uint64_t seq = 0;
    };
    static constexpr int kMaxBufs = 8;
    static bool grow(Buf& b, uint64_t bytes) {
        if (b.cap >= bytes) return true;
        if (b.p) (void)hipHostFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        const uint64_t cap = std::max<uint64_t>(bytes, 1 << 20);
        if (hipHostMalloc((void**)&b.p, cap, hipHostMallocDefault) != hipSuccess) return false;
        b.cap = cap;
        return true;
    }
    std::mutex mu_;
    std::vector<Buf> bufs_;
    uint64_t seq_ = 0;
};

StagingPool& staging_pool(int device) {
    static std::mutex mu;
    static std::map<int, StagingPool*> pools;
    std::lock_guard<std::mutex> lk(mu);
    StagingPool*& p = pools[device];
    if (!p) p = new StagingPool();
    return *p;
}

struct GroupSize {
    size_t nreq = 0, nunits = 0;
};

// Launch group of each request: (storage dtype, radius, piece), a piece being each run of
// kBatchMaxReq requests of one (dtype, radius) in call order.
using GroupKey = std::tuple<int, int, int>;

std::vector<GroupKey> group_keys(const dare_volume* const* vols, int32_t n) {
    std::map<std::pair<int, int>, int> seen;
    std::vector<GroupKey> keys((size_t)n);
    for (int k = 0; k < n; ++k) {
        const int R = (int)vols[k]->p.radius_vox;
        const int i = seen[{vols[k]->dtype, R}]++;
        keys[k] = GroupKey(vols[k]->dtype, R, i / kBatchMaxReq);
    }
    return keys;
}

std::map<GroupKey, GroupSize> group_sizes(const dare_volume* const* vols, const dare_slice_spec* specs, int32_t n) {
    std::map<GroupKey, GroupSize> cnt;
    const std::vector<GroupKey> keys = group_keys(vols, n);
    for (int k = 0; k < n; ++k) {
        const int R = (int)vols[k]->p.radius_vox;
        GroupSize& c = cnt[keys[k]];
        c.nreq += 1;
        c.nunits += (size_t)(R <= 1 ? tile_units_max(specs[k].width, specs[k].height)
                                    : batch_units(R, specs[k].width, specs[k].height));
    }
    return cnt;
}

}  // namespace

namespace dare {

}  // namespace dare

extern "C" {

void dare_default_params(dare_params* p) {
    if (!p) return;
    p->k_normal = 10.0;
    p->k_inplane = 5.0;
    p->thr_normal_deg = 25.0;
    p->thr_inplane_deg = 15.0;
    p->radius_vox = 1.0;
    p->bin_tol_deg = 5.0;
    p->max_bins = 64;
    p->normal_axis = 2;
}

const char* dare_status_str(dare_status s) {
    switch (s) {
        case DARE_OK: return "ok";
        case DARE_ERR_INVALID_ARG: return "invalid argument";
        case DARE_ERR_BAD_POSE: return "pose is not a rigid transform";
        case DARE_ERR_BUDGET: return "arena budget exhausted";
        case DARE_ERR_HIP: return "HIP runtime error";
        case DARE_WARN_BINS_SATURATED: return "direction codebook saturated";
        case DARE_ERR_NOT_READY: return "not ready";
        case DARE_ERR_QUEUE_FULL: return "queue full";
    }
    return "unknown status";
}

uint64_t dare_volume_arena_bytes(const dare_geometry* g, const dare_params* p, dare_dtype dtype, int64_t bricks) {
    if (check_geometry(g) != DARE_OK || check_params(p) != DARE_OK || !valid_dtype(dtype) || bricks < 0) return 0;
    return layout(g, p, dtype, (uint64_t)bricks).end;
}

dare_status dare_volume_create(const dare_geometry* g, const dare_params* p, dare_dtype dtype, void* arena_dev,
                               uint64_t arena_bytes, dare_volume** out) {
    if (!out || !arena_dev || !valid_dtype(dtype)) return DARE_ERR_INVALID_ARG;
    *out = nullptr;
    dare_status st = check_geometry(g);
    if (st != DARE_OK) return st;
    if ((st = check_params(p)) != DARE_OK) return st;
    if (((uintptr_t)arena_dev % kAlign) != 0) return DARE_ERR_INVALID_ARG;
    Layout L0 = layout(g, p, dtype, 0);
    if (arena_bytes <= L0.fixed) return DARE_ERR_INVALID_ARG;
    uint64_t cap = (arena_bytes - L0.off_new) / L0.per_slot;   // upper bound; alignment trims below
    if (cap > 0x7FFFFFFFull) cap = 0x7FFFFFFFull;
    while (cap > 0 && layout(g, p, dtype, cap).end > arena_bytes) --cap;
    if (cap == 0) return DARE_ERR_INVALID_ARG;   // room for at least one brick slot
    const Layout L = layout(g, p, dtype, cap);

    dare_volume* v = new dare_volume();
    if (hipGetDevice(&v->device) != hipSuccess) { delete v; return DARE_ERR_HIP; }
    v->g = *g;
    v->p = *p;
    v->dtype = dtype;
    v->arena = (char*)arena_dev;
    v->arena_bytes = arena_bytes;
    VolDev& h = v->host;
    memset(&h, 0, sizeof(h));
    for (int a = 0; a < 3; ++a) h.origin[a] = g->origin_mm[a];
    h.h = g->spacing_mm;
    h.inv_h = 1.0 / g->spacing_mm;
    h.nx = g->dims[0];
    h.ny = g->dims[1];
    h.nz = g->dims[2];
    h.nbx = (int32_t)L.nbx;
    h.nby = (int32_t)L.nby;
    h.nbz = (int32_t)L.nbz;
    h.nbricks = L.nbricks;
    memcpy(h.calib, g->calib, sizeof(h.calib));
    h.k_normal = p->k_normal;
    h.k_inplane = p->k_inplane;
    h.cos_normal = cos(p->thr_normal_deg * (kPi / 180.0));
    h.cos_inplane = cos(p->thr_inplane_deg * (kPi / 180.0));
    h.cos_tol = cos(p->bin_tol_deg * (kPi / 180.0));
    h.radius = (int32_t)p->radius_vox;
    h.max_bins = p->max_bins;
    h.normal_axis = p->normal_axis;
    h.dtype = dtype;
    h.cap = (uint32_t)cap;
    char* base = v->arena;
    h.table = (int32_t*)(base + L.off_table);
    h.frames = (FrameDesc*)(base + L.off_frames);
    h.frame_bin = (int32_t*)(base + L.off_fbin);
    h.new_list = (int32_t*)(base + L.off_new);
    h.dirty_list = (int32_t*)(base + L.off_dirty);
    h.dirty_flags = (uint32_t*)(base + L.off_flags);
    h.acc = (unsigned long long*)(base + L.off_acc);
    h.data = (void*)(base + L.off_data);
    h.scales = (float2*)(base + L.off_scales);
    v->dev = (VolDev*)base;
    v->stamp.assign(cap, 0);
    if (hipHostMalloc((void**)&v->hdr_pinned, sizeof(VolDev), hipHostMallocDefault) != hipSuccess) {
        delete v;
        return DARE_ERR_HIP;
    }
    hipError_t e = hipMemcpy(v->dev, &h, sizeof(VolDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_table_fill(h.table, (int64_t)p->max_bins * L.nbricks, nullptr);
    if (e == hipSuccess && cap > 0) e = hipMemset(h.dirty_flags, 0, cap * sizeof(uint32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipHostFree(v->hdr_pinned);
        delete v;
        return DARE_ERR_HIP;
    }
    *out = v;
    return DARE_OK;
}

dare_status dare_volume_destroy(dare_volume* v) {
    if (!v) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    hipError_t e = hipDeviceSynchronize();
    (void)hipHostFree(v->hdr_pinned);
    delete v;
    return hip_status(e);
}

namespace {

// Frame batches of linear-array frames (fan == nullptr) or fan frames: per batch, placement and
// bin assignment, one sync to admit the new bricks (spilling cold ones in spill mode), then
// allocation, accumulation and finalisation.
dare_status reconstruct_batches(dare_volume* v, const uint8_t* frames_dev, int32_t n, int32_t w, int32_t h,
                                const double* pitch_mm, const FanArgs* fan, const float* probe_poses_dev,
                                hipStream_t stream) {
    VolDev* vd = v->dev;
    const int G = fan ? fan->sectors : 1;
    const int per_batch = kFrameChunk / G;
    bool retried = false;
    for (int32_t f0 = 0; f0 < n;) {
        const int nf = std::min<int32_t>(per_batch, n - f0);
        const int K0 = v->K, sat0 = v->saturated;
        const uint32_t used = v->used;
        const float* poses = probe_poses_dev + (size_t)f0 * 16;
        if (fan) {
            HIP_TRY(launch_compose_fan(vd, poses, nf, *fan, w, stream));
        } else {
            HIP_TRY(launch_compose_frames(vd, poses, nf, stream));
        }
        HIP_TRY(launch_assign_bins(vd, nf * G, K0, stream));
        if (fan) {
            HIP_TRY(launch_mark_fan(vd, nf, w, h, *fan, stream));
        } else {
            HIP_TRY(launch_mark_pixels(vd, nf, w, h, pitch_mm[0], pitch_mm[1], stream));
        }
        VolState st;
        dare_status s = read_state(v, stream, &st);
        if (s != DARE_OK) return s;
        const bool bad = st.bad_pose != 0;
        const bool over = (uint64_t)used + st.new_count > v->host.cap;
        // slots the batch touches: kept in HBM by a spill, stamped as recently used
        std::vector<int32_t> touched;
        const bool spill = v->spill && !bad && !retried && (uint64_t)st.dirty_count + st.new_count <= v->host.cap;
        if ((over && spill) || (!over && !bad && v->spill)) {
            touched.resize(st.dirty_count);
            if (st.dirty_count) {
                HIP_TRY(hipMemcpyAsync(touched.data(), v->host.dirty_list, (size_t)st.dirty_count * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, stream));
                HIP_TRY(hipStreamSynchronize(stream));
            }
        }
        if (bad || over) {
            HIP_TRY(launch_rollback(vd, st.new_count, st.dirty_count, K0, sat0, stream));
            if (st.new_count > v->host.cap)   // marks beyond the list: clear them table-wide
                HIP_TRY(launch_clear_marks(v->host.table, (int64_t)v->p.max_bins * v->host.nbricks, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            if (over && spill) {   // make room, then the same batch again
                s = spill_for_batch(v, touched, (uint64_t)used + st.new_count - v->host.cap, stream);
                if (s != DARE_OK) return s;
                retried = true;
                continue;
            }
            return bad ? DARE_ERR_BAD_POSE : DARE_ERR_BUDGET;
        }
        HIP_TRY(launch_alloc(vd, st.new_count, used, st.dirty_count, stream));
        const uint8_t* fr = frames_dev + (size_t)f0 * w * h;
        if (fan) {
            HIP_TRY(launch_accumulate_fan(vd, fr, nf, w, h, *fan, stream));
        } else {
            HIP_TRY(launch_accumulate(vd, fr, nf, w, h, pitch_mm[0], pitch_mm[1], stream));
        }
        HIP_TRY(launch_finalize(vd, v->dtype, st.dirty_count + st.new_count, stream));
        v->K = st.K;
        v->saturated = st.saturated;
        v->used = used + st.new_count;
        if (v->spill) {
            ++v->clock;
            for (int32_t t : touched) v->stamp[t] = v->clock;
            for (uint32_t t = used; t < v->used; ++t) v->stamp[t] = v->clock;
        }
        retried = false;
        f0 += nf;
    }
    return v->saturated ? DARE_WARN_BINS_SATURATED : DARE_OK;
}

}  // namespace

dare_status dare_reconstruct_frames(dare_volume* v, const uint8_t* frames_dev, int32_t n, int32_t w, int32_t h,
                                    const double pitch_mm[2], const float* probe_poses_dev, void* stream) {
    if (!v || !pitch_mm || n < 0) return DARE_ERR_INVALID_ARG;
    if (n == 0) return v->saturated ? DARE_WARN_BINS_SATURATED : DARE_OK;
    if (!frames_dev || !probe_poses_dev || w <= 0 || h <= 0 || (int64_t)w * h > (int64_t)1 << 30)
        return DARE_ERR_INVALID_ARG;
    if (!(pitch_mm[0] > 0.0) || !(pitch_mm[1] > 0.0) || !std::isfinite(pitch_mm[0]) || !std::isfinite(pitch_mm[1]))
        return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    return reconstruct_batches(v, frames_dev, n, w, h, pitch_mm, nullptr, probe_poses_dev, (hipStream_t)stream);
}

dare_status dare_reconstruct_fan(dare_volume* v, const uint8_t* frames_dev, int32_t n, int32_t w, int32_t h,
                                 const dare_fan* fan, const double* beams_dev, const float* probe_poses_dev,
                                 void* stream) {
    if (!v || !fan || n < 0) return DARE_ERR_INVALID_ARG;
    if (v->p.normal_axis != 2) return DARE_ERR_INVALID_ARG;
    if (!std::isfinite(fan->apex_mm[0]) || !std::isfinite(fan->apex_mm[1]) || !std::isfinite(fan->r0_mm) ||
        !(fan->r0_mm >= 0.0) || !std::isfinite(fan->dr_mm) || !(fan->dr_mm > 0.0))
        return DARE_ERR_INVALID_ARG;
    if (fan->sectors < 1 || fan->sectors > kMaxBins || (w > 0 && fan->sectors > w) ||
        (int64_t)w * fan->sectors > 0x7FFFFFFF)
        return DARE_ERR_INVALID_ARG;
    if (n == 0) return v->saturated ? DARE_WARN_BINS_SATURATED : DARE_OK;
    if (!frames_dev || !probe_poses_dev || !beams_dev || w <= 0 || h <= 0 || (int64_t)w * h > (int64_t)1 << 30)
        return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    FanArgs a;
    a.apex[0] = fan->apex_mm[0];
    a.apex[1] = fan->apex_mm[1];
    a.r0 = fan->r0_mm;
    a.dr = fan->dr_mm;
    a.beams = beams_dev;
    a.sectors = fan->sectors;
    return reconstruct_batches(v, frames_dev, n, w, h, nullptr, &a, probe_poses_dev, (hipStream_t)stream);
}

dare_status dare_reslice(const dare_volume* v, const dare_slice_spec* spec, float* out_dev, void* stream) {
    if (!v || !out_dev) return DARE_ERR_INVALID_ARG;
    const dare_status st = check_spec(spec);
    if (st != DARE_OK) return st;
    DeviceGuard dg(v->device);
    const SliceArgs a = make_args(spec, out_dev);
    const int R = (int)v->p.radius_vox;
    if (staged_radius(R)) return hip_status(launch_reslice_staged(v->dev, v->dtype, R, a, (hipStream_t)stream));
    return hip_status(launch_reslice(v->dev, v->dtype, R, a, (hipStream_t)stream));
}

uint64_t dare_reslice_batch_workspace_bytes(const dare_volume* const* vols, const dare_slice_spec* specs, int32_t n) {
    if (!vols || !specs || n <= 0) return 0;
    for (int k = 0; k < n; ++k)
        if (!vols[k] || check_spec(specs + k) != DARE_OK) return 0;
    uint64_t total = 0;
    for (auto& kv : group_sizes(vols, specs, n))
        total += group_layout(kv.second.nreq, kv.second.nunits, std::get<1>(kv.first) > 1).total;
    return total;
}

}  // extern "C"

namespace {

// Arguments of a batch call checked, and the device they share; `needed` receives the
// workspace bytes the batch takes.
dare_status check_batch(const dare_volume* const* vols, const dare_slice_spec* specs, float* const* outs_dev,
                        int32_t n, int* device, uint64_t* needed) {
    if (!vols || !specs || !outs_dev || n <= 0) return DARE_ERR_INVALID_ARG;
    *device = -1;
    for (int k = 0; k < n; ++k) {
        if (!vols[k] || !outs_dev[k]) return DARE_ERR_INVALID_ARG;
        const dare_status st = check_spec(specs + k);
        if (st != DARE_OK) return st;
        if (*device < 0) *device = vols[k]->device;
        if (vols[k]->device != *device) return DARE_ERR_INVALID_ARG;
    }
    *needed = dare_reslice_batch_workspace_bytes(vols, specs, n);
    return DARE_OK;
}

// Plan every launch group of a checked batch and launch it into the device workspace `ws`:
// `upload(dst_dev, src_host, bytes)` enqueues the copy of a group's uploaded part on `stream`
// and returns false on failure.  Groups are laid out back to back in call order.
template <class Upload>
dare_status run_batch(const dare_volume* const* vols, const dare_slice_spec* specs, float* const* outs_dev,
                      int32_t n, char* ws, hipStream_t stream, Upload&& upload) {
    std::map<GroupKey, Group> groups;
    const std::vector<GroupKey> keys = group_keys(vols, n);
    for (int k = 0; k < n; ++k) {
        const int R = (int)vols[k]->p.radius_vox;
        Group& g = groups[keys[k]];
        const int r = (int)g.reqs.size();
        BatchReq q{};
        q.vol = vols[k]->dev;
        q.s = make_args(specs + k, outs_dev[k]);
        if (R <= 1) {
            g.nunits += tile_units_max(specs[k].width, specs[k].height);
        } else {
            const int64_t u = batch_units(R, specs[k].width, specs[k].height);
            for (int64_t t = 0; t < u; ++t) g.units.push_back(make_int2(r, (int)t));
            g.nunits += u;
        }
        g.reqs.push_back(q);
    }
    for (auto& kv : groups)   // units are indexed in 32 bits on the device
        if (kv.second.nunits >= INT32_MAX) return DARE_ERR_INVALID_ARG;
    std::vector<char> host;
    for (auto& kv : groups) {
        Group& g = kv.second;
        const int R = std::get<1>(kv.first);
        const bool host_units = R > 1;
        const int nreq = (int)g.reqs.size();
        const GroupLayout L = group_layout(g.reqs.size(), (size_t)g.nunits, host_units);
        host.assign(L.upload, 0);
        BatchHeader hd{};
        hd.counts[0] = host_units ? (int)g.nunits : 0;
        hd.counts[1] = nreq;
        memcpy(host.data(), &hd, sizeof(hd));
        memcpy(host.data() + L.o_req, g.reqs.data(), g.reqs.size() * sizeof(BatchReq));
        if (host_units && !g.units.empty())
            memcpy(host.data() + L.o_units, g.units.data(), g.units.size() * sizeof(int2));
        if (!upload(ws, host.data(), L.upload)) return DARE_ERR_HIP;
        const int grid = R <= 1 ? kBatchGrid : (int)std::min<int64_t>(g.nunits, 65535);
        HIP_TRY(launch_reslice_batch(std::get<0>(kv.first), R, (const BatchReq*)(ws + L.o_req),
                                     (SliceRec*)(ws + L.o_rec), (int2*)(ws + L.o_units), (TileRec*)(ws + L.o_tiles),
                                     (int*)ws, nreq, (int)g.nunits, grid, stream));
        ws += L.total;
    }
    return DARE_OK;
}

}  // namespace

extern "C" {

dare_status dare_reslice_batch(const dare_volume* const* vols, const dare_slice_spec* specs, float* const* outs_dev,
                               int32_t n, void* workspace_dev, uint64_t workspace_bytes, void* stream_) {
    if (n == 0 && vols && specs && outs_dev) return DARE_OK;
    int device = -1;
    uint64_t needed = 0;
    const dare_status st = check_batch(vols, specs, outs_dev, n, &device, &needed);
    if (st != DARE_OK) return st;
    if (!workspace_dev || workspace_bytes < needed || ((uintptr_t)workspace_dev % kAlign) != 0)
        return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(device);
    hipStream_t stream = (hipStream_t)stream_;
    StagingPool& pool = staging_pool(device);
    // uploads go through pinned staging, so the call does not wait for the stream
    auto upload = [&](char* dst, const char* src, uint64_t bytes) {
        const StagingPool::Lease lease = pool.acquire(bytes);
        if (!lease.p) return false;
        memcpy(lease.p, src, bytes);
        const hipError_t ce = hipMemcpyAsync(dst, lease.p, bytes, hipMemcpyHostToDevice, stream);
        const hipError_t re = pool.release(lease, stream);
        return ce == hipSuccess && re == hipSuccess;
    };
    return run_batch(vols, specs, outs_dev, n, (char*)workspace_dev, stream, upload);
}

}  // extern "C"

// Workspace of dare_reslice_batch_noalloc: one copy per device, in device memory until the
// process ends.  In host code this name is not a device address: every use goes through the
// per-device address taken with hipGetSymbolAddress.
static __device__ __align__(256) char scratch[DARE_NOALLOC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on `device` (current), taken on the first call there.
dare_status scratch_address(int device, char** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {nullptr};
    if (device < 0 || device >= kMaxDevices) return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DARE_ERR_HIP;
        addr[device] = p;
    }
    *out = (char*)addr[device];
    return DARE_OK;
}

}  // namespace

extern "C" {

dare_status dare_reslice_batch_noalloc(const dare_volume* const* vols, const dare_slice_spec* specs,
                                       float* const* outs_dev, int32_t n, void* stream_) {
    if (n == 0 && vols && specs && outs_dev) return DARE_OK;
    int device = -1;
    uint64_t needed = 0;
    dare_status st = check_batch(vols, specs, outs_dev, n, &device, &needed);
    if (st != DARE_OK) return st;
    if (needed == 0) return DARE_ERR_INVALID_ARG;
    if (needed > DARE_NOALLOC_WORKSPACE_BYTES) return DARE_ERR_BUDGET;
    DeviceGuard dg(device);
    char* ws = nullptr;
    st = scratch_address(device, &ws);
    if (st != DARE_OK) return st;
    hipStream_t stream = (hipStream_t)stream_;
    // the request table goes from pageable host memory: no pinned staging to allocate
    auto upload = [&](char* dst, const char* src, uint64_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
    };
    return run_batch(vols, specs, outs_dev, n, ws, stream, upload);
}

dare_status dare_bounds_from_frames(const float* poses, int32_t n, int32_t w, int32_t h, const double pitch_mm[2],
                                    const double calib[16], double spacing_mm, dare_geometry* out) {
    if (!poses || n <= 0 || w <= 0 || h <= 0 || !pitch_mm || !calib || !out || !(spacing_mm > 0.0))
        return DARE_ERR_INVALID_ARG;
    if (!rigid(calib)) return DARE_ERR_BAD_POSE;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int f = 0; f < n; ++f) {
        double P[16], T[16];
        for (int k = 0; k < 16; ++k) P[k] = (double)poses[(size_t)f * 16 + k];
        if (!rigid(P)) return DARE_ERR_BAD_POSE;
        compose_host(P, calib, T);
        const int ci[4] = {0, w - 1, 0, w - 1}, cj[4] = {0, 0, h - 1, h - 1};
        for (int k = 0; k < 4; ++k) {
            const double is = (double)ci[k] * pitch_mm[0], js = (double)cj[k] * pitch_mm[1];
            for (int a = 0; a < 3; ++a) {
                const double p = (T[a * 4 + 3] + is * T[a * 4 + 0]) + js * T[a * 4 + 1];
                lo[a] = std::min(lo[a], p);
                hi[a] = std::max(hi[a], p);
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        out->origin_mm[a] = lo[a];
        const double d = ceil((hi[a] - lo[a]) / spacing_mm) + 1.0;
        if (!(d >= 1.0 && d <= (double)(1 << 16))) return DARE_ERR_INVALID_ARG;
        out->dims[a] = (int32_t)d;
    }
    out->spacing_mm = spacing_mm;
    memcpy(out->calib, calib, sizeof(out->calib));
    return DARE_OK;
}

dare_status dare_volume_get_info(const dare_volume* v, dare_volume_info* out) {
    if (!v || !out) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    HIP_TRY(hipDeviceSynchronize());
    out->bins = v->K;
    out->saturated = v->saturated;
    out->bricks_used = v->used;
    out->bricks_capacity = v->host.cap;
    const Layout L = layout(&v->g, &v->p, v->dtype, 0);
    out->bytes_per_brick = (int64_t)L.per_slot;
    out->brick_grid[0] = L.nbx;
    out->brick_grid[1] = L.nby;
    out->brick_grid[2] = L.nbz;
    return DARE_OK;
}

dare_status dare_volume_get_codebook(const dare_volume* v, double* rep_n, double* rep_x, int32_t* bins) {
    if (!v || !rep_n || !rep_x || !bins) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    HIP_TRY(hipDeviceSynchronize());
    VolDev tmp;
    HIP_TRY(hipMemcpy(&tmp, v->dev, sizeof(VolDev), hipMemcpyDeviceToHost));
    *bins = tmp.st.K;
    for (int b = 0; b < tmp.st.K; ++b)
        for (int a = 0; a < 3; ++a) {
            rep_n[b * 3 + a] = tmp.rep_n[b][a];
            rep_x[b * 3 + a] = tmp.rep_x[b][a];
        }
    return DARE_OK;
}

// ------------------------------------------------------------------ persistence
// A saved volume: a fixed header, then the brick table (max_bins x bricks per bin int32), the
// accumulators, stored pairs and FP8 scales of the `used` slots, back to back.
namespace {

struct SavedHeader {
    char magic[8];
    uint32_t version, header_bytes;
    dare_geometry g;
    dare_params p;
    int32_t dtype, K, saturated;
    uint32_t used;
    double rep_n[kMaxBins][3], rep_x[kMaxBins][3];
    uint64_t table_bytes, acc_bytes, data_bytes, scales_bytes;
};

constexpr char kSaveMagic[8] = {'D', 'A', 'R', 'E', 'V', 'O', 'L', '1'};

void saved_sizes(const dare_geometry* g, const dare_params* p, int dtype, uint32_t used, SavedHeader* h) {
    const Layout L = layout(g, p, dtype, 0);
    h->table_bytes = (uint64_t)p->max_bins * L.nbricks * sizeof(int32_t);
    h->acc_bytes = (uint64_t)used * kBrickVox * sizeof(unsigned long long);
    h->data_bytes = (uint64_t)used * kBrickVox * (uint64_t)pair_bytes(dtype);
    h->scales_bytes = (uint64_t)used * sizeof(float2);
}

uint64_t saved_total(const SavedHeader& h) {
    return sizeof(SavedHeader) + h.table_bytes + h.acc_bytes + h.data_bytes + h.scales_bytes;
}

// A saved brick table is used as gather and atomic addresses on the device, so it is checked in
// full before anything is uploaded: every entry -1 or a slot below `used`, each slot owned by
// exactly one entry (the pool is compact), no entry in the rows of bins >= K, and finite
// representatives for the bins in use.
bool saved_table_ok(const SavedHeader& h, const int32_t* table) {
    const uint64_t n = h.table_bytes / sizeof(int32_t);
    const uint64_t nbricks = n / (uint64_t)h.p.max_bins;
    std::vector<uint8_t> owned(h.used, 0);
    for (uint64_t k = 0; k < n; ++k) {
        const int32_t e = table[k];
        if (e == -1) continue;
        if (e < 0 || (uint32_t)e >= h.used || (int64_t)(k / nbricks) >= h.K || owned[e]) return false;
        owned[e] = 1;
    }
    for (uint32_t s = 0; s < h.used; ++s)
        if (!owned[s]) return false;
    for (int b = 0; b < h.K; ++b)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(h.rep_n[b][a]) || !std::isfinite(h.rep_x[b][a])) return false;
    return true;
}

}  // namespace

uint64_t dare_volume_save_bytes(const dare_volume* v) {
    if (!v) return 0;
    DeviceGuard dg(v->device);
    if (hipDeviceSynchronize() != hipSuccess) return 0;
    SavedHeader h{};
    saved_sizes(&v->g, &v->p, v->dtype, v->used, &h);
    return saved_total(h);
}

dare_status dare_volume_save(const dare_volume* v, void* host_out, uint64_t bytes) {
    if (!v || !host_out || !v->held.empty()) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    HIP_TRY(hipDeviceSynchronize());
    VolDev d;
    HIP_TRY(hipMemcpy(&d, v->dev, sizeof(VolDev), hipMemcpyDeviceToHost));
    SavedHeader h{};
    memcpy(h.magic, kSaveMagic, sizeof(h.magic));
    h.version = 1;
    h.header_bytes = sizeof(SavedHeader);
    h.g = v->g;
    h.p = v->p;
    h.dtype = v->dtype;
    h.K = d.st.K;
    h.saturated = d.st.saturated;
    h.used = d.st.used;
    memcpy(h.rep_n, d.rep_n, sizeof(h.rep_n));
    memcpy(h.rep_x, d.rep_x, sizeof(h.rep_x));
    saved_sizes(&v->g, &v->p, v->dtype, h.used, &h);
    if (bytes < saved_total(h)) return DARE_ERR_INVALID_ARG;
    char* o = (char*)host_out;
    memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    HIP_TRY(hipMemcpy(o, d.table, h.table_bytes, hipMemcpyDeviceToHost));
    o += h.table_bytes;
    if (h.used) {
        HIP_TRY(hipMemcpy(o, d.acc, h.acc_bytes, hipMemcpyDeviceToHost));
        o += h.acc_bytes;
        HIP_TRY(hipMemcpy(o, d.data, h.data_bytes, hipMemcpyDeviceToHost));
        o += h.data_bytes;
        HIP_TRY(hipMemcpy(o, d.scales, h.scales_bytes, hipMemcpyDeviceToHost));
    }
    return DARE_OK;
}

dare_status dare_volume_load(const void* host_in, uint64_t bytes, void* arena_dev, uint64_t arena_bytes,
                             dare_volume** out) {
    if (!host_in || !out || bytes < sizeof(SavedHeader)) return DARE_ERR_INVALID_ARG;
    *out = nullptr;
    SavedHeader h;
    memcpy(&h, host_in, sizeof(h));
    if (memcmp(h.magic, kSaveMagic, sizeof(h.magic)) != 0 || h.version != 1 || h.header_bytes != sizeof(SavedHeader))
        return DARE_ERR_INVALID_ARG;
    if (check_geometry(&h.g) != DARE_OK || check_params(&h.p) != DARE_OK || !valid_dtype(h.dtype) || h.K < 0 ||
        h.K > h.p.max_bins)
        return DARE_ERR_INVALID_ARG;
    SavedHeader sz = h;
    saved_sizes(&h.g, &h.p, h.dtype, h.used, &sz);
    if (sz.table_bytes != h.table_bytes || sz.acc_bytes != h.acc_bytes || sz.data_bytes != h.data_bytes ||
        sz.scales_bytes != h.scales_bytes || bytes < saved_total(h))
        return DARE_ERR_INVALID_ARG;
    if ((h.saturated != 0 && h.saturated != 1) ||
        !saved_table_ok(h, (const int32_t*)((const char*)host_in + sizeof(SavedHeader))))
        return DARE_ERR_INVALID_ARG;
    dare_volume* v = nullptr;
    dare_status st = dare_volume_create(&h.g, &h.p, (dare_dtype)h.dtype, arena_dev, arena_bytes, &v);
    if (st != DARE_OK) return st;
    if (h.used > v->host.cap) {
        dare_volume_destroy(v);
        return DARE_ERR_BUDGET;
    }
    const char* in = (const char*)host_in + sizeof(SavedHeader);
    VolDev& d = v->host;
    hipError_t e = hipMemcpy(d.table, in, h.table_bytes, hipMemcpyHostToDevice);
    in += h.table_bytes;
    if (e == hipSuccess && h.used) {
        e = hipMemcpy(d.acc, in, h.acc_bytes, hipMemcpyHostToDevice);
        in += h.acc_bytes;
        if (e == hipSuccess) e = hipMemcpy(d.data, in, h.data_bytes, hipMemcpyHostToDevice);
        in += h.data_bytes;
        if (e == hipSuccess) e = hipMemcpy(d.scales, in, h.scales_bytes, hipMemcpyHostToDevice);
    }
    d.st.K = h.K;
    d.st.saturated = h.saturated;
    d.st.used = h.used;
    memcpy(d.rep_n, h.rep_n, sizeof(d.rep_n));
    memcpy(d.rep_x, h.rep_x, sizeof(d.rep_x));
    if (e == hipSuccess) e = hipMemcpy(v->dev, &d, sizeof(VolDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        dare_volume_destroy(v);
        return DARE_ERR_HIP;
    }
    v->K = h.K;
    v->saturated = h.saturated;
    v->used = h.used;
    *out = v;
    return DARE_OK;
}

dare_status dare_volume_download_sums(const dare_volume* v, uint32_t* S, uint32_t* C, int32_t bins, void* stream) {
    if (!v || !S || !C || bins != v->K) return DARE_ERR_INVALID_ARG;
    if (bins == 0) return DARE_OK;
    DeviceGuard dg(v->device);
    return hip_status(launch_download_sums(v->dev, S, C, bins, v->g.dims[0], v->g.dims[1], v->g.dims[2],
                                           (hipStream_t)stream));
}

dare_status dare_volume_download_storage(const dare_volume* v, float* A, float* C, int32_t bins, void* stream) {
    if (!v || !A || !C || bins != v->K) return DARE_ERR_INVALID_ARG;
    if (bins == 0) return DARE_OK;
    DeviceGuard dg(v->device);
    return hip_status(launch_download_storage(v->dev, v->dtype, A, C, bins, v->g.dims[0], v->g.dims[1],
                                              v->g.dims[2], (hipStream_t)stream));
}

dare_status dare_volume_upload_sums(dare_volume* v, const double* rep_n, const double* rep_x, int32_t bins,
                                    const uint32_t* S, const uint32_t* C, void* stream_) {
    if (!v || bins < 0 || bins > v->p.max_bins) return DARE_ERR_INVALID_ARG;
    if (bins > 0 && (!rep_n || !rep_x || !S || !C)) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    hipStream_t stream = (hipStream_t)stream_;
    VolDev h = v->host;
    memset(&h.st, 0, sizeof(h.st));
    h.st.K = bins;
    for (int b = 0; b < bins; ++b)
        for (int a = 0; a < 3; ++a) {
            h.rep_n[b][a] = rep_n[b * 3 + a];
            h.rep_x[b][a] = rep_x[b * 3 + a];
        }
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(v->dev, &h, sizeof(VolDev), hipMemcpyHostToDevice));
    HIP_TRY(launch_table_fill(h.table, (int64_t)v->p.max_bins * h.nbricks, stream));
    if (h.cap) HIP_TRY(hipMemsetAsync(h.dirty_flags, 0, (size_t)h.cap * sizeof(uint32_t), stream));
    v->host.st = h.st;
    memcpy(v->host.rep_n, h.rep_n, sizeof(h.rep_n));
    memcpy(v->host.rep_x, h.rep_x, sizeof(h.rep_x));
    v->K = bins;
    v->saturated = 0;
    v->used = 0;
    v->held.clear();
    std::fill(v->stamp.begin(), v->stamp.end(), 0);
    if (bins == 0) return hip_status(hipStreamSynchronize(stream));
    HIP_TRY(launch_dense_mark(v->dev, C, bins, stream));
    VolState st;
    dare_status s = read_state(v, stream, &st);
    if (s != DARE_OK) return s;
    if (st.new_count > h.cap) {
        HIP_TRY(launch_rollback(v->dev, st.new_count, 0, 0, 0, stream));
        HIP_TRY(launch_clear_marks(h.table, (int64_t)v->p.max_bins * h.nbricks, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        v->K = 0;
        return DARE_ERR_BUDGET;
    }
    HIP_TRY(launch_alloc(v->dev, st.new_count, 0, 0, stream));
    HIP_TRY(launch_dense_scatter(v->dev, S, C, bins, stream));
    HIP_TRY(launch_finalize(v->dev, v->dtype, st.new_count, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    v->used = st.new_count;
    return DARE_OK;
}

dare_status dare_slice_active_bins(const dare_volume* v, const dare_slice_spec* spec, int32_t* bins_out,
                                   double* weights_out, int32_t* count) {
    if (!v || !count) return DARE_ERR_INVALID_ARG;
    const dare_status st = check_spec(spec);
    if (st != DARE_OK) return st;
    double T[16];
    compose_host(spec->probe_pose, v->g.calib, T);
    int32_t bins[kMaxBins];
    double w[kMaxBins];
    const int n = gate_bins(v, T, bins, w);
    for (int k = 0; k < n; ++k) {
        if (bins_out) bins_out[k] = bins[k];
        if (weights_out) weights_out[k] = w[k];
    }
    *count = n;
    return DARE_OK;
}

dare_status dare_copy_probe(const void* src, void* dst, uint64_t n, void* stream) {
    if (!src || !dst || n == 0 || (n % 16) != 0) return DARE_ERR_INVALID_ARG;
    return hip_status(launch_copy_probe(src, dst, n, (hipStream_t)stream));
}

}  // extern "C"
