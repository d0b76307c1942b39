// Out-of-core bricks: moving bricks between a volume's HBM pool and host memory, so that a
// volume can outgrow its arena (Sec. 4 names support for data sets beyond GPU memory, next to
// incremental integration of newly acquired frames during a scan, as the method's next steps).
//
// A brick's whole state is its 512 accumulators, (sum << 32) | count, exact integers; its
// stored pairs and FP8 scales follow from them by finalisation.  So a brick leaves with its
// accumulators only, and when it comes back they are added to whatever the brick gathered in
// HBM meanwhile, then the brick is finalised.  Integer addition makes the outcome independent of
// when bricks left or came back: once everything is restored, a volume that spilled holds what
// one large arena would have built, bit for bit.
//
// Pool compaction.  Slots stay 0 .. used - 1 (compounding bumps `used`).  Evicting leaves holes
// below the new count `kept`; each hole takes one kept slot from at or above `kept`, so sources
// and destinations are disjoint and one launch moves them all.  A moving slot swaps its
// accumulators with its hole's (the leaving accumulators thereby end up contiguous at
// kept .. used - 1 and come back to the host in one copy) and copies its stored pairs and scale.
#include <string.h>

#include <algorithm>
#include <numeric>
#include <unordered_map>

#include "dare_host.h"

using namespace dare;

namespace {

constexpr uint64_t kStageBytes = 64ull << 20;   // pinned host staging per transfer round

// owner[s] = the table entry pool slot s holds, for every allocated slot.
__global__ void __launch_bounds__(256) k_slot_owner(const int32_t* __restrict__ table, int64_t n,
                                                    int32_t* __restrict__ owner) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int32_t s = table[e];
        if (s >= 0) owner[s] = (int32_t)e;
    }
}

// fate[s], s < used: s (stays), a hole below `kept` (moves there) or -1 (leaves).  Points each
// table entry at its slot's new place; entries own distinct slots, so the writes are disjoint.
__global__ void __launch_bounds__(256) k_relabel(int32_t* __restrict__ table, const int32_t* __restrict__ owner,
                                                 const int32_t* __restrict__ fate, uint32_t used) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= used) return;
    const int32_t f = fate[s];
    if (f != (int32_t)s) table[owner[s]] = f;
}

// One workgroup per slot kept + blockIdx.x: if it moves, swap accumulators with its hole and
// copy its stored pairs (`pair_words` 32-bit words per slot) and scale there.
__global__ void __launch_bounds__(256) k_move_slots(unsigned long long* __restrict__ acc, uint32_t* __restrict__ data,
                                                    float2* __restrict__ scales, const int32_t* __restrict__ fate,
                                                    uint32_t kept, int pair_words) {
    const uint32_t s = kept + blockIdx.x;
    const int32_t h = fate[s];
    if (h < 0) return;   // leaves: its accumulators are read back from here
    unsigned long long* a = acc + (size_t)s * kBrickVox;
    unsigned long long* b = acc + (size_t)h * kBrickVox;
    for (int k = threadIdx.x; k < kBrickVox; k += 256) {
        const unsigned long long x = a[k];
        a[k] = b[k];
        b[k] = x;
    }
    const uint32_t* da = data + (size_t)s * pair_words;
    uint32_t* db = data + (size_t)h * pair_words;
    for (int k = threadIdx.x; k < pair_words; k += 256) db[k] = da[k];
    if (threadIdx.x == 0) scales[h] = scales[s];
}

// Entries brought back into the fresh slots base .. base + n - 1, in order.
__global__ void __launch_bounds__(256) k_adopt(int32_t* __restrict__ table, const int32_t* __restrict__ ent, uint32_t n,
                                               uint32_t base) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) table[ent[k]] = (int32_t)(base + k);
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

struct Pinned {
    void* p = nullptr;
    explicit Pinned(uint64_t bytes) {
        if (bytes && hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) p = nullptr;
    }
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

constexpr uint64_t kAccBytes = (uint64_t)kBrickVox * sizeof(unsigned long long);

// Slot -> table entry of every allocated slot, on the host (the device copy stays in new_list,
// which is free between frame batches).
dare_status read_owners(dare_volume* v, hipStream_t stream, std::vector<int32_t>& owner) {
    owner.assign(v->used, -1);
    if (!v->used) return DARE_OK;
    const int64_t n = (int64_t)v->K * v->host.nbricks;
    HIP_TRY(hipMemsetAsync(v->host.new_list, 0xFF, (size_t)v->used * sizeof(int32_t), stream));
    hipLaunchKernelGGL(k_slot_owner, dim3(blocks_for(n)), dim3(256), 0, stream, v->host.table, n, v->host.new_list);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(owner.data(), v->host.new_list, (size_t)v->used * sizeof(int32_t), hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    // every allocated slot belongs to exactly one entry of a bin in use; anything else would
    // send the table rewrites below astray
    for (int32_t e : owner)
        if (e < 0 || e >= n) return DARE_ERR_HIP;
    return DARE_OK;
}

dare_status set_used(dare_volume* v, uint32_t used, hipStream_t stream) {
    v->used = used;
    HIP_TRY(hipMemcpyAsync(&v->dev->st.used, &v->used, sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return DARE_OK;
}

// Whether the brick of table entry `entry` meets the voxel box lo..hi (never, if the box is empty).
bool meets_box(const dare_volume* v, int64_t entry, const int32_t lo[3], const int32_t hi[3]) {
    if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]) return false;
    const int64_t b = entry % v->host.nbricks;
    const int64_t c[3] = {b % v->host.nbx, (b / v->host.nbx) % v->host.nby, b / ((int64_t)v->host.nbx * v->host.nby)};
    for (int a = 0; a < 3; ++a)
        if (c[a] * kBrick > hi[a] || c[a] * kBrick + kBrick - 1 < lo[a]) return false;
    return true;
}

void hold(dare_volume* v, int64_t entry, const unsigned long long* acc) {
    bool fresh;
    unsigned long long* r = v->held.add(entry, fresh);
    if (fresh) {
        memcpy(r, acc, kAccBytes);
    } else {
        for (int k = 0; k < kBrickVox; ++k) r[k] += acc[k];
    }
}

// Bring the held entries `ents` back (all of them fit: checked by the caller).
dare_status restore_entries(dare_volume* v, const std::vector<int64_t>& ents, hipStream_t stream) {
    if (ents.empty()) return DARE_OK;
    std::vector<int32_t> owner;
    dare_status st = read_owners(v, stream, owner);
    if (st != DARE_OK) return st;
    std::unordered_map<int64_t, uint32_t> slot_of;
    slot_of.reserve(owner.size() * 2);
    for (uint32_t s = 0; s < owner.size(); ++s) slot_of[owner[s]] = s;
    std::vector<int64_t> fresh, merge;
    std::vector<uint32_t> merge_slot;
    for (int64_t e : ents) {
        auto it = slot_of.find(e);
        if (it == slot_of.end()) {
            fresh.push_back(e);
        } else {
            merge.push_back(e);
            merge_slot.push_back(it->second);
        }
    }
    const uint32_t base = v->used;
    if ((uint64_t)base + fresh.size() > v->host.cap) return DARE_ERR_BUDGET;
    const VolDev& d = v->host;
    std::vector<int32_t> targets;
    // fresh slots: the held accumulators as they are, in rounds of the staging size
    const uint64_t per_round = std::max<uint64_t>(1, kStageBytes / kAccBytes);
    Pinned stage(std::min<uint64_t>(std::max(fresh.size(), merge.size()), per_round) * kAccBytes);
    if (!stage.p) return DARE_ERR_HIP;
    unsigned long long* buf = (unsigned long long*)stage.p;
    for (size_t k0 = 0; k0 < fresh.size(); k0 += per_round) {
        const size_t m = std::min<size_t>(per_round, fresh.size() - k0);
        for (size_t k = 0; k < m; ++k) memcpy(buf + k * kBrickVox, v->held.find(fresh[k0 + k]), kAccBytes);
        HIP_TRY(hipMemcpyAsync(d.acc + (size_t)(base + k0) * kBrickVox, buf, m * kAccBytes, hipMemcpyHostToDevice,
                               stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    if (!fresh.empty()) {
        std::vector<int32_t> ent32(fresh.begin(), fresh.end());
        HIP_TRY(hipMemcpyAsync(d.new_list, ent32.data(), ent32.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(k_adopt, dim3(blocks_for((int64_t)ent32.size())), dim3(256), 0, stream, d.table, d.new_list,
                           (uint32_t)ent32.size(), base);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(stream));
        for (size_t k = 0; k < fresh.size(); ++k) targets.push_back((int32_t)(base + k));
    }
    // resident again since they left: read, add on the host (exact), write back
    for (size_t k0 = 0; k0 < merge.size(); k0 += per_round) {
        const size_t m = std::min<size_t>(per_round, merge.size() - k0);
        for (size_t k = 0; k < m; ++k)
            HIP_TRY(hipMemcpyAsync(buf + k * kBrickVox, d.acc + (size_t)merge_slot[k0 + k] * kBrickVox, kAccBytes,
                                   hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (size_t k = 0; k < m; ++k) {
            const unsigned long long* r = v->held.find(merge[k0 + k]);
            for (int i = 0; i < kBrickVox; ++i) buf[k * kBrickVox + i] += r[i];
        }
        for (size_t k = 0; k < m; ++k)
            HIP_TRY(hipMemcpyAsync(d.acc + (size_t)merge_slot[k0 + k] * kBrickVox, buf + k * kBrickVox, kAccBytes,
                                   hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (size_t k = 0; k < m; ++k) targets.push_back((int32_t)merge_slot[k0 + k]);
    }
    HIP_TRY(hipMemcpyAsync(d.dirty_list, targets.data(), targets.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(launch_finalize(v->dev, v->dtype, (uint32_t)targets.size(), stream));
    st = set_used(v, base + (uint32_t)fresh.size(), stream);
    if (st != DARE_OK) return st;
    for (int32_t s : targets) v->stamp[s] = v->clock;
    for (int64_t e : ents) v->held.erase(e);
    return DARE_OK;
}

}  // namespace

namespace dare {

dare_status spill_slots(dare_volume* v, const std::vector<uint32_t>& victims, hipStream_t stream) {
    if (victims.empty()) return DARE_OK;
    const uint32_t used = v->used;
    std::vector<int32_t> owner;
    dare_status st = read_owners(v, stream, owner);
    if (st != DARE_OK) return st;
    std::vector<char> gone(used, 0);
    for (uint32_t s : victims)
        if (s < used) gone[s] = 1;
    const uint32_t nev = (uint32_t)std::count(gone.begin(), gone.end(), 1);
    if (nev == 0) return DARE_OK;
    const uint32_t kept = used - nev;
    std::vector<int32_t> fate(used);
    for (uint32_t s = 0; s < used; ++s) fate[s] = gone[s] ? -1 : (int32_t)s;
    uint32_t t = kept;
    for (uint32_t h = 0; h < kept; ++h) {
        if (!gone[h]) continue;
        while (gone[t]) ++t;   // as many keepers at or above `kept` as holes below it
        fate[t] = (int32_t)h;
        v->stamp[h] = v->stamp[t];
        ++t;
    }
    // after the move, position kept + i holds the accumulators of entry leaving[i]
    std::vector<int64_t> leaving(nev);
    for (uint32_t s = kept; s < used; ++s) leaving[s - kept] = owner[fate[s] >= 0 ? fate[s] : s];
    const VolDev& d = v->host;
    HIP_TRY(hipMemcpyAsync(d.dirty_list, fate.data(), (size_t)used * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_relabel, dim3((used + 255) / 256), dim3(256), 0, stream, d.table, d.new_list, d.dirty_list,
                       used);
    const int pair_words = kBrickVox * pair_bytes(v->dtype) / 4;
    hipLaunchKernelGGL(k_move_slots, dim3(nev), dim3(256), 0, stream, d.acc, (uint32_t*)d.data, d.scales, d.dirty_list,
                       kept, pair_words);
    HIP_TRY(hipGetLastError());
    const uint64_t per_round = std::max<uint64_t>(1, kStageBytes / kAccBytes);
    Pinned stage(std::min<uint64_t>(nev, per_round) * kAccBytes);
    if (!stage.p) return DARE_ERR_HIP;
    const unsigned long long* buf = (const unsigned long long*)stage.p;
    for (uint32_t k0 = 0; k0 < nev; k0 += (uint32_t)per_round) {
        const uint32_t m = (uint32_t)std::min<uint64_t>(per_round, nev - k0);
        HIP_TRY(hipMemcpyAsync(stage.p, d.acc + (size_t)(kept + k0) * kBrickVox, m * kAccBytes, hipMemcpyDeviceToHost,
                               stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (uint32_t k = 0; k < m; ++k) hold(v, leaving[k0 + k], buf + (size_t)k * kBrickVox);
    }
    return set_used(v, kept, stream);
}

dare_status spill_for_batch(dare_volume* v, const std::vector<int32_t>& keep, uint64_t need, hipStream_t stream) {
    const uint32_t used = v->used;
    std::vector<char> busy(used, 0);
    for (int32_t s : keep)
        if (s >= 0 && (uint32_t)s < used) busy[s] = 1;
    std::vector<uint32_t> cand;
    for (uint32_t s = 0; s < used; ++s)
        if (!busy[s]) cand.push_back(s);
    if (cand.size() < need) return DARE_ERR_BUDGET;
    const uint64_t take = std::min<uint64_t>(cand.size(), need + v->host.cap / 16);
    std::stable_sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) { return v->stamp[a] < v->stamp[b]; });
    cand.resize(take);
    return spill_slots(v, cand, stream);
}

}  // namespace dare

extern "C" {

dare_status dare_volume_evict_outside(dare_volume* v, const int32_t lo[3], const int32_t hi[3], void* stream_) {
    if (!v || !lo || !hi) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    hipStream_t stream = (hipStream_t)stream_;
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<int32_t> owner;
    dare_status st = read_owners(v, stream, owner);
    if (st != DARE_OK) return st;
    std::vector<uint32_t> victims;
    for (uint32_t s = 0; s < owner.size(); ++s)
        if (owner[s] >= 0 && !meets_box(v, owner[s], lo, hi)) victims.push_back(s);
    return spill_slots(v, victims, stream);
}

dare_status dare_volume_restore_box(dare_volume* v, const int32_t lo[3], const int32_t hi[3], void* stream_) {
    if (!v || !lo || !hi) return DARE_ERR_INVALID_ARG;
    DeviceGuard dg(v->device);
    hipStream_t stream = (hipStream_t)stream_;
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<int64_t> ents;
    for (const auto& kv : v->held.index())
        if (meets_box(v, kv.first, lo, hi)) ents.push_back(kv.first);
    std::sort(ents.begin(), ents.end());   // fresh slots in entry order, whatever the map's order
    return restore_entries(v, ents, stream);
}

dare_status dare_volume_set_spill(dare_volume* v, int32_t enabled) {
    if (!v) return DARE_ERR_INVALID_ARG;
    v->spill = enabled != 0;
    return DARE_OK;
}

dare_status dare_volume_held(const dare_volume* v, int64_t* bricks, uint64_t* bytes) {
    if (!v || !bricks || !bytes) return DARE_ERR_INVALID_ARG;
    *bricks = (int64_t)v->held.size();
    *bytes = (uint64_t)v->held.size() * kAccBytes;
    return DARE_OK;
}

}  // extern "C"
