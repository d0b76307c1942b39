// Serving: continuous batching of reslice requests from many consoles.
//
// A scheduler thread turns the FIFO of waiting requests into ticks.  A tick
// takes requests from the head of the queue while they fit its pixel and unit
// budget and while a result slot of their size can be allocated in the
// server's arena (the HBM budget of results); the head request waits until
// slots free up, so admission is first come, first served.  Volumes are
// admitted against a second budget, the device bytes of the resident volumes'
// arenas, and can be removed once their requests have completed.  Each tick
// goes to one of up to four streams: its request table is uploaded from pinned
// staging, a captured graph runs the batched reslice (per-request setup pass +
// persistent tile kernel), the results are copied to the callers' host buffers
// and an event marks completion.  Ticks on different streams overlap on the
// device, and requests that arrive meanwhile are admitted into the next tick
// whose stream is free.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dare_alloc.h"
#include "dare_spans.h"
#include "dare_staged.h"

using namespace dare;

namespace dare {
// Views into the C ABI's volume (defined in dare_capi.hip).
const VolDev* volume_device(const dare_volume* v);
int volume_dtype(const dare_volume* v);
int volume_radius(const dare_volume* v);
int volume_device_id(const dare_volume* v);
uint64_t volume_arena_size(const dare_volume* v);
int reslice_lanes(int radius);
dare_status check_slice_spec(const dare_slice_spec* s);
}  // namespace dare

namespace {

constexpr int kMaxStreams = 4;
constexpr uint64_t kAlignS = 256;
constexpr int kServerGrid = 2048;

uint64_t aup(uint64_t x) { return (x + kAlignS - 1) / kAlignS * kAlignS; }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Work units of a request (radius 1: the most the device may append, 16 x 16 tiles).
int64_t units_of(int radius, int W, int H) {
    return radius <= 1 ? tile_units_max(W, H) : batch_units(radius, W, H);
}

enum ReqState { kWaiting = 0, kInFlight = 1, kDone = 2, kFailed = 3 };

struct Request {
    bool frames_job = false;          // a batch of frames to compound, not a reslice
    int vol = 0;
    dare_slice_spec spec{};
    float* host_out = nullptr;
    uint64_t out_off = UINT64_MAX;
    uint64_t bytes = 0;
    int64_t units = 0;
    int state = kWaiting;
    dare_request_times t{};
    // frames job: dare_reconstruct_frames arguments and its status
    const uint8_t* frames = nullptr;
    const float* poses = nullptr;
    int32_t nframes = 0, fw = 0, fh = 0;
    double fpitch[2] = {0.0, 0.0};
    dare_status status = DARE_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr, ev_kernels = nullptr, ev_done = nullptr;
    hipGraphExec_t graph = nullptr;
    char* ws = nullptr;           // device workspace: header, requests, units, setup records
    uint64_t ws_off = UINT64_MAX; // its place in the arena
    char* staging = nullptr;      // pinned host copy of the uploaded part
    bool busy = false;
    bool kernels_seen = false;
    double last_end = 0.0;        // device time at which this slot's last timed tick's kernels ended
    std::vector<uint64_t> tickets;
};

// Device time of the ticks' kernels.  Each tick's kernels lie between two timing events on its
// slot's stream; their spans are summed, and their union (ticks on different streams overlap)
// is the time the device spent on served kernels.  Event times are taken against a reference
// event on an otherwise idle stream, moved forward about once a second so that the single
// precision of hipEventElapsedTime stays well below a microsecond.
struct DeviceClock {
    hipStream_t stream = nullptr;
    hipEvent_t ref[2] = {nullptr, nullptr};
    int cur = 0;
    bool moving = false;          // ref[1 - cur] recorded, not yet reached
    double off = 0.0;             // seconds from the first reference to ref[cur]
    double host_t = 0.0;          // host time at which ref[cur] was taken
    SpanUnion spans;              // the ticks' kernel spans: their sum and their union

    hipError_t init(double now) {
        hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreate(&ref[k]);
        if (e == hipSuccess) e = hipEventRecord(ref[0], stream);
        if (e == hipSuccess) e = hipEventSynchronize(ref[0]);
        host_t = now;
        return e;
    }
    void destroy() {
        for (hipEvent_t& r : ref)
            if (r) (void)hipEventDestroy(r);
        if (stream) (void)hipStreamDestroy(stream);
    }
    // Seconds from the first reference to event `ev` (completed); false if it cannot be timed.
    bool at(hipEvent_t ev, double* t) const {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ref[cur], ev) != hipSuccess) return false;
        *t = off + 1e-3 * (double)ms;
        return true;
    }
    void advance(double now) {
        if (!stream || now - host_t < 1.0) return;
        if (!moving) {
            moving = hipEventRecord(ref[1 - cur], stream) == hipSuccess;
        } else if (hipEventQuery(ref[1 - cur]) == hipSuccess) {
            double t = 0.0;
            if (at(ref[1 - cur], &t)) {
                off = t;
                cur = 1 - cur;
            }
            moving = false;
            host_t = now;
        }
    }
};

}  // namespace

// A registered volume: its device bytes count against the volume budget while it is resident.
struct VolEntry {
    dare_volume* v = nullptr;         // null once removed (ids are never reused)
    uint64_t bytes = 0;
    int64_t pending = 0;              // queued or in-flight requests and frames jobs
    bool closing = false;             // being removed: new requests are refused
};

struct dare_server {
    dare_server_config cfg{};
    int device = 0;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    // workspace layout (identical in every slot, sized for a full tick), set by the first volume
    uint64_t o_req = 0, o_units = 0, o_tiles = 0, o_rec = 0, ws_bytes = 0;
    int64_t max_units = 0;
    Slot slots[kMaxStreams];
    RangeAlloc outs;                  // result slots and the slots' workspaces
    std::vector<VolEntry> vols;
    uint64_t vol_bytes = 0;           // resident volumes' bytes
    int dtype = -1, radius = -1;
    std::mutex mu;
    std::condition_variable cv;       // scheduler: new work or stop
    std::condition_variable done_cv;  // waiters: some request completed
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    dare_server_stats stats{};
    std::atomic<bool> stop{false};
    std::thread th;
    double busy_since = -1.0;
    bool failed = false;
    DeviceClock clock;
};

namespace {

// Launch the tick's kernels on the slot's stream (captured once into a graph when enabled).
hipError_t enqueue_kernels(dare_server* S, Slot& sl) {
    return launch_reslice_batch(S->dtype, S->radius, (const BatchReq*)(sl.ws + S->o_req), (SliceRec*)(sl.ws + S->o_rec),
                                (int2*)(sl.ws + S->o_units), (TileRec*)(sl.ws + S->o_tiles), (int*)sl.ws,
                                S->cfg.max_tick_requests, (int)S->max_units,
                                S->radius <= 1 ? kServerGrid : 4096,
                                sl.stream);
}

hipError_t ensure_graph(dare_server* S, Slot& sl) {
    if (!S->cfg.use_graphs || sl.graph) return hipSuccess;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue_kernels(S, sl);
    e = hipStreamEndCapture(sl.stream, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

// A request leaves the device: its result slot is returned and its volume's count drops.
void release_request(dare_server* S, Request& r) {
    if (r.out_off != UINT64_MAX) S->outs.release(r.out_off, r.bytes);
    r.out_off = UINT64_MAX;
    S->vols[r.vol].pending -= 1;
}

// Device span of a tick whose kernels have finished.  A later tick of a busy slot starts after
// that slot's last timed tick (stream order); an idle slot's next tick starts after now.
void time_tick(dare_server* S, Slot& sl) {
    float ms = 0.0f;
    double t0 = 0.0;
    if (hipEventElapsedTime(&ms, sl.ev_start, sl.ev_kernels) != hipSuccess || !S->clock.at(sl.ev_start, &t0)) {
        S->stats.untimed_ticks += 1;
        return;
    }
    const double t1 = t0 + 1e-3 * (double)std::max(ms, 0.0f);
    sl.last_end = t1;
    double horizon = 1e300;
    for (int k = 0; k < S->cfg.n_streams; ++k) {
        const Slot& o = S->slots[k];
        if (o.busy && &o != &sl && !o.kernels_seen) horizon = std::min(horizon, o.last_end);
    }
    S->clock.spans.add(t0, t1, horizon);
    S->stats.kernel_seconds = S->clock.spans.sum();
}

// Complete finished ticks.  Caller holds the lock.
void reap(dare_server* S) {
    for (int k = 0; k < S->cfg.n_streams; ++k) {
        Slot& sl = S->slots[k];
        if (!sl.busy) continue;
        const double t = now_s();
        if (!sl.kernels_seen && hipEventQuery(sl.ev_kernels) == hipSuccess) {
            sl.kernels_seen = true;
            for (uint64_t id : sl.tickets) S->reqs[id].t.t_device_done = t;
            time_tick(S, sl);
        }
        const hipError_t q = hipEventQuery(sl.ev_done);
        if (q == hipErrorNotReady) continue;
        const bool ok = q == hipSuccess;
        if (ok && !sl.kernels_seen) {
            sl.kernels_seen = true;
            time_tick(S, sl);
        }
        for (uint64_t id : sl.tickets) {
            Request& r = S->reqs[id];
            if (r.t.t_device_done == 0.0) r.t.t_device_done = t;
            r.t.t_host_done = t;
            r.state = ok ? kDone : kFailed;
            release_request(S, r);
            S->stats.completed += 1;
            S->stats.pixels += (int64_t)r.spec.width * r.spec.height;
        }
        if (!ok) S->failed = true;
        sl.tickets.clear();
        sl.busy = false;
        S->done_cv.notify_all();
    }
}

int busy_slots(dare_server* S) {
    int n = 0;
    for (int k = 0; k < S->cfg.n_streams; ++k) n += S->slots[k].busy;
    return n;
}

// Form and launch one tick on a free slot.  Caller holds the lock.  Returns false when
// nothing could be admitted.
bool launch_tick(dare_server* S, Slot& sl) {
    if (S->queue.empty()) return false;
    const double t_admit = now_s();
    int64_t pixels = 0, units = 0;
    int nreq = 0;
    const bool host_units = S->radius > 1;
    std::vector<BatchReq> breqs;
    std::vector<int2> bunits;
    while (!S->queue.empty() && nreq < S->cfg.max_tick_requests) {
        Request& r = S->reqs[S->queue.front()];
        if (r.frames_job) break;               // later requests must see the frames: wait for them
        const int64_t px = (int64_t)r.spec.width * r.spec.height;
        if (nreq > 0 && (pixels + px > S->cfg.max_tick_pixels || units + r.units > S->max_units)) break;
        const uint64_t off = S->outs.alloc(r.bytes);
        if (off == UINT64_MAX) break;          // the head waits for result slots to free up
        r.out_off = off;
        r.state = kInFlight;
        r.t.t_admit = t_admit;
        BatchReq q{};
        q.vol = volume_device(S->vols[r.vol].v);
        q.s.sx = r.spec.pitch_mm[0];
        q.s.sy = r.spec.pitch_mm[1];
        memcpy(q.s.P, r.spec.probe_pose, sizeof(q.s.P));
        q.s.W = r.spec.width;
        q.s.H = r.spec.height;
        q.s.tiles_x = (r.spec.width + kTile - 1) / kTile;
        q.s.tiles = q.s.tiles_x * ((r.spec.height + kTile - 1) / kTile);
        q.s.out = (float*)(S->arena + off);
        breqs.push_back(q);
        if (host_units)
            for (int64_t t = 0; t < r.units; ++t) bunits.push_back(make_int2(nreq, (int)t));
        sl.tickets.push_back(S->queue.front());
        S->queue.pop_front();
        pixels += px;
        units += r.units;
        ++nreq;
    }
    if (nreq == 0) return false;
    BatchHeader hd{};
    hd.counts[0] = host_units ? (int)units : 0;   // radius 1: the setup pass appends the units
    hd.counts[1] = nreq;
    memcpy(sl.staging, &hd, sizeof(hd));
    memcpy(sl.staging + S->o_req, breqs.data(), breqs.size() * sizeof(BatchReq));
    if (host_units) memcpy(sl.staging + S->o_units, bunits.data(), bunits.size() * sizeof(int2));
    const uint64_t upload = host_units ? S->o_units + bunits.size() * sizeof(int2)
                                       : S->o_req + breqs.size() * sizeof(BatchReq);
    hipError_t e = hipMemcpyAsync(sl.ws, sl.staging, upload, hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.ev_start, sl.stream);
    if (e == hipSuccess) e = S->cfg.use_graphs ? hipGraphLaunch(sl.graph, sl.stream) : enqueue_kernels(S, sl);
    if (e == hipSuccess) e = hipEventRecord(sl.ev_kernels, sl.stream);
    for (size_t k = 0; e == hipSuccess && k < sl.tickets.size(); ++k) {
        Request& r = S->reqs[sl.tickets[k]];
        // the result's destination may be host memory or device memory (unified addressing)
        e = hipMemcpyAsync(r.host_out, S->arena + r.out_off, r.bytes, hipMemcpyDefault, sl.stream);
    }
    if (e == hipSuccess) e = hipEventRecord(sl.ev_done, sl.stream);
    const double t_launch = now_s();
    for (uint64_t id : sl.tickets) S->reqs[id].t.t_launch = t_launch;
    sl.busy = true;
    sl.kernels_seen = false;
    S->stats.ticks += 1;
    if (e != hipSuccess) {
        // nothing reliable is in flight on this stream: fail the tick's requests now
        (void)hipStreamSynchronize(sl.stream);
        for (uint64_t id : sl.tickets) {
            Request& r = S->reqs[id];
            r.state = kFailed;
            release_request(S, r);
        }
        sl.tickets.clear();
        sl.busy = false;
        S->failed = true;
        S->done_cv.notify_all();
    }
    return true;
}

// Compound the frames job at the head of the queue once no tick is in flight (ticks read the
// volumes; compounding rewrites them).  Caller holds the lock; it is released while the
// frames are compounded.  Returns true when a job ran.
bool run_frames_job(dare_server* S, std::unique_lock<std::mutex>& lk) {
    if (S->queue.empty() || busy_slots(S) > 0) return false;
    const uint64_t id = S->queue.front();
    Request& r = S->reqs[id];
    if (!r.frames_job) return false;
    r.state = kInFlight;
    r.t.t_admit = r.t.t_launch = now_s();
    dare_volume* v = S->vols[r.vol].v;
    const uint8_t* frames = r.frames;
    const float* poses = r.poses;
    const int32_t n = r.nframes, w = r.fw, h = r.fh;
    const double pitch[2] = {r.fpitch[0], r.fpitch[1]};
    hipStream_t stream = S->slots[0].stream;
    lk.unlock();
    const double t0 = now_s();
    dare_status st = dare_reconstruct_frames(v, frames, n, w, h, pitch, poses, stream);
    if (hipStreamSynchronize(stream) != hipSuccess && (st == DARE_OK || st == DARE_WARN_BINS_SATURATED))
        st = DARE_ERR_HIP;
    const double t1 = now_s();
    lk.lock();
    Request& rr = S->reqs[id];        // the map may have grown meanwhile
    rr.status = st;
    rr.state = (st == DARE_OK || st == DARE_WARN_BINS_SATURATED) ? kDone : kFailed;
    rr.t.t_device_done = rr.t.t_host_done = t1;
    S->stats.compound_seconds += t1 - t0;
    if (rr.state == kDone) S->stats.frames += n;
    S->stats.completed += 1;
    S->vols[rr.vol].pending -= 1;
    S->queue.pop_front();
    S->done_cv.notify_all();
    return true;
}

void scheduler(dare_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop.load()) {
        reap(S);
        while (run_frames_job(S, lk)) reap(S);
        S->clock.advance(now_s());
        for (int k = 0; k < S->cfg.n_streams; ++k) {
            Slot& sl = S->slots[k];
            if (sl.busy) continue;
            if (!launch_tick(S, sl)) break;
        }
        const int busy = busy_slots(S);
        const double t = now_s();
        if (busy > 0 && S->busy_since < 0.0) S->busy_since = t;
        if (busy == 0 && S->busy_since >= 0.0) {
            S->stats.busy_seconds += t - S->busy_since;
            S->busy_since = -1.0;
        }
        if (busy == 0 && S->queue.empty()) {
            S->cv.wait_for(lk, std::chrono::milliseconds(50));
        } else {
            // ticks in flight: poll their events again shortly
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

// A registered volume that still takes requests.  Caller holds the lock.
bool volume_open(const dare_server* S, int32_t id) {
    return id >= 0 && id < (int32_t)S->vols.size() && S->vols[id].v && !S->vols[id].closing;
}

// The slots' workspaces, laid out once the radius is known (the first volume): header,
// request table, unit table (sized for a full tick at this radius) and setup records.
dare_status layout_workspaces(dare_server* S, int radius) {
    const dare_server_config& c = S->cfg;
    // pixels per unit: 16 x 16 tiles up to radius 4, 256 / (lanes per pixel) beyond; a request
    // adds at most one partial tile per row and column of tiles
    const int64_t ppu = radius <= 4 ? 256 : 256 / reslice_lanes(radius);
    int64_t mu = c.max_tick_pixels / ppu + (radius <= 4 ? 300 : 1) * (int64_t)c.max_tick_requests;
    S->max_units = std::min<int64_t>(mu, (int64_t)1 << 28);
    S->o_req = aup(sizeof(BatchHeader));
    S->o_units = S->o_req + aup((uint64_t)c.max_tick_requests * sizeof(BatchReq));
    S->o_tiles = S->o_units + aup((uint64_t)S->max_units * sizeof(int2));
    S->o_rec = S->o_tiles + (radius <= 1 ? aup((uint64_t)S->max_units * sizeof(TileRec)) : 0);
    S->ws_bytes = S->o_rec + aup((uint64_t)c.max_tick_requests * sizeof(SliceRec));
    for (int k = 0; k < c.n_streams; ++k) {
        Slot& sl = S->slots[k];
        const uint64_t off = S->outs.alloc(S->ws_bytes);
        if (off == UINT64_MAX) return DARE_ERR_BUDGET;
        sl.ws_off = off;
        sl.ws = S->arena + off;
        if (hipHostMalloc((void**)&sl.staging, S->o_tiles, hipHostMallocDefault) != hipSuccess) return DARE_ERR_HIP;
    }
    return DARE_OK;
}

void release_workspaces(dare_server* S) {
    for (int k = 0; k < S->cfg.n_streams; ++k) {
        Slot& sl = S->slots[k];
        if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
        sl.graph = nullptr;
        if (sl.staging) (void)hipHostFree(sl.staging);
        sl.staging = nullptr;
        if (sl.ws_off != UINT64_MAX) S->outs.release(sl.ws_off, S->ws_bytes);
        sl.ws_off = UINT64_MAX;
        sl.ws = nullptr;
    }
}

// Validate and queue one request.  Caller holds the lock.
dare_status submit_locked(dare_server* S, int32_t volume_id, const dare_slice_spec* spec, float* host_out,
                          uint64_t* ticket) {
    const dare_status st = check_slice_spec(spec);
    if (st != DARE_OK) return st;
    if (!volume_open(S, volume_id)) return DARE_ERR_INVALID_ARG;
    Request r;
    r.vol = volume_id;
    r.spec = *spec;
    r.host_out = host_out;
    r.bytes = (uint64_t)spec->width * spec->height * sizeof(float);
    r.units = units_of(S->radius, spec->width, spec->height);
    if (!S->outs.fits_ever(r.bytes) || r.units > S->max_units ||
        (int64_t)spec->width * spec->height > S->cfg.max_tick_pixels)
        return DARE_ERR_INVALID_ARG;
    if ((int32_t)S->queue.size() >= S->cfg.max_queue) {
        S->stats.rejected += 1;
        return DARE_ERR_QUEUE_FULL;
    }
    r.t.t_submit = now_s();
    const uint64_t id = S->next_ticket++;
    S->reqs.emplace(id, r);
    S->queue.push_back(id);
    S->stats.submitted += 1;
    S->vols[volume_id].pending += 1;
    *ticket = id;
    return DARE_OK;
}

// State of one ticket; a finished ticket is retired.  Caller holds the lock.
dare_status poll_locked(dare_server* S, uint64_t ticket, dare_request_times* times) {
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return DARE_ERR_INVALID_ARG;
    const int state = it->second.state;
    if (state == kWaiting || state == kInFlight) return DARE_ERR_NOT_READY;
    if (times) *times = it->second.t;
    const bool frames = it->second.frames_job;
    const dare_status fst = it->second.status;
    S->reqs.erase(it);
    if (frames) return fst;
    return state == kDone ? DARE_OK : DARE_ERR_HIP;
}

}  // namespace

extern "C" {

double dare_now_seconds(void) { return now_s(); }

void dare_default_server_config(dare_server_config* c) {
    if (!c) return;
    c->max_tick_pixels = 8 << 20;
    c->max_tick_requests = 64;
    c->n_streams = 3;
    c->max_queue = 4096;
    c->use_graphs = 1;
    c->volume_budget_bytes = 0;
}

dare_status dare_server_create(const dare_server_config* cfg, void* arena_dev, uint64_t arena_bytes,
                               dare_server** out) {
    if (!cfg || !arena_dev || !out) return DARE_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->n_streams < 1 || cfg->n_streams > kMaxStreams || cfg->max_tick_requests < 1 ||
        cfg->max_tick_requests > 4096 || cfg->max_tick_pixels < 1 || cfg->max_tick_pixels > ((int64_t)1 << 32) ||
        cfg->max_queue < 1)
        return DARE_ERR_INVALID_ARG;
    if (((uintptr_t)arena_dev % kAlignS) != 0 || arena_bytes < 2 * kAlignS) return DARE_ERR_INVALID_ARG;
    dare_server* S = new dare_server();
    S->cfg = *cfg;
    S->arena = (char*)arena_dev;
    S->arena_bytes = arena_bytes;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return DARE_ERR_HIP;
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < cfg->n_streams && e == hipSuccess; ++k) {
        Slot& sl = S->slots[k];
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&sl.ev_start);
        if (e == hipSuccess) e = hipEventCreate(&sl.ev_kernels);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev_done, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = S->clock.init(now_s());
    if (e != hipSuccess) {
        dare_server_destroy(S);
        return DARE_ERR_HIP;
    }
    S->outs.reset(0, arena_bytes, kAlignS);
    S->th = std::thread(scheduler, S);
    *out = S;
    return DARE_OK;
}

dare_status dare_server_add_volume(dare_server* S, dare_volume* v, int32_t* volume_id) {
    if (!S || !v || !volume_id) return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    if (volume_device_id(v) != S->device) return DARE_ERR_INVALID_ARG;
    for (const VolEntry& e : S->vols)
        if (e.v == v) return DARE_ERR_INVALID_ARG;   // registered already
    const int dt = volume_dtype(v), R = volume_radius(v);
    const uint64_t bytes = volume_arena_size(v);
    if (S->dtype >= 0 && (dt != S->dtype || R != S->radius))
        return DARE_ERR_INVALID_ARG;   // one storage dtype and radius per server (one graph per stream)
    if (S->cfg.volume_budget_bytes > 0 && S->vol_bytes + bytes > S->cfg.volume_budget_bytes)
        return DARE_ERR_BUDGET;        // admitting it would exceed the resident-volume budget
    if (S->dtype < 0) {
        dare_status st = layout_workspaces(S, R);
        S->dtype = dt;
        S->radius = R;
        for (int k = 0; k < S->cfg.n_streams && st == DARE_OK; ++k)
            if (ensure_graph(S, S->slots[k]) != hipSuccess) st = DARE_ERR_HIP;
        if (st != DARE_OK) {
            release_workspaces(S);
            S->dtype = -1;
            S->radius = -1;
            return st;
        }
    }
    VolEntry e;
    e.v = v;
    e.bytes = bytes;
    S->vols.push_back(e);
    S->vol_bytes += bytes;
    *volume_id = (int32_t)S->vols.size() - 1;
    return DARE_OK;
}

dare_status dare_server_remove_volume(dare_server* S, int32_t volume_id, double wait_seconds) {
    if (!S) return DARE_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    if (!volume_open(S, volume_id)) return DARE_ERR_INVALID_ARG;
    VolEntry& e = S->vols[volume_id];
    e.closing = true;                  // no new requests; the queued ones still run
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(wait_seconds > 0.0 ? std::min(wait_seconds, 3600.0) : 0.0));
    while (S->vols[volume_id].pending > 0) {
        if (!(wait_seconds > 0.0) || S->done_cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            if (S->vols[volume_id].pending == 0) break;
            S->vols[volume_id].closing = false;   // still in use: it stays registered
            return DARE_ERR_NOT_READY;
        }
    }
    VolEntry& f = S->vols[volume_id];
    S->vol_bytes -= f.bytes;
    f.v = nullptr;
    f.bytes = 0;
    f.closing = false;
    return DARE_OK;
}

dare_status dare_server_volume_bytes(dare_server* S, uint64_t* resident_bytes, int32_t* resident_volumes) {
    if (!S || !resident_bytes || !resident_volumes) return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    *resident_bytes = S->vol_bytes;
    int32_t n = 0;
    for (const VolEntry& e : S->vols) n += e.v != nullptr;
    *resident_volumes = n;
    return DARE_OK;
}

dare_status dare_server_submit(dare_server* S, int32_t volume_id, const dare_slice_spec* spec, float* host_out,
                               uint64_t* ticket) {
    if (!S || !host_out || !ticket) return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    const dare_status st = submit_locked(S, volume_id, spec, host_out, ticket);
    if (st == DARE_OK) S->cv.notify_one();
    return st;
}

dare_status dare_server_submit_frames(dare_server* S, int32_t volume_id, const uint8_t* frames_dev, int32_t n,
                                      int32_t w, int32_t h, const double pitch_mm[2], const float* probe_poses_dev,
                                      uint64_t* ticket) {
    if (!S || !ticket || !pitch_mm || n <= 0 || w <= 0 || h <= 0 || !frames_dev || !probe_poses_dev)
        return DARE_ERR_INVALID_ARG;
    if ((int64_t)w * h > (int64_t)1 << 30 || !(pitch_mm[0] > 0.0) || !(pitch_mm[1] > 0.0))
        return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    if (!volume_open(S, volume_id)) return DARE_ERR_INVALID_ARG;
    if ((int32_t)S->queue.size() >= S->cfg.max_queue) {
        S->stats.rejected += 1;
        return DARE_ERR_QUEUE_FULL;
    }
    Request r;
    r.frames_job = true;
    r.vol = volume_id;
    r.frames = frames_dev;
    r.poses = probe_poses_dev;
    r.nframes = n;
    r.fw = w;
    r.fh = h;
    r.fpitch[0] = pitch_mm[0];
    r.fpitch[1] = pitch_mm[1];
    r.t.t_submit = now_s();
    const uint64_t id = S->next_ticket++;
    S->reqs.emplace(id, r);
    S->queue.push_back(id);
    S->stats.submitted += 1;
    S->vols[volume_id].pending += 1;
    *ticket = id;
    S->cv.notify_one();
    return DARE_OK;
}

dare_status dare_server_submit_many(dare_server* S, int32_t n, const int32_t* volume_ids, const dare_slice_spec* specs,
                                    float* const* host_outs, uint64_t* tickets, int32_t* accepted) {
    if (!S || n < 0 || !accepted || (n > 0 && (!volume_ids || !specs || !host_outs || !tickets)))
        return DARE_ERR_INVALID_ARG;
    *accepted = 0;
    std::lock_guard<std::mutex> lk(S->mu);
    dare_status st = DARE_OK;
    int k = 0;
    for (; k < n; ++k) {
        st = host_outs[k] ? submit_locked(S, volume_ids[k], specs + k, host_outs[k], tickets + k)
                          : DARE_ERR_INVALID_ARG;
        if (st != DARE_OK) break;
    }
    *accepted = k;
    if (k > 0) S->cv.notify_one();
    return st;
}

dare_status dare_server_poll(dare_server* S, uint64_t ticket, dare_request_times* times) {
    if (!S) return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    return poll_locked(S, ticket, times);
}

dare_status dare_server_poll_many(dare_server* S, int32_t n, const uint64_t* tickets, dare_request_times* times,
                                  int32_t* states, double wait_seconds, int32_t* n_done) {
    if (!S || n < 0 || !n_done || (n > 0 && (!tickets || !states))) return DARE_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(wait_seconds > 0.0 ? std::min(wait_seconds, 3600.0) : 0.0));
    for (;;) {
        int done = 0;
        for (int k = 0; k < n; ++k) {
            states[k] = (int32_t)poll_locked(S, tickets[k], times ? times + k : nullptr);
            done += states[k] != DARE_ERR_NOT_READY;
        }
        *n_done = done;
        if (done > 0 || n == 0 || !(wait_seconds > 0.0)) return DARE_OK;
        if (S->done_cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            *n_done = 0;
            return DARE_OK;
        }
    }
}

dare_status dare_server_drain(dare_server* S) {
    if (!S) return DARE_ERR_INVALID_ARG;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->queue.empty() && busy_slots(S) == 0) return S->failed ? DARE_ERR_HIP : DARE_OK;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

dare_status dare_server_get_stats(dare_server* S, dare_server_stats* out) {
    if (!S || !out) return DARE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    if (S->busy_since >= 0.0) out->busy_seconds += now_s() - S->busy_since;
    out->device_busy_seconds = S->clock.spans.busy();
    return DARE_OK;
}

dare_status dare_server_destroy(dare_server* S) {
    if (!S) return DARE_ERR_INVALID_ARG;
    if (S->th.joinable()) {
        (void)dare_server_drain(S);
        S->stop.store(true);
        S->cv.notify_all();
        S->th.join();
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < kMaxStreams; ++k) {
        Slot& sl = S->slots[k];
        if (sl.stream) {
            const hipError_t q = hipStreamSynchronize(sl.stream);
            if (q != hipSuccess) e = q;
        }
        if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
        if (sl.ev_kernels) (void)hipEventDestroy(sl.ev_kernels);
        if (sl.ev_done) (void)hipEventDestroy(sl.ev_done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    S->clock.destroy();
    release_workspaces(S);
    delete S;
    return e == hipSuccess ? DARE_OK : DARE_ERR_HIP;
}

}  // extern "C"
