// Continuous-batching server over the simulator's C ABI (srv_* in include/sim.h).
//
// Many virtual cameras, each with its own device-resident simulator state (reference levels,
// previous frame, event buffers) and a device staging ring for frames that arrived and wait for
// the GPU.  Cameras are admitted while their estimated HBM footprint fits the budget and a slot is
// free; releasing a camera returns both.  A step takes every queued frame of every camera and
// runs them as one batched push (sim_push_batch), so different cameras' work overlaps on the
// device.  srv_submit only records where the frame (and flow) is and returns: inputs in device
// memory or in pinned host memory are pulled into the cameras' rings by one copy kernel at the
// start of the step that takes them (the device reads pinned host memory directly over the bus,
// so thousands of small frames cost one launch rather than one DMA request each); pageable host
// inputs are copied at submission.  Cameras without a stream of their own share the server's
// stream, so a step waits on one stream rather than on one per camera.  With the server's worker
// running (srv_start), steps follow one another while frames keep arriving, each step admitting
// every frame queued when it starts.  Per frame, the latency from its arrival stamp to the end of
// the step that ordered its events is recorded.
//
// Locking: `mu` guards the rings, the camera table and the statistics; `push_mu` is held for a
// whole step (and by every call that touches a camera's simulator stream), so a step never sees
// a camera released or drained under it, while srv_submit needs only `mu`.
#include <math.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <mutex>
#include <new>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/sim.h"
#include "evsim_internal.h"

namespace {

// One input to pull into a ring slot at the start of a step.
struct CopyDesc {
    const unsigned char* src;   // device memory, or pinned host memory by its device address
    unsigned char* dst;         // ring slot
    uint64_t bytes;
};

constexpr uint64_t kCopyChunk = 64u << 10;   // bytes per workgroup of the copy kernel
constexpr int kCopyThreads = 256;

struct alignas(16) Vec16 {
    uint64_t lo, hi;
};

// Copies every descriptor's bytes; workgroup b takes chunk b of the concatenation (cstart: the
// descriptors' first chunks, n + 1 entries, the last the total).  Each lane keeps four 16-byte
// loads in flight, which the bus reads of pinned host memory need.
template <typename T>
__device__ void copy_span(const unsigned char* __restrict__ s, unsigned char* __restrict__ t,
                          uint64_t len) {
    const uint64_t nv = len / sizeof(T);
    const T* s4 = reinterpret_cast<const T*>(s);
    T* t4 = reinterpret_cast<T*>(t);
    for (uint64_t base = threadIdx.x; base < nv; base += 4 * kCopyThreads) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (base + u * kCopyThreads < nv) v[u] = s4[base + u * kCopyThreads];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (base + u * kCopyThreads < nv) t4[base + u * kCopyThreads] = v[u];
    }
    for (uint64_t i = nv * sizeof(T) + threadIdx.x; i < len; i += kCopyThreads) t[i] = s[i];
}

__global__ __launch_bounds__(kCopyThreads) void k_gather_copy(const CopyDesc* __restrict__ d,
                                                              const uint64_t* __restrict__ cstart,
                                                              int n) {
    const uint64_t chunk = blockIdx.x;
    int lo = 0, hi = n - 1;   // the last descriptor whose first chunk is at or before this one
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= chunk) lo = mid;
        else hi = mid - 1;
    }
    const CopyDesc cd = d[lo];
    const uint64_t off = (chunk - cstart[lo]) * kCopyChunk;
    const uint64_t len = cd.bytes - off < kCopyChunk ? cd.bytes - off : kCopyChunk;
    const unsigned char* s = cd.src + off;
    unsigned char* t = cd.dst + off;
    const uintptr_t a = (uintptr_t)s | (uintptr_t)t;
    if ((a & 15) == 0) copy_span<Vec16>(s, t, len);
    else if ((a & 7) == 0) copy_span<uint64_t>(s, t, len);
    else if ((a & 3) == 0) copy_span<uint32_t>(s, t, len);
    else copy_span<unsigned char>(s, t, len);
}

struct Camera {
    bool used = false;
    sim_stream* s = nullptr;
    sim_config cfg;
    hipStream_t stream = nullptr;   // the server's shared stream unless the config names one
    uint64_t footprint = 0;
    int64_t npix = 0;
    bool interp = false;          // needs supplied flows
    bool started = false;         // has received its first frame (in a push)
    int head = 0;                 // oldest queued slot of the staging ring
    int q = 0;                    // frames queued in the ring (from head, wrapping)
    uint8_t* d_frames = nullptr;  // ring [qcap][H][W]
    float* d_flows = nullptr;     // ring [qcap][H][W][2], slot j = flow of the interval ending at
                                  // the frame of slot j
    std::vector<int64_t> t_us;
    std::vector<int64_t> arrival_ns;
    std::vector<const unsigned char*> src_frame;   // per slot: input to pull at the step, or
    std::vector<const unsigned char*> src_flow;    // NULL when copied at submission
    int64_t last_t = 0;
    bool any_t = false;
};

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// The device address of pinned host memory, or NULL for pageable memory.
const unsigned char* device_address_of_pinned(const void* p) {
    hipPointerAttribute_t a;
    memset(&a, 0, sizeof(a));
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return a.type == hipMemoryTypeHost ? (const unsigned char*)a.devicePointer : nullptr;
}

void release_camera(Camera& c) {
    if (c.s) sim_destroy(c.s);
    if (c.d_frames) (void)hipFree(c.d_frames);
    if (c.d_flows) (void)hipFree(c.d_flows);
    c = Camera();
}

}  // namespace

// Per-frame latencies kept for the percentiles: the latest kLatencyWindow completed frames.
constexpr size_t kLatencyWindow = size_t(1) << 20;

struct sim_server {
    uint64_t budget = 0;
    uint64_t used = 0;
    int qcap = 0;
    std::vector<Camera> cams;
    std::mutex mu;                 // rings, cameras, statistics
    std::mutex push_mu;            // a step; calls on a camera's simulator stream
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool running = false, stopping = false;
    uint64_t queued = 0;           // frames in the rings, not yet completed
    int last_rc = SIM_OK;          // first error of a worker step since srv_sync
    // Everything below is reserved at creation, so that serving allocates no host memory.
    std::vector<float> lat_ms;     // ring of per-frame latencies
    size_t lat_next = 0;           // slot the next latency overwrites once the ring is full
    std::vector<float> lat_sort;   // scratch for the percentiles
    std::vector<sim_stream*> step_handles;
    std::vector<sim_frames> step_items;
    std::vector<int> step_cams;
    std::vector<int> step_n;       // frames each camera contributes to the step
    std::vector<std::pair<hipStream_t, CopyDesc>> step_copies;   // the step's ring fills
    std::vector<hipStream_t> fill_streams;   // streams of the last ring fills (reading h_desc)
    hipStream_t stream = nullptr;  // shared by the cameras without a stream of their own
    CopyDesc* h_desc = nullptr;    // pinned: the step's descriptors, then their chunk starts
    char* d_desc = nullptr;
    size_t desc_cap = 0;           // descriptors the buffers hold
    sim_server_stats st;
};

namespace {

void record_latency(sim_server* srv, float ms) {
    if (srv->lat_ms.size() < kLatencyWindow) {
        srv->lat_ms.push_back(ms);   // within the reserved capacity
    } else {
        srv->lat_ms[srv->lat_next] = ms;
        srv->lat_next = (srv->lat_next + 1) % kLatencyWindow;
    }
}

// Queues the step's ring fills: per stream (in the usual case only the server's), one upload of
// the descriptors and one copy kernel, ordered before the batched push, which waits for the
// cameras' streams.  Holds push_mu (the descriptor buffers belong to the running step).
int fill_rings(sim_server* srv, std::vector<std::pair<hipStream_t, CopyDesc>>& copies) {
    if (copies.empty()) return SIM_OK;
    // the previous step's uploads and copy kernels read these buffers; a step whose cameras all
    // sent only their first frame runs no batched window, so nothing has waited for them yet
    for (hipStream_t st : srv->fill_streams)
        if (hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            return SIM_E_HIP;
        }
    srv->fill_streams.clear();
    const size_t n = copies.size();
    if (n > srv->desc_cap) {
        size_t cap = 1024;
        while (cap < n) cap *= 2;
        if (srv->h_desc) (void)hipHostFree(srv->h_desc);
        if (srv->d_desc) (void)hipFree(srv->d_desc);
        srv->h_desc = nullptr;
        srv->d_desc = nullptr;
        srv->desc_cap = 0;
        const size_t bytes = cap * sizeof(CopyDesc) + (2 * cap + 2) * sizeof(uint64_t);
        if (hipHostMalloc((void**)&srv->h_desc, bytes, 0) != hipSuccess ||
            hipMalloc((void**)&srv->d_desc, bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (srv->h_desc) (void)hipHostFree(srv->h_desc);
            srv->h_desc = nullptr;
            return SIM_E_NOMEM;
        }
        srv->desc_cap = cap;
    }
    std::stable_sort(copies.begin(), copies.end(),
                     [](const std::pair<hipStream_t, CopyDesc>& a,
                        const std::pair<hipStream_t, CopyDesc>& b) {
                         return (uintptr_t)a.first < (uintptr_t)b.first;
                     });
    const size_t starts_off = srv->desc_cap * sizeof(CopyDesc);
    uint64_t* h_starts = (uint64_t*)((char*)srv->h_desc + starts_off);
    size_t si = 0;   // next free chunk-start slot
    for (size_t a = 0; a < n;) {
        size_t b = a;
        while (b < n && copies[b].first == copies[a].first) ++b;
        uint64_t chunks = 0;
        for (size_t k = a; k < b; ++k) {
            srv->h_desc[k] = copies[k].second;
            h_starts[si + (k - a)] = chunks;
            chunks += (copies[k].second.bytes + kCopyChunk - 1) / kCopyChunk;
        }
        h_starts[si + (b - a)] = chunks;
        const hipStream_t st = copies[a].first;
        const CopyDesc* d = (const CopyDesc*)(srv->d_desc + a * sizeof(CopyDesc));
        const uint64_t* ds = (const uint64_t*)(srv->d_desc + starts_off + si * sizeof(uint64_t));
        if (hipMemcpyAsync((void*)d, srv->h_desc + a, (b - a) * sizeof(CopyDesc),
                           hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync((void*)ds, h_starts + si, (b - a + 1) * sizeof(uint64_t),
                           hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipGetLastError();
            return SIM_E_HIP;
        }
        if (chunks) {
            hipLaunchKernelGGL(k_gather_copy, dim3((unsigned)chunks), dim3(kCopyThreads), 0, st,
                               d, ds, (int)(b - a));
            if (hipGetLastError() != hipSuccess) return SIM_E_HIP;
        }
        srv->fill_streams.push_back(st);
        si += b - a + 1;
        a = b;
    }
    return SIM_OK;
}

// One step: every camera's queued frames (those contiguous in its ring from its head) as one
// batched push.  Holds push_mu throughout, mu while reading and updating the rings.  Returns
// SIM_OK or the first per-camera error; *n_frames receives the frames completed.
int run_step(sim_server* srv, uint64_t* n_frames) {
    const int64_t asked = now_ns();
    std::lock_guard<std::mutex> step(srv->push_mu);
    const int64_t began = now_ns();
    std::vector<sim_stream*>& handles = srv->step_handles;   // capacity: one per camera slot
    std::vector<sim_frames>& items = srv->step_items;
    std::vector<int>& which = srv->step_cams;
    std::vector<int>& taken = srv->step_n;
    std::vector<std::pair<hipStream_t, CopyDesc>>& copies = srv->step_copies;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        handles.clear();
        items.clear();
        which.clear();
        taken.clear();
        copies.clear();
        for (int i = 0; i < (int)srv->cams.size(); ++i) {
            Camera& c = srv->cams[i];
            if (!c.used || c.q == 0) continue;
            const int n = std::min(c.q, srv->qcap - c.head);   // contiguous part of the ring
            sim_frames it;
            memset(&it, 0, sizeof(it));
            it.n_frames = n;
            it.mem_kind = SIM_MEM_DEVICE;
            it.frames = c.d_frames + (size_t)c.head * c.npix;
            // a camera's very first frame only initialises its state: its flow slot is unused
            const int fl0 = c.started ? c.head : c.head + 1;
            it.flows = c.interp ? c.d_flows + (size_t)fl0 * c.npix * 2 : nullptr;
            it.t_us = c.t_us.data() + c.head;
            for (int f = c.head; f < c.head + n; ++f) {
                if (c.src_frame[f])
                    copies.push_back({c.stream, {c.src_frame[f], c.d_frames + (size_t)f * c.npix,
                                                 (uint64_t)c.npix}});
                if (c.src_flow[f])
                    copies.push_back(
                        {c.stream, {c.src_flow[f], (unsigned char*)(c.d_flows + (size_t)f * c.npix * 2),
                                    (uint64_t)c.npix * 2 * sizeof(float)}});
                c.src_frame[f] = c.src_flow[f] = nullptr;
            }
            handles.push_back(c.s);
            items.push_back(it);
            which.push_back(i);
            taken.push_back(n);
        }
    }
    if (n_frames) *n_frames = 0;
    if (items.empty()) return SIM_OK;
    int rc = fill_rings(srv, copies);
    if (rc != SIM_OK) {
        for (sim_frames& it : items) it.status = rc;
    } else {
        rc = sim_push_batch(handles.data(), items.data(), (int32_t)items.size());
    }
    if (rc != SIM_OK) {
        // the fills may still be running: the descriptor buffers are reused by the next step
        for (const auto& cp : copies) (void)hipStreamSynchronize(cp.first);
        (void)hipGetLastError();
    }
    const int64_t done = now_ns();
    uint64_t frames = 0;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        for (size_t j = 0; j < items.size(); ++j) {
            Camera& c = srv->cams[which[j]];
            const int n = taken[j];
            if (items[j].status == SIM_OK) {
                for (int f = 0; f < n; ++f)
                    record_latency(srv,
                                   (float)((double)(done - c.arrival_ns[c.head + f]) * 1e-6));
                frames += (uint64_t)n;
                srv->st.events += items[j].n_new_events;
                c.started = true;
            } else {
                srv->st.failed_frames += (uint64_t)n;
            }
            c.head = (c.head + n) % srv->qcap;
            c.q -= n;
            srv->queued -= (uint64_t)n;
        }
        srv->st.completed += frames;
        srv->st.steps++;
        srv->st.busy_ms += (double)(now_ns() - began) * 1e-6;
        srv->st.lock_wait_ms += (double)(began - asked) * 1e-6;
    }
    srv->cv_done.notify_all();
    if (n_frames) *n_frames = frames;
    return rc;
}

// The worker of a running server: steps while frames are queued, sleeps otherwise.
void worker_loop(sim_server* srv) {
    for (;;) {
        {
            std::unique_lock<std::mutex> lock(srv->mu);
            srv->cv_work.wait(lock, [&] { return srv->stopping || srv->queued > 0; });
            if (srv->stopping) return;
        }
        const int rc = run_step(srv, nullptr);
        if (rc) {
            std::lock_guard<std::mutex> lock(srv->mu);
            if (srv->last_rc == SIM_OK) srv->last_rc = rc;
        }
    }
}

void stop_worker(sim_server* srv) {
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        if (!srv->running) return;
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    srv->worker.join();
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->running = false;
    srv->stopping = false;
}

}  // namespace

extern "C" {

int srv_footprint(const sim_config* cfg, int32_t queue_depth, uint64_t* bytes) {
    if (!cfg || !bytes || queue_depth < 1) return SIM_E_INVAL;
    if (cfg->width < 1 || cfg->height < 1 || cfg->width > 4096 || cfg->height > 4096)
        return SIM_E_INVAL;
    const uint64_t npix = (uint64_t)cfg->width * (uint64_t)cfg->height;
    const bool sparse = cfg->method == SIM_SPARSE;
    const bool interp = cfg->method != SIM_BASIC && cfg->flow_source == SIM_FLOW_SUPPLIED;
    // reference levels 4, previous frames 2, chain resume points 4, event arena at its initial
    // capacity of 2 keys per pixel 16, sort buffers 32, FIFO 16; sparse: selection masks 16 and
    // active lists 8 (the selection's and the length-ordered one); difference method: the
    // frames before the previous ones 2; staging: one frame (+ flow) per queued slot
    uint64_t per_px = 4 + 2 + 4 + 16 + 32 + 16 + (sparse ? 24 : 0) +
                      (cfg->method == SIM_DIFFERENCE ? 2 : 0);
    per_px += (uint64_t)queue_depth * (1 + (interp ? 8 : 0));
    // estimated flow: a pyramid (at most 4/3 of a float frame) per frame of a step and one
    // flow field per interval
    if (cfg->flow_source == SIM_FLOW_LK) per_px += (uint64_t)(queue_depth + 1) * 6 + 8 * queue_depth;
    *bytes = npix * per_px + (1u << 20);
    return SIM_OK;
}

int srv_create(uint64_t hbm_budget_bytes, int32_t max_cameras, int32_t queue_depth,
               sim_server** out) {
    if (!out || max_cameras < 1 || max_cameras > 65536 || queue_depth < 1 || queue_depth > 128)
        return SIM_E_INVAL;
    *out = nullptr;
    sim_server* srv = new (std::nothrow) sim_server();
    if (!srv) return SIM_E_NOMEM;
    srv->budget = hbm_budget_bytes;
    srv->qcap = queue_depth;
    try {
        srv->cams.resize(max_cameras);
        srv->lat_ms.reserve(kLatencyWindow);
        srv->lat_sort.reserve(kLatencyWindow);
        srv->step_handles.reserve(max_cameras);
        srv->step_items.reserve(max_cameras);
        srv->step_cams.reserve(max_cameras);
        srv->step_n.reserve(max_cameras);
        srv->fill_streams.reserve(max_cameras);
        srv->step_copies.reserve(std::min<size_t>((size_t)max_cameras * queue_depth * 2,
                                                  size_t(1) << 16));
    } catch (...) {
        delete srv;
        return SIM_E_NOMEM;
    }
    memset(&srv->st, 0, sizeof(srv->st));
    srv->st.hbm_budget = hbm_budget_bytes;
    *out = srv;
    return SIM_OK;
}

int srv_destroy(sim_server* srv) {
    if (!srv) return SIM_E_INVAL;
    stop_worker(srv);
    for (Camera& c : srv->cams)
        if (c.used) release_camera(c);
    if (srv->stream) (void)hipStreamDestroy(srv->stream);
    if (srv->h_desc) (void)hipHostFree(srv->h_desc);
    if (srv->d_desc) (void)hipFree(srv->d_desc);
    delete srv;
    return SIM_OK;
}

int srv_admit(sim_server* srv, const sim_config* cfg, int32_t* cam) {
    if (!srv || !cfg || !cam) return SIM_E_INVAL;
    *cam = -1;
    std::lock_guard<std::mutex> step(srv->push_mu);
    std::lock_guard<std::mutex> lock(srv->mu);
    uint64_t fp = 0;
    int rc = srv_footprint(cfg, srv->qcap, &fp);
    if (rc) return rc;
    int slot = -1;
    for (int i = 0; i < (int)srv->cams.size(); ++i)
        if (!srv->cams[i].used) {
            slot = i;
            break;
        }
    if (slot < 0 || srv->used + fp > srv->budget) {
        srv->st.rejected_admissions++;
        return SIM_E_BUSY;
    }
    Camera c;
    c.cfg = *cfg;
    c.npix = (int64_t)cfg->width * cfg->height;
    c.interp = cfg->method != SIM_BASIC && cfg->flow_source == SIM_FLOW_SUPPLIED;
    c.footprint = fp;
    if (cfg->hip_stream) {
        c.stream = (hipStream_t)cfg->hip_stream;
    } else {
        if (!srv->stream &&
            hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
            srv->stream = nullptr;
            (void)hipGetLastError();
            return SIM_E_NOMEM;
        }
        c.stream = srv->stream;
        c.cfg.hip_stream = (void*)c.stream;
    }
    rc = sim_create(&c.cfg, &c.s);
    bool ok = rc == SIM_OK;
    ok = ok && hipMalloc((void**)&c.d_frames, (size_t)srv->qcap * c.npix) == hipSuccess;
    if (ok && c.interp)
        ok = hipMalloc((void**)&c.d_flows, (size_t)srv->qcap * c.npix * 2 * sizeof(float)) ==
             hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        c.used = true;
        release_camera(c);
        return rc ? rc : SIM_E_NOMEM;
    }
    try {
        c.t_us.resize(srv->qcap);
        c.arrival_ns.resize(srv->qcap);
        c.src_frame.assign(srv->qcap, nullptr);
        c.src_flow.assign(srv->qcap, nullptr);
    } catch (...) {
        c.used = true;
        release_camera(c);
        return SIM_E_NOMEM;
    }
    c.used = true;
    srv->cams[slot] = std::move(c);   // no copy of its vectors
    srv->used += fp;
    srv->st.cameras++;
    srv->st.admissions++;
    srv->st.hbm_used = srv->used;
    *cam = slot;
    return SIM_OK;
}

int srv_release(sim_server* srv, int32_t cam) {
    if (!srv) return SIM_E_INVAL;
    std::lock_guard<std::mutex> step(srv->push_mu);
    std::lock_guard<std::mutex> lock(srv->mu);
    if (cam < 0 || cam >= (int)srv->cams.size() || !srv->cams[cam].used) return SIM_E_INVAL;
    // frames still queued for the camera are dropped
    srv->st.failed_frames += (uint64_t)srv->cams[cam].q;
    srv->queued -= (uint64_t)srv->cams[cam].q;
    srv->used -= srv->cams[cam].footprint;
    release_camera(srv->cams[cam]);
    srv->st.cameras--;
    srv->st.hbm_used = srv->used;
    return SIM_OK;
}

int srv_submit(sim_server* srv, int32_t cam, const uint8_t* frame, const float* flow,
               int64_t t_us, int32_t mem_kind, int64_t arrival_ns) {
    if (!srv || !frame) return SIM_E_INVAL;
    if (mem_kind != SIM_MEM_HOST && mem_kind != SIM_MEM_DEVICE && mem_kind != SIM_MEM_HOST_FRAME)
        return SIM_E_INVAL;
    // inputs the step's copy kernel can read: device memory, and pinned host memory (by its
    // device address); pageable host memory is copied now
    const unsigned char* pull_frame = mem_kind == SIM_MEM_DEVICE
                                          ? (const unsigned char*)frame
                                          : device_address_of_pinned(frame);
    const unsigned char* pull_flow = nullptr;
    if (flow)
        pull_flow = mem_kind == SIM_MEM_HOST ? device_address_of_pinned(flow)
                                             : (const unsigned char*)flow;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        if (cam < 0 || cam >= (int)srv->cams.size() || !srv->cams[cam].used) return SIM_E_INVAL;
        Camera& c = srv->cams[cam];
        const bool first_ever = !c.started && c.q == 0;
        if (c.interp && !first_ever && !flow) return SIM_E_INVAL;
        if (c.any_t && t_us <= c.last_t) return SIM_E_ORDER;
        if (c.q >= srv->qcap) {
            srv->st.rejected_frames++;
            return SIM_E_BUSY;
        }
        const int slot = (c.head + c.q) % srv->qcap;
        // pageable inputs: queued on the camera's stream, which the step waits for
        if (!pull_frame && hipMemcpyAsync(c.d_frames + (size_t)slot * c.npix, frame,
                                          (size_t)c.npix, hipMemcpyHostToDevice,
                                          c.stream) != hipSuccess) {
            (void)hipGetLastError();
            return SIM_E_HIP;
        }
        if (c.interp && flow && !pull_flow &&
            hipMemcpyAsync(c.d_flows + (size_t)slot * c.npix * 2, flow,
                           (size_t)c.npix * 2 * sizeof(float), hipMemcpyHostToDevice,
                           c.stream) != hipSuccess) {
            (void)hipGetLastError();
            return SIM_E_HIP;
        }
        c.src_frame[slot] = pull_frame;
        c.src_flow[slot] = c.interp ? pull_flow : nullptr;
        c.t_us[slot] = t_us;
        c.arrival_ns[slot] = arrival_ns ? arrival_ns : now_ns();
        c.q++;
        c.last_t = t_us;
        c.any_t = true;
        srv->queued++;
        srv->st.submitted++;
    }
    srv->cv_work.notify_one();
    return SIM_OK;
}

int srv_step(sim_server* srv, uint64_t* n_frames) {
    if (!srv) return SIM_E_INVAL;
    if (n_frames) *n_frames = 0;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        if (srv->running) return SIM_E_BUSY;   // the worker steps
    }
    return run_step(srv, n_frames);
}

int srv_start(sim_server* srv) {
    if (!srv) return SIM_E_INVAL;
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->running) return SIM_OK;
    try {
        srv->worker = std::thread(worker_loop, srv);
    } catch (...) {
        return SIM_E_NOMEM;
    }
    srv->running = true;
    return SIM_OK;
}

int srv_stop(sim_server* srv) {
    if (!srv) return SIM_E_INVAL;
    stop_worker(srv);
    return SIM_OK;
}

int srv_sync(sim_server* srv) {
    if (!srv) return SIM_E_INVAL;
    std::unique_lock<std::mutex> lock(srv->mu);
    // with the worker running, wait for it; if it is being stopped, run what is left here
    if (srv->running)
        srv->cv_done.wait(lock, [&] { return srv->queued == 0 || srv->stopping; });
    int rc = srv->last_rc;
    srv->last_rc = SIM_OK;
    lock.unlock();
    for (;;) {
        {
            std::lock_guard<std::mutex> l(srv->mu);
            if (srv->queued == 0) break;
        }
        const int r = run_step(srv, nullptr);
        if (r && rc == SIM_OK) rc = r;
    }
    return rc;
}

int srv_drain(sim_server* srv, int32_t cam, uint64_t* dst, uint64_t max_events, int32_t mem_kind,
              uint64_t* n_written) {
    if (!srv) return SIM_E_INVAL;
    std::lock_guard<std::mutex> step(srv->push_mu);
    if (cam < 0 || cam >= (int)srv->cams.size() || !srv->cams[cam].used) return SIM_E_INVAL;
    return sim_drain_keys(srv->cams[cam].s, dst, max_events, mem_kind, n_written);
}

int srv_pending(sim_server* srv, int32_t cam, uint64_t* n) {
    if (!srv || !n) return SIM_E_INVAL;
    std::lock_guard<std::mutex> step(srv->push_mu);
    if (cam < 0 || cam >= (int)srv->cams.size() || !srv->cams[cam].used) return SIM_E_INVAL;
    return sim_pending_events(srv->cams[cam].s, n);
}

int srv_stream(sim_server* srv, int32_t cam, sim_stream** out) {
    if (!srv || !out) return SIM_E_INVAL;
    std::lock_guard<std::mutex> lock(srv->mu);
    if (cam < 0 || cam >= (int)srv->cams.size() || !srv->cams[cam].used) return SIM_E_INVAL;
    *out = srv->cams[cam].s;
    return SIM_OK;
}

int srv_get_stats(sim_server* srv, sim_server_stats* out) {
    if (!srv || !out) return SIM_E_INVAL;
    std::lock_guard<std::mutex> lock(srv->mu);
    *out = srv->st;
    const size_t n = srv->lat_ms.size();
    if (n) {
        std::vector<float>& v = srv->lat_sort;   // reserved: no allocation
        v.assign(srv->lat_ms.begin(), srv->lat_ms.end());
        auto pct = [&](double q) {
            size_t k = (size_t)floor(q * (double)(n - 1) + 0.5);
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return (double)v[k];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = (double)*std::max_element(v.begin(), v.end());
    }
    return SIM_OK;
}

int srv_clear_stats(sim_server* srv) {
    if (!srv) return SIM_E_INVAL;
    std::lock_guard<std::mutex> lock(srv->mu);
    const uint64_t cams = srv->st.cameras;
    memset(&srv->st, 0, sizeof(srv->st));
    srv->st.cameras = cams;
    srv->st.hbm_budget = srv->budget;
    srv->st.hbm_used = srv->used;
    srv->lat_ms.clear();
    srv->lat_next = 0;
    return SIM_OK;
}

int64_t srv_now_ns(void) { return now_ns(); }

}  // extern "C"
