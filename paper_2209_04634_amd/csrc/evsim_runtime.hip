// Host runtime of the event simulator: the C ABI declared in include/sim.h.
//
// Per stream the device holds the 256-entry transform table, the per-pixel reference levels
// (updated in place), two previous-frame buffers (ping-pong; two more for the difference
// method), the sparse method's selection masks and active list, an event arena of 256 striped
// sub-arenas, sort buffers, and a FIFO of sorted packed keys awaiting drain.  A push runs in
// windows of up to 128 intervals (host inputs are copied to the device one window at a time):
// the selection pass (or the frame copies), flow estimation when
// it is on, one chain launch, a read of the overflow counters, re-runs of the chains that ran out
// of arena space after growing it, the gather of the sub-arenas, and the sort whose last pass
// appends to the FIFO.  A batched push runs each phase of every stream's window in one fused
// launch (fused_window).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sim.h"
#include "evsim_internal.h"

using namespace evsim;

namespace {

constexpr uint64_t kMaxInterval = 1ull << 31;
constexpr int64_t kMaxEpochSpan = (int64_t)1 << 39;

int bits_for(uint64_t v) {  // number of bits to represent values 0..v (at least 1)
    int b = 1;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

template <class T>
hipError_t dev_alloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    return hipMalloc((void**)p, n * sizeof(T));
}

}  // namespace

struct sim_stream {
    sim_config cfg;
    int S = 1;
    float m = 0.0f;
    float lut_host[256];
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    hipEvent_t ev_ready = nullptr;   // marks the stream's queued work for a batched push to wait on

    int64_t npix = 0;
    float* d_lut = nullptr;
    float* d_lref = nullptr;
    uint8_t* d_prev[2] = {nullptr, nullptr};
    uint8_t* d_prev2[2] = {nullptr, nullptr};    // difference method: the frame before d_prev
    int cur = 0;
    uint64_t n_int = 0;                          // intervals simulated since the first frame
    uint64_t est_events = 0;                     // most events of a batched window so far
                                                 // (sizes the sort grid of the next one)

    bool started = false;
    int64_t epoch = 0, t_prev = 0;

    // window scratch
    uint64_t* d_arena = nullptr;                 // kArenaStripes sub-arenas of stripe_cap keys
    uint64_t stripe_cap = 0;
    unsigned long long* d_reserve = nullptr;     // per sub-arena reservation counters
    unsigned long long* d_stats = nullptr;       // striped selection statistics
    uint64_t* d_alt = nullptr;                   // gathered keys (sort input)
    uint64_t alt_cap = 0;
    uint64_t* d_alt2 = nullptr;                  // sort ping-pong buffer; never the arena, which
    uint64_t alt2_cap = 0;                       // must survive until the overflow check
    uint32_t* d_hist = nullptr;
    size_t hist_cap = 0;
    uint32_t* d_totals = nullptr;
    unsigned long long* d_counters = nullptr;
    unsigned long long* h_counters = nullptr;   // pinned
    unsigned long long* h_stats = nullptr;      // pinned copy of d_stats (sim_get_stats)
    float* d_delta = nullptr;
    int64_t* d_tbase = nullptr;
    int* d_resume = nullptr;                     // per chain slot
    uint32_t* d_mask = nullptr;                  // sparse: [kMaskWords][npix]
    uint32_t* d_act = nullptr;                   // sparse: the selection blocks' runs
    uint32_t* d_olist = nullptr;                 // sparse: per-block class counts, run places,
                                                 // selected counts, the ordered list's length
    uint32_t* d_ord = nullptr;                   // sparse: active pixels ordered by chain length
    float* h_delta = nullptr;                    // pinned
    int64_t* h_tbase = nullptr;                  // pinned

    // staging for host inputs
    uint8_t* d_stage_frames = nullptr;
    size_t stage_frames_cap = 0;
    float* d_stage_flows = nullptr;
    size_t stage_flows_cap = 0;

    // FIFO of sorted packed keys
    uint64_t* d_fifo = nullptr;
    uint64_t fifo_cap = 0, fifo_head = 0, fifo_tail = 0;

    // flow estimation (SIM_FLOW_LK): pyramids of a window's frames, estimated flow fields
    LkParams lk;
    float* d_pyr = nullptr;
    uint64_t pyr_cap = 0;
    float* d_lkflow = nullptr;
    uint64_t lkflow_cap = 0;

    // accumulated-frame scratch (sim_accumulate with host counts, sim_event_rate)
    uint32_t* d_acc = nullptr;
    uint64_t acc_cap = 0;
    unsigned long long* d_moments = nullptr;     // per-block partial sums (sim_event_rate)
    uint64_t moments_cap = 0;

    sim_stats stats;
    char last_error[256] = {0};

    // window in flight (between the launch, check and order phases of a push)
    struct Job {
        bool active = false;
        int K = 0;
        int nbits = 0;
        int max_slots = 0;
        KeyLayout lay;
        ChainArgs a;
        int64_t t_last = 0;
        int variant = kDefaultChainVariant;
    } job;

    int forced_variant = -1;                     // sim_set_chain_variant; -1: autotuned
    int last_variant = -1;                       // variant of the last window's chain pass

    // kernel timing (sim_set_kernel_timing)
    bool timing = false;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

int hip_fail_at(sim_stream* s, hipError_t e, const char* what, int line) {
    s->poisoned = true;
    snprintf(s->last_error, sizeof(s->last_error), "%s (line %d): %s", what, line,
             hipGetErrorString(e));
    (void)hipGetLastError();
    return SIM_E_HIP;
}

int hip_fail(sim_stream* s) { return hip_fail_at(s, hipGetLastError(), "HIP call", 0); }

// A failure after a window's chains have run: the reference levels and the previous frame have
// advanced on the device while the host state has not, so the stream cannot continue.
int fail_mid_push(sim_stream* s, int rc, const char* what) {
    s->poisoned = true;
    snprintf(s->last_error, sizeof(s->last_error), "%s failed in the middle of a push (%s)",
             what, rc == SIM_E_NOMEM ? "out of memory" : "error");
    return rc;
}

#define HIP_TRY(s, expr)                                                 \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) return hip_fail_at(s, e_, #expr, __LINE__); \
    } while (0)

void free_stream(sim_stream* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->ev_ready) (void)hipEventDestroy(s->ev_ready);
    dfree(s->d_lut);
    dfree(s->d_lref);
    dfree(s->d_prev[0]);
    dfree(s->d_prev[1]);
    dfree(s->d_prev2[0]);
    dfree(s->d_prev2[1]);
    dfree(s->d_acc);
    dfree(s->d_moments);
    dfree(s->d_pyr);
    dfree(s->d_lkflow);
    dfree(s->d_arena);
    dfree(s->d_reserve);
    dfree(s->d_stats);
    dfree(s->d_alt);
    dfree(s->d_alt2);
    dfree(s->d_hist);
    dfree(s->d_totals);
    dfree(s->d_counters);
    dfree(s->d_mask);
    dfree(s->d_act);
    dfree(s->d_olist);
    dfree(s->d_ord);
    dfree(s->d_delta);
    dfree(s->d_tbase);
    dfree(s->d_resume);
    dfree(s->d_stage_frames);
    dfree(s->d_stage_flows);
    dfree(s->d_fifo);
    if (s->h_counters) (void)hipHostFree(s->h_counters);
    if (s->h_stats) (void)hipHostFree(s->h_stats);
    if (s->h_delta) (void)hipHostFree(s->h_delta);
    if (s->h_tbase) (void)hipHostFree(s->h_tbase);
    for (hipEvent_t& e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Grows a device buffer to at least n elements, keeping the first `keep` elements.
template <class T>
int grow(sim_stream* s, T** buf, uint64_t* cap, uint64_t n, uint64_t keep) {
    if (n <= *cap) return SIM_OK;
    T* nb = nullptr;
    if (hipMalloc((void**)&nb, n * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return SIM_E_NOMEM;
    }
    if (keep) {
        if (hipMemcpyAsync(nb, *buf, keep * sizeof(T), hipMemcpyDeviceToDevice, s->stream) !=
                hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess) {
            dfree(nb);
            return hip_fail(s);
        }
    } else if (*buf) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) {
            dfree(nb);
            return hip_fail(s);
        }
    }
    dfree(*buf);
    *buf = nb;
    *cap = n;
    return SIM_OK;
}

int ensure_alt(sim_stream* s, uint64_t n) {
    int rc = grow(s, &s->d_alt, &s->alt_cap, n, 0);
    if (!rc) rc = grow(s, &s->d_alt2, &s->alt2_cap, n, 0);
    return rc;
}

int ensure_sort_scratch(sim_stream* s, uint64_t n) {
    uint64_t hc = s->hist_cap;
    int rc = grow(s, &s->d_hist, &hc, sort_hist_entries(n), 0);
    s->hist_cap = (size_t)hc;
    return rc;
}

// Grows every sub-arena to new_stripe_cap keys, keeping the first stripe_cap keys of each.
int grow_arena(sim_stream* s, uint64_t new_stripe_cap) {
    if (new_stripe_cap <= s->stripe_cap) return SIM_OK;
    if (new_stripe_cap * kArenaStripes >= kArenaKeyLimit) return SIM_E_NOMEM;
    uint64_t* nb = nullptr;
    if (hipMalloc((void**)&nb, new_stripe_cap * kArenaStripes * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return SIM_E_NOMEM;
    }
    if (hipMemcpy2DAsync(nb, new_stripe_cap * sizeof(uint64_t), s->d_arena,
                         s->stripe_cap * sizeof(uint64_t), s->stripe_cap * sizeof(uint64_t),
                         kArenaStripes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        dfree(nb);
        return hip_fail(s);
    }
    dfree(s->d_arena);
    s->d_arena = nb;
    s->stripe_cap = new_stripe_cap;
    s->stats.event_capacity = new_stripe_cap * kArenaStripes;
    return SIM_OK;
}

void build_lut(sim_stream* s) {
    for (int v = 0; v < 256; ++v) {
        if (s->cfg.transform == SIM_LOG)
            s->lut_host[v] = (float)log((double)v / 255.0 + (double)s->cfg.log_eps);
        else
            s->lut_host[v] = (float)v;
    }
}

int check_mem_kind(int32_t k) { return (k == SIM_MEM_HOST || k == SIM_MEM_DEVICE) ? SIM_OK : SIM_E_INVAL; }

bool lk_ok(const sim_lk_params& p) {
    return p.levels >= 0 && p.levels <= kLkMaxLevels && p.radius >= 1 && p.radius <= 15 &&
           p.iterations >= 1 && p.iterations <= 100 && p.eps >= 0.0f && p.min_trace >= 0.0f &&
           p.min_ratio >= 0.0f;
}

LkParams lk_from(const sim_lk_params& p) {
    LkParams r;
    r.levels = p.levels;
    r.radius = p.radius;
    r.iters = p.iterations;
    r.eps = p.eps;
    r.min_trace = p.min_trace;
    r.min_ratio = p.min_ratio;
    return r;
}

// A window of K intervals whose frames/flows are already on the device runs in three phases, so
// that a batch of streams can interleave them: every stream's kernels are queued on its own HIP
// stream before any host wait.
//   launch: per-interval tables, counter resets, selection (or frame save), chain kernel, and an
//           asynchronous read of the overflow counters;
//   check:  wait for the counters; re-run overflowed chains after growing the arena until none
//           overflows; concatenate the sub-arenas and read the event count asynchronously;
//   order:  wait for the count; sort into the FIFO; advance the stream's state.
// Host side of a window (no device work): per-interval tables into h_delta / h_tbase, the key
// layout, and the selection and chain arguments, whose table pointers are d_delta / d_tbase.
int plan_window(sim_stream* s, const uint8_t* frames, const float* flows, const int64_t* t_us,
                int K, float* h_delta, int64_t* h_tbase, const float* d_delta, KeyLayout* lay_out,
                int* nbits_out, SelectArgs* sa, OrderArgs* oa, ChainArgs* a) {
    const int W = s->cfg.width, H = s->cfg.height;
    uint64_t max_delta = 0;
    for (int i = 0; i < K; ++i) {
        const int64_t t0 = i == 0 ? s->t_prev : t_us[i - 1];
        const int64_t d = t_us[i] - t0;
        h_delta[i] = (float)d;
        h_tbase[i] = t0 - s->epoch;
        const uint64_t dr = (uint64_t)ceil((double)h_delta[i]);
        max_delta = std::max(max_delta, dr);
    }
    KeyLayout lay;
    lay.xb = bits_for((uint64_t)(W - 1));
    lay.yb = bits_for((uint64_t)(H - 1));
    lay.tb = bits_for(max_delta);
    lay.ib = K > 1 ? bits_for((uint64_t)(K - 1)) : 0;
    const int nbits = lay.total_bits() + 1;   // + sentinel bit
    if (nbits > 64) return SIM_E_RANGE;
    *lay_out = lay;
    *nbits_out = nbits;

    const bool sparse = s->cfg.method == SIM_SPARSE;
    sa->prev = s->d_prev[s->cur];
    sa->frames = frames;
    sa->fstride = s->npix;
    sa->lut = s->d_lut;
    sa->prev_out = s->d_prev[1 - s->cur];
    sa->mask = s->d_mask;
    const int nblk = select_blocks(s->npix);
    uint32_t* counts = s->d_olist;
    uint32_t* goff = counts ? counts + (size_t)nblk * kClasses : nullptr;
    uint32_t* bsel = goff ? goff + (size_t)nblk * kClasses : nullptr;
    unsigned int* n_total = bsel ? bsel + nblk : nullptr;
    sa->act_px = s->d_act;
    sa->counts = counts;
    sa->bsel = bsel;
    sa->npix = (int)s->npix;
    sa->K = K;
    sa->m = s->m;

    oa->act_px = s->d_act;
    oa->counts = counts;
    oa->bsel = bsel;
    oa->nblocks = nblk;
    oa->goff = goff;
    oa->n_total = n_total;
    oa->stats = s->d_stats;
    oa->ord = s->d_ord;
    oa->resume = s->d_resume;

    const bool estimate = s->cfg.flow_source == SIM_FLOW_LK && s->S > 1;
    a->prev = s->d_prev[s->cur];
    a->frames = frames;
    a->fstride = s->npix;
    a->flows = estimate ? s->d_lkflow : flows;
    a->flstride = 2 * s->npix;
    a->lut = s->d_lut;
    a->delta = d_delta;
    a->lref = s->d_lref;
    a->mask = sparse ? s->d_mask : nullptr;
    a->act_px = sparse ? s->d_ord : nullptr;
    a->n_active = sparse ? n_total : nullptr;
    a->resume = s->d_resume;
    a->reserve = s->d_reserve;
    a->fails = s->d_counters;          // [0] failed reservations, [1] sentinels, [2] gathered
    a->W = W;
    a->H = H;
    a->S = s->S;
    a->K = K;
    a->npix = (int)s->npix;
    a->cpos = s->cfg.c_pos;
    a->cneg = s->cfg.c_neg;
    a->lay = lay;
    if (s->cfg.method == SIM_DIFFERENCE)
        a->mode = kModeDifference;
    else
        a->mode = s->cfg.thresh_mode == SIM_THRESH_MEMORYLESS ? kModeMemoryless : kModeReference;
    a->prev2 = s->d_prev2[s->cur];
    a->first_emit = s->n_int == 0 ? 1 : 0;   // difference method: three frames are needed
    a->arena = s->d_arena;
    a->stripe_cap = s->stripe_cap;
    return SIM_OK;
}

// Slots of the chain pass: the ordered active list (sparse) or every pixel.
int chain_slots(const sim_stream* s) { return (int)s->npix; }

// Words of d_olist: counts and run places per (block, class), selected counts per block, the
// ordered list's length.
size_t olist_words(int64_t npix) {
    const size_t nblk = (size_t)select_blocks(npix);
    return 2 * nblk * kClasses + nblk + 1;
}

// Estimated flow (SIM_FLOW_LK): buffers for a window of K intervals.
int ensure_lk_buffers(sim_stream* s, int K) {
    const PyrLayout pl = pyr_layout(s->cfg.width, s->cfg.height, s->lk.levels);
    uint64_t cap = s->pyr_cap;
    int rc = grow(s, &s->d_pyr, &cap, (uint64_t)(K + 1) * pl.total, 0);
    s->pyr_cap = cap;
    if (!rc) {
        cap = s->lkflow_cap;
        rc = grow(s, &s->d_lkflow, &cap, (uint64_t)K * 2 * (uint64_t)s->npix, 0);
        s->lkflow_cap = cap;
    }
    return rc;
}

// Flow of every selected pixel-interval of the window, from the pyramids of the previous frame
// and the window's frames, into the layout of supplied flows (after the selection pass).
hipError_t launch_lk(sim_stream* s, const uint8_t* frames, int K, hipStream_t stream) {
    const bool sparse = s->cfg.method == SIM_SPARSE;
    const PyrLayout pl = pyr_layout(s->cfg.width, s->cfg.height, s->lk.levels);
    hipError_t e = launch_pyramids(s->d_prev[s->cur], frames, s->npix, K + 1, pl, s->d_pyr, stream);
    if (e != hipSuccess) return e;
    LkWindowArgs la;
    la.pyr = s->d_pyr;
    la.lay = pl;
    la.P = s->lk;
    la.mask = sparse ? s->d_mask : nullptr;
    la.act_px = sparse ? s->d_ord : nullptr;
    la.n_active = sparse ? s->d_olist + olist_words(s->npix) - 1 : nullptr;
    la.npix = (int)s->npix;
    la.W = s->cfg.width;
    la.K = K;
    la.flow = s->d_lkflow;
    return launch_lk_window(la, chain_slots(s), stream);
}

// ------------------------------------------------------------------------------------------
// Chain-pass autotuner.  The variants differ only in how many interior samples' loads a lane
// keeps in flight (registers against waves per SIMD); the fastest depends on the image size, the
// method and mode, S and the selected fraction.  On the first window of each (device
// architecture, W, H, method, mode, S), every variant runs on that window against scratch copies
// of what the pass writes -- reference levels, resume points, event arena and counters -- so the
// stream itself is untouched, timed with HIP events (a warm-up round, then the best of three
// rounds, variants interleaved); the fastest is kept for the process.  All variants give
// identical results.
// ------------------------------------------------------------------------------------------
struct TuneKey {
    std::string arch;
    int W, H, method, mode, S;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, W, H, method, mode, S) <
               std::tie(o.arch, o.W, o.H, o.method, o.mode, o.S);
    }
};

struct Tuner {
    std::mutex mu;
    std::map<TuneKey, int> best;
    std::map<int, std::string> arch;   // per device
};

Tuner& tuner() {
    static Tuner* t = new Tuner();   // lives until the process ends
    return *t;
}

std::string device_arch(Tuner& t) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return "?";
    }
    auto it = t.arch.find(dev);
    if (it != t.arch.end()) return it->second;
    hipDeviceProp_t p;
    std::string name = "?";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess)
        name = p.gcnArchName;
    else
        (void)hipGetLastError();
    t.arch[dev] = name;
    return name;
}

// Times every variant of the chain pass `a` (max_slots slots) on `st`; returns the fastest, or
// the default variant if anything fails.  Waits on `st`.
int tune_chain(sim_stream* s, const ChainArgs& a, int max_slots, hipStream_t st) {
    ChainArgs t = a;
    float* lref = nullptr;
    int* resume = nullptr;
    uint64_t* arena = nullptr;
    unsigned long long* reserve = nullptr;
    unsigned long long* fails = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = (a.mode != kModeReference || dev_alloc(&lref, (size_t)s->npix) == hipSuccess) &&
              dev_alloc(&resume, (size_t)max_slots) == hipSuccess &&
              dev_alloc(&reserve, (size_t)kArenaStripes * kCounterStride) == hipSuccess &&
              dev_alloc(&fails, 4) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
              hipEventCreate(&e1) == hipSuccess;
    float ms[kChainVariants];
    // The scratch arena starts at the stream's capacity and grows fourfold (up to 2^28 keys)
    // while a timed pass runs out of space: a pass whose waves stop early would be timed on
    // part of the work.
    uint64_t cap = std::max<uint64_t>(a.stripe_cap, 1);
    for (int attempt = 0; ok; ++attempt) {
        dfree(arena);
        arena = nullptr;
        ok = dev_alloc(&arena, (size_t)kArenaStripes * cap) == hipSuccess;
        if (!ok) break;
        if (lref) t.lref = lref;
        t.resume = resume;
        t.arena = arena;
        t.stripe_cap = cap;
        t.reserve = reserve;
        t.fails = fails;
        for (int v = 0; v < kChainVariants; ++v) ms[v] = 1e30f;
        bool overflow = false;
        for (int rep = 0; rep < 4 && ok && !overflow; ++rep) {   // a warm-up, then best of three
            for (int v = 0; v < kChainVariants && ok && !overflow; ++v) {
                // the state the real pass starts from: levels as they are, every chain at its
                // first interval, empty arena counters
                ok = (!lref || hipMemcpyAsync(lref, a.lref, (size_t)s->npix * sizeof(float),
                                              hipMemcpyDeviceToDevice, st) == hipSuccess) &&
                     launch_zero(resume, (size_t)max_slots * sizeof(int), st) == hipSuccess &&
                     launch_zero(reserve, (size_t)kArenaStripes * kCounterStride *
                                              sizeof(unsigned long long), st) == hipSuccess &&
                     launch_zero(fails, 4 * sizeof(unsigned long long), st) == hipSuccess &&
                     hipEventRecord(e0, st) == hipSuccess &&
                     launch_chain(t, max_slots, v, st) == hipSuccess &&
                     hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
                unsigned long long failed = 0;
                ok = ok &&
                     hipMemcpyAsync(&failed, fails, sizeof(failed), hipMemcpyDeviceToHost, st) ==
                         hipSuccess &&
                     hipStreamSynchronize(st) == hipSuccess;
                overflow = ok && failed != 0;
                float m = 0.0f;
                if (ok && !overflow && rep > 0 && hipEventElapsedTime(&m, e0, e1) == hipSuccess)
                    ms[v] = std::min(ms[v], m);
            }
        }
        if (!overflow || (uint64_t)kArenaStripes * cap * 4 > (1ull << 28)) {
            if (overflow)   // timed on part of the work: fall back to the default
                for (int v = 0; v < kChainVariants; ++v) ms[v] = 1e30f;
            break;
        }
        cap *= 4;
    }
    if (!ok) (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(lref);
    dfree(resume);
    dfree(arena);
    dfree(reserve);
    dfree(fails);
    int best = kDefaultChainVariant;
    if (ok)
        for (int v = 0; v < kChainVariants; ++v)
            if (ms[v] < ms[best]) best = v;
    return best;
}

// The variant for the window `a` of stream s: forced, cached for its key, or tuned now (the
// window's selection and order pass must be queued on `st` already).
int chain_variant_for(sim_stream* s, const ChainArgs& a, int max_slots, hipStream_t st) {
    if (s->forced_variant >= 0) return s->forced_variant;
    if (s->S <= 1) return kDefaultChainVariant;   // no interior samples: variants coincide
    if (s->cfg.flow_source == SIM_FLOW_LK) return kDefaultChainVariant;
    Tuner& tu = tuner();
    std::lock_guard<std::mutex> lock(tu.mu);
    TuneKey k{device_arch(tu), s->cfg.width, s->cfg.height, s->cfg.method, a.mode, s->S};
    auto it = tu.best.find(k);
    if (it != tu.best.end()) return it->second;
    const int v = tune_chain(s, a, max_slots, st);
    tu.best[k] = v;
    return v;
}

int win_launch(sim_stream* s, const uint8_t* frames, const float* flows, const int64_t* t_us,
               int K) {
    const bool estimate = s->cfg.flow_source == SIM_FLOW_LK && s->S > 1;
    if (estimate) {
        int rc = ensure_lk_buffers(s, K);
        if (rc) return rc;
    }
    KeyLayout lay;
    int nbits = 0;
    SelectArgs sa;
    OrderArgs oa;
    ChainArgs a;
    int rc = plan_window(s, frames, flows, t_us, K, s->h_delta, s->h_tbase, s->d_delta, &lay,
                         &nbits, &sa, &oa, &a);
    if (rc) return rc;

    HIP_TRY(s, hipMemcpyAsync(s->d_delta, s->h_delta, K * sizeof(float), hipMemcpyHostToDevice,
                              s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->d_tbase, s->h_tbase, K * sizeof(int64_t), hipMemcpyHostToDevice,
                              s->stream));
    const bool sparse = s->cfg.method == SIM_SPARSE;
    HIP_TRY(s, launch_prep_window(s->d_counters, s->d_reserve, sparse ? nullptr : s->d_resume,
                                  s->npix, s->stream));
    if (s->timing) HIP_TRY(s, hipEventRecord(s->ev[0], s->stream));
    if (sparse) {
        HIP_TRY(s, launch_select(sa, s->stream));
        HIP_TRY(s, launch_order(oa, s->stream));
    } else {
        HIP_TRY(s, launch_copy_u8(frames + (size_t)(K - 1) * s->npix, sa.prev_out, s->npix,
                                  s->stream));
        if (s->cfg.method == SIM_DIFFERENCE) {
            // the frame before the window's last one becomes the next window's second-to-last
            const uint8_t* src = K >= 2 ? frames + (size_t)(K - 2) * s->npix : s->d_prev[s->cur];
            HIP_TRY(s, launch_copy_u8(src, s->d_prev2[1 - s->cur], s->npix, s->stream));
        }
    }
    if (estimate) HIP_TRY(s, launch_lk(s, frames, K, s->stream));
    if (s->timing) HIP_TRY(s, hipEventRecord(s->ev[1], s->stream));

    const int max_slots = chain_slots(s);
    s->job.active = true;
    s->job.K = K;
    s->job.nbits = nbits;
    s->job.max_slots = max_slots;
    s->job.lay = lay;
    s->job.t_last = t_us[K - 1];
    s->job.variant = chain_variant_for(s, a, max_slots, s->stream);
    s->last_variant = s->job.variant;
    HIP_TRY(s, launch_chain(a, max_slots, s->job.variant, s->stream));
    if (s->timing) HIP_TRY(s, hipEventRecord(s->ev[2], s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->h_counters, s->d_counters, 2 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s->stream));
    s->job.a = a;
    return SIM_OK;
}

int win_check(sim_stream* s) {
    ChainArgs& a = s->job.a;
    bool first = true;
    for (;;) {
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        if (s->timing) {
            float ms = 0.0f;
            if (first) {
                HIP_TRY(s, hipEventElapsedTime(&ms, s->ev[0], s->ev[1]));
                s->stats.select_ms += ms;
                s->stats.select_launches++;
            }
            HIP_TRY(s, hipEventElapsedTime(&ms, s->ev[1], s->ev[2]));
            s->stats.simulate_ms += ms;
            s->stats.simulate_launches++;
        }
        first = false;
        if (s->h_counters[0] == 0) break;
        // Some waves ran out of sub-arena space: grow every sub-arena (keeping what was
        // written, including the sentinels of abandoned reservations) and re-run only the
        // unfinished pixel chains.  Nothing else reads or writes the arena in between.
        const uint64_t old = s->stripe_cap;
        int rc = grow_arena(s, 2 * old);
        // finished chains have already advanced their reference levels: no roll-back
        if (rc) return fail_mid_push(s, rc, "event arena growth");
        HIP_TRY(s, launch_clamp(s->d_reserve, old, s->stream));
        HIP_TRY(s, launch_zero(s->d_counters, sizeof(unsigned long long), s->stream));
        s->stats.retries++;
        a.arena = s->d_arena;
        a.stripe_cap = s->stripe_cap;
        if (s->timing) HIP_TRY(s, hipEventRecord(s->ev[1], s->stream));
        HIP_TRY(s, launch_chain(a, s->job.max_slots, s->job.variant, s->stream));
        if (s->timing) HIP_TRY(s, hipEventRecord(s->ev[2], s->stream));
        HIP_TRY(s, hipMemcpyAsync(s->h_counters, s->d_counters, 2 * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s->stream));
    }
    // every chain has finished: concatenate the sub-arenas, then order the events
    {
        int rc = ensure_alt(s, kArenaStripes * s->stripe_cap);
        if (rc) return fail_mid_push(s, rc, "sort buffer growth");
    }
    HIP_TRY(s, launch_gather(s->d_arena, s->stripe_cap, s->d_reserve, s->d_alt,
                             s->d_counters + 2, s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->h_counters, s->d_counters, 3 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s->stream));
    return SIM_OK;
}

int win_order(sim_stream* s, uint64_t* n_new) {
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const uint64_t n_total = s->h_counters[2];
    const uint64_t n_valid = n_total - s->h_counters[1];
    if (n_valid > 0) {
        int rc = ensure_sort_scratch(s, n_total);
        if (!rc && s->fifo_tail + n_valid > s->fifo_cap)
            rc = grow(s, &s->d_fifo, &s->fifo_cap,
                      std::max<uint64_t>(s->fifo_tail + n_valid, 2 * s->fifo_cap),
                      s->fifo_tail);
        if (rc) return fail_mid_push(s, rc, "event buffer growth");
        ConvertArgs cv;
        cv.enabled = 1;
        cv.n_sentinel = s->d_counters + 1;
        cv.tbase = s->d_tbase;
        cv.K = s->job.K;
        cv.lay = s->job.lay;
        if (s->timing) HIP_TRY(s, hipEventRecord(s->ev[3], s->stream));
        HIP_TRY(s, launch_sort(s->d_alt, s->d_alt2, s->d_counters + 2, n_total, s->job.nbits,
                               s->d_hist, s->d_totals, s->d_fifo + s->fifo_tail, cv, s->stream));
        if (s->timing) {
            HIP_TRY(s, hipEventRecord(s->ev[4], s->stream));
            HIP_TRY(s, hipEventSynchronize(s->ev[4]));
            float ms = 0.0f;
            HIP_TRY(s, hipEventElapsedTime(&ms, s->ev[3], s->ev[4]));
            s->stats.sort_ms += ms;
            s->stats.sort_launches++;
        }
    }
    s->fifo_tail += n_valid;
    s->cur = 1 - s->cur;
    s->t_prev = s->job.t_last;
    s->n_int += (uint64_t)s->job.K;
    s->stats.intervals += (uint64_t)s->job.K;
    s->stats.frames += (uint64_t)s->job.K;
    s->stats.events += n_valid;
    s->job.active = false;
    if (n_new) *n_new += n_valid;
    return SIM_OK;
}

// Argument and timestamp validation of a push (no state change, no device work).
int push_validate(sim_stream* s, int32_t n_frames, const uint8_t* frames, const float* flows,
                  const int64_t* t_us, int32_t mem_kind) {
    if (!s) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    if (n_frames < 1 || !frames || !t_us || check_mem_kind(mem_kind)) return SIM_E_INVAL;
    const int first = s->started ? 0 : 1;     // frames consumed by initialisation
    const int n_int = n_frames - first;
    if (n_int > 0 && s->S > 1 && !flows && s->cfg.flow_source == SIM_FLOW_SUPPLIED)
        return SIM_E_INVAL;
    int64_t prev = s->started ? s->t_prev : t_us[0];
    const int64_t epoch = s->started ? s->epoch : t_us[0];
    for (int j = first; j < n_frames; ++j) {
        if (t_us[j] <= prev) return SIM_E_ORDER;
        if ((uint64_t)(t_us[j] - prev) >= kMaxInterval) return SIM_E_RANGE;
        if (t_us[j] - epoch >= kMaxEpochSpan) return SIM_E_RANGE;
        prev = t_us[j];
    }
    return SIM_OK;
}

struct Staged {
    const uint8_t* frames = nullptr;   // the caller's frames (host or device, see `host`)
    const float* flows = nullptr;      // the caller's flows
    bool host = false;                 // host inputs: copied to the device one window at a time
    int first = 0;                     // frames consumed by initialisation
    int n_int = 0;                     // intervals to simulate
};

bool uses_flows(const sim_stream* s) {
    return s->S > 1 && s->cfg.flow_source == SIM_FLOW_SUPPLIED;
}

// Reserves what the push needs whatever its events (host inputs: staging for one window of
// frames and flows) and initialises a fresh stream from its first frame.
int push_stage(sim_stream* s, int32_t n_frames, const uint8_t* frames, const float* flows,
               const int64_t* t_us, int32_t mem_kind, Staged* out) {
    const size_t fbytes = (size_t)s->npix;
    const size_t flfloats = (size_t)s->npix * 2;
    out->first = s->started ? 0 : 1;
    out->n_int = n_frames - out->first;
    out->frames = frames;
    out->flows = flows;
    out->host = mem_kind == SIM_MEM_HOST;
    const uint8_t* init_frame = frames;
    if (out->host) {
        const int win = std::min(kMaxWindow, out->n_int);
        uint64_t cap = s->stage_frames_cap;
        int rc = grow(s, &s->d_stage_frames, &cap, (uint64_t)std::max(win, 1) * fbytes, 0);
        s->stage_frames_cap = (size_t)cap;
        if (rc) return rc;
        if (win > 0 && uses_flows(s)) {
            cap = s->stage_flows_cap;
            rc = grow(s, &s->d_stage_flows, &cap, (uint64_t)win * flfloats, 0);
            s->stage_flows_cap = (size_t)cap;
            if (rc) return rc;
        }
        init_frame = s->d_stage_frames;
    }
    if (out->n_int > 0) {
        // every buffer whose size is known now, before anything changes: a failure here leaves
        // the stream as it was (later growth with the event count fails mid-push and poisons)
        int rc = SIM_OK;
        if (s->cfg.flow_source == SIM_FLOW_LK && s->S > 1)
            rc = ensure_lk_buffers(s, std::min(kMaxWindow, out->n_int));
        if (!rc) rc = ensure_alt(s, kArenaStripes * s->stripe_cap);
        if (!rc) rc = ensure_sort_scratch(s, kArenaStripes * s->stripe_cap);
        if (rc) return rc;
    }
    if (!s->started) {
        if (out->host)
            HIP_TRY(s, hipMemcpyAsync(s->d_stage_frames, frames, fbytes, hipMemcpyHostToDevice,
                                      s->stream));
        HIP_TRY(s, launch_init(init_frame, s->d_lut, s->d_lref, s->d_prev[s->cur], s->npix,
                               s->stream));
        s->started = true;
        s->epoch = t_us[0];
        s->t_prev = t_us[0];
        s->n_int = 0;
        s->stats.frames += 1;
    }
    return SIM_OK;
}

// Device frames and flows of the window of K intervals starting at interval j.  Host inputs are
// copied into the staging buffers on the stream, after the work queued before (the previous
// window, which read the same buffers, has completed by then: every window ends with a host
// wait).
int stage_window(sim_stream* s, const Staged& st, int j, int K, const uint8_t** frames,
                 const float** flows) {
    const size_t npix = (size_t)s->npix;
    const uint8_t* f = st.frames + (size_t)(st.first + j) * npix;
    const float* fl = uses_flows(s) ? st.flows + (size_t)j * 2 * npix : nullptr;
    if (st.host) {
        HIP_TRY(s, hipMemcpyAsync(s->d_stage_frames, f, (size_t)K * npix, hipMemcpyHostToDevice,
                                  s->stream));
        f = s->d_stage_frames;
        if (fl) {
            HIP_TRY(s, hipMemcpyAsync(s->d_stage_flows, fl, (size_t)K * 2 * npix * sizeof(float),
                                      hipMemcpyHostToDevice, s->stream));
            fl = s->d_stage_flows;
        }
    }
    *frames = f;
    *flows = fl;
    return SIM_OK;
}

int run_window(sim_stream* s, const uint8_t* frames, const float* flows, const int64_t* t_us,
               int K, uint64_t* n_new) {
    int rc = win_launch(s, frames, flows, t_us, K);
    if (!rc) rc = win_check(s);
    if (!rc) rc = win_order(s, n_new);
    if (rc) s->job.active = false;
    return rc;
}

// ------------------------------------------------------------------------------------------
// Fused batched push: the streams of a sim_push_batch call share one launch per phase (clear,
// selection or frame copies, chains per thresholding mode, overflow readback, gather, counts,
// and every pass of the sort), on one library stream, with one host wait per phase instead of
// one per stream.  Per stream the kernels run the same block bodies on the same data as its
// own launches, so every stream's result is that of the stream pushed alone.
// ------------------------------------------------------------------------------------------
// Launch shape of a fused chunk: what a recorded graph's nodes depend on besides the blob's
// contents (grid sizes, sizes of the copies, the buffers the nodes read and write).
struct BatchShape {
    int n = 0;
    size_t tab = 0;
    std::array<int, 14> totals{};
    const void* blob = nullptr;
    const void* out = nullptr;
    bool operator==(const BatchShape& o) const {
        return n == o.n && tab == o.tab && totals == o.totals && blob == o.blob && out == o.out;
    }
};

struct BatchCtx {
    std::mutex mu;                   // one fused batch at a time (shared buffers below)
    hipStream_t stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;   // the recorded chunk of the last shape
    BatchShape graph_key;
    uint64_t graph_captures = 0, graph_launches = 0, redo_windows = 0;
    sim_batch_timing times{};        // accumulated phase times of the chunks
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    char* h_blob = nullptr;          // pinned: entries, block offsets, per-interval tables
    size_t h_cap = 0;
    char* d_blob = nullptr;
    size_t d_cap = 0;
    unsigned long long* h_out = nullptr;   // pinned readback of per-entry counters
    unsigned long long* d_out = nullptr;
    size_t out_cap = 0;
};

BatchCtx& batch_ctx() {
    static BatchCtx* ctx = new BatchCtx();   // lives until the process ends
    return *ctx;
}

size_t align8(size_t v) { return (v + 7) & ~(size_t)7; }

// Grows the context's buffers; returns false on allocation failure.
bool batch_reserve(BatchCtx& c, size_t blob, size_t outs) {
    if (!c.stream && hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess)
        return false;
    if (!c.ev_begin && hipEventCreate(&c.ev_begin) != hipSuccess) return false;
    if (!c.ev_end && hipEventCreate(&c.ev_end) != hipSuccess) return false;
    if (blob > c.h_cap || blob > c.d_cap) {
        if (hipStreamSynchronize(c.stream) != hipSuccess) return false;
        if (c.graph_exec) {   // its nodes point at the buffers being replaced
            (void)hipGraphExecDestroy(c.graph_exec);
            c.graph_exec = nullptr;
        }
        if (c.h_blob) (void)hipHostFree(c.h_blob);
        if (c.d_blob) (void)hipFree(c.d_blob);
        c.h_blob = nullptr;
        c.d_blob = nullptr;
        c.h_cap = c.d_cap = 0;
        const size_t cap = std::max(blob, (size_t)1 << 16);
        if (hipHostMalloc((void**)&c.h_blob, cap, 0) != hipSuccess) return false;
        if (hipMalloc((void**)&c.d_blob, cap) != hipSuccess) return false;
        c.h_cap = c.d_cap = cap;
    }
    if (outs > c.out_cap) {
        if (hipStreamSynchronize(c.stream) != hipSuccess) return false;
        if (c.graph_exec) {
            (void)hipGraphExecDestroy(c.graph_exec);
            c.graph_exec = nullptr;
        }
        if (c.h_out) (void)hipHostFree(c.h_out);
        if (c.d_out) (void)hipFree(c.d_out);
        c.h_out = nullptr;
        c.d_out = nullptr;
        c.out_cap = 0;
        const size_t cap = std::max(outs, (size_t)256);
        if (hipHostMalloc((void**)&c.h_out, cap * sizeof(unsigned long long), 0) != hipSuccess)
            return false;
        if (hipMalloc((void**)&c.d_out, cap * sizeof(unsigned long long)) != hipSuccess)
            return false;
        c.out_cap = cap;
    }
    return true;
}

struct FusedItem {
    sim_stream* s;
    sim_frames* it;
    const uint8_t* frames;           // the window's frames on the device
    const float* flows;              // its supplied flows (or null)
    const int64_t* t_us;
    int K;
    KeyLayout lay;
    int nbits;
    size_t tab_off;                  // offset of its tables in the blob
    uint64_t n_valid;
};

// Block offsets of one launch: start[e] = blocks of entries before e; returns the total.
int fill_starts(int* start, const std::vector<int>& blocks) {
    int acc = 0;
    for (size_t e = 0; e < blocks.size(); ++e) {
        start[e] = acc;
        acc += blocks[e];
    }
    start[blocks.size()] = acc;
    return acc;
}

// One window chunk of a batch: the streams in `items` (each with K >= 1 intervals).  Returns
// SIM_OK or the status every participating item gets.
//
// Every grid is sized on the host before any work is queued (the event arena's capacity bounds a
// window's events; the sort's grid follows a running estimate of the stream's events per window),
// so the whole chunk -- upload of the entries, clears, selection and order, chains, gather, every
// sort pass and the readback of each entry's status -- is queued with no host wait in between and
// ends with one wait.  Without estimated flow (whose launches take per-window pointers) that
// sequence is recorded once as a HIP graph per launch shape and replayed: its kernels find their
// per-window arguments in the entry blob that the graph's first node uploads from pinned memory.
// Entries whose chains ran out of arena space, or whose events outgrew the sort's grid, are
// finished afterwards by the re-run path (grow the arena, resume the unfinished chains, gather and
// sort again), which overwrites what the chunk's gather and sort wrote for them.
double ms_between(std::chrono::steady_clock::time_point a,
                  std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

int fused_window(std::vector<FusedItem>& items) {
    using clk = std::chrono::steady_clock;
    const clk::time_point t_start = clk::now();
    BatchCtx& c = batch_ctx();
    const int n = (int)items.size();
    // blob: entries | 8 offset arrays of n + 1 ints | per-item delta (K floats) + tbase (K int64)
    const size_t ent_bytes = align8((size_t)n * sizeof(BatchEntry));
    const size_t starts_bytes = align8((size_t)8 * (n + 1) * sizeof(int));
    size_t tab = ent_bytes + starts_bytes;
    for (FusedItem& f : items) {
        f.tab_off = tab;
        tab += align8((size_t)f.K * sizeof(float)) + (size_t)f.K * sizeof(int64_t);
    }
    if (!batch_reserve(c, tab, 3 * (size_t)n)) {
        (void)hipGetLastError();
        return SIM_E_NOMEM;
    }
    BatchEntry* he = (BatchEntry*)c.h_blob;
    BatchEntry* de = (BatchEntry*)c.d_blob;
    int* hs = (int*)(c.h_blob + ent_bytes);
    int* ds = (int*)(c.d_blob + ent_bytes);
    auto hstart = [&](int k) { return hs + (size_t)k * (n + 1); };
    auto dstart = [&](int k) { return ds + (size_t)k * (n + 1); };
    enum { kSel = 0, kChain0 = 1, kGather = 4, kSort = 5, kOrder = 6 };

#define BATCH_TRY(expr)                       \
    do {                                      \
        if ((expr) != hipSuccess) {           \
            (void)hipGetLastError();          \
            return SIM_E_HIP;                 \
        }                                     \
    } while (0)
    // every stream's staged inputs and earlier work are complete before the batch stream reads
    // them: the batch stream waits on the device for an event marking each distinct stream's
    // queued work (no host wait; entries that share a stream wait once)
    {
        std::vector<std::pair<hipStream_t, sim_stream*>> qs(n);
        for (int e = 0; e < n; ++e) qs[e] = {items[e].s->stream, items[e].s};
        std::sort(qs.begin(), qs.end(), [](const std::pair<hipStream_t, sim_stream*>& a,
                                           const std::pair<hipStream_t, sim_stream*>& b) {
            return (uintptr_t)a.first < (uintptr_t)b.first;
        });
        for (int e = 0; e < n; ++e) {
            if (e && qs[e].first == qs[e - 1].first) continue;
            sim_stream* s = qs[e].second;
            if (!s->ev_ready &&
                hipEventCreateWithFlags(&s->ev_ready, hipEventDisableTiming) != hipSuccess) {
                s->ev_ready = nullptr;
                (void)hipGetLastError();
                return SIM_E_HIP;
            }
            if (hipEventRecord(s->ev_ready, qs[e].first) != hipSuccess ||
                hipStreamWaitEvent(c.stream, s->ev_ready, 0) != hipSuccess) {
                (void)hipGetLastError();
                return SIM_E_HIP;
            }
        }
    }
    const clk::time_point t_inputs = clk::now();

    std::vector<int> sel_blocks(n), order_blocks(n), chain_blocks[3], gather_blocks(n),
        sort_blocks(n), blocks(n);
    std::vector<uint64_t> sort_cap(n);
    for (int m = 0; m < 3; ++m) chain_blocks[m].assign(n, 0);
    int max_stash[3] = {0, 0, 0};
    int max_nbits = 1;
    bool capturable = true;
    for (int e = 0; e < n; ++e) {
        FusedItem& f = items[e];
        sim_stream* s = f.s;
        if (s->cfg.flow_source == SIM_FLOW_LK && s->S > 1) {
            int rc = ensure_lk_buffers(s, f.K);
            if (rc) return rc;
            capturable = false;
        }
        // buffers for the most events the arena can hold, before anything changes
        const uint64_t n_max = (uint64_t)kArenaStripes * s->stripe_cap;
        // the sort's grid: twice the most events a window of this stream has had, rounded up to
        // a power of two, so that steps of a steady stream keep one launch shape (the first
        // window: the whole arena)
        uint64_t want = n_max;
        if (s->est_events) {
            want = kSortTile;
            while (want < 2 * s->est_events) want *= 2;
        }
        sort_cap[e] = std::min<uint64_t>(n_max, want);
        int rc = ensure_alt(s, n_max);
        if (!rc) rc = ensure_sort_scratch(s, n_max);
        if (!rc && s->fifo_tail + n_max > s->fifo_cap)
            rc = grow(s, &s->d_fifo, &s->fifo_cap,
                      std::max<uint64_t>(s->fifo_tail + n_max, 2 * s->fifo_cap), s->fifo_tail);
        if (rc) return rc;
        float* h_delta = (float*)(c.h_blob + f.tab_off);
        int64_t* h_tbase = (int64_t*)(c.h_blob + f.tab_off + align8((size_t)f.K * sizeof(float)));
        const float* d_delta = (const float*)(c.d_blob + f.tab_off);
        const int64_t* d_tbase =
            (const int64_t*)(c.d_blob + f.tab_off + align8((size_t)f.K * sizeof(float)));
        BatchEntry& b = he[e];
        memset(&b, 0, sizeof(b));
        rc = plan_window(s, f.frames, f.flows, f.t_us, f.K, h_delta, h_tbase, d_delta, &f.lay,
                         &f.nbits, &b.sel, &b.ord, &b.chain);
        if (rc) return rc;
        b.sparse = s->cfg.method == SIM_SPARSE ? 1 : 0;
        b.vec = (b.sel.fstride % 4) == 0 && ((uintptr_t)b.sel.frames % 4) == 0 &&
                ((uintptr_t)b.sel.prev % 4) == 0 && ((uintptr_t)b.sel.prev_out % 4) == 0;
        b.copy_src = f.frames + (size_t)(f.K - 1) * s->npix;
        b.copy_dst = b.sel.prev_out;
        if (s->cfg.method == SIM_DIFFERENCE) {
            b.copy2_src = f.K >= 2 ? f.frames + (size_t)(f.K - 2) * s->npix : s->d_prev[s->cur];
            b.copy2_dst = s->d_prev2[1 - s->cur];
        }
        b.npix = s->npix;
        b.counters = s->d_counters;
        b.gathered = s->d_alt;
        b.sort_alt = s->d_alt2;
        b.hist = s->d_hist;
        b.totals = s->d_totals;
        b.out = s->d_fifo + s->fifo_tail;
        b.cv.enabled = 1;
        b.cv.n_sentinel = s->d_counters + 1;
        b.cv.tbase = d_tbase;
        b.cv.K = f.K;
        b.cv.lay = f.lay;
        b.sort_blocks = (int)std::max<uint64_t>(1, (sort_cap[e] + kSortTile - 1) / kSortTile);
        sort_blocks[e] = b.sort_blocks;
        sel_blocks[e] = select_blocks(s->npix);
        order_blocks[e] = b.sparse ? select_blocks(s->npix) : 0;
        gather_blocks[e] =
            (int)(std::max<uint64_t>(1, (s->stripe_cap + kSortTile - 1) / kSortTile) *
                  kArenaStripes);
        const int m = b.chain.mode;
        chain_blocks[m][e] = (chain_slots(s) + kSimThreads - 1) / kSimThreads;
        max_stash[m] = std::max(max_stash[m], (s->S - 1 <= kMaxStash) ? s->S - 1 : 0);
        max_nbits = std::max(max_nbits, f.nbits);
    }
    // chain-pass variant per thresholding mode: that of the entry with the most chain slots
    // (tuned now if its key is new: its selection and order pass run alone first)
    int variant[3] = {kDefaultChainVariant, kDefaultChainVariant, kDefaultChainVariant};
    {
        int lead[3] = {-1, -1, -1};
        for (int e = 0; e < n; ++e) {
            const int m = he[e].chain.mode;
            if (lead[m] < 0 || chain_slots(items[lead[m]].s) < chain_slots(items[e].s))
                lead[m] = e;
        }
        bool uploaded = false;
        for (int m = 0; m < 3; ++m) {
            if (lead[m] < 0) continue;
            FusedItem& f = items[lead[m]];
            BatchEntry& b = he[lead[m]];
            if (!uploaded) {   // the per-interval tables the chain pass reads
                BATCH_TRY(
                    hipMemcpyAsync(c.d_blob, c.h_blob, tab, hipMemcpyHostToDevice, c.stream));
                uploaded = true;
            }
            if (b.sparse) {
                OrderArgs oa = b.ord;
                oa.stats = nullptr;   // the chunk's own order pass counts the statistics
                BATCH_TRY(launch_select(b.sel, c.stream));
                BATCH_TRY(launch_order(oa, c.stream));
            }
            variant[m] = chain_variant_for(f.s, b.chain, chain_slots(f.s), c.stream);
            f.s->last_variant = variant[m];
        }
    }
    const int sel_total = fill_starts(hstart(kSel), sel_blocks);
    const int order_total = fill_starts(hstart(kOrder), order_blocks);
    int chain_total[3];
    for (int m = 0; m < 3; ++m) chain_total[m] = fill_starts(hstart(kChain0 + m), chain_blocks[m]);
    const int gather_total = fill_starts(hstart(kGather), gather_blocks);
    const int sort_total = fill_starts(hstart(kSort), sort_blocks);
    // every entry's sort takes the batch's digit width and pass count (an entry with fewer key
    // bits takes the extra passes harmlessly)
    const int radix_bits = sort_radix_bits(max_nbits);
    const int passes = sort_passes(max_nbits);
    hipStream_t st = c.stream;
    const size_t head = ent_bytes + starts_bytes;

    // the chunk's whole device sequence (entries with fewer sort passes than `passes` take the
    // extra ones harmlessly: their keys are zero, their sentinels all ones, in those digits)
    auto enqueue = [&]() -> hipError_t {
        hipError_t r = hipMemcpyAsync(c.d_blob, c.h_blob, tab, hipMemcpyHostToDevice, st);
        if (r == hipSuccess) r = launch_batch_prep(de, n, st);
        if (r == hipSuccess) r = launch_batch_select(de, dstart(kSel), n, sel_total, st);
        if (r == hipSuccess) r = launch_batch_order(de, dstart(kOrder), n, order_total, st);
        for (FusedItem& f : items)
            if (r == hipSuccess && f.s->cfg.flow_source == SIM_FLOW_LK && f.s->S > 1)
                r = launch_lk(f.s, f.frames, f.K, st);
        for (int m = 0; m < 3 && r == hipSuccess; ++m)
            r = launch_batch_chain(de, dstart(kChain0 + m), n, chain_total[m], m, max_stash[m],
                                   variant[m], st);
        if (r == hipSuccess) r = launch_batch_gather(de, dstart(kGather), n, gather_total, st);
        if (r == hipSuccess)
            r = launch_batch_sort(de, dstart(kSort), n, sort_total, passes, radix_bits, st);
        if (r == hipSuccess) r = launch_batch_status(de, n, c.d_out, st);
        if (r == hipSuccess)
            r = hipMemcpyAsync(c.h_out, c.d_out, 3 * (size_t)n * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st);
        return r;
    };
    const clk::time_point t_plan = clk::now();
    BATCH_TRY(hipEventRecord(c.ev_begin, st));
    if (capturable) {
        BatchShape key;
        key.n = n;
        key.tab = tab;
        key.totals = {sel_total,    order_total,   chain_total[0],          chain_total[1],
                      chain_total[2], gather_total, sort_total, passes * 16 + radix_bits,
                      max_stash[0], max_stash[1],  max_stash[2],  variant[0],
                      variant[1],   variant[2]};
        key.blob = c.d_blob;
        key.out = c.d_out;
        if (!(c.graph_exec && c.graph_key == key)) {
            if (c.graph_exec) {
                (void)hipGraphExecDestroy(c.graph_exec);
                c.graph_exec = nullptr;
            }
            hipGraph_t g = nullptr;
            BATCH_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const hipError_t er = enqueue();
            const hipError_t ee = hipStreamEndCapture(st, &g);
            if (er != hipSuccess || ee != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                return SIM_E_HIP;
            }
            const hipError_t ei = hipGraphInstantiate(&c.graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) {
                c.graph_exec = nullptr;
                (void)hipGetLastError();
                return SIM_E_HIP;
            }
            c.graph_key = key;
            c.graph_captures++;
        }
        BATCH_TRY(hipGraphLaunch(c.graph_exec, st));
        c.graph_launches++;
    } else {
        BATCH_TRY(enqueue());
    }
    BATCH_TRY(hipEventRecord(c.ev_end, st));
    const clk::time_point t_launch = clk::now();
    BATCH_TRY(hipStreamSynchronize(st));
    const clk::time_point t_wait = clk::now();
    float dev_ms = 0.f;
    if (hipEventElapsedTime(&dev_ms, c.ev_begin, c.ev_end) != hipSuccess) {
        (void)hipGetLastError();
        dev_ms = 0.f;
    }

    // entries that need the re-run path: chains out of arena space, or more events than the
    // sort's grid covered
    std::vector<int> redo;
    for (int e = 0; e < n; ++e) {
        he[e].clamp_cap = 0;
        const unsigned long long fails = c.h_out[3 * e], gathered = c.h_out[3 * e + 2];
        if (fails != 0 || gathered > sort_cap[e]) redo.push_back(e);
    }
    if (!redo.empty()) {
        // chains that ran out of event-buffer space: grow those buffers, re-run only them
        for (;;) {
            bool any = false;
            for (int m = 0; m < 3; ++m) std::fill(chain_blocks[m].begin(), chain_blocks[m].end(), 0);
            for (int e : redo) {
                he[e].clamp_cap = 0;
                if (c.h_out[3 * e] == 0) continue;
                any = true;
                sim_stream* s = items[e].s;
                const uint64_t old = s->stripe_cap;
                int rc = grow_arena(s, 2 * old);
                if (rc) return fail_mid_push(s, rc, "event arena growth");
                s->stats.retries++;
                he[e].clamp_cap = old;
                he[e].chain.arena = s->d_arena;
                he[e].chain.stripe_cap = s->stripe_cap;
                chain_blocks[he[e].chain.mode][e] = (chain_slots(s) + kSimThreads - 1) / kSimThreads;
            }
            if (!any) break;
            for (int m = 0; m < 3; ++m)
                chain_total[m] = fill_starts(hstart(kChain0 + m), chain_blocks[m]);
            BATCH_TRY(hipMemcpyAsync(c.d_blob, c.h_blob, head, hipMemcpyHostToDevice, st));
            BATCH_TRY(launch_batch_clamp(de, n, st));
            for (int m = 0; m < 3; ++m)
                BATCH_TRY(launch_batch_chain(de, dstart(kChain0 + m), n, chain_total[m], m,
                                             max_stash[m], variant[m], st));
            BATCH_TRY(launch_batch_status(de, n, c.d_out, st));
            BATCH_TRY(hipMemcpyAsync(c.h_out, c.d_out, 3 * (size_t)n * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, st));
            BATCH_TRY(hipStreamSynchronize(st));
        }
        // every chain has finished: gather and sort the re-run entries again, grids from counts
        std::fill(blocks.begin(), blocks.end(), 0);
        for (int e : redo) {
            sim_stream* s = items[e].s;
            int rc = ensure_alt(s, kArenaStripes * s->stripe_cap);
            if (rc) return fail_mid_push(s, rc, "sort buffer growth");
            he[e].clamp_cap = 0;
            he[e].gathered = s->d_alt;
            he[e].sort_alt = s->d_alt2;
            blocks[e] = (int)(std::max<uint64_t>(1, (s->stripe_cap + kSortTile - 1) / kSortTile) *
                              kArenaStripes);
        }
        const int gt = fill_starts(hstart(kGather), blocks);
        BATCH_TRY(hipMemcpyAsync(c.d_blob, c.h_blob, head, hipMemcpyHostToDevice, st));
        BATCH_TRY(launch_batch_gather(de, dstart(kGather), n, gt, st));
        BATCH_TRY(launch_batch_status(de, n, c.d_out, st));
        BATCH_TRY(hipMemcpyAsync(c.h_out, c.d_out, 3 * (size_t)n * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st));
        BATCH_TRY(hipStreamSynchronize(st));
        std::fill(blocks.begin(), blocks.end(), 0);
        int rnbits = 1;
        for (int e : redo) {
            FusedItem& f = items[e];
            sim_stream* s = f.s;
            const uint64_t n_total = c.h_out[3 * e + 2];
            int rc = ensure_sort_scratch(s, n_total);
            if (!rc && s->fifo_tail + n_total > s->fifo_cap)
                rc = grow(s, &s->d_fifo, &s->fifo_cap,
                          std::max<uint64_t>(s->fifo_tail + n_total, 2 * s->fifo_cap),
                          s->fifo_tail);
            if (rc) return fail_mid_push(s, rc, "event buffer growth");
            BatchEntry& b = he[e];
            b.hist = s->d_hist;
            b.out = s->d_fifo + s->fifo_tail;
            b.sort_blocks = (int)std::max<uint64_t>(1, (n_total + kSortTile - 1) / kSortTile);
            blocks[e] = b.sort_blocks;
            rnbits = std::max(rnbits, f.nbits);
        }
        const int rt = fill_starts(hstart(kSort), blocks);
        BATCH_TRY(hipMemcpyAsync(c.d_blob, c.h_blob, head, hipMemcpyHostToDevice, st));
        BATCH_TRY(launch_batch_sort(de, dstart(kSort), n, rt, sort_passes(rnbits),
                                    sort_radix_bits(rnbits), st));
        BATCH_TRY(hipStreamSynchronize(st));
        c.redo_windows += redo.size();
    }
#undef BATCH_TRY
    for (int e = 0; e < n; ++e) {
        FusedItem& f = items[e];
        sim_stream* s = f.s;
        const uint64_t n_total = c.h_out[3 * e + 2];
        f.n_valid = n_total - c.h_out[3 * e + 1];
        s->est_events = std::max<uint64_t>(s->est_events, n_total);
        s->fifo_tail += f.n_valid;
        s->cur = 1 - s->cur;
        s->t_prev = f.t_us[f.K - 1];
        s->n_int += (uint64_t)f.K;
        s->stats.intervals += (uint64_t)f.K;
        s->stats.frames += (uint64_t)f.K;
        s->stats.events += f.n_valid;
        f.it->n_new_events += f.n_valid;
    }
    sim_batch_timing& tm = c.times;
    tm.chunks++;
    tm.inputs_ms += ms_between(t_start, t_inputs);
    tm.plan_ms += ms_between(t_inputs, t_plan);
    tm.launch_ms += ms_between(t_plan, t_launch);
    tm.wait_ms += ms_between(t_launch, t_wait);
    tm.finish_ms += ms_between(t_wait, clk::now());
    tm.device_ms += dev_ms;
    return SIM_OK;
}

}  // namespace

// The window loop of a batched push: chunk by chunk, every stream's window of the chunk runs in
// the fused launches.  A failure poisons the streams of its chunk (their device state may have
// advanced); the others go on.  *chunk receives the first interval of the chunk being run.  May
// throw std::bad_alloc.
void batch_windows(sim_stream** streams, sim_frames* items, const std::vector<Staged>& st, int n,
                   int max_int, int* chunk) {
    std::lock_guard<std::mutex> lock(batch_ctx().mu);
    for (int j = 0; j < max_int; j += kMaxWindow) {
        *chunk = j;
        std::vector<FusedItem> fi;
        for (int i = 0; i < n; ++i) {
            sim_frames& it = items[i];
            if (it.status || j >= st[i].n_int) continue;
            FusedItem f;
            memset(&f, 0, sizeof(f));
            f.s = streams[i];
            f.it = &it;
            f.K = std::min(kMaxWindow, st[i].n_int - j);
            it.status = stage_window(streams[i], st[i], j, f.K, &f.frames, &f.flows);
            if (it.status) continue;
            f.t_us = it.t_us + st[i].first + j;
            fi.push_back(f);
        }
        if (fi.empty()) continue;
        const int rc = fused_window(fi);
        if (rc) {
            // device state of the chunk's streams may have advanced: they cannot continue
            for (FusedItem& f : fi) {
                f.it->status = rc;
                f.s->poisoned = true;
                if (!f.s->last_error[0])
                    snprintf(f.s->last_error, sizeof(f.s->last_error),
                             "batched push failed (%s)", sim_strerror(rc));
            }
        }
    }
}

// Fixed device scratch of sim_lk_flow_noalloc (the two pyramids of one call), for callers that
// cannot allocate.  Every GPU the library runs on holds its own copy from module load until the
// process ends; host code reaches it only through the address hipGetSymbolAddress returns for
// the current device (the array's name is a host-side stand-in, not a device address).
constexpr uint64_t kLkScratchFloats = 6ull << 20;   // 24 MiB: two 1920x1080 pyramids, any depth
static __device__ __align__(256) float scratch[kLkScratchFloats];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int lk_scratch_of_current_device(float** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        (void)hipGetLastError();
        return SIM_E_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return SIM_E_HIP;
        }
        g_scratch_dev[dev] = (float*)ptr;
    }
    *out = g_scratch_dev[dev];
    return SIM_OK;
}

}  // namespace

extern "C" {

void sim_config_init(sim_config* cfg) {
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->method = SIM_BASIC;
    cfg->transform = SIM_LOG;
    cfg->c_pos = 0.2f;
    cfg->c_neg = 0.2f;
    cfg->log_eps = 1e-3f;
    cfg->n_interp = 10;
    cfg->mask_threshold = -1.0f;
    cfg->event_capacity = 0;
    cfg->hip_stream = nullptr;
}

const char* sim_strerror(int status) {
    switch (status) {
        case SIM_OK: return "ok";
        case SIM_E_INVAL: return "invalid argument";
        case SIM_E_ORDER: return "frame timestamps must strictly increase";
        case SIM_E_NOMEM: return "out of memory";
        case SIM_E_RANGE: return "value out of range";
        case SIM_E_HIP: return "HIP runtime error (handle poisoned)";
        case SIM_E_POISONED: return "handle poisoned by an earlier HIP error";
        case SIM_E_BUSY: return "no capacity for the request";
        case SIM_E_EMPTY: return "nothing available";
        case SIM_E_TOO_BIG: return "request exceeds the fixed scratch of the non-allocating call";
        default: return "unknown status";
    }
}

int sim_create(const sim_config* cfg, sim_stream** out) {
    if (!cfg || !out) return SIM_E_INVAL;
    *out = nullptr;
    if (cfg->width < 1 || cfg->height < 1 || cfg->width > 4096 || cfg->height > 4096)
        return SIM_E_INVAL;
    if (cfg->method < SIM_BASIC || cfg->method > SIM_DIFFERENCE) return SIM_E_INVAL;
    if (cfg->thresh_mode != SIM_THRESH_REFERENCE && cfg->thresh_mode != SIM_THRESH_MEMORYLESS)
        return SIM_E_INVAL;
    if (cfg->flow_source != SIM_FLOW_SUPPLIED && cfg->flow_source != SIM_FLOW_LK)
        return SIM_E_INVAL;
    if (cfg->flow_source == SIM_FLOW_LK && cfg->method != SIM_DENSE &&
        cfg->method != SIM_SPARSE)
        return SIM_E_INVAL;
    if (cfg->transform != SIM_LOG && cfg->transform != SIM_LINEAR) return SIM_E_INVAL;
    if (!(cfg->c_pos > 0.0f) || !(cfg->c_neg > 0.0f) || !isfinite(cfg->c_pos) ||
        !isfinite(cfg->c_neg))
        return SIM_E_INVAL;
    if (cfg->transform == SIM_LOG && !(cfg->log_eps > 0.0f && isfinite(cfg->log_eps)))
        return SIM_E_INVAL;
    if (cfg->n_interp < 0 || cfg->n_interp > 255) return SIM_E_INVAL;
    if (isnan(cfg->mask_threshold)) return SIM_E_INVAL;

    sim_stream* s = new (std::nothrow) sim_stream();
    if (!s) return SIM_E_NOMEM;
    s->cfg = *cfg;
    build_lut(s);
    // The crossing loop advances R by C each step; C must be large enough that R + C != R for
    // every level the loop can reach (|R| <= max|T| + C).
    float maxabs = 0.0f;
    for (int v = 0; v < 256; ++v) maxabs = std::max(maxabs, fabsf(s->lut_host[v]));
    const float cmin = (maxabs + 1.0f) * ldexpf(1.0f, -20);
    if (cfg->c_pos < cmin || cfg->c_neg < cmin) {
        delete s;
        return SIM_E_INVAL;
    }
    s->S = cfg->method == SIM_BASIC ? 1 : cfg->n_interp + 1;
    // With a reference level one pixel may fire at most kMaxLaneCount events per interval.  Above
    // cmin a level step loses less than C/8 to rounding and R stays within C/8 of the samples, so
    // one sub-interval fires at most 2 (max T - min T) / C + 3 events.
    if (cfg->thresh_mode == SIM_THRESH_REFERENCE && cfg->method != SIM_DIFFERENCE) {
        float tmin = s->lut_host[0], tmax = s->lut_host[0];
        for (int v = 1; v < 256; ++v) {
            tmin = std::min(tmin, s->lut_host[v]);
            tmax = std::max(tmax, s->lut_host[v]);
        }
        const double c = std::min(cfg->c_pos, cfg->c_neg);
        const double per_interval = (double)s->S * (2.0 * ((double)tmax - tmin) / c + 3.0);
        if (per_interval > (double)kMaxLaneCount) {
            delete s;
            return SIM_E_INVAL;
        }
    }
    s->m = cfg->mask_threshold < 0.0f ? std::min(cfg->c_pos, cfg->c_neg) : cfg->mask_threshold;
    s->npix = (int64_t)cfg->width * cfg->height;
    {
        sim_lk_params d;
        sim_lk_params_init(&d);
        s->lk = lk_from(d);
    }
    memset(&s->stats, 0, sizeof(s->stats));

    bool ok = true;
    if (cfg->hip_stream) {
        s->stream = (hipStream_t)cfg->hip_stream;
    } else {
        ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
        s->own_stream = ok;
    }
    uint64_t cap0 = cfg->event_capacity ? cfg->event_capacity : 2 * (uint64_t)s->npix;
    s->stripe_cap = std::max<uint64_t>(1, (cap0 + kArenaStripes - 1) / kArenaStripes);
    if (s->stripe_cap * kArenaStripes >= kArenaKeyLimit) {
        delete s;
        return SIM_E_INVAL;
    }
    const int sel_blocks = (int)((s->npix + kSelectPx - 1) / kSelectPx);
    const size_t slots = (size_t)s->npix;
    ok = ok && dev_alloc(&s->d_lut, 256) == hipSuccess;
    ok = ok && dev_alloc(&s->d_lref, s->npix) == hipSuccess;
    ok = ok && dev_alloc(&s->d_prev[0], s->npix) == hipSuccess;
    ok = ok && dev_alloc(&s->d_prev[1], s->npix) == hipSuccess;
    ok = ok && dev_alloc(&s->d_arena, s->stripe_cap * kArenaStripes) == hipSuccess;
    ok = ok && dev_alloc(&s->d_reserve, (size_t)kArenaStripes * kCounterStride) == hipSuccess;
    ok = ok && dev_alloc(&s->d_stats, (size_t)kStatStripes * kCounterStride) == hipSuccess;
    ok = ok && dev_alloc(&s->d_totals, kRadixDigits) == hipSuccess;
    ok = ok && dev_alloc(&s->d_counters, 4) == hipSuccess;
    if (cfg->method == SIM_DIFFERENCE) {
        ok = ok && dev_alloc(&s->d_prev2[0], s->npix) == hipSuccess;
        ok = ok && dev_alloc(&s->d_prev2[1], s->npix) == hipSuccess;
    }
    if (cfg->method == SIM_SPARSE) {
        ok = ok && dev_alloc(&s->d_mask, (size_t)kMaskWords * s->npix) == hipSuccess;
        ok = ok && dev_alloc(&s->d_act, (size_t)sel_blocks * kSelectPx) == hipSuccess;
        ok = ok && dev_alloc(&s->d_olist, olist_words(s->npix)) == hipSuccess;
        ok = ok && dev_alloc(&s->d_ord, (size_t)s->npix) == hipSuccess;
    }
    ok = ok && dev_alloc(&s->d_delta, kMaxWindow) == hipSuccess;
    ok = ok && dev_alloc(&s->d_tbase, kMaxWindow) == hipSuccess;
    ok = ok && dev_alloc(&s->d_resume, slots) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->h_counters, 4 * sizeof(unsigned long long), 0) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->h_stats,
                             (size_t)kStatStripes * kCounterStride * sizeof(unsigned long long),
                             0) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->h_delta, kMaxWindow * sizeof(float), 0) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->h_tbase, kMaxWindow * sizeof(int64_t), 0) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_stream(s);
        return SIM_E_NOMEM;
    }
    if (hipMemcpyAsync(s->d_lut, s->lut_host, sizeof(s->lut_host), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess ||
        launch_zero(s->d_stats,
                    (size_t)kStatStripes * kCounterStride * sizeof(unsigned long long),
                    s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        free_stream(s);
        return SIM_E_HIP;
    }
    s->stats.event_capacity = s->stripe_cap * kArenaStripes;
    *out = s;
    return SIM_OK;
}

int sim_destroy(sim_stream* s) {
    if (!s) return SIM_E_INVAL;
    free_stream(s);
    return SIM_OK;
}

int sim_reset(sim_stream* s) {
    if (!s) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->started = false;
    s->fifo_head = s->fifo_tail = 0;
    return SIM_OK;
}

int sim_clear_stats(sim_stream* s) {
    if (!s) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    HIP_TRY(s, launch_zero(s->d_stats,
                           (size_t)kStatStripes * kCounterStride * sizeof(unsigned long long),
                           s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    memset(&s->stats, 0, sizeof(s->stats));
    s->stats.event_capacity = s->stripe_cap * kArenaStripes;
    return SIM_OK;
}

int sim_push_frames(sim_stream* s, int32_t n_frames, const uint8_t* frames, const float* flows,
                    const int64_t* t_us, int32_t mem_kind, uint64_t* n_new_events) {
    if (n_new_events) *n_new_events = 0;
    int rc = push_validate(s, n_frames, frames, flows, t_us, mem_kind);
    if (rc) return rc;
    Staged st;
    rc = push_stage(s, n_frames, frames, flows, t_us, mem_kind, &st);
    if (rc) return rc;
    uint64_t total = 0;
    for (int j = 0; j < st.n_int; j += kMaxWindow) {
        const int K = std::min(kMaxWindow, st.n_int - j);
        uint64_t nn = 0;
        const uint8_t* wf = nullptr;
        const float* wfl = nullptr;
        rc = stage_window(s, st, j, K, &wf, &wfl);
        if (!rc) rc = run_window(s, wf, wfl, t_us + st.first + j, K, &nn);
        if (rc) return rc;
        total += nn;
    }
    if (n_new_events) *n_new_events = total;
    return SIM_OK;
}

int sim_push_batch(sim_stream** streams, sim_frames* items, int32_t n) {
    if (!streams || !items || n < 0) return SIM_E_INVAL;
    // validate everything (and reject a handle listed twice) before queueing any work
    int first_err = SIM_OK;
    for (int i = 0; i < n; ++i) {
        items[i].n_new_events = 0;
        items[i].status = push_validate(streams[i], items[i].n_frames, items[i].frames,
                                        items[i].flows, items[i].t_us, items[i].mem_kind);
        for (int j = 0; j < i && items[i].status == SIM_OK; ++j)
            if (streams[j] == streams[i]) items[i].status = SIM_E_INVAL;
        if (items[i].status && !first_err) first_err = items[i].status;
    }
    if (first_err) return first_err;
    std::vector<Staged> st;
    try {
        st.resize(n);
    } catch (...) {
        return SIM_E_NOMEM;   // nothing has changed yet
    }
    int max_int = 0;
    for (int i = 0; i < n; ++i) {
        sim_frames& it = items[i];
        it.status = push_stage(streams[i], it.n_frames, it.frames, it.flows, it.t_us, it.mem_kind,
                               &st[i]);
        if (it.status && !first_err) first_err = it.status;
        if (!it.status) max_int = std::max(max_int, st[i].n_int);
    }
    int chunk = 0;
    try {
        batch_windows(streams, items, st, n, max_int, &chunk);
    } catch (...) {
        // host memory ran out: a staged stream with a window in this chunk or later may have
        // advanced part of the way
        for (int i = 0; i < n; ++i) {
            if (items[i].status || st[i].n_int <= chunk) continue;
            items[i].status = SIM_E_NOMEM;
            streams[i]->poisoned = true;
            if (!streams[i]->last_error[0])
                snprintf(streams[i]->last_error, sizeof(streams[i]->last_error),
                         "batched push failed (host allocation)");
        }
    }
    for (int i = 0; i < n; ++i)
        if (items[i].status && !first_err) first_err = items[i].status;
    return first_err;
}

int sim_set_chain_variant(sim_stream* s, int32_t variant) {
    if (!s || variant < -1 || variant >= kChainVariants) return SIM_E_INVAL;
    s->forced_variant = variant;
    return SIM_OK;
}

int sim_get_chain_variant(sim_stream* s, int32_t* variant) {
    if (!s || !variant) return SIM_E_INVAL;
    *variant = s->last_variant;
    return SIM_OK;
}

int sim_batch_stats(uint64_t* graphs_recorded, uint64_t* graph_launches, uint64_t* rerun_windows) {
    BatchCtx& c = batch_ctx();
    std::lock_guard<std::mutex> lock(c.mu);
    if (graphs_recorded) *graphs_recorded = c.graph_captures;
    if (graph_launches) *graph_launches = c.graph_launches;
    if (rerun_windows) *rerun_windows = c.redo_windows;
    return SIM_OK;
}

int sim_batch_times(sim_batch_timing* out) {
    if (!out) return SIM_E_INVAL;
    BatchCtx& c = batch_ctx();
    std::lock_guard<std::mutex> lock(c.mu);
    *out = c.times;
    return SIM_OK;
}

int sim_push_frame(sim_stream* s, const uint8_t* frame, const float* flow, int64_t t_us,
                   int32_t mem_kind, uint64_t* n_new_events) {
    return sim_push_frames(s, 1, frame, flow, &t_us, mem_kind, n_new_events);
}

int sim_pending_events(sim_stream* s, uint64_t* n) {
    if (!s || !n) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    *n = s->fifo_tail - s->fifo_head;
    return SIM_OK;
}

int sim_drain_keys(sim_stream* s, uint64_t* dst, uint64_t max_events, int32_t mem_kind,
                   uint64_t* n_written) {
    if (!s || (!dst && max_events) || check_mem_kind(mem_kind)) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    const uint64_t n = std::min(max_events, s->fifo_tail - s->fifo_head);
    if (n) {
        HIP_TRY(s, hipMemcpyAsync(dst, s->d_fifo + s->fifo_head, n * sizeof(uint64_t),
                                  mem_kind == SIM_MEM_HOST ? hipMemcpyDeviceToHost
                                                           : hipMemcpyDeviceToDevice,
                                  s->stream));
        HIP_TRY(s, hipStreamSynchronize(s->stream));
    }
    s->fifo_head += n;
    if (s->fifo_head == s->fifo_tail) s->fifo_head = s->fifo_tail = 0;
    if (n_written) *n_written = n;
    return SIM_OK;
}

int sim_drain_events(sim_stream* s, sim_event* dst, uint64_t max_events, uint64_t* n_written) {
    if (!s || (!dst && max_events)) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    const uint64_t n = std::min(max_events, s->fifo_tail - s->fifo_head);
    // keys come over in chunks, so the host buffer stays small whatever the count
    std::vector<uint64_t> keys;
    try {
        keys.resize((size_t)std::min<uint64_t>(n, 1u << 20));
    } catch (...) {
        return SIM_E_NOMEM;
    }
    uint64_t done = 0;
    while (done < n) {
        uint64_t got = 0;
        int rc = sim_drain_keys(s, keys.data(), std::min<uint64_t>(n - done, keys.size()),
                                SIM_MEM_HOST, &got);
        if (rc) {
            if (n_written) *n_written = done;
            return rc;
        }
        if (got == 0) break;
        for (uint64_t j = 0; j < got; ++j) {
            const uint64_t k = keys[j];
            sim_event& e = dst[done + j];
            e.t_us = s->epoch + (int64_t)(k >> 25);
            e.y = (uint16_t)((k >> 13) & 0xFFF);
            e.x = (uint16_t)((k >> 1) & 0xFFF);
            e.p = (k & 1) ? 1 : -1;
            e.pad[0] = e.pad[1] = e.pad[2] = 0;
        }
        done += got;
    }
    if (n_written) *n_written = done;
    return SIM_OK;
}

int sim_epoch(sim_stream* s, int64_t* epoch) {
    if (!s || !epoch) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    if (!s->started) return SIM_E_INVAL;
    *epoch = s->epoch;
    return SIM_OK;
}

int sim_get_reference(sim_stream* s, float* dst, int32_t mem_kind) {
    if (!s || !dst || check_mem_kind(mem_kind)) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    HIP_TRY(s, hipMemcpyAsync(dst, s->d_lref, (size_t)s->npix * sizeof(float),
                              mem_kind == SIM_MEM_HOST ? hipMemcpyDeviceToHost
                                                       : hipMemcpyDeviceToDevice,
                              s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return SIM_OK;
}

namespace {

// Window [t_begin, t_end) in the key's time field (t - epoch); false when it holds no key time.
bool key_window(const sim_stream* s, int64_t t_begin, int64_t t_end, uint64_t* lo, uint64_t* hi) {
    if (!s->started || t_end <= s->epoch || t_end <= t_begin) return false;
    *lo = t_begin > s->epoch ? (uint64_t)(t_begin - s->epoch) : 0;
    *hi = (uint64_t)(t_end - s->epoch);
    return *lo < *hi;
}

}  // namespace

int sim_accumulate(sim_stream* s, int64_t t_begin, int64_t t_end, uint32_t* counts,
                   int32_t mem_kind) {
    if (!s || !counts || t_end < t_begin || check_mem_kind(mem_kind)) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    uint64_t lo = 0, hi = 0;
    const uint64_t n = s->fifo_tail - s->fifo_head;
    if (n == 0 || !key_window(s, t_begin, t_end, &lo, &hi)) return SIM_OK;
    const size_t bytes = 2 * (size_t)s->npix * sizeof(uint32_t);
    uint32_t* dst = counts;
    if (mem_kind == SIM_MEM_HOST) {
        int rc = grow(s, &s->d_acc, &s->acc_cap, 2 * (uint64_t)s->npix, 0);
        if (rc) return rc;
        HIP_TRY(s, hipMemcpyAsync(s->d_acc, counts, bytes, hipMemcpyHostToDevice, s->stream));
        dst = s->d_acc;
    }
    HIP_TRY(s, launch_accumulate(s->d_fifo + s->fifo_head, n, lo, hi, s->cfg.width,
                                 s->cfg.height, dst, s->stream));
    if (mem_kind == SIM_MEM_HOST) {
        HIP_TRY(s, hipMemcpyAsync(counts, s->d_acc, bytes, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(s, hipStreamSynchronize(s->stream));
    }
    return SIM_OK;
}

int sim_event_rate(sim_stream* s, int64_t t_begin, int64_t t_end, double* mean, double* stddev,
                   uint64_t* sums) {
    if (!s || !mean || !stddev || t_end <= t_begin) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    const uint64_t plane = (uint64_t)s->npix;
    int rc = grow(s, &s->d_acc, &s->acc_cap, 2 * plane, 0);
    if (!rc) rc = grow(s, &s->d_moments, &s->moments_cap, 2 * (uint64_t)moments_blocks(plane), 0);
    if (rc) return rc;
    HIP_TRY(s, launch_zero(s->d_acc, 2 * plane * sizeof(uint32_t), s->stream));
    uint64_t lo = 0, hi = 0;
    const uint64_t n = s->fifo_tail - s->fifo_head;
    if (n && key_window(s, t_begin, t_end, &lo, &hi))
        HIP_TRY(s, launch_accumulate(s->d_fifo + s->fifo_head, n, lo, hi, s->cfg.width,
                                     s->cfg.height, s->d_acc, s->stream));
    HIP_TRY(s, launch_moments(s->d_acc, plane, s->d_moments, s->stream));
    const int nb = moments_blocks(plane);
    std::vector<unsigned long long> part;
    try {
        part.resize(2 * (size_t)nb);
    } catch (...) {
        return SIM_E_NOMEM;
    }
    HIP_TRY(s, hipMemcpyAsync(part.data(), s->d_moments, part.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    uint64_t s1 = 0, s2 = 0;
    for (int b = 0; b < nb; ++b) {
        s1 += part[2 * b];
        s2 += part[2 * b + 1];
    }
    const double seconds = (double)(t_end - t_begin) * 1e-6;
    const double m1 = (double)s1 / (double)plane;
    const double m2 = (double)s2 / (double)plane;
    const double var = m2 - m1 * m1;
    *mean = m1 / seconds;
    *stddev = sqrt(var > 0.0 ? var : 0.0) / seconds;
    if (sums) {
        sums[0] = s1;
        sums[1] = s2;
    }
    return SIM_OK;
}

void sim_lk_params_init(sim_lk_params* p) {
    if (!p) return;
    p->levels = 3;
    p->radius = 7;
    p->iterations = 10;
    p->eps = 1e-4f;
    p->min_trace = 1.0f;
    p->min_ratio = 1e-3f;
}

int sim_set_lk_params(sim_stream* s, const sim_lk_params* p) {
    if (!s || !p || !lk_ok(*p)) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    s->lk = lk_from(*p);
    return SIM_OK;
}

int sim_lk_flow(const uint8_t* f0, const uint8_t* f1, int32_t width, int32_t height,
                const uint32_t* points, uint64_t n_points, float* flow, uint8_t* valid,
                const sim_lk_params* params, int32_t mem_kind, void* hip_stream) {
    sim_lk_params P;
    if (params)
        P = *params;
    else
        sim_lk_params_init(&P);
    if (!lk_ok(P) || width < 1 || height < 1 || width > 4096 || height > 4096 ||
        check_mem_kind(mem_kind))
        return SIM_E_INVAL;
    if (n_points == 0) return SIM_OK;
    if (!f0 || !f1 || !points || !flow) return SIM_E_INVAL;
    const bool host = mem_kind == SIM_MEM_HOST;
    const size_t npix = (size_t)width * (size_t)height;
    const PyrLayout pl = pyr_layout(width, height, P.levels);
    hipStream_t st = (hipStream_t)hip_stream;
    bool own = false;
    if (!st) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return SIM_E_HIP;
        }
        own = true;
    }
    float* d_pyr = nullptr;
    uint8_t* d_frames = nullptr;
    uint32_t* d_pts = nullptr;
    float* d_flow = nullptr;
    uint8_t* d_valid = nullptr;
    int rc = SIM_OK;
    bool ok = dev_alloc(&d_pyr, 2 * pl.total) == hipSuccess;
    if (ok && host) {
        ok = dev_alloc(&d_frames, 2 * npix) == hipSuccess &&
             dev_alloc(&d_pts, n_points) == hipSuccess &&
             dev_alloc(&d_flow, 2 * n_points) == hipSuccess &&
             (!valid || dev_alloc(&d_valid, n_points) == hipSuccess);
    }
    if (!ok) {
        (void)hipGetLastError();
        rc = SIM_E_NOMEM;
    }
    const uint8_t* a = f0;
    const uint8_t* b = f1;
    const uint32_t* pts = points;
    float* fl = flow;
    uint8_t* va = valid;
    if (!rc && host) {
        a = d_frames;
        b = d_frames + npix;
        pts = d_pts;
        fl = d_flow;
        va = d_valid;
        if (hipMemcpyAsync(d_frames, f0, npix, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(d_frames + npix, f1, npix, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(d_pts, points, n_points * sizeof(uint32_t), hipMemcpyHostToDevice,
                           st) != hipSuccess)
            rc = SIM_E_HIP;
    }
    if (!rc && (launch_pyramids(a, nullptr, 0, 1, pl, d_pyr, st) != hipSuccess ||
                launch_pyramids(b, nullptr, 0, 1, pl, d_pyr + pl.total, st) != hipSuccess ||
                launch_lk_points(d_pyr, d_pyr + pl.total, pl, lk_from(P), pts, n_points, fl, va,
                                 st) != hipSuccess))
        rc = SIM_E_HIP;
    if (!rc && host) {
        if (hipMemcpyAsync(flow, d_flow, 2 * n_points * sizeof(float), hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            (valid && hipMemcpyAsync(valid, d_valid, n_points, hipMemcpyDeviceToHost, st) !=
                          hipSuccess))
            rc = SIM_E_HIP;
    }
    if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = SIM_E_HIP;
    if (rc == SIM_E_HIP) (void)hipGetLastError();
    dfree(d_pyr);
    dfree(d_frames);
    dfree(d_pts);
    dfree(d_flow);
    dfree(d_valid);
    if (own) (void)hipStreamDestroy(st);
    return rc;
}

int sim_lk_flow_noalloc(const uint8_t* f0, const uint8_t* f1, int32_t width, int32_t height,
                        const uint32_t* points, uint64_t n_points, float* flow, uint8_t* valid,
                        const sim_lk_params* params, void* hip_stream) {
    sim_lk_params P;
    if (params)
        P = *params;
    else
        sim_lk_params_init(&P);
    if (!lk_ok(P) || width < 1 || height < 1 || width > 4096 || height > 4096)
        return SIM_E_INVAL;
    if (n_points == 0) return SIM_OK;
    if (!f0 || !f1 || !points || !flow) return SIM_E_INVAL;
    const PyrLayout pl = pyr_layout(width, height, P.levels);
    if (2 * pl.total > kLkScratchFloats) return SIM_E_TOO_BIG;
    float* pyr = nullptr;
    int rc = lk_scratch_of_current_device(&pyr);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if (launch_pyramids(f0, nullptr, 0, 1, pl, pyr, st) != hipSuccess ||
        launch_pyramids(f1, nullptr, 0, 1, pl, pyr + pl.total, st) != hipSuccess ||
        launch_lk_points(pyr, pyr + pl.total, pl, lk_from(P), points, n_points, flow, valid,
                         st) != hipSuccess) {
        (void)hipGetLastError();
        return SIM_E_HIP;
    }
    return SIM_OK;
}

int sim_sync(sim_stream* s) {
    if (!s) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return SIM_OK;
}

const char* sim_last_error(sim_stream* s) {
    if (!s) return "";
    return s->last_error;
}

int sim_get_stats(sim_stream* s, sim_stats* out) {
    if (!s || !out) return SIM_E_INVAL;
    *out = s->stats;
    if (!s->poisoned && s->cfg.method == SIM_SPARSE) {
        // the whole striped block (16 KiB) in one plain copy to pinned memory
        HIP_TRY(s, hipMemcpyAsync(s->h_stats, s->d_stats,
                                  (size_t)kStatStripes * kCounterStride *
                                      sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        uint64_t tot = 0, act = 0;
        for (int i = 0; i < kStatStripes; ++i) {
            tot += s->h_stats[(size_t)i * kCounterStride];
            act += s->h_stats[(size_t)i * kCounterStride + 1];
        }
        out->selected = tot;
        out->active = act;
    }
    return SIM_OK;
}

int sim_set_kernel_timing(sim_stream* s, int32_t enable) {
    if (!s) return SIM_E_INVAL;
    if (s->poisoned) return SIM_E_POISONED;
    if (enable && !s->ev[0]) {
        for (hipEvent_t& e : s->ev) HIP_TRY(s, hipEventCreate(&e));
    }
    s->timing = enable != 0;
    return SIM_OK;
}

}  // extern "C"
