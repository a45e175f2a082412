/*
 * sim.h -- C ABI of the MI355X event simulator (libevsim.so).
 *
 * The library turns camera frames into the events an event camera would have produced between
 * them, following Ziegler et al., "Real-time event simulation with frame-based cameras"
 * (arXiv 2209.04634):
 *   - inputs are consecutive grayscale camera frames taken at t_{i-1} and t_i (Sec. III-A,
 *     Fig. 1 caption), plus, for the interpolating methods, a dense optical-flow field per frame
 *     interval (Sec. III-A, III-B; here supplied by the caller instead of estimated);
 *   - parameters are the contrast thresholds C_pos / C_neg and the number of interpolated frames
 *     (Sec. IV-A, Table I);
 *   - outputs are events <x, y, t, p> (Sec. III-A, Fig. 1 caption).
 * Four methods: BASIC (difference of consecutive frames, Sec. III and IV-A reference bar),
 * DENSE (dense flow interpolation, Sec. III-A), SPARSE (interpolation only at pixels whose
 * frame-to-frame change reaches a threshold, Sec. III-B) and DIFFERENCE (interpolation of
 * difference frames, Sec. III-C).  Outputs can also be read as a frame of accumulated events
 * (Fig. 1 caption) and as the events/(pixel s) statistic (Sec. IV-C).
 *
 * Arithmetic (identical on every entry point; fp32, one rounding per operation, no contraction):
 *   L = T[I] with T the 256-entry transform table (LOG: ln(v/255 + eps) rounded once from double;
 *   LINEAR: v).  Per pixel and interval, with S = n_interp + 1 sub-intervals (BASIC: S = 1),
 *   samples V_0 = L0, V_S = L1 and, for 0 < k < S, tau = k/S, w = 1 - tau, (u, v) = flow at the
 *   pixel: V_k = w * bil(L0, x - tau u, y - tau v) + tau * bil(L1, x + w u, y + w v) with
 *   clamp-to-edge bilinear sampling.  A per-pixel reference level R (device resident, initialised
 *   from the first frame) fires a positive event while V_{k+1} - R >= C_pos (R += C_pos) and a
 *   negative one while V_{k+1} - R <= -C_neg (R -= C_neg); the event time is
 *   t_{i-1} + floor(((k + theta) / S) * (t_i - t_{i-1})) with theta the crossing fraction inside
 *   the sub-interval (0 when the level was already passed at its start).  SPARSE skips pixels
 *   with |L1 - L0| < mask_threshold entirely (no events, R unchanged).
 * Memoryless thresholding (thresh_mode = SIM_THRESH_MEMORYLESS; the paper's Sec. III-A equations
 *   taken literally): no reference level; each difference D = V_{k+1} - V_k fires once, positive
 *   if D > C_pos, negative if D < -C_neg (strict), at t_{i-1} + floor(((k + 1) / S) * delta).
 * DIFFERENCE (always memoryless): from three consecutive frames the difference frames
 *   D1 = L_{i-1} - L_{i-2} and D2 = L_i - L_{i-1} (texel by texel); the flow supplied for the
 *   interval is the flow from D1 to D2; D_k = w * bil(D1, x - tau u, y - tau v) +
 *   tau * bil(D2, x + w u, y + w v) for 0 < k < S and D_S = D2; each D_k (k = 1..S) fires as
 *   above at t_{i-1} + floor((k / S) * delta).  The first interval (two frames, one difference
 *   frame) emits nothing; its flow is not read.
 *
 * Event order: within each frame interval events are sorted by (t, y, x, p) with p = -1 before
 * p = +1; intervals follow in push order.
 *
 * Packed key (sim_drain_keys): ((t - epoch) << 25) | (y << 13) | (x << 1) | (p > 0), where
 * epoch is the timestamp of the first frame pushed (sim_epoch).
 *
 * Conventions for every call: the return value is SIM_OK (0) or a negative status.  No C++
 * exception crosses the ABI.  SIM_E_INVAL, SIM_E_ORDER, SIM_E_RANGE and SIM_E_NOMEM leave the
 * stream exactly as it was before the call, with one exception: when a device buffer sized by
 * the number of events (the event arena, the sort buffers, the event FIFO) has to grow in the
 * middle of a push and that allocation fails, part of the image has already advanced, so the
 * push returns SIM_E_NOMEM and poisons the handle.  The same holds when the events of one window
 * (the up to 128 intervals a push simulates in one launch) exceed what that buffer can hold:
 * fewer than 2^31 events, in 256 equal parts of at most 2^23 - 1 events; the pixels are taken in
 * groups of 64 consecutive ones (consecutive selected pixels for SPARSE) and group g writes into
 * part g mod 256.  Pushing fewer frames per call makes windows smaller.  SIM_E_HIP poisons the
 * handle: every later call except sim_destroy, sim_get_stats and sim_strerror returns
 * SIM_E_POISONED.  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef EVSIM_SIM_H
#define EVSIM_SIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_E_INVAL (-1)     /* bad argument or configuration                                   */
#define SIM_E_ORDER (-2)     /* frame timestamp not strictly increasing                         */
#define SIM_E_NOMEM (-3)     /* device or host allocation failed                                */
#define SIM_E_RANGE (-4)     /* timestamp or key field out of range (see sim_push_frames)       */
#define SIM_E_HIP (-5)       /* HIP runtime error; the handle is now poisoned                   */
#define SIM_E_POISONED (-6)  /* handle poisoned by an earlier SIM_E_HIP                         */
#define SIM_E_BUSY (-7)      /* server: no slot or memory for the request (nothing changed)     */
#define SIM_E_EMPTY (-8)     /* server: nothing to return yet                                   */
#define SIM_E_TOO_BIG (-9)   /* sim_lk_flow_noalloc: the request needs more than its fixed scratch */

enum { SIM_BASIC = 0, SIM_DENSE = 1, SIM_SPARSE = 2, SIM_DIFFERENCE = 3 };
enum { SIM_THRESH_REFERENCE = 0, SIM_THRESH_MEMORYLESS = 1 };
enum { SIM_FLOW_SUPPLIED = 0, SIM_FLOW_LK = 1 };
enum { SIM_LOG = 0, SIM_LINEAR = 1 };
enum { SIM_MEM_HOST = 0, SIM_MEM_DEVICE = 1 };
/* srv_submit only: the frame in host memory, the flow in device memory (cameras stream frames
 * while flows are produced on the device). */
enum { SIM_MEM_HOST_FRAME = 2 };

typedef struct sim_config {
    int32_t width, height;      /* 1..4096 each (12-bit x and y fields of the packed key)          */
    int32_t method;             /* SIM_BASIC | SIM_DENSE | SIM_SPARSE | SIM_DIFFERENCE              */
    int32_t transform;          /* SIM_LOG (default) | SIM_LINEAR (the paper's linear difference)  */
    float c_pos, c_neg;         /* threshold magnitudes > 0; the paper writes C_neg as negative     */
    float log_eps;              /* SIM_LOG offset inside the logarithm, > 0 (default 1e-3)          */
    int32_t n_interp;           /* N >= 0 interpolated frames per interval, S = N + 1 (<= 255);     */
                                /* ignored by SIM_BASIC (S = 1)                                     */
    float mask_threshold;       /* SIM_SPARSE selection m: < 0 -> min(c_pos, c_neg); 0 -> all px   */
    uint64_t event_capacity;    /* initial device event buffer (events, < 2^31 - 255); grows on    */
                                /* demand; 0 = auto (2 per pixel)                                  */
    void* hip_stream;           /* hipStream_t to order all work on; NULL -> library-owned stream   */
    int32_t thresh_mode;        /* SIM_THRESH_REFERENCE (default: reference level, event pixel) |   */
                                /* SIM_THRESH_MEMORYLESS (paper's equations); DIFFERENCE: ignored   */
    int32_t flow_source;        /* SIM_FLOW_SUPPLIED (default: flow passed with each frame) |       */
                                /* SIM_FLOW_LK (estimated on the device, see sim_lk_flow; DENSE and */
                                /* SPARSE only; the flow arguments are then ignored and may be NULL) */
} sim_config;

/* Parameters of the pyramidal Lucas-Kanade estimator (sim_lk_flow, SIM_FLOW_LK). */
typedef struct sim_lk_params {
    int32_t levels;             /* pyramid levels above full resolution, 0..4 (default 3)           */
    int32_t radius;             /* window half size r: (2r+1)^2 texels, 1..15 (default 7)            */
    int32_t iterations;         /* Gauss-Newton steps per level, 1..100 (default 10)                */
    float eps;                  /* stop a level once |step|^2 < eps, px^2 (default 1e-4)            */
    float min_trace;            /* texture: trace(G) >= min_trace * (2r+1)^2 (default 1)            */
    float min_ratio;            /* aperture: det(G) >= min_ratio * trace(G)^2 (default 1e-3)       */
} sim_lk_params;

/* One event as drained to the host (16 bytes). */
typedef struct sim_event {
    int64_t t_us;               /* absolute timestamp, microseconds                                 */
    uint16_t x, y;              /* pixel                                                            */
    int8_t p;                   /* +1 or -1                                                         */
    uint8_t pad[3];
} sim_event;

typedef struct sim_stats {
    uint64_t frames;            /* frames pushed (including the first)                              */
    uint64_t intervals;         /* frame intervals simulated                                        */
    uint64_t events;            /* events produced                                                  */
    uint64_t selected;          /* SIM_SPARSE: pixel-intervals selected for interpolation           */
    uint64_t active;            /* SIM_SPARSE: pixels selected at least once, summed over windows  */
    uint64_t retries;           /* event-buffer growths that re-ran part of a window                */
    uint64_t event_capacity;    /* current device event buffer (events)                             */
    /* Filled only while kernel timing is on (sim_set_kernel_timing): HIP-event durations on the  */
    /* stream of the launches, summed over launches.                                               */
    uint64_t select_launches;   /* selection passes (SIM_SPARSE) or frame saves (others), 1/window */
    double select_ms;           /* their summed duration                                            */
    uint64_t simulate_launches; /* per-pixel chain kernel launches (one per window, plus re-runs)   */
    double simulate_ms;         /* their summed duration                                            */
    uint64_t sort_launches;     /* ordering passes (each: histogram, scan, scatter kernels)         */
    double sort_ms;             /* their summed duration                                            */
} sim_stats;

typedef struct sim_stream sim_stream;

/* Fills cfg with defaults: 0x0 image, SIM_BASIC, SIM_LOG, C = 0.2, eps = 1e-3, N = 10, m = -1,
 * automatic capacity, library-owned stream, reference-level thresholding.  Width and height must
 * be set before sim_create. */
void sim_config_init(sim_config* cfg);

/* Creates a stream (device state: reference levels, previous frame, table, event buffers).
 * cfg is copied.  On success *out owns the handle until sim_destroy.  Errors: SIM_E_INVAL
 * (dimension out of 1..4096, method/transform/thresh_mode/flow_source unknown, SIM_FLOW_LK
 * with a method other than DENSE or SPARSE, thresholds not > 0 or so small that R + C == R for
 * some reachable R, n_interp outside 0..255, log_eps not > 0, event_capacity >= 2^31 - 255, and,
 * with a reference level (SIM_THRESH_REFERENCE, methods other than DIFFERENCE), thresholds so
 * small that one pixel could fire more than 2^24 events in one interval:
 * S * (2 * (max T - min T) / min(c_pos, c_neg) + 3) > 2^24), SIM_E_NOMEM. */
int sim_create(const sim_config* cfg, sim_stream** out);

/* Releases every resource of the handle after the work queued on its stream completes. */
int sim_destroy(sim_stream* s);

/* Forgets all frames and pending events; the next push is a first frame again.  Device
 * buffers keep their (grown) sizes and sim_stats keeps counting. */
int sim_reset(sim_stream* s);

/* Pushes one frame taken at t_us (frame interval semantics of Sec. III-A: the pair of frames
 * (previous, this one) defines one interval).  frame: uint8 [height][width], row-major, no
 * padding.  flow: float32 [height][width][2] (dx, dy in pixels per interval, motion from the
 * previous frame to this one; for SIM_DIFFERENCE the flow between the interval's difference
 * frames); required for SIM_DENSE / SIM_SPARSE / SIM_DIFFERENCE except on the first frame,
 * ignored otherwise (may be NULL).  mem_kind tells whether frame and flow are host or device
 * pointers; host inputs are copied before the call returns (one window of frames and flows at a
 * time, through a device staging buffer of that size), device inputs must stay valid until
 * the work queued on the stream has completed.  The first push only initialises the reference
 * levels (no events).  n_new_events (may be NULL) receives the number of events this push
 * produced.  Errors: SIM_E_INVAL (NULL frame, missing flow), SIM_E_ORDER (t_us not greater than
 * the previous frame's), SIM_E_RANGE (t_us - epoch >= 2^39 or interval longer than 2^31 us). */
int sim_push_frame(sim_stream* s, const uint8_t* frame, const float* flow, int64_t t_us,
                   int32_t mem_kind, uint64_t* n_new_events);

/* Pushes n_frames frames at once: the same result as n_frames calls of sim_push_frame, computed
 * by one persistent launch that carries the reference levels across the frame intervals.
 * frames: uint8 [n_frames][height][width]; t_us: host array of n_frames timestamps; flows:
 * float32 [n_intervals][height][width][2] with n_intervals = n_frames - 1 when the stream has no
 * frame yet (the first frame only initialises) and n_frames otherwise; flows[j] belongs to the
 * j-th interval produced by this call.  Same memory, error and ordering rules as
 * sim_push_frame; every timestamp is validated before any work is queued. */
int sim_push_frames(sim_stream* s, int32_t n_frames, const uint8_t* frames, const float* flows,
                    const int64_t* t_us, int32_t mem_kind, uint64_t* n_new_events);

/* One entry of a batched push: the arguments of sim_push_frames for one stream (inputs), plus
 * the per-stream results (outputs). */
typedef struct sim_frames {
    int32_t n_frames;
    int32_t mem_kind;           /* SIM_MEM_HOST or SIM_MEM_DEVICE for frames and flows            */
    const uint8_t* frames;      /* uint8 [n_frames][height][width]                                 */
    const float* flows;         /* float32 [n_intervals][height][width][2] (see sim_push_frames)   */
    const int64_t* t_us;        /* host array of n_frames timestamps                               */
    uint64_t n_new_events;      /* out: events produced for this stream                            */
    int32_t status;             /* out: SIM_OK or this stream's error                              */
    int32_t pad;
} sim_frames;

/* Pushes frames to n distinct streams at once, with exactly the result of n sim_push_frames
 * calls.  Streams of any resolution, method, thresholding mode and flow source may be combined:
 * each window of all streams runs as one launch per phase (clearing, selection and ordering,
 * chains, gather, every sort pass) on a library stream, all queued before one host wait; unless
 * a stream estimates its flow, that sequence is recorded once as a HIP graph per launch shape
 * (streams, sizes, sort passes) and replayed for later windows of the same shape.  Streams whose
 * window ran out of event-buffer space, or produced more events than the sort was sized for,
 * are finished after that wait by re-runs (one host wait per phase).  The
 * streams' earlier work is completed first; their events are ordered when the call returns.
 * Validation of every entry (and a handle listed twice, SIM_E_INVAL) happens before any work is
 * queued; on a validation error nothing changes.  Staging and buffer reservation follow per
 * entry (an entry failing there stays untouched while the others proceed).  A failure inside the
 * fused launches poisons every stream of that window; a host allocation failure between windows
 * returns SIM_E_NOMEM and poisons every stream that still had a window to run.  Errors are
 * reported per entry in `status`;
 * returns SIM_OK or the first error.  One batched push runs at a time per process. */
int sim_push_batch(sim_stream** streams, sim_frames* items, int32_t n);

/* Chain-pass variant: how many interior samples' texel loads a lane keeps in flight (0: 2, 1: 5,
 * 2: 10 for the frame methods; 1, 2 and 4 for difference frames).  Every variant computes the
 * same events bit for bit; they differ in speed.  -1 (the default) lets the library's autotuner
 * choose: on the first window of each (device architecture, width, height, method, thresholding
 * mode, S) it times every variant on that window against scratch copies of the state the pass
 * writes and keeps the fastest for the process (streams with estimated flow, and S = 1, use
 * variant 2).  A batched push runs each thresholding mode's streams with the variant of its
 * stream with the most pixels.  sim_get_chain_variant reports the variant the stream's last
 * window used (-1 before its first window).
 * Errors: SIM_E_INVAL (NULL, variant outside -1..2). */
int sim_set_chain_variant(sim_stream* s, int32_t variant);
int sim_get_chain_variant(sim_stream* s, int32_t* variant);

/* Process-wide counts of the batched pushes since the library was loaded: graphs recorded,
 * graph launches, and stream windows finished by re-runs (sim_push_batch).  Any pointer may be
 * NULL.  Errors: none (returns SIM_OK). */
int sim_batch_stats(uint64_t* graphs_recorded, uint64_t* graph_launches, uint64_t* rerun_windows);

/* Process-wide time spent by batched pushes since the library was loaded, per fused chunk (one
 * chunk per window of up to 120 intervals of every stream of a sim_push_batch call): host time
 * waiting for work already queued on the streams (their staged inputs), planning (per-stream
 * tables, buffer checks, tuning), recording or replaying the chunk's graph, blocked until the
 * chunk's counts are back, and finishing (re-runs, per-stream bookkeeping); and the device time
 * of the chunks' sequences, from events recorded around them. */
typedef struct sim_batch_timing {
    uint64_t chunks;
    double inputs_ms, plan_ms, launch_ms, wait_ms, finish_ms;
    double device_ms;
} sim_batch_timing;
int sim_batch_times(sim_batch_timing* out);

/* Number of events produced and not yet drained. */
int sim_pending_events(sim_stream* s, uint64_t* n);

/* Copies up to max_events of the oldest pending events, in canonical order, into dst (host
 * memory owned by the caller) and removes them from the stream.  *n_written receives the count.
 * Partial drains are allowed; the next drain continues where this one stopped. */
int sim_drain_events(sim_stream* s, sim_event* dst, uint64_t max_events, uint64_t* n_written);

/* As sim_drain_events, but writes packed 64-bit keys (format above) to dst, which is host
 * memory (SIM_MEM_HOST) or device memory (SIM_MEM_DEVICE, copied on the stream). */
int sim_drain_keys(sim_stream* s, uint64_t* dst, uint64_t max_events, int32_t mem_kind,
                   uint64_t* n_written);

/* Timestamp of the first frame (the epoch of packed keys).  SIM_E_INVAL before the first push. */
int sim_epoch(sim_stream* s, int64_t* epoch);

/* Copies the per-pixel reference levels, float32 [height][width], to host or device memory. */
int sim_get_reference(sim_stream* s, float* dst, int32_t mem_kind);

/* Waits until all work queued by this stream has completed. */
int sim_sync(sim_stream* s);

/* Counters since creation or the last sim_clear_stats. */
int sim_get_stats(sim_stream* s, sim_stats* out);

/* Zeroes the counters of sim_stats (event_capacity excepted). */
int sim_clear_stats(sim_stream* s);

/* Turns per-kernel timing on (enable != 0) or off.  While on, every simulation launch and every
 * ordering sort is bracketed by HIP events recorded on the stream's own queue, and each push
 * waits for its sort to finish before returning so the durations can be read.  The durations
 * accumulate in sim_stats until sim_clear_stats. */
int sim_set_kernel_timing(sim_stream* s, int32_t enable);

/* Static text for a status code. */
const char* sim_strerror(int status);

/* Frame of accumulated events (Fig. 1 caption: the methods output either the events or a frame
 * of accumulated events): adds, for every pending (not yet drained) event with
 * t_begin <= t < t_end, one to counts[0][y][x] if it is positive or to counts[1][y][x] if it is
 * negative.  counts: uint32 [2][height][width], caller-owned, host or device (mem_kind); it is
 * added to, not cleared (each count wraps modulo 2^32).  Host counts are complete when the call
 * returns; device counts are written in stream order on the handle's stream.  Pending events are
 * not consumed.  Errors: SIM_E_INVAL (NULL counts, t_end < t_begin, bad mem_kind). */
int sim_accumulate(sim_stream* s, int64_t t_begin, int64_t t_end, uint32_t* counts,
                   int32_t mem_kind);

/* Events per pixel and second (the statistic of Sec. IV-C) of the pending events with
 * t_begin <= t < t_end: with c the per-pixel count of both polarities over all width * height
 * pixels, S1 = sum c and S2 = sum c^2 (exact integers), m1 = S1 / npix, m2 = S2 / npix and
 * T = (t_end - t_begin) * 1e-6 s, *mean = m1 / T and *stddev = sqrt(max(m2 - m1 * m1, 0)) / T
 * (population deviation over pixels; double precision).  sums (may be NULL) receives S1, S2.
 * S1 and S2 are exact while S2 < 2^64 (so every c < 2^32).
 * Synchronises the stream.  Errors: SIM_E_INVAL (NULL mean or stddev, t_end <= t_begin). */
int sim_event_rate(sim_stream* s, int64_t t_begin, int64_t t_end, double* mean, double* stddev,
                   uint64_t* sums);

/* Fills p with the defaults listed in sim_lk_params. */
void sim_lk_params_init(sim_lk_params* p);

/* Parameters used by a SIM_FLOW_LK stream from its next push on (defaults until called).
 * Errors: SIM_E_INVAL (NULL, a field out of its range). */
int sim_set_lk_params(sim_stream* s, const sim_lk_params* p);

/* Pyramidal Lucas-Kanade flow (the sparse method's flow estimator, Sec. III-B; the method of
 * Lucas and Kanade, iterated coarse to fine) from frame f0 to frame f1 (uint8 [height][width])
 * at the pixel indices points[j] = y * width + x: flow[2j], flow[2j+1] = (dx, dy) in pixels,
 * valid[j] (may be NULL) = 1, or 0 with flow (0, 0) where the window lacks texture, has only
 * one-dimensional structure, or the index is outside the image.
 *   Pyramid: level 0 = intensity; level l+1 (ceil(W/2) x ceil(H/2)) = 1-2-1 x 1-2-1 binomial
 *   average / 16 around (2x, 2y), clamped.  Gradients: central differences / 2, clamped.
 *   Samples: clamp-to-edge bilinear.  From the coarsest level, guess g = 0, window offsets
 *   d in [-r, r]^2 around u = p / 2^l: G = sum [ix^2, ix iy; ix iy, iy^2]; valid only if
 *   trace(G) >= min_trace (2r+1)^2 and det(G) >= min_ratio trace(G)^2; up to `iterations` steps
 *   b = sum (I(u+d) - J(u+d+g+v)) [ix, iy], step = G^-1 b, v += step, until |step|^2 < eps;
 *   g = 2 (g + v) between levels; flow = g + v.  fp32, one rounding per operation.
 * Every pointer is host or device memory as mem_kind says; work is ordered on hip_stream (NULL:
 * a stream of the call) and complete when the call returns.  params NULL: defaults.
 * Errors: SIM_E_INVAL (NULL pointers with n_points > 0, dimensions outside 1..4096, params out
 * of range), SIM_E_NOMEM, SIM_E_HIP. */
int sim_lk_flow(const uint8_t* f0, const uint8_t* f1, int32_t width, int32_t height,
                const uint32_t* points, uint64_t n_points, float* flow, uint8_t* valid,
                const sim_lk_params* params, int32_t mem_kind, void* hip_stream);

/* sim_lk_flow without any allocation, for callers that cannot allocate device memory: code
 * recorded into a HIP graph, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, arithmetic and results as sim_lk_flow with mem_kind = SIM_MEM_DEVICE: f0, f1,
 * points, flow and valid (may be NULL) are device memory owned by the caller.  The two pyramids
 * live in a fixed device array that the library holds on every GPU it runs on until the process
 * ends: 6 * 2^20 floats (24 MiB), enough for two pyramids of 1920x1080 frames at any level
 * count; larger requests return SIM_E_TOO_BIG before any device work.  Work is queued on
 * hip_stream (NULL: the null stream) and the call returns without waiting for it; read the
 * outputs after synchronising with that stream.  Every call on one GPU shares that GPU's array:
 * calls whose work overlaps on one GPU (queued on different streams, or from several threads)
 * race and give undefined results; calls queued on one stream are ordered and safe.  No
 * hipMalloc, hipFree, memset node or host wait is issued.
 * Errors: as sim_lk_flow (SIM_E_INVAL, SIM_E_HIP) plus SIM_E_TOO_BIG; never SIM_E_NOMEM. */
int sim_lk_flow_noalloc(const uint8_t* f0, const uint8_t* f1, int32_t width, int32_t height,
                        const uint32_t* points, uint64_t n_points, float* flow, uint8_t* valid,
                        const sim_lk_params* params, void* hip_stream);

/* Text describing the HIP failure that poisoned the handle (call, source line, HIP's message);
 * empty when there was none.  Valid until the next call on the handle. */
const char* sim_last_error(sim_stream* s);

/* ------------------------------------------------------------------------------------------
 * Serving: many virtual cameras, continuous batching.
 *
 * A server owns cameras (one simulator stream each, with its device-resident state and a device
 * staging ring of `queue_depth` frames (+ flows)).  srv_admit creates a camera if a slot is free
 * and its estimated HBM footprint (srv_footprint) fits the remaining budget, else returns
 * SIM_E_BUSY and changes nothing; srv_release frees both (frames still queued for it are dropped
 * and counted as failed).  srv_submit queues one frame into the camera's ring and returns
 * (SIM_E_BUSY when the ring is full, SIM_E_ORDER when t_us does not increase).  Cameras whose
 * configuration names no HIP stream share one stream of the server.  A step runs every queued frame of every camera as one batched push
 * (sim_push_batch), so the cameras' GPU work overlaps.  srv_start runs steps on a worker thread
 * of the server: each step admits every frame queued when it starts, frames that arrive while
 * it runs are admitted by the next one, which starts as soon as it ends (continuous
 * batching).  Without the worker, srv_step
 * runs one step on the calling thread.  The latency of a frame is the time from its arrival stamp
 * (srv_now_ns clock; 0 = now) to the end of the step that ordered its events.  Results per camera
 * are exactly those of the camera's frames pushed alone.  Every srv_* call may come from any
 * thread: calls are serialised inside the server, except that srv_submit (and srv_get_stats) do
 * not wait for a running step.  srv_create reserves the server's own host bookkeeping (about 8 MB
 * of latency record, plus a little per camera slot), so it does not grow while serving.
 * ------------------------------------------------------------------------------------------ */
typedef struct sim_server sim_server;

typedef struct sim_server_stats {
    uint64_t cameras;             /* admitted and not released                                     */
    uint64_t admissions;
    uint64_t rejected_admissions; /* SIM_E_BUSY from srv_admit                                     */
    uint64_t submitted;           /* frames accepted by srv_submit                                 */
    uint64_t rejected_frames;     /* SIM_E_BUSY from srv_submit (queue full)                       */
    uint64_t completed;           /* frames whose events are ordered                               */
    uint64_t failed_frames;       /* frames of a camera whose push failed in a step                */
    uint64_t steps;
    uint64_t events;
    uint64_t hbm_used, hbm_budget;/* footprint estimates of the admitted cameras, and the budget   */
    double p50_ms, p99_ms, max_ms;/* per-frame latency, arrival to ordered events, over the latest */
                                  /* 2^20 completed frames since srv_clear_stats                  */
    double busy_ms;               /* wall time inside steps                                        */
    double lock_wait_ms;          /* time steps waited for other calls on the cameras (drains,     */
                                  /* admissions, releases) to finish                               */
} sim_server_stats;

/* Estimated device bytes of one camera with this configuration and staging queue depth. */
int srv_footprint(const sim_config* cfg, int32_t queue_depth, uint64_t* bytes);
int srv_create(uint64_t hbm_budget_bytes, int32_t max_cameras, int32_t queue_depth,
               sim_server** out);
int srv_destroy(sim_server* srv);
int srv_admit(sim_server* srv, const sim_config* cfg, int32_t* cam);
int srv_release(sim_server* srv, int32_t cam);
/* frame: uint8 [H][W]; flow: float32 [H][W][2] for the interval ending at this frame (required
 * for SIM_DENSE / SIM_SPARSE / SIM_DIFFERENCE except on a camera's first frame); both host
 * (SIM_MEM_HOST), both device (SIM_MEM_DEVICE), or a host frame with a device flow
 * (SIM_MEM_HOST_FRAME).  Device inputs and pinned host inputs (hipHostMalloc) are read
 * asynchronously by the step that takes the frame (one copy kernel per step pulls every queued
 * input into the cameras' rings; the device reads pinned host memory directly); pageable host
 * inputs are copied at the call.  A device input must be complete (its writes synchronised) at
 * the call, and inputs must stay valid and unchanged until the frame completes (srv_sync, or the
 * stats count it).  SIM_E_BUSY when the camera's ring is full (a step frees it), SIM_E_ORDER
 * when t_us does not increase. */
int srv_submit(sim_server* srv, int32_t cam, const uint8_t* frame, const float* flow,
               int64_t t_us, int32_t mem_kind, int64_t arrival_ns);
/* One continuous-batching step on the calling thread; *n_frames receives the frames completed.
 * Returns SIM_OK or the first per-camera error (that camera's frames of the step are dropped
 * and counted as failed); SIM_E_BUSY while the worker runs (it steps by itself). */
int srv_step(sim_server* srv, uint64_t* n_frames);
/* Starts the server's worker thread (steps back to back while frames are queued); a started
 * server stays started until srv_stop or srv_destroy.  Errors: SIM_E_NOMEM (no thread). */
int srv_start(sim_server* srv);
/* Stops the worker after its current step (queued frames stay queued). */
int srv_stop(sim_server* srv);
/* Waits until every queued frame has completed (with the worker running: until it has run
 * them; otherwise by running steps).  Returns SIM_OK or the first step error since the last
 * srv_sync. */
int srv_sync(sim_server* srv);
/* Drains a camera's ordered events as packed keys (as sim_drain_keys). */
int srv_drain(sim_server* srv, int32_t cam, uint64_t* dst, uint64_t max_events, int32_t mem_kind,
              uint64_t* n_written);
/* Ordered events of a camera not yet drained (as sim_pending_events). */
int srv_pending(sim_server* srv, int32_t cam, uint64_t* n);
/* The simulator stream of a camera (owned by the server; not to be used while the worker runs). */
int srv_stream(sim_server* srv, int32_t cam, sim_stream** out);
int srv_get_stats(sim_server* srv, sim_server_stats* out);
int srv_clear_stats(sim_server* srv);
int64_t srv_now_ns(void);

#ifdef __cplusplus
}
#endif

#endif /* EVSIM_SIM_H */
