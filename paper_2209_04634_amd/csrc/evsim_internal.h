// Internal interface between the HIP kernels (evsim_kernels.hip) and the host runtime
// (evsim_runtime.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace evsim {

constexpr int kSimThreads = 256;     // pixels per simulation tile (one per thread)
constexpr int kMaxSubIntervals = 256;   // S = n_interp + 1 <= 256
constexpr int kMaxStash = 31;        // interior samples kept in LDS per pixel (S - 1 <= 31)
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per sort block
// Sort digit width: 9 bits where that saves a pass (45-bit keys: five passes instead of six), 8
// otherwise (a 9-bit pass costs about 15% more).  Scratch is sized for the wider digits.
constexpr int kRadixDigits = 512;    // histogram and totals entries per block at the widest
inline int sort_radix_bits(int nbits) { return (nbits + 8) / 9 < (nbits + 7) / 8 ? 9 : 8; }
inline int sort_passes(int nbits) {
    const int b = sort_radix_bits(nbits);
    return (nbits + b - 1) / b;
}
constexpr uint64_t kSentinel = ~0ull;
constexpr int kMaskWords = 4;        // selected-interval bitmask words per pixel
constexpr int kMaxWindow = 32 * kMaskWords;   // frame intervals per launch
// Device-scope atomics on one address serialise (about 12 ns each on MI355X), so every counter
// that many waves hit is striped: each stripe lives on its own 256-byte line.
constexpr int kCounterStride = 32;   // u64 / u32 elements between stripe counters
constexpr int kArenaStripes = 256;   // event sub-arenas, one reservation counter each
constexpr int kActStripes = 8;       // active-pixel sub-lists (one per group of select blocks)
constexpr int kStatStripes = 64;     // statistics counters
constexpr int kSelectPx = 1024;      // pixels per selection block (4 per thread)
// Chain-length classes of the sparse method's active pixels: class c holds the pixels with c + 1
// selected intervals in the window (the last class: kClasses or more).  The chain pass takes the
// classes longest first, so the 64 lanes of a wave walk chains of (nearly) equal length.
constexpr int kClasses = 16;
// The event arena of one window holds fewer than kArenaKeyLimit keys (so every count, offset and
// prefix sum over it fits 32 bits), hence each sub-arena fewer than kArenaKeyLimit / kArenaStripes.
constexpr uint64_t kArenaKeyLimit = 1ull << 31;
// Most events one pixel may fire in one frame interval with a reference level (the stream's
// configuration is refused otherwise): the chain kernel sums 64 lanes' counts in an int, and each
// lane's crossing loop runs at most this many steps per pass.  (Memoryless thresholding fires at
// most S <= 256 events per pixel and interval.)
constexpr int kMaxLaneCount = 1 << 24;
static_assert(64ull * kMaxLaneCount < (1ull << 31), "wave totals fit an int");

enum Method { kBasic = 0, kDense = 1, kSparse = 2, kDifference = 3 };

// What the chain pass compares with the thresholds.
//   kModeReference:  the interpolated series against a per-pixel reference level (event pixel);
//   kModeMemoryless: each difference of consecutive samples on its own (paper's equations);
//   kModeDifference: each interpolated difference frame on its own (difference method).
enum ChainMode { kModeReference = 0, kModeMemoryless = 1, kModeDifference = 2 };

// Layout of the unsorted "sort key" written by the simulation kernel, low bits first:
//   p (1) | x (xb) | y (yb) | t_rel (tb) | interval index within the window (ib)
// Sorting these keys ascending gives interval-major (t, y, x, p) order.  One extra bit above the
// layout is always sorted so that the all-ones sentinel (unused slots) sorts after every key.
struct KeyLayout {
    int xb, yb, tb, ib;
    __host__ __device__ int pix_bits() const { return xb + yb + 1; }
    __host__ __device__ int total_bits() const { return ib + tb + xb + yb + 1; }
};

// Selection pass (sparse method): streams every frame of the window once, writes the per-pixel
// bitmask of selected intervals, and writes each block's pixels selected at least once as one run
// (at block * kSelectPx of act_px), longest length class first, pixel order within a class.  No
// atomics: per-block counts go to plain arrays for the order pass.
struct SelectArgs {
    const uint8_t* prev;        // frame before the window, uint8 [H][W]
    const uint8_t* frames;      // window frames; frame j at frames + j * fstride
    int64_t fstride;
    const float* lut;           // 256-entry transform table
    uint8_t* prev_out;          // receives the window's last frame
    uint32_t* mask;             // [kMaskWords][npix] selected-interval bits
    uint32_t* act_px;           // per block: its run of active pixels (kSelectPx slots)
    uint32_t* counts;           // [kClasses][block] active pixels per length class
    uint32_t* bsel;             // [block] selected pixel-intervals
    int npix, K;
    float m;
};

// Order pass (sparse method): the selection blocks' runs into one list of active pixels, length
// classes longest first, blocks in order within a class (so the list is deterministic), resume
// points cleared.  Two kernels: a one-block scan of the per-block counts, then the copy.
struct OrderArgs {
    const uint32_t* act_px;     // the selection's runs
    const uint32_t* counts;     // [kClasses][block] (class-major: a class's counts are adjacent)
    const uint32_t* bsel;       // [block]
    int nblocks;
    uint32_t* goff;             // [kClasses][block]: place of the block's class run in ord
    unsigned int* n_total;      // length of ord
    unsigned long long* stats;  // += selected pixel-intervals, active pixels (one atomic each)
    uint32_t* ord;
    int* resume;                // per ordered slot: set to 0
};

// Chain pass: one lane per active pixel (sparse) or per pixel (dense, basic) walks its selected
// intervals in order, carrying the reference level in a register.
struct ChainArgs {
    const uint8_t* prev;
    const uint8_t* frames;
    int64_t fstride;
    const float* flows;         // flow of interval j at flows + j * flstride (null for basic)
    int64_t flstride;
    const float* lut;
    const float* delta;         // per interval: (float)(t_j - t_{j-1})
    float* lref;                // per-pixel reference level, updated in place
    const uint32_t* mask;       // sparse: [kMaskWords][npix]; null: every interval selected
    const uint32_t* act_px;     // sparse: the ordered active list; null: slot = pixel
    const unsigned int* n_active;  // sparse: its length (one counter); null: npix slots
    int* resume;                // per slot: first interval still to run (updated on exit)
    uint64_t* arena;            // kArenaStripes sub-arenas of stripe_cap keys
    uint64_t stripe_cap;
    unsigned long long* reserve;   // kArenaStripes reservation counters (stride kCounterStride)
    unsigned long long* fails;     // [0] failed reservations, [1] sentinel slots written
    int W, H, S, K, npix;
    float cpos, cneg;
    KeyLayout lay;
    int mode;                   // ChainMode
    const uint8_t* prev2;       // difference method: frame before `prev`
    int first_emit;             // difference method: intervals below this emit nothing
};

struct ConvertArgs {
    int enabled;                // final pass: write packed ABI keys instead of sort keys
    const unsigned long long* n_sentinel;  // keys below n - *n_sentinel are real events
    const int64_t* tbase;       // per interval: t_{j-1} - epoch
    int K;                      // intervals in the window (bound of the interval field)
    KeyLayout lay;
};

// Launchers (all asynchronous on `stream`).
hipError_t launch_init(const uint8_t* frame, const float* lut, float* lref, uint8_t* prev,
                       int64_t npix, hipStream_t stream);
hipError_t launch_select(const SelectArgs& a, hipStream_t stream);
hipError_t launch_order(const OrderArgs& a, hipStream_t stream);
// Blocks of the selection (and of the order copy) for npix pixels.
inline int select_blocks(int64_t npix) { return (int)((npix + kSelectPx - 1) / kSelectPx); }
// Chain-pass variants (interior samples in flight per lane: 2 / 5 / 10 for the frame methods,
// 1 / 2 / 4 for difference frames); identical results.
constexpr int kChainVariants = 3;
constexpr int kDefaultChainVariant = 2;
hipError_t launch_chain(const ChainArgs& a, int max_slots, int variant, hipStream_t stream);
// Concatenates the used part of every sub-arena into `out`; writes the total to *n_total.
hipError_t launch_gather(const uint64_t* arena, uint64_t stripe_cap,
                         const unsigned long long* reserve, uint64_t* out,
                         unsigned long long* n_total, hipStream_t stream);
// reserve[s] = min(reserve[s], cap) for every stripe (before re-running failed chains).
hipError_t launch_clamp(unsigned long long* reserve, uint64_t cap, hipStream_t stream);
hipError_t launch_copy_u8(const uint8_t* src, uint8_t* dst, int64_t n, hipStream_t stream);
// Zero-fills `bytes` (a multiple of 4) at p with a kernel (no memset node in a captured graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);
// Clears a window's counters[4], the reservation counters and resume[npix] (if not null: every
// method but the sparse one, whose order pass clears its own) in one launch.
hipError_t launch_prep_window(unsigned long long* counters, unsigned long long* reserve,
                              int* resume, int64_t npix, hipStream_t stream);
// Sorts keys[0, *n) on bits [0, nbits) (stable LSD radix, 8-bit digits); the last pass writes
// into `out` converted by `cv`.  The count is read on the device; grids are sized for n_max.
// `alt` holds n_max keys; `hist` holds sort_hist_entries(n_max) counters and `totals` 256.
hipError_t launch_sort(uint64_t* keys, uint64_t* alt, const unsigned long long* n,
                       uint64_t n_max, int nbits, uint32_t* hist, uint32_t* totals,
                       uint64_t* out, const ConvertArgs& cv, hipStream_t stream);
size_t sort_hist_entries(uint64_t n_max);

// Adds every packed key of keys[0, n) whose time field (t - epoch) lies in [t_lo, t_hi) to the
// accumulated frame counts[2][H][W] (plane 0 positive, plane 1 negative).
hipError_t launch_accumulate(const uint64_t* keys, uint64_t n, uint64_t t_lo, uint64_t t_hi,
                             int W, int H, uint32_t* counts, hipStream_t stream);
// Per-block partial sums (sum c, sum c^2) of c = counts[p] + counts[plane + p] over p < plane
// into part[2 * block], part[2 * block + 1] for `blocks` = moments_blocks(plane) blocks.
int moments_blocks(uint64_t plane);
hipError_t launch_moments(const uint32_t* counts, uint64_t plane, unsigned long long* part,
                          hipStream_t stream);

// ------------------------------------------------------------------------------------------
// Fused batch: one launch per phase over every stream of a batched push.  Each stream of the
// launch is one BatchEntry in device memory; a block finds its entry by binary search over the
// launch's block offsets (entry e owns blocks [start[e], start[e + 1])) and runs the same block
// body as the stream's own kernel with its block index inside the stream.
// ------------------------------------------------------------------------------------------
struct BatchEntry {
    int sparse;                      // 1: selection pass; 0: frame copies
    int vec;                         // selection: 4-byte aligned frames (vector loads)
    SelectArgs sel;
    OrderArgs ord;
    const uint8_t* copy_src;         // non-sparse: the window's last frame -> prev_out
    uint8_t* copy_dst;
    const uint8_t* copy2_src;        // difference method: the frame before it -> prev2 out
    uint8_t* copy2_dst;
    int64_t npix;
    unsigned long long* counters;    // [0] failed reservations [1] sentinels [2] gathered
    ChainArgs chain;
    uint64_t clamp_cap;              // re-run: clamp reservations to this (old) stripe capacity
    uint64_t* gathered;              // gather output = sort input
    uint64_t* sort_alt;              // sort ping-pong buffer
    uint32_t* hist;
    uint32_t* totals;
    uint64_t* out;                   // the stream's FIFO tail
    ConvertArgs cv;
    int sort_blocks;                 // 0: nothing to sort
};

// Block offsets of each fused launch live in device memory as n + 1 ints.
hipError_t launch_batch_prep(const BatchEntry* e, int n, hipStream_t stream);
hipError_t launch_batch_select(const BatchEntry* e, const int* start, int n, int blocks,
                               hipStream_t stream);
// Order pass of the sparse entries: one scan block per entry (non-sparse entries' blocks return),
// then the copy (entries without one own no block).
hipError_t launch_batch_order(const BatchEntry* e, const int* start, int n, int blocks,
                              hipStream_t stream);
hipError_t launch_batch_chain(const BatchEntry* e, const int* start, int n, int blocks, int mode,
                              int max_stash, int variant, hipStream_t stream);
// out[e] = failed reservations of entry e (counters[0]).
hipError_t launch_batch_fails(const BatchEntry* e, int n, unsigned long long* out,
                              hipStream_t stream);
// For every entry with a nonzero clamp_cap: clamp its reservations, clear its failure count.
hipError_t launch_batch_clamp(const BatchEntry* e, int n, hipStream_t stream);
hipError_t launch_batch_gather(const BatchEntry* e, const int* start, int n, int blocks,
                               hipStream_t stream);
// out[2e] = sentinels, out[2e + 1] = gathered keys of entry e.
// out[3e], out[3e + 1], out[3e + 2] = failed reservations, sentinels, gathered keys of entry e.
hipError_t launch_batch_status(const BatchEntry* e, int n, unsigned long long* out,
                               hipStream_t stream);
hipError_t launch_batch_counts(const BatchEntry* e, int n, unsigned long long* out,
                               hipStream_t stream);
// Every pass of the sort of every entry (`passes` passes; the last converts into `out`).
hipError_t launch_batch_sort(const BatchEntry* e, const int* start, int n, int blocks, int passes,
                             int radix_bits,
                             hipStream_t stream);

// ------------------------------------------------------------------------------------------
// Pyramidal Lucas-Kanade flow (evsim_lk.hip).
// ------------------------------------------------------------------------------------------
constexpr int kLkMaxLevels = 4;      // pyramid levels above full resolution

struct LkParams {
    int levels, radius, iters;
    float eps, min_trace, min_ratio;
};

// Layout of one frame's pyramid inside a float buffer: level l has w[l] x h[l] texels at off[l].
struct PyrLayout {
    int levels;
    int w[kLkMaxLevels + 1], h[kLkMaxLevels + 1];
    uint64_t off[kLkMaxLevels + 1];
    uint64_t total;                  // floats per frame
};
PyrLayout pyr_layout(int W, int H, int levels);

// Pyramids of n uint8 frames, frame f's written at pyr + f * lay.total.  Frame 0 is `first`,
// frame f > 0 is rest + (f - 1) * fstride (a window's previous frame, then its frames).
hipError_t launch_pyramids(const uint8_t* first, const uint8_t* rest, int64_t fstride, int n,
                           const PyrLayout& lay, float* pyr, hipStream_t stream);

// Flow of every pixel index points[j] from pyramid a to pyramid b.
hipError_t launch_lk_points(const float* a, const float* b, const PyrLayout& lay,
                            const LkParams& P, const uint32_t* points, uint64_t n, float* flow,
                            uint8_t* valid, hipStream_t stream);

// Flow of a window: for every chain slot's pixel (active list of the sparse method, or every
// pixel) and every selected interval i, the flow from pyramid i to pyramid i + 1 into
// flow + i * 2 * npix + 2 * p (the layout of supplied flows).
struct LkWindowArgs {
    const float* pyr;                // K + 1 pyramids (previous frame, then the window's frames)
    PyrLayout lay;
    LkParams P;
    const uint32_t* mask;            // sparse: [kMaskWords][npix]; null: every interval
    const uint32_t* act_px;          // sparse: the ordered active list; null: slot = pixel
    const unsigned int* n_active;    // sparse: its length
    int npix, W, K;
    float* flow;
};
hipError_t launch_lk_window(const LkWindowArgs& a, int max_slots, hipStream_t stream);

}  // namespace evsim
