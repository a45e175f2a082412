// Internal interface between the HIP kernels (evsim_kernels.hip) and the host runtime
// (evsim_runtime.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace evsim {

constexpr int kSimThreads = 256;     // pixels per simulation tile (one per thread)
constexpr int kMaxStash = 31;        // interior samples kept in LDS per pixel (S - 1 <= 31)
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per sort block
constexpr uint64_t kSentinel = ~0ull;

enum Method { kBasic = 0, kDense = 1, kSparse = 2 };

// Layout of the unsorted "sort key" written by the simulation kernel, low bits first:
//   p (1) | x (xb) | y (yb) | t_rel (tb) | interval index within the window (ib)
// Sorting these keys ascending gives interval-major (t, y, x, p) order.  One extra bit above the
// layout is always sorted so that the all-ones sentinel (unused slots) sorts after every key.
struct KeyLayout {
    int xb, yb, tb, ib;
    __host__ __device__ int pix_bits() const { return xb + yb + 1; }
    __host__ __device__ int total_bits() const { return ib + tb + xb + yb + 1; }
};

struct SimArgs {
    const uint8_t* prev;        // frame before the window, uint8 [H][W]
    const uint8_t* frames;      // window frames; frame j at frames + j * fstride
    int64_t fstride;
    const float* flows;         // flow of interval j at flows + j * flstride (null for basic)
    int64_t flstride;
    const float* lut;           // 256-entry transform table
    const float* delta;         // per interval: (float)(t_j - t_{j-1})
    float* lref;                // per-pixel reference level, updated in place
    uint8_t* prev_out;          // receives the window's last frame (may be null)
    uint64_t* arena;            // unsorted sort keys
    uint64_t cap;               // arena capacity (keys)
    unsigned long long* counters;  // [0] reserved, [1] committed, [2] failed tiles, [3] selected
    unsigned int* icount;       // committed events per interval of the window
    int* resume;                // per tile: first interval to run; on exit the first not run
    int W, H, S, K, method, ntiles;
    float cpos, cneg, m;
    KeyLayout lay;
};

struct ConvertArgs {
    int enabled;                // final pass: write packed ABI keys instead of sort keys
    uint64_t n_valid;           // keys below this position are real events
    const int64_t* tbase;       // per interval: t_{j-1} - epoch
    KeyLayout lay;
};

// Launchers (all asynchronous on `stream`).
hipError_t launch_init(const uint8_t* frame, const float* lut, float* lref, uint8_t* prev,
                       int64_t npix, hipStream_t stream);
hipError_t launch_simulate(const SimArgs& a, hipStream_t stream);
// Sorts keys[0, n) on bits [0, nbits) (stable LSD radix, 8-bit digits); the last pass writes
// into `out` converted by `cv`.  `alt` holds n keys; `hist` holds 256 * ceil(n / kSortTile)
// counters and `totals` 256.
hipError_t launch_sort(uint64_t* keys, uint64_t* alt, uint64_t n, int nbits, uint32_t* hist,
                       uint32_t* totals, uint64_t* out, const ConvertArgs& cv, hipStream_t stream);
size_t sort_hist_entries(uint64_t n);

}  // namespace evsim
