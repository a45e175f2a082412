// HIP kernels of the event simulator for gfx950 (MI355X).
//
// Arithmetic follows the paper's pipeline (Ziegler et al., arXiv 2209.04634): transformed camera
// frames (Sec. III), flow-driven intermediate frames (Sec. III-A; sparse selection, Sec. III-B),
// difference against a per-pixel reference level thresholded with C_pos / C_neg (Sec. III-A
// threshold equations, in the event-pixel form of Sec. I), events <x, y, t, p> (Fig. 1 caption).
// Every floating-point operation is one fp32 operation with one rounding in the order written
// here; the file is compiled with -ffp-contract=off so no multiply-add is fused.
#include "evsim_internal.h"

#pragma clang fp contract(off)

namespace evsim {

// ------------------------------------------------------------------------------------------
// Helpers
// ------------------------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
// tiles so that neighbouring tiles (which gather the same texels) share an L2.
__device__ __forceinline__ int xcd_tile(int b, int g) {
    const int q = g >> 3, r = g & 7;
    const int xcd = b & 7, idx = b >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Exclusive scan over a 256-thread block; returns this thread's prefix and the block total.
// `wsum` is 4 ints of LDS; the caller must synchronise before `wsum` is reused.
__device__ __forceinline__ int block_scan_256(int v, int* wsum, int* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int before = 0;
    for (int j = 0; j < w; ++j) before += wsum[j];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    return before + inc - v;
}

// Clamp-to-edge bilinear sample of T[F] at (sx, sy).
__device__ __forceinline__ float bilinear(const uint8_t* __restrict__ F, const float* lut, int W,
                                          int H, float sx, float sy) {
    sx = fminf(fmaxf(sx, 0.0f), (float)(W - 1));
    sy = fminf(fmaxf(sy, 0.0f), (float)(H - 1));
    const int x0 = (int)floorf(sx);
    const int y0 = (int)floorf(sy);
    const float fx = sx - (float)x0;
    const float fy = sy - (float)y0;
    const int x1 = min(x0 + 1, W - 1);
    const int y1 = min(y0 + 1, H - 1);
    const float gx = 1.0f - fx;
    const float gy = 1.0f - fy;
    const uint8_t* r0 = F + (int64_t)y0 * W;
    const uint8_t* r1 = F + (int64_t)y1 * W;
    const float top = gx * lut[r0[x0]] + fx * lut[r0[x1]];
    const float bot = gx * lut[r1[x0]] + fx * lut[r1[x1]];
    return gy * top + fy * bot;
}

// Interior sample V_k (0 < k < S) of the flow-guided blend between frames F0 and F1.
__device__ __forceinline__ float interp_sample(const uint8_t* F0, const uint8_t* F1,
                                               const float* lut, int W, int H, int x, int y,
                                               float u, float v, int k, int S) {
    const float tau = (float)k / (float)S;
    const float om = 1.0f - tau;
    const float a = bilinear(F0, lut, W, H, (float)x - tau * u, (float)y - tau * v);
    const float b = bilinear(F1, lut, W, H, (float)x + om * u, (float)y + om * v);
    return om * a + tau * b;
}

struct PixelCtx {
    const uint8_t* F0;
    const uint8_t* F1;
    const float* lut;
    const float* stash;     // column of this thread's interior samples (stride 256) or null
    int W, H, x, y, S;
    float u, v;
};

__device__ __forceinline__ float sample_k(const PixelCtx& c, int k, float A1) {
    if (k == c.S) return A1;
    if (c.stash) return c.stash[(k - 1) * kSimThreads];
    return interp_sample(c.F0, c.F1, c.lut, c.W, c.H, c.x, c.y, c.u, c.v, k, c.S);
}

// Threshold crossings of one pixel's series V_0 = A0 .. V_S = A1 against reference level R.
// Counts (WRITE = false) or writes (WRITE = true) the events; returns the count and leaves the
// final level in *Rout.
template <bool WRITE>
__device__ __forceinline__ int crossings(const PixelCtx& c, float R, float A0, float A1,
                                         float cpos, float cneg, float delta, uint64_t keyhi,
                                         int pbits, uint64_t pixkey, uint64_t* out, float* Rout) {
    int n = 0;
    float A = A0;
    for (int k = 0; k < c.S; ++k) {
        const float B = sample_k(c, k + 1, A1);
        const float D = B - A;
        for (;;) {
            int pol;
            float Rn;
            if (B - R >= cpos) {
                Rn = R + cpos;
                pol = 1;
            } else if (B - R <= -cneg) {
                Rn = R - cneg;
                pol = -1;
            } else {
                break;
            }
            if (WRITE) {
                float theta;
                const bool backlog = pol > 0 ? (A >= Rn) : (A <= Rn);
                if (backlog) {
                    theta = 0.0f;
                } else {
                    theta = (D == 0.0f) ? 0.0f : (Rn - A) / D;
                    theta = fminf(fmaxf(theta, 0.0f), 1.0f);
                }
                const float phi = ((float)k + theta) / (float)c.S;
                const uint64_t trel = (uint64_t)(int64_t)floorf(phi * delta);
                out[n] = keyhi | (trel << pbits) | pixkey | (pol > 0 ? 1ull : 0ull);
            }
            ++n;
            R = Rn;
        }
        A = B;
    }
    *Rout = R;
    return n;
}

// ------------------------------------------------------------------------------------------
// First frame: reference levels from the transformed frame, previous-frame copy.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(const uint8_t* __restrict__ frame,
                                              const float* __restrict__ lut,
                                              float* __restrict__ lref, uint8_t* __restrict__ prev,
                                              int64_t npix) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npix) {
        const uint8_t v = frame[p];
        lref[p] = lut[v];
        prev[p] = v;
    }
}

// ------------------------------------------------------------------------------------------
// Simulation of a window of K frame intervals.  One workgroup owns a tile of 256 consecutive
// pixels (row-major) for the whole window and carries their reference levels in registers from
// interval to interval (the only temporal dependency is per pixel).  Per interval:
//   1. transform, sparse selection, interior samples into LDS, count the events;
//   2. block scan of the counts, one arena reservation per workgroup;
//   3. if it fits, write the events; otherwise fill the reserved slots with sentinels, keep the
//      levels of the last completed interval and record where to resume (the host grows the
//      arena and relaunches only the unfinished tiles).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kSimThreads) void k_simulate(SimArgs a) {
    extern __shared__ float smem[];
    __shared__ int s_wsum[4];
    __shared__ int s_wsel[4];
    __shared__ unsigned long long s_base;
    __shared__ int s_fail;

    float* lut = smem;
    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    lut[tid] = a.lut[tid];
    const int start = a.resume[tile];
    __syncthreads();
    if (start >= a.K) return;

    const int stash_n = (a.S - 1 <= kMaxStash) ? (a.S - 1) : 0;
    float* stash = smem + 256 + tid;

    const int64_t npix = (int64_t)a.W * a.H;
    const int64_t p = (int64_t)tile * kSimThreads + tid;
    const bool inb = p < npix;
    const int y = inb ? (int)(p / a.W) : 0;
    const int x = inb ? (int)(p - (int64_t)y * a.W) : 0;
    const int pbits = a.lay.pix_bits();
    const int ishift = a.lay.tb + pbits;
    const uint64_t pixkey = ((uint64_t)y << (a.lay.xb + 1)) | ((uint64_t)x << 1);

    float R = inb ? a.lref[p] : 0.0f;
    const uint8_t* Fs = start == 0 ? a.prev : a.frames + (int64_t)(start - 1) * a.fstride;
    float A0 = inb ? lut[Fs[p]] : 0.0f;

    int i = start;
    for (; i < a.K; ++i) {
        const uint8_t* F0 = i == 0 ? a.prev : a.frames + (int64_t)(i - 1) * a.fstride;
        const uint8_t* F1 = a.frames + (int64_t)i * a.fstride;
        const float A1 = inb ? lut[F1[p]] : 0.0f;
        const float delta = a.delta[i];
        const bool sel = inb && (a.method != kSparse || fabsf(A1 - A0) >= a.m);

        PixelCtx c;
        c.F0 = F0; c.F1 = F1; c.lut = lut; c.W = a.W; c.H = a.H; c.x = x; c.y = y; c.S = a.S;
        c.u = 0.0f; c.v = 0.0f; c.stash = nullptr;
        float Rn = R;
        int n = 0;
        if (sel) {
            if (a.S > 1) {
                const float* fl = a.flows + (int64_t)i * a.flstride + 2 * p;
                c.u = fl[0];
                c.v = fl[1];
                for (int k = 1; k <= stash_n; ++k)
                    stash[(k - 1) * kSimThreads] =
                        interp_sample(F0, F1, lut, a.W, a.H, x, y, c.u, c.v, k, a.S);
                if (stash_n) c.stash = stash;
            }
            n = crossings<false>(c, R, A0, A1, a.cpos, a.cneg, delta, 0, pbits, 0, nullptr, &Rn);
        }
        const uint64_t wsel = __ballot(sel);
        if ((tid & 63) == 0) s_wsel[tid >> 6] = __popcll(wsel);
        int total;
        const int off = block_scan_256(n, s_wsum, &total);
        if (tid == 0) {
            int fail = 0;
            unsigned long long base = 0;
            if (total > 0) {
                base = atomicAdd(&a.counters[0], (unsigned long long)total);
                if (base + (unsigned long long)total > a.cap) {
                    fail = 1;
                    atomicAdd(&a.counters[2], 1ull);
                } else {
                    atomicAdd(&a.counters[1], (unsigned long long)total);
                    atomicAdd(&a.icount[i], (unsigned int)total);
                }
            }
            if (!fail) {
                const int nsel = s_wsel[0] + s_wsel[1] + s_wsel[2] + s_wsel[3];
                if (nsel) atomicAdd(&a.counters[3], (unsigned long long)nsel);
            }
            s_base = base;
            s_fail = fail;
        }
        __syncthreads();
        if (s_fail) {
            const unsigned long long b = s_base;
            const unsigned long long e = min(b + (unsigned long long)total, (unsigned long long)a.cap);
            for (unsigned long long j = b + tid; j < e; j += kSimThreads) a.arena[j] = kSentinel;
            break;
        }
        if (n > 0) {
            const uint64_t keyhi = (uint64_t)i << ishift;
            crossings<true>(c, R, A0, A1, a.cpos, a.cneg, delta, keyhi, pbits, pixkey,
                            a.arena + s_base + off, &Rn);
        }
        if (sel) R = Rn;
        A0 = A1;
    }
    if (inb) a.lref[p] = R;
    if (tid == 0) a.resume[tile] = i;
    if (i == a.K && a.prev_out && inb) a.prev_out[p] = a.frames[(int64_t)(a.K - 1) * a.fstride + p];
}

// ------------------------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, three kernels per pass.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                             uint64_t n, int shift,
                                                             uint32_t* __restrict__ hist,
                                                             int nblocks) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
        const uint64_t idx = base + (uint64_t)j * kSortThreads + tid;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = h[tid];
}

// One block per digit: exclusive scan of that digit's per-block counts; row total to totals[d].
__global__ __launch_bounds__(kSortThreads) void k_radix_rowscan(uint32_t* __restrict__ hist,
                                                                int nblocks,
                                                                uint32_t* __restrict__ totals) {
    __shared__ int s_wsum[4];
    uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int b = 0; b < nblocks; b += kSortThreads) {
        const int j = b + threadIdx.x;
        const int v = j < nblocks ? (int)row[j] : 0;
        int tot;
        const int ex = block_scan_256(v, s_wsum, &tot);
        if (j < nblocks) row[j] = carry + (uint32_t)ex;
        carry += (uint32_t)tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__device__ __forceinline__ uint64_t convert_key(uint64_t k, const ConvertArgs& cv) {
    const KeyLayout& L = cv.lay;
    const int pb = L.pix_bits();
    const uint64_t pix = k & ((1ull << pb) - 1);
    const uint64_t trel = (k >> pb) & ((1ull << L.tb) - 1);
    const uint64_t iv = k >> (pb + L.tb);
    const uint64_t x = (pix >> 1) & ((1ull << L.xb) - 1);
    const uint64_t y = (pix >> (L.xb + 1)) & ((1ull << L.yb) - 1);
    const uint64_t t = (uint64_t)cv.tbase[iv] + trel;
    return (t << 25) | (y << 13) | (x << 1) | (pix & 1ull);
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t n, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int nblocks,
    ConvertArgs cv) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wcnt[4][256];
    __shared__ int s_wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int tot;
    const int dex = block_scan_256((int)totals[tid], s_wsum, &tot);
    s_base[tid] = (uint32_t)dex + hist[(size_t)tid * nblocks + blockIdx.x];
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortItems; ++j) {
        s_wcnt[0][tid] = 0;
        s_wcnt[1][tid] = 0;
        s_wcnt[2][tid] = 0;
        s_wcnt[3][tid] = 0;
        __syncthreads();
        const uint64_t idx = base + (uint64_t)j * kSortThreads + tid;
        const bool valid = idx < n;
        const uint64_t key = valid ? in[idx] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int q = 0; q < w; ++q) pre += s_wcnt[q][d];
            const uint64_t pos = (uint64_t)s_base[d] + pre + rank;
            if (!cv.enabled) {
                out[pos] = key;
            } else if (pos < cv.n_valid) {
                out[pos] = convert_key(key, cv);
            }
        }
        __syncthreads();
        s_base[tid] += s_wcnt[0][tid] + s_wcnt[1][tid] + s_wcnt[2][tid] + s_wcnt[3][tid];
    }
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
hipError_t launch_init(const uint8_t* frame, const float* lut, float* lref, uint8_t* prev,
                       int64_t npix, hipStream_t stream) {
    const int64_t blocks = (npix + 255) / 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, stream, frame, lut, lref,
                       prev, npix);
    return hipGetLastError();
}

hipError_t launch_simulate(const SimArgs& a, hipStream_t stream) {
    const int stash_n = (a.S - 1 <= kMaxStash) ? (a.S - 1) : 0;
    const size_t shmem = (size_t)(256 + stash_n * kSimThreads) * sizeof(float);
    hipLaunchKernelGGL(k_simulate, dim3((unsigned)a.ntiles), dim3(kSimThreads), shmem, stream, a);
    return hipGetLastError();
}

size_t sort_hist_entries(uint64_t n) {
    const uint64_t nb = (n + kSortTile - 1) / kSortTile;
    return (size_t)(nb ? nb : 1) * 256;
}

hipError_t launch_sort(uint64_t* keys, uint64_t* alt, uint64_t n, int nbits, uint32_t* hist,
                       uint32_t* totals, uint64_t* out, const ConvertArgs& cv,
                       hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
    const int passes = (nbits + 7) / 8;
    uint64_t* src = keys;
    uint64_t* dst = alt;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        const bool last = pass == passes - 1;
        ConvertArgs c = cv;
        if (!last) c.enabled = 0;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kSortThreads), 0, stream, src, n,
                           shift, hist, nblocks);
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, stream, hist,
                           nblocks, totals);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortThreads), 0, stream, src,
                           last ? out : dst, n, shift, hist, totals, nblocks, c);
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    return hipGetLastError();
}

}  // namespace evsim
