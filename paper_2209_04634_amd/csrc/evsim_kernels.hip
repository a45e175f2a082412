// HIP kernels of the event simulator for gfx950 (MI355X).
//
// Arithmetic follows the paper's pipeline (Ziegler et al., arXiv 2209.04634): transformed camera
// frames (Sec. III), flow-driven intermediate frames (Sec. III-A; sparse selection, Sec. III-B),
// difference against a per-pixel reference level thresholded with C_pos / C_neg (Sec. III-A
// threshold equations, in the event-pixel form of Sec. I), events <x, y, t, p> (Fig. 1 caption).
// Every floating-point operation is one fp32 operation with one rounding in the order written
// here; the file is compiled with -ffp-contract=off so no multiply-add is fused.
#include "evsim_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace evsim {

// ------------------------------------------------------------------------------------------
// Helpers
// ------------------------------------------------------------------------------------------

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

// Clamp-to-edge bilinear footprint of the sample position (sx, sy): the offsets of its four
// texels and its weights.  Callers load every texel of a sample before blending any, so that
// the loads of one sample are in flight together.
struct BilTap {
    int64_t o00, o01, o10, o11;
    float fx, fy, gx, gy;
};

__device__ __forceinline__ BilTap bil_tap(int W, int H, float sx, float sy) {
    sx = fminf(fmaxf(sx, 0.0f), (float)(W - 1));
    sy = fminf(fmaxf(sy, 0.0f), (float)(H - 1));
    const int x0 = (int)floorf(sx);
    const int y0 = (int)floorf(sy);
    BilTap t;
    t.fx = sx - (float)x0;
    t.fy = sy - (float)y0;
    const int x1 = min(x0 + 1, W - 1);
    const int y1 = min(y0 + 1, H - 1);
    t.gx = 1.0f - t.fx;
    t.gy = 1.0f - t.fy;
    const int64_t r0 = (int64_t)y0 * W;
    const int64_t r1 = (int64_t)y1 * W;
    t.o00 = r0 + x0;
    t.o01 = r0 + x1;
    t.o10 = r1 + x0;
    t.o11 = r1 + x1;
    return t;
}

// Bilinear blend of four texel values v (already transformed) with the tap's weights.
__device__ __forceinline__ float bil_blend(const BilTap& t, float v00, float v01, float v10,
                                           float v11) {
    const float top = t.gx * v00 + t.fx * v01;
    const float bot = t.gx * v10 + t.fx * v11;
    return t.gy * top + t.fy * bot;
}

// Interior sample V_k (0 < k < S) of the flow-guided blend between frames F0 and F1, at
// tau = k / S (one fp32 division, taken from the block's table): clamp-to-edge bilinear samples
// of T[F0] at p - tau F and of T[F1] at p + (1 - tau) F.
__device__ __forceinline__ float interp_sample(const uint8_t* F0, const uint8_t* F1,
                                               const float* lut, int W, int H, int x, int y,
                                               float u, float v, float tau) {
    const float om = 1.0f - tau;
    const BilTap ta = bil_tap(W, H, (float)x - tau * u, (float)y - tau * v);
    const BilTap tb = bil_tap(W, H, (float)x + om * u, (float)y + om * v);
    const uint32_t a00 = F0[ta.o00], a01 = F0[ta.o01], a10 = F0[ta.o10], a11 = F0[ta.o11];
    const uint32_t b00 = F1[tb.o00], b01 = F1[tb.o01], b10 = F1[tb.o10], b11 = F1[tb.o11];
    const float a = bil_blend(ta, lut[a00], lut[a01], lut[a10], lut[a11]);
    const float b = bil_blend(tb, lut[b00], lut[b01], lut[b10], lut[b11]);
    return om * a + tau * b;
}

// The same footprint with 32-bit texel offsets (a frame has fewer than 2^24 pixels) and the
// bounds as floats (wm1 = W - 1, hm1 = H - 1).  fx = sx - floor(sx) equals sx - (float)x0
// exactly: floor is exact and x0 < 2^24.
struct Tap32 {
    uint32_t o00, o01, o10, o11;
    float fx, fy;
};

__device__ __forceinline__ Tap32 tap32(int W, int H, float wm1, float hm1, float sx, float sy) {
    sx = fminf(fmaxf(sx, 0.0f), wm1);
    sy = fminf(fmaxf(sy, 0.0f), hm1);
    const float flx = floorf(sx);
    const float fly = floorf(sy);
    const int x0 = (int)flx;
    const int y0 = (int)fly;
    const int x1 = min(x0 + 1, W - 1);
    const int y1 = min(y0 + 1, H - 1);
    Tap32 t;
    t.fx = sx - flx;
    t.fy = sy - fly;
    const uint32_t r0 = __umul24((uint32_t)y0, (uint32_t)W);
    const uint32_t r1 = __umul24((uint32_t)y1, (uint32_t)W);
    t.o00 = r0 + (uint32_t)x0;
    t.o01 = r0 + (uint32_t)x1;
    t.o10 = r1 + (uint32_t)x0;
    t.o11 = r1 + (uint32_t)x1;
    return t;
}

// bil_blend with the weights given as (fx, fy).
__device__ __forceinline__ float blend_w(float fx, float fy, float v00, float v01, float v10,
                                         float v11) {
    const float gx = 1.0f - fx;
    const float gy = 1.0f - fy;
    const float top = gx * v00 + fx * v01;
    const float bot = gx * v10 + fx * v11;
    return gy * top + fy * bot;
}

// Interior samples V_k, k = k0 .. min(k0 + G - 1, klast), of the frame methods into the stash
// (stride kSimThreads): the same arithmetic as interp_sample, with every texel load of the G
// samples issued before any of them is blended, so that a lane has 8 G loads in flight at once.
template <int G>
__device__ __forceinline__ void stash_frame_samples(const uint8_t* F0, const uint8_t* F1,
                                                    const float* lut, const float* tau, int W,
                                                    int H, float wm1, float hm1, float xf,
                                                    float yf, float u, float v, int k0, int klast,
                                                    float* stash) {
    uint32_t t[G][8];
    float w[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int k = k0 + g;
        if (k <= klast) {
            const float tk = tau[k];
            const float om = 1.0f - tk;
            const Tap32 ta = tap32(W, H, wm1, hm1, xf - tk * u, yf - tk * v);
            const Tap32 tb = tap32(W, H, wm1, hm1, xf + om * u, yf + om * v);
            t[g][0] = F0[ta.o00];
            t[g][1] = F0[ta.o01];
            t[g][2] = F0[ta.o10];
            t[g][3] = F0[ta.o11];
            t[g][4] = F1[tb.o00];
            t[g][5] = F1[tb.o01];
            t[g][6] = F1[tb.o10];
            t[g][7] = F1[tb.o11];
            w[g][0] = ta.fx;
            w[g][1] = ta.fy;
            w[g][2] = tb.fx;
            w[g][3] = tb.fy;
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int k = k0 + g;
        if (k <= klast) {
            const float tk = tau[k];
            const float om = 1.0f - tk;
            const float a = blend_w(w[g][0], w[g][1], lut[t[g][0]], lut[t[g][1]], lut[t[g][2]],
                                    lut[t[g][3]]);
            const float b = blend_w(w[g][2], w[g][3], lut[t[g][4]], lut[t[g][5]], lut[t[g][6]],
                                    lut[t[g][7]]);
            stash[(k - 1) * kSimThreads] = om * a + tk * b;
        }
    }
}

// The difference method's interior difference frames D_k into the stash, batched the same way
// (16 texel loads per sample): the arithmetic of interp_diff_sample.
template <int G>
__device__ __forceinline__ void stash_diff_samples(const uint8_t* Fm, const uint8_t* F0,
                                                   const uint8_t* F1, const float* lut,
                                                   const float* tau, int W, int H, float wm1,
                                                   float hm1, float xf, float yf, float u,
                                                   float v, int k0, int klast, float* stash) {
    uint32_t t[G][16];
    float w[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int k = k0 + g;
        if (k <= klast) {
            const float tk = tau[k];
            const float om = 1.0f - tk;
            const Tap32 ta = tap32(W, H, wm1, hm1, xf - tk * u, yf - tk * v);
            const Tap32 tb = tap32(W, H, wm1, hm1, xf + om * u, yf + om * v);
            t[g][0] = Fm[ta.o00];
            t[g][1] = Fm[ta.o01];
            t[g][2] = Fm[ta.o10];
            t[g][3] = Fm[ta.o11];
            t[g][4] = F0[ta.o00];
            t[g][5] = F0[ta.o01];
            t[g][6] = F0[ta.o10];
            t[g][7] = F0[ta.o11];
            t[g][8] = F0[tb.o00];
            t[g][9] = F0[tb.o01];
            t[g][10] = F0[tb.o10];
            t[g][11] = F0[tb.o11];
            t[g][12] = F1[tb.o00];
            t[g][13] = F1[tb.o01];
            t[g][14] = F1[tb.o10];
            t[g][15] = F1[tb.o11];
            w[g][0] = ta.fx;
            w[g][1] = ta.fy;
            w[g][2] = tb.fx;
            w[g][3] = tb.fy;
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int k = k0 + g;
        if (k <= klast) {
            const float tk = tau[k];
            const float om = 1.0f - tk;
            const float a = blend_w(w[g][0], w[g][1], lut[t[g][4]] - lut[t[g][0]],
                                    lut[t[g][5]] - lut[t[g][1]], lut[t[g][6]] - lut[t[g][2]],
                                    lut[t[g][7]] - lut[t[g][3]]);
            const float b = blend_w(w[g][2], w[g][3], lut[t[g][12]] - lut[t[g][8]],
                                    lut[t[g][13]] - lut[t[g][9]], lut[t[g][14]] - lut[t[g][10]],
                                    lut[t[g][15]] - lut[t[g][11]]);
            stash[(k - 1) * kSimThreads] = om * a + tk * b;
        }
    }
}

// Chain-pass variants: interior samples whose texel loads a lane keeps in flight at once (frame
// methods / difference method).  More samples in flight hide more memory latency per wave but
// take registers and so waves per SIMD; which is faster depends on the image, the method and the
// selected fraction, so the runtime times the variants on the device (autotuner).  Every variant
// performs the same arithmetic in the same order.
template <int V> struct ChainVariant;
template <> struct ChainVariant<0> { static constexpr int frame = 2, diff = 1; };
template <> struct ChainVariant<1> { static constexpr int frame = 5, diff = 2; };
template <> struct ChainVariant<2> { static constexpr int frame = 10, diff = 4; };

struct PixelCtx {
    const uint8_t* F0;
    const uint8_t* F1;
    const float* lut;
    const float* stash;     // column of this thread's interior samples (stride 256) or null
    const float* tau;       // tau[k] = k / S, k = 0..S (LDS table of the block)
    int W, H, x, y, S;
    float u, v;
    const uint8_t* Fm;      // difference method: the frame before F0
};

__device__ __forceinline__ float sample_k(const PixelCtx& c, int k, float A1) {
    if (k == c.S) return A1;
    if (c.stash) return c.stash[(k - 1) * kSimThreads];
    return interp_sample(c.F0, c.F1, c.lut, c.W, c.H, c.x, c.y, c.u, c.v, c.tau[k]);
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

// Interior interpolated difference frame D_k (0 < k < S) of the difference method (Sec. III-C):
// the same flow-guided blend as interp_sample, between D1 = T[F0] - T[Fm] and D2 = T[F1] - T[F0],
// each texel difference one fp32 subtraction before the bilinear blend.
__device__ __forceinline__ float interp_diff_sample(const uint8_t* Fm, const uint8_t* F0,
                                                    const uint8_t* F1, const float* lut, int W,
                                                    int H, int x, int y, float u, float v,
                                                    float tau) {
    const float om = 1.0f - tau;
    const BilTap ta = bil_tap(W, H, (float)x - tau * u, (float)y - tau * v);
    const BilTap tb = bil_tap(W, H, (float)x + om * u, (float)y + om * v);
    const uint32_t m00 = Fm[ta.o00], m01 = Fm[ta.o01], m10 = Fm[ta.o10], m11 = Fm[ta.o11];
    const uint32_t p00 = F0[ta.o00], p01 = F0[ta.o01], p10 = F0[ta.o10], p11 = F0[ta.o11];
    const uint32_t q00 = F0[tb.o00], q01 = F0[tb.o01], q10 = F0[tb.o10], q11 = F0[tb.o11];
    const uint32_t c00 = F1[tb.o00], c01 = F1[tb.o01], c10 = F1[tb.o10], c11 = F1[tb.o11];
    const float a = bil_blend(ta, lut[p00] - lut[m00], lut[p01] - lut[m01], lut[p10] - lut[m10],
                              lut[p11] - lut[m11]);
    const float b = bil_blend(tb, lut[c00] - lut[q00], lut[c01] - lut[q01], lut[c10] - lut[q10],
                              lut[c11] - lut[q11]);
    return om * a + tau * b;
}

template <int MODE>
__device__ __forceinline__ float sample_mode(const PixelCtx& c, int k, float A1) {
    if (k == c.S) return A1;
    if (c.stash) return c.stash[(k - 1) * kSimThreads];
    if constexpr (MODE == kModeDifference)
        return interp_diff_sample(c.Fm, c.F0, c.F1, c.lut, c.W, c.H, c.x, c.y, c.u, c.v,
                                  c.tau[k]);
    else
        return interp_sample(c.F0, c.F1, c.lut, c.W, c.H, c.x, c.y, c.u, c.v, c.tau[k]);
}

// Memoryless thresholding of one pixel's interval (the paper's Sec. III-A equations taken
// literally): the value compared at sub-frame k + 1 is V_{k+1} - V_k (kModeMemoryless, series
// V_0 = A0 .. V_S = A1) or the interpolated difference frame D_{k+1} (kModeDifference, D_S = A1).
// Strictly above C_pos fires positive, strictly below -C_neg negative, at most once per sub-frame,
// stamped at the sub-frame's time t0 + floor((k + 1) / S * delta).  Counts (WRITE = false) or
// writes (WRITE = true) the events and returns the count.
template <int MODE, bool WRITE>
__device__ __forceinline__ int flips(const PixelCtx& c, float A0, float A1, float cpos,
                                     float cneg, float delta, uint64_t keyhi, int pbits,
                                     uint64_t pixkey, uint64_t* out) {
    int n = 0;
    float A = A0;
    for (int k = 0; k < c.S; ++k) {
        const float B = sample_mode<MODE>(c, k + 1, A1);
        const float D = (MODE == kModeMemoryless) ? B - A : B;
        int pol = 0;
        if (D > cpos)
            pol = 1;
        else if (D < -cneg)
            pol = -1;
        if (pol != 0) {
            if (WRITE) {
                const float phi = c.tau[k + 1];   // (k + 1) / S
                const uint64_t trel = (uint64_t)(int64_t)floorf(phi * delta);
                out[n] = keyhi | (trel << pbits) | pixkey | (pol > 0 ? 1ull : 0ull);
            }
            ++n;
        }
        A = B;
    }
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
// Wave-level helpers (wave64)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Per-class counts over a wave, without atomics on shared addresses: every lane contributes
// packed 16-bit counts of the kClasses length classes (four classes per word); returns the lane's
// exclusive prefix in *excl and the wave's totals in *tot (both packed the same way).  Each field
// stays below 2^16 (a wave counts at most 256 pixels).
constexpr int kClassWords = 4;   // kClasses / 4
__device__ __forceinline__ void wave_class_counts(const uint64_t (&mine)[kClassWords],
                                                  uint64_t (&excl)[kClassWords],
                                                  uint64_t (&tot)[kClassWords]) {
#pragma unroll
    for (int k = 0; k < kClassWords; ++k) {
        const uint64_t inc = wave_incl_scan_u64(mine[k]);
        excl[k] = inc - mine[k];
        tot[k] = __shfl(inc, 63, 64);
    }
}

// Field c of packed class counts (selects, no indexed access, so the words stay in registers).
__device__ __forceinline__ uint32_t class_field(const uint64_t (&w)[kClassWords], uint32_t c) {
    const uint32_t k = c >> 2;
    const uint64_t v = k == 0 ? w[0] : (k == 1 ? w[1] : (k == 2 ? w[2] : w[3]));
    return (uint32_t)(v >> (16 * (c & 3u))) & 0xFFFFu;
}

// Adds one to field c of packed class counts.
__device__ __forceinline__ void class_add(uint64_t (&w)[kClassWords], uint32_t c) {
    const uint64_t one = 1ull << (16 * (c & 3u));
    const uint32_t k = c >> 2;
    w[0] += k == 0 ? one : 0ull;
    w[1] += k == 1 ? one : 0ull;
    w[2] += k == 2 ? one : 0ull;
    w[3] += k == 3 ? one : 0ull;
}

__device__ __forceinline__ uint32_t pick4(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3,
                                          int w) {
    return w == 0 ? m0 : (w == 1 ? m1 : (w == 2 ? m2 : m3));
}

// First selected interval >= i (K when none is left).
__device__ __forceinline__ int next_selected(bool all, uint32_t m0, uint32_t m1, uint32_t m2,
                                             uint32_t m3, int i, int K) {
    if (all) return min(i, K);
    while (i < K) {
        const int w = i >> 5;
        const uint32_t bits = pick4(m0, m1, m2, m3, w) >> (i & 31);
        if (bits) return min(i + __ffs(bits) - 1, K);
        i = (w + 1) << 5;
    }
    return K;
}

// ------------------------------------------------------------------------------------------
// Selection pass of the sparse method (Sec. III-B): a pixel-interval is interpolated only if the
// transformed frame-to-frame change reaches m.  Each thread streams 4 consecutive pixels through
// every frame of the window once, builds their selected-interval bitmasks, saves the window's
// last frame for the next window, and appends the pixels selected at least once to the active
// list (wave-aggregated reservation).
// ------------------------------------------------------------------------------------------
template <bool VEC>
__device__ __forceinline__ void select_block(SelectArgs a, unsigned bid) {
    __shared__ float lut[256];
    const int tid = threadIdx.x;
    lut[tid] = a.lut[tid];
    __syncthreads();
    const int lane = tid & 63, wv = tid >> 6;
    const int base = (bid * 256 + tid) * 4;
    const int cnt = max(0, min(4, a.npix - base));

    uint32_t last = 0;
    float A0[4];
    if (VEC && cnt == 4) {
        last = *(const uint32_t*)(a.prev + base);
    } else {
        for (int q = 0; q < cnt; ++q) last |= (uint32_t)a.prev[base + q] << (8 * q);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) A0[q] = lut[(last >> (8 * q)) & 255u];

    uint32_t any[4] = {0u, 0u, 0u, 0u};
    int plen[4] = {0, 0, 0, 0};     // selected intervals per pixel
    int nsel = 0;
    for (int w = 0; w < kMaskWords && w * 32 < a.K; ++w) {
        uint32_t mw[4] = {0u, 0u, 0u, 0u};
        const int jend = min(32, a.K - w * 32);
        const uint8_t* Fw = a.frames + (int64_t)(w * 32) * a.fstride + base;
        // one frame's four pixels: transform, compare with the previous frame, set bit jj
        auto step = [&](uint32_t v, int jj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float A1 = lut[(v >> (8 * q)) & 255u];
                mw[q] |= (uint32_t)(fabsf(A1 - A0[q]) >= a.m) << jj;
                A0[q] = A1;
            }
            last = v;
        };
        if (VEC && cnt == 4) {
            // sixteen frames' loads issued before any is used, so that they are in flight together
            int jj = 0;
            for (; jj + 16 <= jend; jj += 16) {
                uint32_t v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    v[u] = *(const uint32_t*)(Fw + (int64_t)(jj + u) * a.fstride);
#pragma unroll
                for (int u = 0; u < 16; ++u) step(v[u], jj + u);
            }
            for (; jj < jend; ++jj) step(*(const uint32_t*)(Fw + (int64_t)jj * a.fstride), jj);
        } else {
            for (int jj = 0; jj < jend; ++jj) {
                const uint8_t* F = Fw + (int64_t)jj * a.fstride;
                uint32_t v = 0;
                for (int q = 0; q < cnt; ++q) v |= (uint32_t)F[q] << (8 * q);
                step(v, jj);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < cnt) {
                a.mask[(int64_t)w * a.npix + base + q] = mw[q];
                any[q] |= mw[q];
                plen[q] += __popc(mw[q]);
            }
        }
    }
    if (VEC && cnt == 4) {
        *(uint32_t*)(a.prev_out + base) = last;
    } else {
        for (int q = 0; q < cnt; ++q) a.prev_out[base + q] = (uint8_t)(last >> (8 * q));
    }

    // The block's run of active pixels: class kClasses-1 first, pixel order within a class.
    // Ranks come from a block-wide exclusive scan of packed per-class counts (no atomics).
    __shared__ uint64_t s_wt[4][kClassWords];   // per wave: class totals
    __shared__ uint32_t s_cs[kClasses];         // start of each class in the run
    __shared__ uint32_t s_nsel[4];
    uint32_t cls[4];
    bool act[4];
    uint64_t cw[kClassWords] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        nsel += plen[q];
        cls[q] = (uint32_t)(min(plen[q], kClasses) - 1);
        act[q] = q < cnt && any[q] != 0u;
        if (act[q]) class_add(cw, cls[q]);
    }
    uint64_t ex[kClassWords], wt[kClassWords];
    wave_class_counts(cw, ex, wt);
    const int wsel = wave_incl_scan(nsel);
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < kClassWords; ++k) s_wt[wv][k] = wt[k];
        s_nsel[wv] = (uint32_t)wsel;
    }
    __syncthreads();
    uint64_t bt[kClassWords], wp[kClassWords];
#pragma unroll
    for (int k = 0; k < kClassWords; ++k) {
        bt[k] = s_wt[0][k] + s_wt[1][k] + s_wt[2][k] + s_wt[3][k];
        wp[k] = 0ull;
        for (int j = 0; j < wv; ++j) wp[k] += s_wt[j][k];
    }
    if (tid < kClasses) {
        uint32_t start = 0u;
        for (int c = kClasses - 1; c > tid; --c) start += class_field(bt, (uint32_t)c);
        s_cs[tid] = start;
        const int nblocks = (a.npix + kSelectPx - 1) / kSelectPx;
        a.counts[(size_t)tid * nblocks + bid] = class_field(bt, (uint32_t)tid);
    }
    if (tid == 0) a.bsel[bid] = s_nsel[0] + s_nsel[1] + s_nsel[2] + s_nsel[3];
    __syncthreads();
    uint32_t* run = a.act_px + (size_t)bid * kSelectPx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (act[q]) {
            uint32_t r = class_field(ex, cls[q]) + class_field(wp, cls[q]);
#pragma unroll
            for (int q2 = 0; q2 < 3; ++q2)
                if (q2 < q) r += (act[q2] && cls[q2] == cls[q]) ? 1u : 0u;
            run[s_cs[cls[q]] + r] = (uint32_t)(base + q);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Order pass of the sparse method: the selection blocks' runs into one list, length classes
// longest first and, within a class, blocks in order (a deterministic list), resume points
// cleared.  k_order_scan (one block, a wave per class) places every (block, class) run; k_order_copy
// (a block per selection block) moves the runs.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void order_scan_block(const OrderArgs& a) {
    static_assert(kClasses * 64 == 1024, "one wave per class");
    __shared__ uint32_t s_tot[kClasses];
    __shared__ uint64_t s_sel[kClasses];
    const int tid = threadIdx.x, lane = tid & 63;
    const int c = kClasses - 1 - (tid >> 6);      // wave w scans class kClasses-1-w
    const int nb = a.nblocks;
    const int per = (nb + 63) / 64;
    const int b0 = min(nb, lane * per), b1 = min(nb, b0 + per);
    // loads in groups of 16, issued before they are summed
    uint32_t sum = 0u;
    uint64_t sel = 0ull;
    for (int b = b0; b < b1; b += 16) {
        uint32_t v[16], w[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            v[u] = b + u < b1 ? a.counts[(size_t)c * nb + b + u] : 0u;
            w[u] = (c == 0 && b + u < b1) ? a.bsel[b + u] : 0u;   // selected, counted once
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            sum += v[u];
            sel += w[u];
        }
    }
    const int inc = wave_incl_scan((int)sum);
    const uint64_t sinc = wave_incl_scan_u64(sel);
    if (lane == 63) {
        s_tot[c] = (uint32_t)inc;
        s_sel[c] = sinc;
    }
    __syncthreads();
    uint32_t cbase = 0u;
    for (int c2 = kClasses - 1; c2 > c; --c2) cbase += s_tot[c2];
    uint32_t pos = cbase + (uint32_t)(inc - (int)sum);
    for (int b = b0; b < b1; b += 16) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = b + u < b1 ? a.counts[(size_t)c * nb + b + u] : 0u;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (b + u < b1) a.goff[(size_t)c * nb + b + u] = pos;
            pos += v[u];
        }
    }
    if (tid == 0) {
        uint32_t total = 0u;
        for (int c2 = 0; c2 < kClasses; ++c2) total += s_tot[c2];
        *a.n_total = total;
        if (a.stats && s_sel[0] > 0) atomicAdd(a.stats, (unsigned long long)s_sel[0]);
        if (a.stats && total > 0) atomicAdd(a.stats + 1, (unsigned long long)total);
    }
}

__device__ __forceinline__ void order_copy_block(const OrderArgs& a, unsigned bid) {
    __shared__ uint32_t s_start[kClasses + 1];    // class starts within the run, descending
    __shared__ uint32_t s_goff[kClasses];
    const int tid = threadIdx.x;
    if (tid == 0) {
        uint32_t pos = 0u;
        for (int c = kClasses - 1; c >= 0; --c) {
            s_start[c] = pos;
            pos += a.counts[(size_t)c * a.nblocks + bid];
        }
        s_start[kClasses] = pos;
    }
    if (tid < kClasses) s_goff[tid] = a.goff[(size_t)tid * a.nblocks + bid];
    __syncthreads();
    const uint32_t n = s_start[kClasses];
    const uint32_t* run = a.act_px + (size_t)bid * kSelectPx;
    for (uint32_t i = tid; i < n; i += 256) {
        int c = kClasses - 1;
        while (c > 0 && i >= s_start[c - 1]) --c;   // the class whose part of the run holds i
        const uint32_t dst = s_goff[c] + (i - s_start[c]);
        a.ord[dst] = run[i];
        a.resume[dst] = 0;
    }
}

__global__ __launch_bounds__(1024) void k_order_scan(OrderArgs a) { order_scan_block(a); }
__global__ __launch_bounds__(256) void k_order_copy(OrderArgs a) {
    order_copy_block(a, blockIdx.x);
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_select(SelectArgs a) {
    select_block<VEC>(a, blockIdx.x);
}

// ------------------------------------------------------------------------------------------
// Chain pass.  One lane per pixel (per active pixel for the sparse method) walks that pixel's
// selected intervals in order, carrying its reference level in a register: the only temporal
// dependency of the method is per pixel, so no lane ever waits for another.  Per step, each
// active lane computes its interior samples into LDS, counts its crossings, the wave reserves
// arena space with one atomic (no block barrier), and the lanes write their events.  If the
// arena is full the wave fills its reservation with sentinels, stores each lane's current
// interval as its resume point and stops; the host grows the arena and launches again.
// MODE selects what is thresholded (ChainMode): the reference-level crossings of the event pixel,
// or the paper's memoryless thresholding of sample differences or of interpolated difference
// frames (no reference level, which is then neither read nor written).
// ------------------------------------------------------------------------------------------
template <int MODE, int V>
__device__ __forceinline__ void chain_block(ChainArgs a, unsigned bid) {
    constexpr int kFrameBatch = ChainVariant<V>::frame;
    constexpr int kDiffBatch = ChainVariant<V>::diff;
    extern __shared__ float smem[];
    __shared__ float tau[kMaxSubIntervals + 1];   // k / S for k = 0..S, shared by every sample
    float* lut = smem;
    const int tid = threadIdx.x, lane = tid & 63;
    lut[tid] = a.lut[tid];
    for (int k = tid; k <= a.S; k += kSimThreads) tau[k] = (float)k / (float)a.S;
    __syncthreads();

    const int slot = bid * kSimThreads + tid;
    bool valid;
    if (a.act_px) {
        valid = slot < (int)*a.n_active;
    } else {
        valid = slot < a.npix;
    }
    if (!__any(valid)) return;

    const int p = valid ? (a.act_px ? (int)a.act_px[slot] : slot) : 0;
    const int astripe = (slot >> 6) % kArenaStripes;   // this wave's sub-arena
    uint64_t* arena = a.arena + (uint64_t)astripe * a.stripe_cap;
    const int y = p / a.W;
    const int x = p - y * a.W;
    const float xf = (float)x, yf = (float)y;
    const float wm1 = (float)(a.W - 1), hm1 = (float)(a.H - 1);
    const bool all = a.mask == nullptr;
    uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    if (valid && !all) {
        m0 = a.mask[p];
        if (a.K > 32) m1 = a.mask[(int64_t)a.npix + p];
        if (a.K > 64) m2 = a.mask[2 * (int64_t)a.npix + p];
        if (a.K > 96) m3 = a.mask[3 * (int64_t)a.npix + p];
    }
    int i = valid ? next_selected(all, m0, m1, m2, m3, a.resume[slot], a.K) : a.K;
    if constexpr (MODE == kModeDifference) i = max(i, a.first_emit);
    float R = (MODE == kModeReference && valid) ? a.lref[p] : 0.0f;

    const int stash_n = (a.S - 1 <= kMaxStash) ? (a.S - 1) : 0;
    float* stash = smem + 256 + tid;
    const int pbits = a.lay.pix_bits();
    const int ishift = a.lay.tb + pbits;
    const uint64_t pixkey = ((uint64_t)y << (a.lay.xb + 1)) | ((uint64_t)x << 1);
    bool failed = false;

    for (;;) {
        const bool have = i < a.K;
        if (!__any(have)) break;
        int n = 0;
        float Rn = R, A0 = 0.0f, A1 = 0.0f, delta = 0.0f;
        PixelCtx c;
        c.W = a.W; c.H = a.H; c.x = x; c.y = y; c.S = a.S; c.lut = lut; c.tau = tau;
        c.u = 0.0f; c.v = 0.0f; c.stash = nullptr;
        c.F0 = i == 0 ? a.prev : a.frames + (int64_t)(i - 1) * a.fstride;
        c.F1 = a.frames + (int64_t)i * a.fstride;
        if constexpr (MODE == kModeDifference)
            c.Fm = i == 0 ? a.prev2 : (i == 1 ? a.prev : a.frames + (int64_t)(i - 2) * a.fstride);
        if (have) {
            // frame methods: the flow vector is loaded before the frame bytes, so that all of
            // the interval's loads at this pixel are in flight together (the difference method
            // keeps the later load: the earlier one costs it a wave of occupancy)
            if constexpr (MODE != kModeDifference) {
                if (a.S > 1) {
                    const float* fl = a.flows + (int64_t)i * a.flstride + 2 * (int64_t)p;
                    c.u = fl[0];
                    c.v = fl[1];
                }
            }
            A0 = lut[c.F0[p]];
            A1 = lut[c.F1[p]];
            if constexpr (MODE == kModeDifference) {
                // the two difference frames at this pixel: D1 (series start), D2 = D_S
                const float Am = lut[c.Fm[p]];
                const float D2 = A1 - A0;
                A0 = A0 - Am;
                A1 = D2;
            }
            delta = a.delta[i];
            if (a.S > 1) {
                if constexpr (MODE == kModeDifference) {
                    const float* fl = a.flows + (int64_t)i * a.flstride + 2 * (int64_t)p;
                    c.u = fl[0];
                    c.v = fl[1];
                }
                if constexpr (MODE == kModeDifference) {
                    for (int k0 = 1; k0 <= stash_n; k0 += kDiffBatch)
                        stash_diff_samples<kDiffBatch>(c.Fm, c.F0, c.F1, lut, tau, a.W, a.H, wm1,
                                                       hm1, xf, yf, c.u, c.v, k0, stash_n,
                                                       stash);
                } else {
                    for (int k0 = 1; k0 <= stash_n; k0 += kFrameBatch)
                        stash_frame_samples<kFrameBatch>(c.F0, c.F1, lut, tau, a.W, a.H, wm1,
                                                         hm1, xf, yf, c.u, c.v, k0, stash_n,
                                                         stash);
                }
                if (stash_n) c.stash = stash;
            }
            if constexpr (MODE == kModeReference)
                n = crossings<false>(c, R, A0, A1, a.cpos, a.cneg, delta, 0, pbits, 0, nullptr,
                                     &Rn);
            else
                n = flips<MODE, false>(c, A0, A1, a.cpos, a.cneg, delta, 0, pbits, 0, nullptr);
        }
        const int inc = wave_incl_scan(n);
        const int total = __shfl(inc, 63, 64);
        unsigned long long base = 0;
        int fail = 0;
        if (lane == 0 && total > 0) {
            base = atomicAdd(a.reserve + astripe * kCounterStride, (unsigned long long)total);
            if (base + (unsigned long long)total > a.stripe_cap) {
                fail = 1;
                atomicAdd(&a.fails[0], 1ull);
                if (base < a.stripe_cap) atomicAdd(&a.fails[1], a.stripe_cap - base);
            }
        }
        base = __shfl(base, 0, 64);
        fail = __shfl(fail, 0, 64);
        if (fail) {
            const unsigned long long e =
                min(base + (unsigned long long)total, (unsigned long long)a.stripe_cap);
            for (unsigned long long j = base + lane; j < e; j += 64) arena[j] = kSentinel;
            failed = true;
            break;
        }
        if (have) {
            if (n > 0) {
                const uint64_t keyhi = (uint64_t)i << ishift;
                if constexpr (MODE == kModeReference)
                    crossings<true>(c, R, A0, A1, a.cpos, a.cneg, delta, keyhi, pbits, pixkey,
                                    arena + base + (inc - n), &Rn);
                else
                    flips<MODE, true>(c, A0, A1, a.cpos, a.cneg, delta, keyhi, pbits, pixkey,
                                      arena + base + (inc - n));
            }
            R = Rn;
            i = next_selected(all, m0, m1, m2, m3, i + 1, a.K);
        }
    }
    if (valid) {
        if constexpr (MODE == kModeReference) a.lref[p] = R;
        a.resume[slot] = failed ? i : a.K;
    }
}

template <int MODE, int V>
__global__ __launch_bounds__(kSimThreads) void k_chain(ChainArgs a) {
    chain_block<MODE, V>(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_copy_u8(const uint8_t* __restrict__ src,
                                                 uint8_t* __restrict__ dst, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

// Concatenation of the sub-arenas.  Block b copies chunk b / kArenaStripes of stripe
// b % kArenaStripes; its destination offset is the exclusive prefix of the stripe lengths.
__device__ __forceinline__ void gather_block(const uint64_t* __restrict__ arena,
                                             uint64_t stripe_cap,
                                             const unsigned long long* reserve,
                                             uint64_t* __restrict__ out,
                                             unsigned long long* n_total, unsigned bid) {
    static_assert(kArenaStripes == 256, "one thread per stripe");
    __shared__ int s_wsum[4];
    __shared__ unsigned long long s_len[kArenaStripes];
    const int tid = threadIdx.x;
    const unsigned long long len = min(reserve[tid * kCounterStride], (unsigned long long)stripe_cap);
    s_len[tid] = len;
    // 64-bit exclusive prefix via two 32-bit scans would be overkill: stripe lengths and their
    // sum stay below 2^31 (the arena holds fewer than 2^31 keys).
    int tot;
    const int ex = block_scan_256((int)len, s_wsum, &tot);
    __shared__ unsigned long long s_off[kArenaStripes];
    s_off[tid] = (unsigned long long)ex;
    __syncthreads();
    const int stripe = bid % kArenaStripes;
    const uint64_t chunk = bid / kArenaStripes;
    if (bid == 0 && tid == 0) *n_total = (unsigned long long)tot;
    const uint64_t n = s_len[stripe];
    const uint64_t b0 = chunk * kSortTile;
    if (b0 >= n) return;
    const uint64_t* src = arena + (uint64_t)stripe * stripe_cap;
    uint64_t* dst = out + s_off[stripe];
    const uint64_t e = min(b0 + (uint64_t)kSortTile, n);
    for (uint64_t j = b0 + tid; j < e; j += kArenaStripes) dst[j] = src[j];
}

__global__ __launch_bounds__(kArenaStripes) void k_gather(const uint64_t* __restrict__ arena,
                                                          uint64_t stripe_cap,
                                                          const unsigned long long* reserve,
                                                          uint64_t* __restrict__ out,
                                                          unsigned long long* n_total) {
    gather_block(arena, stripe_cap, reserve, out, n_total, blockIdx.x);
}

__global__ void k_clamp(unsigned long long* reserve, uint64_t cap) {
    const int s = threadIdx.x;
    if (s < kArenaStripes) {
        unsigned long long* r = reserve + s * kCounterStride;
        if (*r > cap) *r = cap;
    }
}

// ------------------------------------------------------------------------------------------
// Frame of accumulated events (Fig. 1 caption) and its per-pixel moments (the events/(pixel s)
// statistic of Sec. IV-C).  Keys are packed ABI keys: (t - epoch) << 25 | y << 13 | x << 1 | p.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accumulate(const uint64_t* __restrict__ keys, uint64_t n,
                                                    uint64_t t_lo, uint64_t t_hi, int W, int H,
                                                    uint32_t* __restrict__ counts) {
    const uint64_t plane = (uint64_t)W * (uint64_t)H;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = keys[i];
        const uint64_t t = k >> 25;
        if (t < t_lo || t >= t_hi) continue;
        const uint32_t y = (uint32_t)(k >> 13) & 0xFFFu;
        const uint32_t x = (uint32_t)(k >> 1) & 0xFFFu;
        if (x >= (uint32_t)W || y >= (uint32_t)H) continue;
        atomicAdd(counts + ((k & 1ull) ? 0ull : plane) + (uint64_t)y * W + x, 1u);
    }
}

constexpr int kMomentBlocks = 1024;

__global__ __launch_bounds__(256) void k_moments(const uint32_t* __restrict__ counts,
                                                 uint64_t plane,
                                                 unsigned long long* __restrict__ part) {
    __shared__ unsigned long long r1[256], r2[256];
    const int tid = threadIdx.x;
    unsigned long long s1 = 0, s2 = 0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + tid; p < plane; p += stride) {
        const unsigned long long c = (unsigned long long)counts[p] + counts[plane + p];
        s1 += c;
        s2 += c * c;
    }
    r1[tid] = s1;
    r2[tid] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            r1[tid] += r1[tid + h];
            r2[tid] += r2[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[2 * blockIdx.x] = r1[0];
        part[2 * blockIdx.x + 1] = r2[0];
    }
}

// ------------------------------------------------------------------------------------------
// Stable LSD radix sort, kRadixBits-bit digits, three kernels per pass.
// ------------------------------------------------------------------------------------------
template <int BITS>
__device__ __forceinline__ void hist_block(const uint64_t* __restrict__ keys,
                                           const unsigned long long* n_dev, int shift,
                                           uint32_t* __restrict__ hist, int nblocks, unsigned bid) {
    constexpr int D = 1 << BITS;
    __shared__ uint32_t h[D];
    const int tid = threadIdx.x;
    const uint64_t n = *n_dev;
    for (int d = tid; d < D; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)bid * kSortTile;
    if (base < n) {
        // every key of the thread is loaded before any is counted (indices past the end re-read
        // the last key and are not counted), so that the loads are in flight together
        uint64_t kv[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const uint64_t idx = base + (uint64_t)j * kSortThreads + tid;
            kv[j] = keys[idx < n ? idx : n - 1];
        }
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const uint64_t idx = base + (uint64_t)j * kSortThreads + tid;
            if (idx < n) atomicAdd(&h[(kv[j] >> shift) & (D - 1u)], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < D; d += kSortThreads) hist[(size_t)d * nblocks + bid] = h[d];
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                             const unsigned long long* n_dev,
                                                             int shift,
                                                             uint32_t* __restrict__ hist,
                                                             int nblocks) {
    hist_block<BITS>(keys, n_dev, shift, hist, nblocks, blockIdx.x);
}

// One block per digit: exclusive scan of that digit's per-block counts; row total to totals[d].
__device__ __forceinline__ void rowscan_block(uint32_t* __restrict__ hist, int nblocks,
                                              uint32_t* __restrict__ totals, unsigned digit) {
    __shared__ int s_wsum[4];
    uint32_t* row = hist + (size_t)digit * nblocks;
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
    if (threadIdx.x == 0) totals[digit] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_rowscan(uint32_t* __restrict__ hist,
                                                                int nblocks,
                                                                uint32_t* __restrict__ totals) {
    rowscan_block(hist, nblocks, totals, blockIdx.x);
}

__device__ __forceinline__ uint64_t convert_key(uint64_t k, const ConvertArgs& cv) {
    const KeyLayout& L = cv.lay;
    const int pb = L.pix_bits();
    const uint64_t pix = k & ((1ull << pb) - 1);
    const uint64_t trel = (k >> pb) & ((1ull << L.tb) - 1);
    const uint64_t iv = k >> (pb + L.tb);
    if (iv >= (uint64_t)cv.K) return kSentinel;   // never for a real key; keeps reads in bounds
    const uint64_t x = (pix >> 1) & ((1ull << L.xb) - 1);
    const uint64_t y = (pix >> (L.xb + 1)) & ((1ull << L.yb) - 1);
    const uint64_t t = (uint64_t)cv.tbase[iv] + trel;
    return (t << 25) | (y << 13) | (x << 1) | (pix & 1ull);
}

// One pass's scatter of a block's tile.  Each wave ranks its own quarter of the tile (keys
// base + w * 1024 + j * 64 + lane, j = 0..15, the tile's order) against wave-private digit counts
// in LDS: ballot peer matching gives the rank among the wave's lanes, the count before it the
// rank among the wave's earlier keys, so no block barrier is needed until the quarters are
// combined (the waves before w, per digit).  Stable: a key's place follows every key before it
// in the tile with the same digit.
template <int BITS>
__device__ __forceinline__ void scatter_block(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
    const unsigned long long* n_dev, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, int nblocks, ConvertArgs cv, unsigned bid) {
    static_assert(kSortThreads == 256 && kSortItems == 16, "four waves of 16 x 64 keys");
    constexpr int D = 1 << BITS;
    constexpr int PER = D / kSortThreads;   // digits per thread: 1 or 2
    static_assert(PER == 1 || PER == 2, "8- or 9-bit digits");
    __shared__ uint32_t s_base[D];
    __shared__ uint32_t s_wc[4][D];
    __shared__ int s_wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t n = *n_dev;
    const uint64_t base = (uint64_t)bid * kSortTile;
    if (base >= n) return;
    const uint64_t n_valid = cv.enabled ? n - *cv.n_sentinel : n;
    const uint64_t wbase = base + (uint64_t)w * (kSortItems * 64) + lane;
    uint64_t kv[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const uint64_t idx = wbase + (uint64_t)j * 64;
        kv[j] = in[idx < n ? idx : n - 1];
    }
    int tot;
    const int d0 = PER * tid;   // this thread's digits: d0 .. d0 + PER - 1
    uint32_t tv[PER];
    uint32_t tsum = 0u;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        tv[q] = totals[d0 + q];
        tsum += tv[q];
    }
    const int dex = block_scan_256((int)tsum, s_wsum, &tot);
    uint32_t run = (uint32_t)dex;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        s_base[d0 + q] = run + hist[(size_t)(d0 + q) * nblocks + bid];
        run += tv[q];
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) s_wc[w2][d0 + q] = 0u;
    }
    __syncthreads();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    uint32_t lrank[kSortItems];
    uint32_t* wc = s_wc[w];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const bool valid = wbase + (uint64_t)j * 64 < n;
        const uint32_t d = (uint32_t)(kv[j] >> shift) & (D - 1u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        // the first lane of each digit group reads the wave's count and hands it to its group;
        // after the exchange it advances the count (the next key's read comes after the next
        // key's ballots, which every lane reaches only after this write)
        const bool leader = valid && rank == 0;
        const int src = valid ? __ffsll((long long)peers) - 1 : lane;
        const uint32_t mine = leader ? wc[d] : 0u;
        const uint32_t before = (uint32_t)__shfl((int)mine, src, 64);
        lrank[j] = before + rank;
        if (leader) wc[d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit (PER per thread): the counts of the waves before each wave, in place
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int d = d0 + q;
        const uint32_t c0 = s_wc[0][d], c1 = s_wc[1][d], c2 = s_wc[2][d];
        s_wc[0][d] = 0u;
        s_wc[1][d] = c0;
        s_wc[2][d] = c0 + c1;
        s_wc[3][d] = c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (wbase + (uint64_t)j * 64 < n) {
            const uint32_t d = (uint32_t)(kv[j] >> shift) & (D - 1u);
            const uint64_t pos = (uint64_t)s_base[d] + wc[d] + lrank[j];
            if (!cv.enabled) {
                out[pos] = kv[j];
            } else if (pos < n_valid) {
                out[pos] = convert_key(kv[j], cv);
            }
        }
    }
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
    const unsigned long long* n_dev, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, int nblocks, ConvertArgs cv) {
    scatter_block<BITS>(in, out, n_dev, shift, hist, totals, nblocks, cv, blockIdx.x);
}

// ------------------------------------------------------------------------------------------
// Clearing, as kernels rather than memset nodes, so that pushes recorded into a HIP graph replay
// correctly.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0u;
}

// Start of a window: its counters, the reservation counters, the active-list counters (sparse)
// and the per-pixel resume points (every other method).
__global__ __launch_bounds__(256) void k_prep_window(unsigned long long* __restrict__ counters,
                                                     unsigned long long* __restrict__ reserve,
                                                     int* __restrict__ resume, int64_t npix) {
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        if (tid < 4) counters[tid] = 0ull;
        for (int i = tid; i < kArenaStripes * kCounterStride; i += 256) reserve[i] = 0ull;
    }
    if (resume) {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < npix; i += stride)
            resume[i] = 0;
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

hipError_t launch_select(const SelectArgs& a, hipStream_t stream) {
    const int blocks = (a.npix + kSelectPx - 1) / kSelectPx;
    const bool vec = (a.fstride % 4) == 0 && ((uintptr_t)a.frames % 4) == 0 &&
                     ((uintptr_t)a.prev % 4) == 0 && ((uintptr_t)a.prev_out % 4) == 0;
    if (vec)
        hipLaunchKernelGGL(k_select<true>, dim3(blocks), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_select<false>, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_order(const OrderArgs& a, hipStream_t stream) {
    if (a.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, stream, a);
    hipLaunchKernelGGL(k_order_copy, dim3(a.nblocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <int MODE, int V>
hipError_t launch_chain_v(const ChainArgs& a, int blocks, size_t shmem, hipStream_t stream) {
    hipLaunchKernelGGL((k_chain<MODE, V>), dim3(blocks), dim3(kSimThreads), shmem, stream, a);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_chain_m(const ChainArgs& a, int blocks, size_t shmem, int variant,
                          hipStream_t stream) {
    switch (variant) {
        case 0: return launch_chain_v<MODE, 0>(a, blocks, shmem, stream);
        case 1: return launch_chain_v<MODE, 1>(a, blocks, shmem, stream);
        case 2: return launch_chain_v<MODE, 2>(a, blocks, shmem, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chain(const ChainArgs& a, int max_slots, int variant, hipStream_t stream) {
    const int stash_n = (a.S - 1 <= kMaxStash) ? (a.S - 1) : 0;
    const size_t shmem = (size_t)(256 + stash_n * kSimThreads) * sizeof(float);
    const int blocks = (max_slots + kSimThreads - 1) / kSimThreads;
    if (blocks == 0) return hipSuccess;
    switch (a.mode) {
        case kModeReference:
            return launch_chain_m<kModeReference>(a, blocks, shmem, variant, stream);
        case kModeMemoryless:
            return launch_chain_m<kModeMemoryless>(a, blocks, shmem, variant, stream);
        case kModeDifference:
            return launch_chain_m<kModeDifference>(a, blocks, shmem, variant, stream);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_gather(const uint64_t* arena, uint64_t stripe_cap,
                         const unsigned long long* reserve, uint64_t* out,
                         unsigned long long* n_total, hipStream_t stream) {
    const uint64_t chunks = (stripe_cap + kSortTile - 1) / kSortTile;
    const uint64_t blocks = std::max<uint64_t>(1, chunks) * kArenaStripes;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(kArenaStripes), 0, stream, arena,
                       stripe_cap, reserve, out, n_total);
    return hipGetLastError();
}

hipError_t launch_clamp(unsigned long long* reserve, uint64_t cap, hipStream_t stream) {
    hipLaunchKernelGGL(k_clamp, dim3(1), dim3(kArenaStripes), 0, stream, reserve, cap);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
    const uint64_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t*)p,
                       words);
    return hipGetLastError();
}

hipError_t launch_prep_window(unsigned long long* counters, unsigned long long* reserve,
                              int* resume, int64_t npix, hipStream_t stream) {
    const int64_t blocks = resume ? std::max<int64_t>(1, std::min<int64_t>((npix + 255) / 256,
                                                                            1024))
                                  : 1;
    hipLaunchKernelGGL(k_prep_window, dim3((unsigned)blocks), dim3(256), 0, stream, counters,
                       reserve, resume, npix);
    return hipGetLastError();
}

hipError_t launch_copy_u8(const uint8_t* src, uint8_t* dst, int64_t n, hipStream_t stream) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_copy_u8, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

size_t sort_hist_entries(uint64_t n_max) {
    const uint64_t nb = (n_max + kSortTile - 1) / kSortTile;
    return (size_t)(nb ? nb : 1) * kRadixDigits;
}

hipError_t launch_sort(uint64_t* keys, uint64_t* alt, const unsigned long long* n,
                       uint64_t n_max, int nbits, uint32_t* hist, uint32_t* totals,
                       uint64_t* out, const ConvertArgs& cv, hipStream_t stream) {
    const int nblocks = (int)std::max<uint64_t>(1, (n_max + kSortTile - 1) / kSortTile);
    const int bits = sort_radix_bits(nbits);
    const int passes = sort_passes(nbits);
    uint64_t* src = keys;
    uint64_t* dst = alt;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = bits * pass;
        const bool last = pass == passes - 1;
        ConvertArgs c = cv;
        if (!last) c.enabled = 0;
        if (bits == 9) {
            hipLaunchKernelGGL(k_radix_hist<9>, dim3(nblocks), dim3(kSortThreads), 0, stream, src,
                               n, shift, hist, nblocks);
            hipLaunchKernelGGL(k_radix_rowscan, dim3(512), dim3(kSortThreads), 0, stream, hist,
                               nblocks, totals);
            hipLaunchKernelGGL(k_radix_scatter<9>, dim3(nblocks), dim3(kSortThreads), 0, stream,
                               src, last ? out : dst, n, shift, hist, totals, nblocks, c);
        } else {
            hipLaunchKernelGGL(k_radix_hist<8>, dim3(nblocks), dim3(kSortThreads), 0, stream, src,
                               n, shift, hist, nblocks);
            hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, stream, hist,
                               nblocks, totals);
            hipLaunchKernelGGL(k_radix_scatter<8>, dim3(nblocks), dim3(kSortThreads), 0, stream,
                               src, last ? out : dst, n, shift, hist, totals, nblocks, c);
        }
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    return hipGetLastError();
}

hipError_t launch_accumulate(const uint64_t* keys, uint64_t n, uint64_t t_lo, uint64_t t_hi,
                             int W, int H, uint32_t* counts, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)blocks), dim3(256), 0, stream, keys, n, t_lo,
                       t_hi, W, H, counts);
    return hipGetLastError();
}

int moments_blocks(uint64_t plane) {
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((plane + 255) / 256, kMomentBlocks));
}

hipError_t launch_moments(const uint32_t* counts, uint64_t plane, unsigned long long* part,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_moments, dim3((unsigned)moments_blocks(plane)), dim3(256), 0, stream,
                       counts, plane, part);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Fused batch: one launch per phase over the streams of a batched push.  A block finds its
// stream's entry by binary search over the launch's block offsets and runs that stream's block
// body with its block index inside the stream.
// ------------------------------------------------------------------------------------------
// Largest e with start[e] <= b: the entry owning block b (entries owning no block share their
// offset with the next owner, which has the larger index).
__device__ __forceinline__ int batch_entry(const int* __restrict__ start, int n, unsigned b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((unsigned)start[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Per entry: clear the reservation counters, the window counters and (sparse) the active-list
// lengths.
__global__ __launch_bounds__(256) void k_batch_prep(const BatchEntry* __restrict__ entries) {
    const BatchEntry* e = entries + blockIdx.x;
    const int tid = threadIdx.x;
    unsigned long long* reserve = e->chain.reserve;
    for (int i = tid; i < kArenaStripes * kCounterStride; i += 256) reserve[i] = 0ull;
    if (tid < 4) e->counters[tid] = 0ull;
}

// Selection pass of sparse entries; frame copies and chain resets of the others (kSelectPx
// pixels per block either way).
__global__ __launch_bounds__(256) void k_batch_select(const BatchEntry* __restrict__ entries,
                                                      const int* __restrict__ start, int n) {
    const int ei = batch_entry(start, n, blockIdx.x);
    const unsigned lb = blockIdx.x - (unsigned)start[ei];
    const BatchEntry* e = entries + ei;
    if (e->sparse) {
        if (e->vec)
            select_block<true>(e->sel, lb);
        else
            select_block<false>(e->sel, lb);
        return;
    }
    const int64_t base = (int64_t)lb * kSelectPx;
    const int64_t end = min(base + (int64_t)kSelectPx, e->npix);
    for (int64_t p = base + threadIdx.x; p < end; p += 256) {
        e->copy_dst[p] = e->copy_src[p];
        if (e->copy2_dst) e->copy2_dst[p] = e->copy2_src[p];
        e->chain.resume[p] = 0;
    }
}

// One scan block per entry (blockIdx.x = entry); entries that are not sparse return.
__global__ __launch_bounds__(1024) void k_batch_order_scan(const BatchEntry* __restrict__ entries) {
    const BatchEntry* e = entries + blockIdx.x;
    if (!e->sparse) return;
    order_scan_block(e->ord);
}

__global__ __launch_bounds__(256) void k_batch_order_copy(const BatchEntry* __restrict__ entries,
                                                          const int* __restrict__ start, int n) {
    const int ei = batch_entry(start, n, blockIdx.x);
    order_copy_block(entries[ei].ord, blockIdx.x - (unsigned)start[ei]);
}

template <int MODE, int V>
__global__ __launch_bounds__(kSimThreads) void k_batch_chain(const BatchEntry* __restrict__ entries,
                                                             const int* __restrict__ start,
                                                             int n) {
    const int ei = batch_entry(start, n, blockIdx.x);
    chain_block<MODE, V>(entries[ei].chain, blockIdx.x - (unsigned)start[ei]);
}

__global__ void k_batch_fails(const BatchEntry* __restrict__ entries, int n,
                              unsigned long long* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = entries[e].counters[0];
}

__global__ void k_batch_clamp(const BatchEntry* __restrict__ entries) {
    const BatchEntry* e = entries + blockIdx.x;
    if (e->clamp_cap == 0) return;
    unsigned long long* r = e->chain.reserve + threadIdx.x * kCounterStride;
    if (*r > e->clamp_cap) *r = e->clamp_cap;
    if (threadIdx.x == 0) e->counters[0] = 0ull;
}

__global__ __launch_bounds__(kArenaStripes) void k_batch_gather(
    const BatchEntry* __restrict__ entries, const int* __restrict__ start, int n) {
    const int ei = batch_entry(start, n, blockIdx.x);
    const BatchEntry* e = entries + ei;
    gather_block(e->chain.arena, e->chain.stripe_cap, e->chain.reserve, e->gathered,
                 e->counters + 2, blockIdx.x - (unsigned)start[ei]);
}

// out[3e .. 3e+2] = failed reservations, sentinels, gathered keys of entry e.
__global__ void k_batch_status(const BatchEntry* __restrict__ entries, int n,
                               unsigned long long* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        out[3 * e] = entries[e].counters[0];
        out[3 * e + 1] = entries[e].counters[1];
        out[3 * e + 2] = entries[e].counters[2];
    }
}

__global__ void k_batch_counts(const BatchEntry* __restrict__ entries, int n,
                               unsigned long long* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        out[2 * e] = entries[e].counters[1];
        out[2 * e + 1] = entries[e].counters[2];
    }
}

// One pass of every entry's sort: pass p reads the gathered keys (p even) or the ping-pong
// buffer (p odd) and writes the other one, or the FIFO on the last pass.
template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_batch_hist(const BatchEntry* __restrict__ entries,
                                                             const int* __restrict__ start, int n,
                                                             int pass) {
    const int ei = batch_entry(start, n, blockIdx.x);
    const BatchEntry* e = entries + ei;
    const uint64_t* src = (pass & 1) ? e->sort_alt : e->gathered;
    hist_block<BITS>(src, e->counters + 2, BITS * pass, e->hist, e->sort_blocks,
                     blockIdx.x - (unsigned)start[ei]);
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_batch_rowscan(
    const BatchEntry* __restrict__ entries) {
    const BatchEntry* e = entries + blockIdx.x / (1 << BITS);
    if (e->sort_blocks == 0) return;
    rowscan_block(e->hist, e->sort_blocks, e->totals, blockIdx.x % (1 << BITS));
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_batch_scatter(
    const BatchEntry* __restrict__ entries, const int* __restrict__ start, int n, int pass,
    int last) {
    const int ei = batch_entry(start, n, blockIdx.x);
    const BatchEntry* e = entries + ei;
    const uint64_t* src = (pass & 1) ? e->sort_alt : e->gathered;
    uint64_t* dst = last ? e->out : ((pass & 1) ? e->gathered : e->sort_alt);
    ConvertArgs c = e->cv;
    if (!last) c.enabled = 0;
    scatter_block<BITS>(src, dst, e->counters + 2, BITS * pass, e->hist, e->totals,
                        e->sort_blocks, c,
                  blockIdx.x - (unsigned)start[ei]);
}

hipError_t launch_batch_prep(const BatchEntry* e, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_prep, dim3(n), dim3(256), 0, stream, e);
    return hipGetLastError();
}

hipError_t launch_batch_select(const BatchEntry* e, const int* start, int n, int blocks,
                               hipStream_t stream) {
    if (n <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_select, dim3(blocks), dim3(256), 0, stream, e, start, n);
    return hipGetLastError();
}

hipError_t launch_batch_order(const BatchEntry* e, const int* start, int n, int blocks,
                              hipStream_t stream) {
    if (n <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_order_scan, dim3(n), dim3(1024), 0, stream, e);
    hipLaunchKernelGGL(k_batch_order_copy, dim3(blocks), dim3(256), 0, stream, e, start, n);
    return hipGetLastError();
}

template <int MODE, int V>
hipError_t launch_batch_chain_v(const BatchEntry* e, const int* start, int n, int blocks,
                                size_t shmem, hipStream_t stream) {
    hipLaunchKernelGGL((k_batch_chain<MODE, V>), dim3(blocks), dim3(kSimThreads), shmem, stream,
                       e, start, n);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_batch_chain_m(const BatchEntry* e, const int* start, int n, int blocks,
                                size_t shmem, int variant, hipStream_t stream) {
    switch (variant) {
        case 0: return launch_batch_chain_v<MODE, 0>(e, start, n, blocks, shmem, stream);
        case 1: return launch_batch_chain_v<MODE, 1>(e, start, n, blocks, shmem, stream);
        case 2: return launch_batch_chain_v<MODE, 2>(e, start, n, blocks, shmem, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_chain(const BatchEntry* e, const int* start, int n, int blocks, int mode,
                              int max_stash, int variant, hipStream_t stream) {
    if (n <= 0 || blocks <= 0) return hipSuccess;
    const size_t shmem = (size_t)(256 + max_stash * kSimThreads) * sizeof(float);
    switch (mode) {
        case kModeReference:
            return launch_batch_chain_m<kModeReference>(e, start, n, blocks, shmem, variant,
                                                        stream);
        case kModeMemoryless:
            return launch_batch_chain_m<kModeMemoryless>(e, start, n, blocks, shmem, variant,
                                                         stream);
        case kModeDifference:
            return launch_batch_chain_m<kModeDifference>(e, start, n, blocks, shmem, variant,
                                                         stream);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_fails(const BatchEntry* e, int n, unsigned long long* out,
                              hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_fails, dim3((n + 255) / 256), dim3(256), 0, stream, e, n, out);
    return hipGetLastError();
}

hipError_t launch_batch_clamp(const BatchEntry* e, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_clamp, dim3(n), dim3(kArenaStripes), 0, stream, e);
    return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchEntry* e, const int* start, int n, int blocks,
                               hipStream_t stream) {
    if (n <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_gather, dim3(blocks), dim3(kArenaStripes), 0, stream, e, start,
                       n);
    return hipGetLastError();
}

hipError_t launch_batch_status(const BatchEntry* e, int n, unsigned long long* out,
                               hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_status, dim3((n + 255) / 256), dim3(256), 0, stream, e, n, out);
    return hipGetLastError();
}

hipError_t launch_batch_counts(const BatchEntry* e, int n, unsigned long long* out,
                               hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_counts, dim3((n + 255) / 256), dim3(256), 0, stream, e, n, out);
    return hipGetLastError();
}

template <int BITS>
void launch_batch_sort_bits(const BatchEntry* e, const int* start, int n, int blocks, int passes,
                            hipStream_t stream) {
    for (int pass = 0; pass < passes; ++pass) {
        const int last = pass == passes - 1;
        hipLaunchKernelGGL(k_batch_hist<BITS>, dim3(blocks), dim3(kSortThreads), 0, stream, e,
                           start, n, pass);
        hipLaunchKernelGGL(k_batch_rowscan<BITS>, dim3((1 << BITS) * n), dim3(kSortThreads), 0,
                           stream, e);
        hipLaunchKernelGGL(k_batch_scatter<BITS>, dim3(blocks), dim3(kSortThreads), 0, stream, e,
                           start, n, pass, last);
    }
}

hipError_t launch_batch_sort(const BatchEntry* e, const int* start, int n, int blocks, int passes,
                             int radix_bits, hipStream_t stream) {
    if (n <= 0 || blocks <= 0) return hipSuccess;
    if (radix_bits == 9)
        launch_batch_sort_bits<9>(e, start, n, blocks, passes, stream);
    else
        launch_batch_sort_bits<8>(e, start, n, blocks, passes, stream);
    return hipGetLastError();
}

}  // namespace evsim
