// Pyramidal Lucas-Kanade flow on gfx950: the flow the sparse method needs at its selected pixels
// (Sec. III-B, where the paper estimates it with Lucas-Kanade) estimated on the device instead of
// supplied.  The method is Lucas and Kanade's least-squares window fit, iterated, coarse to fine:
//   pyramid level 0 = the frame's intensity; level l+1 (ceil(W/2) x ceil(H/2)) = the 1-2-1 x 1-2-1
//   binomial average (/16) of level l around (2x, 2y), clamped; gradient texels are central
//   differences (T(x+1) - T(x-1)) / 2, clamped; samples at real positions are clamp-to-edge
//   bilinear blends of texels.  Per pixel p, from the coarsest level down with guess g (0 at the
//   top), window offsets (dx, dy) in [-r, r]^2 around u = p / 2^l: G = sum [ix^2, ix iy; ix iy,
//   iy^2]; the pixel is invalid (flow 0) unless trace(G) >= min_trace (2r+1)^2 and det(G) >=
//   min_ratio trace(G)^2; then up to `iters` steps b = sum (I(u+d) - J(u+d+g+v)) [ix, iy],
//   step = G^-1 b (Cramer's rule), v += step, stopping once |step|^2 < eps; g = 2 (g + v) for the
//   next level, flow = g + v at level 0.
// Every value of the pyramid and of the gradients is exact in fp32 (dyadic with at most 24
// significant bits for <= 4 levels of 8-bit input), and every other operation is one fp32
// operation with one rounding in the order written (-ffp-contract=off).  Each window sum is taken
// in one fixed order: position q = (dy + r)(2r + 1) + (dx + r) goes to partial q mod 64, in order
// of q from 0, and the 64 partials combine pairwise (partial l takes l + 32, then l + 16, ..., l + 1).
// That is one wave's lanes each summing their own positions, then a six-step shuffle tree.
#include "evsim_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace evsim {

PyrLayout pyr_layout(int W, int H, int levels) {
    PyrLayout L;
    L.levels = levels;
    uint64_t off = 0;
    int w = W, h = H;
    for (int l = 0; l <= kLkMaxLevels; ++l) {
        L.w[l] = w;
        L.h[l] = h;
        L.off[l] = off;
        if (l <= levels) off += (uint64_t)w * (uint64_t)h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    L.total = off;
    return L;
}

namespace {

struct Level {
    const float* v;
    int w, h;
};

__device__ __forceinline__ Level level_of(const float* pyr, const PyrLayout& L, int l) {
    Level r;
    r.v = pyr + L.off[l];
    r.w = L.w[l];
    r.h = L.h[l];
    return r;
}

__device__ __forceinline__ float texel_at(const Level& T, int x, int y) {
    x = x < 0 ? 0 : (x >= T.w ? T.w - 1 : x);
    y = y < 0 ? 0 : (y >= T.h ? T.h - 1 : y);
    return T.v[(int64_t)y * T.w + x];
}

struct Tap {
    int x0, y0, x1, y1;
    float fx, fy, gx, gy;
};

__device__ __forceinline__ Tap tap_at(const Level& T, float sx, float sy) {
    Tap t;
    sx = fminf(fmaxf(sx, 0.0f), (float)(T.w - 1));
    sy = fminf(fmaxf(sy, 0.0f), (float)(T.h - 1));
    t.x0 = (int)floorf(sx);
    t.y0 = (int)floorf(sy);
    t.fx = sx - (float)t.x0;
    t.fy = sy - (float)t.y0;
    t.x1 = min(t.x0 + 1, T.w - 1);
    t.y1 = min(t.y0 + 1, T.h - 1);
    t.gx = 1.0f - t.fx;
    t.gy = 1.0f - t.fy;
    return t;
}

// kind 0: intensity; 1: x gradient; 2: y gradient texel at (x, y) (inside the level).
template <int KIND>
__device__ __forceinline__ float texel(const Level& T, int x, int y) {
    if constexpr (KIND == 0)
        return T.v[(int64_t)y * T.w + x];
    else if constexpr (KIND == 1)
        return (texel_at(T, x + 1, y) - texel_at(T, x - 1, y)) * 0.5f;
    else
        return (texel_at(T, x, y + 1) - texel_at(T, x, y - 1)) * 0.5f;
}

template <int KIND>
__device__ __forceinline__ float bil_tap(const Level& T, const Tap& t) {
    const float top = t.gx * texel<KIND>(T, t.x0, t.y0) + t.fx * texel<KIND>(T, t.x1, t.y0);
    const float bot = t.gx * texel<KIND>(T, t.x0, t.y1) + t.fx * texel<KIND>(T, t.x1, t.y1);
    return t.gy * top + t.fy * bot;
}

// Wide reads of a tap's texels.  They read exactly the texels the one-texel forms above read (so
// every sample is bit-identical) with fewer load instructions: a row's (x0, x1) pair in one 8-byte
// read, the first frame's (x0 - 1 .. x0 + 2) run in one 16-byte read, where those texels are
// adjacent inside the row (4-byte aligned, which multi-dword reads need); the clamped edge cases
// read texel by texel.
struct Pair {
    float a, b;
};
struct Quad {
    float a, b, c, d;
};
// Vector views of 2 and 4 adjacent texels at 4-byte alignment: one 8- or 16-byte read.
typedef float TexelPair __attribute__((vector_size(8), aligned(4)));
typedef float TexelQuad __attribute__((vector_size(16), aligned(4)));

// (T(x0, y), T(x1, y)), x1 = min(x0 + 1, w - 1)
__device__ __forceinline__ Pair row_pair(const Level& T, int x0, int x1, int y) {
    const float* p = T.v + (int64_t)y * T.w + x0;
    Pair r;
    if (x1 > x0) {
        const TexelPair v = *(const TexelPair*)p;
        r.a = v[0];
        r.b = v[1];
    } else {
        r.a = r.b = *p;
    }
    return r;
}

// (T(xm, y), T(x0, y), T(x1, y), T(x2, y)), xm = max(x0 - 1, 0), x2 = min(x1 + 1, w - 1)
__device__ __forceinline__ Quad row_quad(const Level& T, int x0, int x1, int y) {
    const float* row = T.v + (int64_t)y * T.w;
    Quad r;
    if (x0 >= 1 && x0 + 2 <= T.w - 1) {
        const TexelQuad v = *(const TexelQuad*)(row + x0 - 1);
        r.a = v[0];
        r.b = v[1];
        r.c = v[2];
        r.d = v[3];
    } else {
        r.a = row[x0 >= 1 ? x0 - 1 : 0];
        r.b = row[x0];
        r.c = row[x1];
        r.d = row[x1 + 1 <= T.w - 1 ? x1 + 1 : T.w - 1];
    }
    return r;
}

// bil_tap<0> of the second frame through row_pair
__device__ __forceinline__ float bil0_wide(const Level& T, const Tap& t) {
    const Pair r0 = row_pair(T, t.x0, t.x1, t.y0), r1 = row_pair(T, t.x0, t.x1, t.y1);
    const float top = t.gx * r0.a + t.fx * r0.b;
    const float bot = t.gx * r1.a + t.fx * r1.b;
    return t.gy * top + t.fy * bot;
}

// bil_tap<0>, <1> and <2> of one tap from its 12 distinct texels: rows y0 and y1 at xm .. x2,
// rows ym = max(y0 - 1, 0) and y2 = min(y1 + 1, h - 1) at x0 and x1.  A gradient texel at x1 takes
// its left neighbour max(x1 - 1, 0): x0 when x1 = x0 + 1, else (right edge, x1 = x0) xm; likewise
// for rows.
__device__ __forceinline__ void bil_all_wide(const Level& T, const Tap& t, float* i0, float* ix,
                                             float* iy) {
    const Quad q0 = row_quad(T, t.x0, t.x1, t.y0), q1 = row_quad(T, t.x0, t.x1, t.y1);
    const int ym = t.y0 >= 1 ? t.y0 - 1 : 0, y2 = t.y1 + 1 <= T.h - 1 ? t.y1 + 1 : T.h - 1;
    const Pair pm = row_pair(T, t.x0, t.x1, ym), p2 = row_pair(T, t.x0, t.x1, y2);
    const bool xs = t.x1 > t.x0, ys = t.y1 > t.y0;
    const float gx00 = (q0.c - q0.a) * 0.5f, gx10 = (q0.d - (xs ? q0.b : q0.a)) * 0.5f;
    const float gx01 = (q1.c - q1.a) * 0.5f, gx11 = (q1.d - (xs ? q1.b : q1.a)) * 0.5f;
    const float gy00 = (q1.b - pm.a) * 0.5f, gy10 = (q1.c - pm.b) * 0.5f;
    const float gy01 = (p2.a - (ys ? q0.b : pm.a)) * 0.5f, gy11 = (p2.b - (ys ? q0.c : pm.b)) * 0.5f;
    {
        const float top = t.gx * gx00 + t.fx * gx10;
        const float bot = t.gx * gx01 + t.fx * gx11;
        *ix = t.gy * top + t.fy * bot;
    }
    {
        const float top = t.gx * gy00 + t.fx * gy10;
        const float bot = t.gx * gy01 + t.fx * gy11;
        *iy = t.gy * top + t.fy * bot;
    }
    {
        const float top = t.gx * q0.b + t.fx * q0.c;
        const float bot = t.gx * q1.b + t.fx * q1.c;
        *i0 = t.gy * top + t.fy * bot;
    }
}

// Level 0 of every frame: intensity as float.
__global__ __launch_bounds__(256) void k_pyr_base(const uint8_t* __restrict__ first,
                                                  const uint8_t* __restrict__ rest,
                                                  int64_t fstride, int n, int64_t npix,
                                                  uint64_t total, float* __restrict__ pyr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t all = (int64_t)n * npix;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < all; i += stride) {
        const int64_t f = i / npix, p = i - f * npix;
        const uint8_t* src = f == 0 ? first : rest + (f - 1) * fstride;
        pyr[(uint64_t)f * total + (uint64_t)p] = (float)src[p];
    }
}

// Level l of every frame from level l - 1.
__global__ __launch_bounds__(256) void k_pyr_down(PyrLayout L, int l, int n,
                                                  float* __restrict__ pyr) {
    const int w = L.w[l], h = L.h[l];
    const int64_t per = (int64_t)w * h;
    const int64_t all = (int64_t)n * per;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < all; i += stride) {
        const int64_t f = i / per, q = i - f * per;
        const int y = (int)(q / w), x = (int)(q - (int64_t)y * w);
        Level a;
        a.v = pyr + (uint64_t)f * L.total + L.off[l - 1];
        a.w = L.w[l - 1];
        a.h = L.h[l - 1];
        const int cx = 2 * x, cy = 2 * y;
        const float c = texel_at(a, cx, cy);
        const float edges = texel_at(a, cx - 1, cy) + texel_at(a, cx + 1, cy) +
                            texel_at(a, cx, cy - 1) + texel_at(a, cx, cy + 1);
        const float corners = texel_at(a, cx - 1, cy - 1) + texel_at(a, cx + 1, cy - 1) +
                              texel_at(a, cx - 1, cy + 1) + texel_at(a, cx + 1, cy + 1);
        pyr[(uint64_t)f * L.total + L.off[l] + (uint64_t)q] =
            ((4.0f * c + 2.0f * edges) + corners) * 0.0625f;
    }
}

// ------------------------------------------------------------------------------------------
// One wave per point.  The lanes share the window's positions (position q, lane q mod 64, PL
// positions per lane): per level each lane samples the first frame's intensity and gradients at
// its positions once and keeps them in registers for every iteration, so an iteration samples
// only the second frame.  Each lane adds its positions' products in order of q, and the wave
// combines the 64 partials pairwise (wave_window_sum): the order the file header fixes.
// ------------------------------------------------------------------------------------------
constexpr int kLkWave = 64;
constexpr int kLkMaxPerLane = 16;   // (2 * 15 + 1)^2 = 961 <= 64 * 16 positions
// The kernels are built for PL = 4, 8 and 16 positions per lane (radius <= 7, <= 11, <= 15), so
// that a small window does not hold registers for the largest.

// Lane l's partial plus lane l + 32's, then l + 16's, ..., l + 1's; the total (lane 0's) to every
// lane.  Lanes at or above 64 - off read their own value at that step and are not used after it.
__device__ __forceinline__ float wave_window_sum(float part) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) part = part + __shfl_down(part, off, 64);
    return __shfl(part, 0, 64);
}

// Flow of integer pixel (px, py) from pyramid A to pyramid B; every lane returns the same result
// (true if valid).
template <int PL>
__device__ bool lk_point_wave(const float* A, const float* B, const PyrLayout& L,
                              const LkParams& P, int px, int py, float* fx, float* fy) {
    const int lane = threadIdx.x & 63;
    const int r = P.radius, side = 2 * r + 1, n = side * side;
    const float N = (float)n;
    float gx = 0.0f, gy = 0.0f;
    for (int l = P.levels; l >= 0; --l) {
        const Level I = level_of(A, L, l);
        const Level J = level_of(B, L, l);
        const float sc = ldexpf(1.0f, -l);
        const float ux = (float)px * sc, uy = (float)py * sc;
        float cix[PL], ciy[PL], ci0[PL];
        float sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
#pragma unroll
        for (int j = 0; j < PL; ++j) {
            const int q = lane + kLkWave * j;
            cix[j] = ciy[j] = ci0[j] = 0.0f;
            if (q < n) {
                const int dy = q / side - r, dx = q - (q / side) * side - r;
                const Tap t = tap_at(I, ux + (float)dx, uy + (float)dy);
                bil_all_wide(I, t, &ci0[j], &cix[j], &ciy[j]);
                sxx += cix[j] * cix[j];
                sxy += cix[j] * ciy[j];
                syy += ciy[j] * ciy[j];
            }
        }
        const float Gxx = wave_window_sum(sxx), Gxy = wave_window_sum(sxy),
                    Gyy = wave_window_sum(syy);
        const float trace = Gxx + Gyy;
        const float det = Gxx * Gyy - Gxy * Gxy;
        if (!(trace >= P.min_trace * N) || !(det >= P.min_ratio * trace * trace)) {
            *fx = 0.0f;
            *fy = 0.0f;
            return false;
        }
        float vx = 0.0f, vy = 0.0f;
        for (int k = 0; k < P.iters; ++k) {
            float sbx = 0.0f, sby = 0.0f;
#pragma unroll
            for (int j = 0; j < PL; ++j) {
                const int q = lane + kLkWave * j;
                if (q < n) {
                    const int dy = q / side - r, dx = q - (q / side) * side - r;
                    const float x = ux + (float)dx, y = uy + (float)dy;
                    const Tap u = tap_at(J, x + (gx + vx), y + (gy + vy));
                    const float d = ci0[j] - bil0_wide(J, u);
                    sbx += d * cix[j];
                    sby += d * ciy[j];
                }
            }
            const float bx = wave_window_sum(sbx), by = wave_window_sum(sby);
            const float ex = (Gyy * bx - Gxy * by) / det;
            const float ey = (Gxx * by - Gxy * bx) / det;
            vx += ex;
            vy += ey;
            if (ex * ex + ey * ey < P.eps) break;
        }
        if (l > 0) {
            gx = 2.0f * (gx + vx);
            gy = 2.0f * (gy + vy);
        } else {
            *fx = gx + vx;
            *fy = gy + vy;
        }
    }
    return true;
}

// Block b (one wave): slot b of the active list (sparse) or pixel b, every selected interval.
template <int PL>
__global__ __launch_bounds__(kLkWave) void k_lk_window(LkWindowArgs a) {
    const int slot = blockIdx.x;
    int p;
    if (a.act_px) {
        if (slot >= (int)*a.n_active) return;
        p = (int)a.act_px[slot];
    } else {
        if (slot >= a.npix) return;
        p = slot;
    }
    const int py = p / a.W, px = p - py * a.W;
    for (int i = 0; i < a.K; ++i) {
        if (a.mask && !((a.mask[(int64_t)(i >> 5) * a.npix + p] >> (i & 31)) & 1u)) continue;
        float fx = 0.0f, fy = 0.0f;
        lk_point_wave<PL>(a.pyr + (uint64_t)i * a.lay.total,
                          a.pyr + (uint64_t)(i + 1) * a.lay.total, a.lay, a.P, px, py, &fx, &fy);
        if (threadIdx.x == 0) {
            float* out = a.flow + (int64_t)i * 2 * a.npix + 2 * (int64_t)p;
            out[0] = fx;
            out[1] = fy;
        }
    }
}

// Points j = block, block + grid, ...: one wave each.  An index outside the image is invalid
// (flow 0) rather than read out of bounds.
template <int PL>
__global__ __launch_bounds__(kLkWave) void k_lk_points(const float* __restrict__ A,
                                                       const float* __restrict__ B, PyrLayout L,
                                                       LkParams P, const uint32_t* __restrict__ pts,
                                                       uint64_t n, float* __restrict__ flow,
                                                       uint8_t* __restrict__ valid) {
    const uint32_t W = (uint32_t)L.w[0];
    for (uint64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const uint32_t p = pts[j];
        const bool inside = (uint64_t)p < (uint64_t)W * (uint64_t)L.h[0];
        const int py = inside ? (int)(p / W) : 0, px = inside ? (int)(p - (uint32_t)py * W) : 0;
        float fx = 0.0f, fy = 0.0f;
        const bool ok = inside && lk_point_wave<PL>(A, B, L, P, px, py, &fx, &fy);
        if (threadIdx.x == 0) {
            flow[2 * j] = fx;
            flow[2 * j + 1] = fy;
            if (valid) valid[j] = ok ? 1 : 0;
        }
    }
}

}  // namespace

hipError_t launch_pyramids(const uint8_t* first, const uint8_t* rest, int64_t fstride, int n,
                           const PyrLayout& lay, float* pyr, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t npix = (int64_t)lay.w[0] * lay.h[0];
    int64_t blocks = std::min<int64_t>(((int64_t)n * npix + 255) / 256, 8192);
    hipLaunchKernelGGL(k_pyr_base, dim3((unsigned)blocks), dim3(256), 0, stream, first, rest,
                       fstride, n, npix, lay.total, pyr);
    for (int l = 1; l <= lay.levels; ++l) {
        const int64_t per = (int64_t)lay.w[l] * lay.h[l];
        blocks = std::min<int64_t>(((int64_t)n * per + 255) / 256, 8192);
        hipLaunchKernelGGL(k_pyr_down, dim3((unsigned)blocks), dim3(256), 0, stream, lay, l, n,
                           pyr);
    }
    return hipGetLastError();
}

hipError_t launch_lk_points(const float* a, const float* b, const PyrLayout& lay,
                            const LkParams& P, const uint32_t* points, uint64_t n, float* flow,
                            uint8_t* valid, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    if (P.radius < 1 || (2 * P.radius + 1) * (2 * P.radius + 1) > kLkWave * kLkMaxPerLane)
        return hipErrorInvalidValue;
    const int n_win = (2 * P.radius + 1) * (2 * P.radius + 1);
    const unsigned blocks = (unsigned)std::min<uint64_t>(n, 1u << 20);
    if (n_win <= kLkWave * 4)
        hipLaunchKernelGGL(k_lk_points<4>, dim3(blocks), dim3(kLkWave), 0, stream, a, b, lay, P,
                           points, n, flow, valid);
    else if (n_win <= kLkWave * 8)
        hipLaunchKernelGGL(k_lk_points<8>, dim3(blocks), dim3(kLkWave), 0, stream, a, b, lay, P,
                           points, n, flow, valid);
    else
        hipLaunchKernelGGL(k_lk_points<16>, dim3(blocks), dim3(kLkWave), 0, stream, a, b, lay, P,
                           points, n, flow, valid);
    return hipGetLastError();
}

hipError_t launch_lk_window(const LkWindowArgs& a, int max_slots, hipStream_t stream) {
    if (max_slots <= 0) return hipSuccess;
    if (a.P.radius < 1 || (2 * a.P.radius + 1) * (2 * a.P.radius + 1) > kLkWave * kLkMaxPerLane)
        return hipErrorInvalidValue;
    const int side = 2 * a.P.radius + 1, n = side * side;
    if (n <= kLkWave * 4)
        hipLaunchKernelGGL(k_lk_window<4>, dim3(max_slots), dim3(kLkWave), 0, stream, a);
    else if (n <= kLkWave * 8)
        hipLaunchKernelGGL(k_lk_window<8>, dim3(max_slots), dim3(kLkWave), 0, stream, a);
    else
        hipLaunchKernelGGL(k_lk_window<16>, dim3(max_slots), dim3(kLkWave), 0, stream, a);
    return hipGetLastError();
}

}  // namespace evsim
