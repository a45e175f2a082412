/*
 * oracle.c -- plain, slow, single-threaded CPU reference of the frame-to-event simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or loads this file; it
 * exists so that tests, the smoke check and the benchmark's CPU-baseline leg can compare the HIP
 * path against an implementation a reader can check against the paper line by line.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared (no -march: no FMA).
 * Every floating-point operation is a single fp32 operation with one rounding, written in the
 * order given below; integers are exact.
 *
 * Paper: Ziegler et al., "Real-time event simulation with frame-based cameras" (arXiv 2209.04634).
 *   - Event pixel model: a pixel fires when its log-brightness change reaches a threshold (Sec. I).
 *   - Difference frames of consecutive frames, thresholded with C_pos / C_neg into polarities
 *     (Sec. III, Sec. III-A threshold equations).
 *   - Temporal up-sampling by flow-driven linear interpolation of intermediate frames (Sec. III,
 *     Sec. III-A); sparse variant interpolates only pixels whose frame-to-frame change passes a
 *     threshold, unselected pixels emit nothing (Sec. III-B, Sec. IV-B discussion).
 *   - Output: events <x, y, t, p> (Sec. III-A, Fig. 1 caption), or a frame of accumulated events
 *     (same caption); the events/(pixel s) statistic of the statistical comparison (Sec. IV-C).
 *   - Memoryless thresholding: every difference of consecutive (interpolated) frames is compared
 *     with C_pos / C_neg on its own, strictly, one event at most per pixel and sub-frame
 *     (Sec. III-A threshold equations, taken literally).
 *   - Difference-frame interpolation: from three consecutive frames, two difference frames; the
 *     flow between them interpolates further difference frames, each thresholded (Sec. III-C).
 *   - Flow at the selected pixels estimated with Lucas-Kanade (Sec. III-B, IV-A), here the
 *     published pyramidal form of Lucas and Kanade's window least-squares fit (oracle_lk_flow).
 *
 * Readings where the paper is silent:
 *   log transform ln(v/255 + eps) via a 256-entry table; interpolation of the transformed frames;
 *   S = N + 1 sub-intervals for N interpolated frames; gather-form bidirectional flow-guided blend
 *   with clamp-to-edge bilinear sampling; threshold crossing against a per-pixel reference level
 *   with ties counted (>= C_pos, <= -C_neg); crossing times linear within a sub-interval, floored
 *   to integer microseconds; backlog crossings stamped at the sub-interval start; sparse selection
 *   |L1 - L0| >= m; first frame initialises state only; canonical order by (t, y, x, p) per
 *   interval, intervals in push order.  Memoryless mode: strict > C_pos / < -C_neg on each
 *   difference of consecutive samples, stamped at the later sample's time t0 + floor(k/S delta),
 *   no reference level.  Difference method: events from the third frame on (the second gives the
 *   first difference frame only); the supplied flow of an interval is the flow from the previous
 *   difference frame to the current one; difference frames of transformed frames; always
 *   memoryless; interpolated difference frames are not rescaled (the paper's larger thresholds
 *   for this method, Table I, fit unscaled frames).  Accumulated frame: counts per pixel and
 *   polarity over a half-open time window.  Events/(pixel s): mean and population standard
 *   deviation over all pixels of the per-pixel count divided by the window length.  Lucas-Kanade
 *   window sums: 64 strided partial sums combined pairwise, in one fixed order (window_sum).
 *
 * Parity is pinned (tests/test_oracle_*.py) by: the exhaustive table check against an exact
 * logarithm, zero-event invariants, the closed-form per-pixel count floor(|dL|/C) of the basic
 * method, endpoint exactness (dense with S = 1 equals basic), zero-flow and translating-edge
 * closed forms, time reversal, reference bookkeeping, hand-worked fixtures under tests/golden/ and
 * an independent float64 brute-force solver on 8x8 inputs; for the memoryless mode and the
 * difference method by hand-worked fixtures, the float64 solver, a translating-edge closed form
 * and invariants; for the accumulated frame and the event rate by hand-worked examples and exact
 * rational arithmetic; for Lucas-Kanade by recovered known translations, rejection of flat and
 * edge windows, invalidity of indices outside the image and an independent float64
 * implementation (tests/lk64.py).  Planted one-token
 * mistakes each fail a pin (tests/test_oracle_mutants*.py).  The exact interpolation formula has
 * no anchor in the paper beyond those properties ("parity unpinned" against the paper itself for
 * that formula; pinned through endpoint exactness, the zero-flow and translating-edge closed forms
 * and the brute-force solver), and the estimator's quality on real scenes is unpinned (no data
 * or reference implementation here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_ORDER (-2)
#define OR_E_NOMEM (-3)
#define OR_E_RANGE (-4)

enum { OR_BASIC = 0, OR_DENSE = 1, OR_SPARSE = 2, OR_DIFFERENCE = 3 };
enum { OR_LOG = 0, OR_LINEAR = 1 };
enum { OR_REFERENCE = 0, OR_MEMORYLESS = 1 };
enum { OR_FLOW_SUPPLIED = 0, OR_FLOW_LK = 1 };

typedef struct {
    int32_t width, height;
    int32_t method, transform;
    float c_pos, c_neg;      /* magnitudes, > 0 */
    float log_eps;
    int32_t n_interp;        /* N interpolated frames; S = N + 1 (basic: S = 1) */
    float mask_threshold;    /* sparse: < 0 -> min(c_pos, c_neg) */
    int32_t thresh_mode;     /* OR_REFERENCE or OR_MEMORYLESS; the difference method is always
                                memoryless */
    int32_t flow_source;     /* OR_FLOW_SUPPLIED or OR_FLOW_LK (dense and sparse methods) */
    int32_t lk_levels, lk_radius, lk_iters;
    float lk_eps, lk_min_trace, lk_min_ratio;
} oracle_cfg;

typedef struct {
    int32_t levels, radius, iters;
    float eps, min_trace, min_ratio;
} oracle_lk;

typedef struct {
    oracle_cfg cfg;
    int S;
    float m;                 /* sparse selection threshold */
    float lut[256];
    uint8_t* prev;           /* previous camera frame */
    uint8_t* prev2;          /* the frame before it (difference method) */
    uint64_t n_int;          /* intervals pushed so far */
    float* lref;             /* per-pixel reference level */
    float* L0;               /* scratch: transformed previous frame */
    float* L1;               /* scratch: transformed current frame */
    float* V;                /* scratch: S + 1 samples of one pixel */
    int started;
    int64_t t_prev, epoch;
    float* lkflow;           /* flow estimated by Lucas-Kanade for the current interval */
    uint64_t* ev;            /* events of the last pushed interval (sorted keys) */
    uint64_t n_ev, cap_ev;
    uint64_t n_selected;     /* sparse: pixels selected in the last interval */
} oracle_sim;

/* Intensity transform table.  The event pixel responds to log-scale brightness change (Sec. I);
 * the paper itself thresholds linear differences (Sec. III).  LOG: ln(v/255 + eps) evaluated in
 * double and rounded once to float.  LINEAR: the raw value, thresholds in 0..255 units. */
int oracle_lut(int32_t transform, float log_eps, float* lut) {
    if (transform == OR_LOG) {
        if (!(log_eps > 0.0f)) return OR_E_INVAL;
        for (int v = 0; v < 256; ++v)
            lut[v] = (float)log((double)v / 255.0 + (double)log_eps);
    } else if (transform == OR_LINEAR) {
        for (int v = 0; v < 256; ++v) lut[v] = (float)v;
    } else {
        return OR_E_INVAL;
    }
    return OR_OK;
}

static int lk_params_ok(const oracle_lk* P);

static void or_destroy(oracle_sim* s) {
    if (!s) return;
    free(s->prev); free(s->prev2); free(s->lref); free(s->L0); free(s->L1); free(s->V);
    free(s->lkflow); free(s->ev);
    free(s);
}

void oracle_destroy(oracle_sim* s) { or_destroy(s); }

int oracle_create(const oracle_cfg* cfg, oracle_sim** out) {
    if (!cfg || !out) return OR_E_INVAL;
    *out = NULL;
    if (cfg->width < 1 || cfg->height < 1 || cfg->width > 4096 || cfg->height > 4096)
        return OR_E_INVAL;
    if (cfg->method < OR_BASIC || cfg->method > OR_DIFFERENCE) return OR_E_INVAL;
    if (cfg->thresh_mode != OR_REFERENCE && cfg->thresh_mode != OR_MEMORYLESS) return OR_E_INVAL;
    if (cfg->flow_source != OR_FLOW_SUPPLIED && cfg->flow_source != OR_FLOW_LK) return OR_E_INVAL;
    if (cfg->flow_source == OR_FLOW_LK) {
        const oracle_lk P = {cfg->lk_levels, cfg->lk_radius, cfg->lk_iters, cfg->lk_eps,
                             cfg->lk_min_trace, cfg->lk_min_ratio};
        if (!lk_params_ok(&P)) return OR_E_INVAL;
        if (cfg->method != OR_DENSE && cfg->method != OR_SPARSE) return OR_E_INVAL;
    }
    if (!(cfg->c_pos > 0.0f) || !(cfg->c_neg > 0.0f)) return OR_E_INVAL;
    if (cfg->n_interp < 0 || cfg->n_interp > 255) return OR_E_INVAL;
    oracle_sim* s = (oracle_sim*)calloc(1, sizeof(oracle_sim));
    if (!s) return OR_E_NOMEM;
    s->cfg = *cfg;
    if (oracle_lut(cfg->transform, cfg->log_eps, s->lut) != OR_OK) { free(s); return OR_E_INVAL; }
    s->S = (cfg->method == OR_BASIC) ? 1 : cfg->n_interp + 1;
    s->m = cfg->mask_threshold < 0.0f ? fminf(cfg->c_pos, cfg->c_neg) : cfg->mask_threshold;
    size_t n = (size_t)cfg->width * (size_t)cfg->height;
    s->prev = (uint8_t*)malloc(n);
    s->prev2 = (uint8_t*)malloc(n);
    s->lref = (float*)malloc(n * sizeof(float));
    s->L0 = (float*)malloc(n * sizeof(float));
    s->L1 = (float*)malloc(n * sizeof(float));
    s->V = (float*)malloc((size_t)(s->S + 1) * sizeof(float));
    if (cfg->flow_source == OR_FLOW_LK) s->lkflow = (float*)calloc(2 * n, sizeof(float));
    if (!s->prev || !s->prev2 || !s->lref || !s->L0 || !s->L1 || !s->V ||
        (cfg->flow_source == OR_FLOW_LK && !s->lkflow)) {
        or_destroy(s);
        return OR_E_NOMEM;
    }
    *out = s;
    return OR_OK;
}

/* Clamp-to-edge bilinear sample of a transformed frame at a real-valued position. */
static float bil(const float* L, int W, int H, float sx, float sy) {
    sx = fminf(fmaxf(sx, 0.0f), (float)(W - 1));
    sy = fminf(fmaxf(sy, 0.0f), (float)(H - 1));
    int x0 = (int)floorf(sx);
    int y0 = (int)floorf(sy);
    float fx = sx - (float)x0;
    float fy = sy - (float)y0;
    int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    float gx = 1.0f - fx;
    float gy = 1.0f - fy;
    float top = gx * L[(size_t)y0 * W + x0] + fx * L[(size_t)y0 * W + x1];
    float bot = gx * L[(size_t)y1 * W + x0] + fx * L[(size_t)y1 * W + x1];
    return gy * top + fy * bot;
}

/* ------------------------------------------------------------------------------------------
 * Pyramidal Lucas-Kanade flow (the sparse method estimates flow with Lucas-Kanade at the selected
 * pixels, Sec. III-B, IV-A; here written from the published method: Lucas and Kanade's
 * least-squares window fit, iterated, coarse to fine over an image pyramid).
 *   Pyramid: level 0 is the frame's intensity; level l+1 has ceil(W/2) x ceil(H/2) texels, each
 *   the 1-2-1 x 1-2-1 binomial average (/16) of level l around (2x, 2y), clamped at the border.
 *   Gradient texels: central differences (T(x+1) - T(x-1)) / 2, clamped.  Samples at real
 *   positions: clamp-to-edge bilinear of texels.
 *   Per pixel p, from the coarsest level down, with guess g (0 at the top) and window offsets
 *   (dx, dy) in [-r, r]^2 around u = p / 2^l: G = sum of [ix^2, ix iy; ix iy, iy^2] of the
 *   gradients of I; the level is rejected (flow 0, invalid) unless trace(G) >= min_trace * N
 *   (N = (2r+1)^2 texels: enough texture) and det(G) >= min_ratio * trace(G)^2 (no aperture
 *   problem).  Then up to `iters` steps: b = sum of (I(u + d) - J(u + d + g + v)) [ix, iy],
 *   step = G^-1 b (by Cramer's rule), v += step, stop once |step|^2 < eps.  Next level:
 *   g = 2 (g + v); at level 0 the flow is g + v.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    int W, H;
    float* v;
} or_img;

static float img_at(const or_img* im, int x, int y) {
    x = x < 0 ? 0 : (x >= im->W ? im->W - 1 : x);
    y = y < 0 ? 0 : (y >= im->H ? im->H - 1 : y);
    return im->v[(size_t)y * im->W + x];
}

static void pyr_down(const or_img* a, or_img* b) {
    for (int y = 0; y < b->H; ++y) {
        for (int x = 0; x < b->W; ++x) {
            const int cx = 2 * x, cy = 2 * y;
            const float c = img_at(a, cx, cy);
            const float edges = img_at(a, cx - 1, cy) + img_at(a, cx + 1, cy) +
                                img_at(a, cx, cy - 1) + img_at(a, cx, cy + 1);
            const float corners = img_at(a, cx - 1, cy - 1) + img_at(a, cx + 1, cy - 1) +
                                  img_at(a, cx - 1, cy + 1) + img_at(a, cx + 1, cy + 1);
            b->v[(size_t)y * b->W + x] = ((4.0f * c + 2.0f * edges) + corners) * 0.0625f;
        }
    }
}

static float grad_x(const or_img* im, int x, int y) {
    return (img_at(im, x + 1, y) - img_at(im, x - 1, y)) * 0.5f;
}

static float grad_y(const or_img* im, int x, int y) {
    return (img_at(im, x, y + 1) - img_at(im, x, y - 1)) * 0.5f;
}

typedef struct {
    int x0, y0, x1, y1;
    float fx, fy, gx, gy;
} or_tap;

static or_tap tap_at(int W, int H, float sx, float sy) {
    or_tap t;
    sx = fminf(fmaxf(sx, 0.0f), (float)(W - 1));
    sy = fminf(fmaxf(sy, 0.0f), (float)(H - 1));
    t.x0 = (int)floorf(sx);
    t.y0 = (int)floorf(sy);
    t.fx = sx - (float)t.x0;
    t.fy = sy - (float)t.y0;
    t.x1 = t.x0 + 1 < W ? t.x0 + 1 : W - 1;
    t.y1 = t.y0 + 1 < H ? t.y0 + 1 : H - 1;
    t.gx = 1.0f - t.fx;
    t.gy = 1.0f - t.fy;
    return t;
}

/* kind 0: intensity, 1: x gradient, 2: y gradient texels */
static float texel(const or_img* im, int kind, int x, int y) {
    return kind == 0 ? im->v[(size_t)y * im->W + x] : (kind == 1 ? grad_x(im, x, y) : grad_y(im, x, y));
}

static float bil_tap(const or_img* im, int kind, or_tap t) {
    const float top = t.gx * texel(im, kind, t.x0, t.y0) + t.fx * texel(im, kind, t.x1, t.y0);
    const float bot = t.gx * texel(im, kind, t.x0, t.y1) + t.fx * texel(im, kind, t.x1, t.y1);
    return t.gy * top + t.fy * bot;
}

/* A window sum in a fixed order (the paper does not fix one; this order is exact to reproduce
 * with 64 parallel partial sums): position q of the window, row-major, goes to partial q mod 64
 * in order of q, each partial starting from 0; then partial l takes partial l + 32, l + 16, ...,
 * l + 1 in turn (pairwise, 6 levels); the sum is partial 0.  One rounding per addition. */
#define OR_WINDOW_MAX 961   /* (2 * 15 + 1)^2 */
static float window_sum(const float* v, int n) {
    float part[64];
    for (int l = 0; l < 64; ++l) part[l] = 0.0f;
    for (int q = 0; q < n; ++q) part[q % 64] += v[q];
    for (int off = 32; off >= 1; off /= 2)
        for (int l = 0; l < off; ++l) part[l] = part[l] + part[l + off];
    return part[0];
}

/* Flow of integer pixel (px, py) from pyramid I to pyramid J; returns 1 if valid. */
static int lk_point(const or_img* I, const or_img* J, const oracle_lk* P, int px, int py,
                    float* fx, float* fy) {
    const int r = P->radius, side = 2 * r + 1, n = side * side;
    const float N = (float)n;
    /* per window position q = (dy + r) side + (dx + r): the products whose window sums form the
     * normal matrix and the right-hand side */
    float pxx[OR_WINDOW_MAX], pxy[OR_WINDOW_MAX], pyy[OR_WINDOW_MAX];
    float pbx[OR_WINDOW_MAX], pby[OR_WINDOW_MAX];
    float gx = 0.0f, gy = 0.0f;
    for (int l = P->levels; l >= 0; --l) {
        const float sc = ldexpf(1.0f, -l);
        const float ux = (float)px * sc, uy = (float)py * sc;
        memset(pxx, 0, sizeof pxx);
        memset(pxy, 0, sizeof pxy);
        memset(pyy, 0, sizeof pyy);
        for (int dy = -r; dy <= r; ++dy) {
            for (int dx = -r; dx <= r; ++dx) {
                const or_tap t = tap_at(I[l].W, I[l].H, ux + (float)dx, uy + (float)dy);
                const float ix = bil_tap(&I[l], 1, t), iy = bil_tap(&I[l], 2, t);
                const int q = (dy + r) * side + (dx + r);
                pxx[q] = ix * ix;
                pxy[q] = ix * iy;
                pyy[q] = iy * iy;
            }
        }
        const float Gxx = window_sum(pxx, n), Gxy = window_sum(pxy, n), Gyy = window_sum(pyy, n);
        const float trace = Gxx + Gyy;
        const float det = Gxx * Gyy - Gxy * Gxy;
        if (!(trace >= P->min_trace * N) || !(det >= P->min_ratio * trace * trace)) {
            *fx = 0.0f;
            *fy = 0.0f;
            return 0;
        }
        float vx = 0.0f, vy = 0.0f;
        for (int k = 0; k < P->iters; ++k) {
            memset(pbx, 0, sizeof pbx);
            memset(pby, 0, sizeof pby);
            for (int dy = -r; dy <= r; ++dy) {
                for (int dx = -r; dx <= r; ++dx) {
                    const float x = ux + (float)dx, y = uy + (float)dy;
                    const or_tap t = tap_at(I[l].W, I[l].H, x, y);
                    const float ix = bil_tap(&I[l], 1, t), iy = bil_tap(&I[l], 2, t);
                    const float i0 = bil_tap(&I[l], 0, t);
                    const or_tap u = tap_at(J[l].W, J[l].H, x + (gx + vx), y + (gy + vy));
                    const float d = i0 - bil_tap(&J[l], 0, u);
                    const int q = (dy + r) * side + (dx + r);
                    pbx[q] = d * ix;
                    pby[q] = d * iy;
                }
            }
            const float bx = window_sum(pbx, n), by = window_sum(pby, n);
            const float ex = (Gyy * bx - Gxy * by) / det;
            const float ey = (Gxx * by - Gxy * bx) / det;
            vx += ex;
            vy += ey;
            if (ex * ex + ey * ey < P->eps) break;
        }
        if (l > 0) {
            gx = 2.0f * (gx + vx);
            gy = 2.0f * (gy + vy);
        } else {
            *fx = gx + vx;
            *fy = gy + vy;
        }
    }
    return 1;
}

static int lk_params_ok(const oracle_lk* P) {
    return P->levels >= 0 && P->levels <= 4 && P->radius >= 1 && P->radius <= 15 &&
           P->iters >= 1 && P->iters <= 100 && P->eps >= 0.0f && P->min_trace >= 0.0f &&
           P->min_ratio >= 0.0f;
}

/* Pyramids of one frame: levels 0..L in one allocation; returns NULL on failure. */
static float* build_pyramid(const uint8_t* f, int W, int H, int L, or_img* lv) {
    size_t total = 0;
    int w = W, h = H;
    for (int l = 0; l <= L; ++l) {
        total += (size_t)w * h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    float* mem = (float*)malloc(total * sizeof(float));
    if (!mem) return NULL;
    size_t off = 0;
    w = W;
    h = H;
    for (int l = 0; l <= L; ++l) {
        lv[l].W = w;
        lv[l].H = h;
        lv[l].v = mem + off;
        off += (size_t)w * h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    for (size_t i = 0; i < (size_t)W * H; ++i) lv[0].v[i] = (float)f[i];
    for (int l = 1; l <= L; ++l) pyr_down(&lv[l - 1], &lv[l]);
    return mem;
}

/* Lucas-Kanade flow from f0 to f1 at pixel indices points[j] = y * W + x: flow[2j], flow[2j+1]
 * (dx, dy), valid[j] (may be NULL). */
int oracle_lk_flow(const uint8_t* f0, const uint8_t* f1, int W, int H, const oracle_lk* P,
                   const uint32_t* points, uint64_t n, float* flow, uint8_t* valid) {
    if (!f0 || !f1 || !P || W < 1 || H < 1 || !lk_params_ok(P)) return OR_E_INVAL;
    or_img I[5], J[5];
    float* a = build_pyramid(f0, W, H, P->levels, I);
    float* b = build_pyramid(f1, W, H, P->levels, J);
    if (!a || !b) { free(a); free(b); return OR_E_NOMEM; }
    for (uint64_t j = 0; j < n; ++j) {
        int ok = 0;
        flow[2 * j] = flow[2 * j + 1] = 0.0f;
        /* an index at or beyond W * H names no pixel: invalid, flow (0, 0) */
        if ((uint64_t)points[j] < (uint64_t)W * (uint64_t)H) {
            const int px = (int)(points[j] % (uint32_t)W), py = (int)(points[j] / (uint32_t)W);
            ok = lk_point(I, J, P, px, py, &flow[2 * j], &flow[2 * j + 1]);
        }
        if (valid) valid[j] = (uint8_t)ok;
    }
    free(a);
    free(b);
    return OR_OK;
}

static int push_event(oracle_sim* s, int64_t t, int x, int y, int pol) {
    if (s->n_ev == s->cap_ev) {
        uint64_t nc = s->cap_ev ? 2 * s->cap_ev : 1024;
        uint64_t* p = (uint64_t*)realloc(s->ev, nc * sizeof(uint64_t));
        if (!p) return OR_E_NOMEM;
        s->ev = p;
        s->cap_ev = nc;
    }
    uint64_t key = ((uint64_t)(t - s->epoch) << 25) | ((uint64_t)y << 13) | ((uint64_t)x << 1) |
                   (uint64_t)(pol > 0 ? 1 : 0);
    s->ev[s->n_ev++] = key;
    return OR_OK;
}

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Difference-frame interpolation (Sec. III-C) for the interval (t0, t0 + delta]: difference frames
 * D1 = T[prev] - T[prev2] and D2 = T[frame] - T[prev]; with the flow F between them, the
 * interpolated difference frame at tau = k / S is (1 - tau) * D1(p - tau F) + tau * D2(p +
 * (1 - tau) F) (the same gather-form blend and clamp-to-edge bilinear sampling as the frame
 * methods, applied to difference frames); D_S = D2.  Each of D_1 .. D_S is thresholded on its
 * own (> C_pos: positive, < -C_neg: negative) and its events are stamped at t0 + floor(k/S delta).
 * On allocation failure n_ev is set to all ones. */
static void difference_events(oracle_sim* s, const uint8_t* frame, const float* flow, int64_t t0,
                              float delta) {
    const int W = s->cfg.width, H = s->cfg.height, S = s->S;
    const size_t n = (size_t)W * (size_t)H;
    const float cp = s->cfg.c_pos, cn = s->cfg.c_neg;
    float* D1 = s->L0;
    float* D2 = s->L1;
    for (size_t i = 0; i < n; ++i) {
        D1[i] = s->lut[s->prev[i]] - s->lut[s->prev2[i]];
        D2[i] = s->lut[frame[i]] - s->lut[s->prev[i]];
    }
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            for (int k = 1; k <= S; ++k) {
                float Dk;
                if (k == S) {
                    Dk = D2[p];
                } else {
                    const float u = flow[2 * p], v = flow[2 * p + 1];
                    const float tau = (float)k / (float)S;
                    const float om = 1.0f - tau;
                    const float a = bil(D1, W, H, (float)x - tau * u, (float)y - tau * v);
                    const float b = bil(D2, W, H, (float)x + om * u, (float)y + om * v);
                    Dk = om * a + tau * b;
                }
                int pol = 0;
                if (Dk > cp) pol = 1;
                else if (Dk < -cn) pol = -1;
                if (!pol) continue;
                const float phi = (float)k / (float)S;
                const int64_t t = t0 + (int64_t)floorf(phi * delta);
                if (push_event(s, t, x, y, pol) != OR_OK) {
                    s->n_ev = (uint64_t)-1;
                    return;
                }
            }
        }
    }
}

/* Push one camera frame taken at t_us.  The first frame only initialises the reference levels.
 * For later frames, the interval (t_prev, t_us] is simulated and its events are left, sorted by
 * key, in the internal buffer (oracle_events).  flow is [H][W][2] (dx, dy) in pixels per interval,
 * required for the dense and sparse methods. */
int oracle_push(oracle_sim* s, const uint8_t* frame, const float* flow, int64_t t_us,
                uint64_t* n_events) {
    if (!s || !frame) return OR_E_INVAL;
    const int W = s->cfg.width, H = s->cfg.height, S = s->S;
    const size_t n = (size_t)W * (size_t)H;
    s->n_ev = 0;
    s->n_selected = 0;
    if (n_events) *n_events = 0;
    if (!s->started) {
        for (size_t i = 0; i < n; ++i) s->lref[i] = s->lut[frame[i]];
        memcpy(s->prev, frame, n);
        s->t_prev = t_us;
        s->epoch = t_us;
        s->started = 1;
        return OR_OK;
    }
    if (t_us <= s->t_prev) return OR_E_ORDER;
    if (t_us - s->epoch >= ((int64_t)1 << 39)) return OR_E_RANGE;
    const int diff = s->cfg.method == OR_DIFFERENCE;
    /* the difference method's first interval has one difference frame only: nothing to
     * interpolate and no flow needed */
    const int diff_first = diff && s->n_int == 0;
    if (s->cfg.method != OR_BASIC && !diff_first && !flow && s->cfg.flow_source != OR_FLOW_LK)
        return OR_E_INVAL;

    const int64_t t0 = s->t_prev;
    const float delta = (float)(t_us - t0);
    const float cp = s->cfg.c_pos, cn = s->cfg.c_neg;
    if (diff) {
        if (!diff_first) difference_events(s, frame, flow, t0, delta);
        if (s->n_ev == (uint64_t)-1) return OR_E_NOMEM;
        qsort(s->ev, s->n_ev, sizeof(uint64_t), cmp_u64);
        memcpy(s->prev2, s->prev, n);
        memcpy(s->prev, frame, n);
        s->t_prev = t_us;
        s->n_int++;
        if (n_events) *n_events = s->n_ev;
        return OR_OK;
    }
    const int memoryless = s->cfg.thresh_mode == OR_MEMORYLESS;
    for (size_t i = 0; i < n; ++i) {
        s->L0[i] = s->lut[s->prev[i]];
        s->L1[i] = s->lut[frame[i]];
    }
    if (s->cfg.flow_source == OR_FLOW_LK && S > 1) {
        /* estimate the flow at every pixel that will be interpolated (sparse: the selected) */
        uint32_t* pts = (uint32_t*)malloc(n * sizeof(uint32_t));
        float* fl = (float*)malloc(2 * n * sizeof(float));
        if (!pts || !fl) { free(pts); free(fl); return OR_E_NOMEM; }
        uint64_t np = 0;
        for (size_t i = 0; i < n; ++i)
            if (s->cfg.method != OR_SPARSE || fabsf(s->L1[i] - s->L0[i]) >= s->m)
                pts[np++] = (uint32_t)i;
        const oracle_lk P = {s->cfg.lk_levels, s->cfg.lk_radius, s->cfg.lk_iters, s->cfg.lk_eps,
                             s->cfg.lk_min_trace, s->cfg.lk_min_ratio};
        int rc = oracle_lk_flow(s->prev, frame, W, H, &P, pts, np, fl, NULL);
        if (rc == OR_OK)
            for (uint64_t j = 0; j < np; ++j) {
                s->lkflow[2 * (size_t)pts[j]] = fl[2 * j];
                s->lkflow[2 * (size_t)pts[j] + 1] = fl[2 * j + 1];
            }
        free(pts);
        free(fl);
        if (rc != OR_OK) return rc;
        flow = s->lkflow;
    }
    float* V = s->V;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            const float A0 = s->L0[p], A1 = s->L1[p];
            if (s->cfg.method == OR_SPARSE) {
                if (!(fabsf(A1 - A0) >= s->m)) continue;   /* not selected: no samples, no events */
                s->n_selected++;
            }
            /* samples of the interpolated series at tau = k / S */
            V[0] = A0;
            V[S] = A1;
            if (S > 1) {
                const float u = flow[2 * p], v = flow[2 * p + 1];
                for (int k = 1; k < S; ++k) {
                    const float tau = (float)k / (float)S;
                    const float om = 1.0f - tau;
                    const float a = bil(s->L0, W, H, (float)x - tau * u, (float)y - tau * v);
                    const float b = bil(s->L1, W, H, (float)x + om * u, (float)y + om * v);
                    V[k] = om * a + tau * b;
                }
            }
            if (memoryless) {
                /* each difference of consecutive samples on its own: one event at most, stamped
                 * at the later sample's time */
                for (int k = 0; k < S; ++k) {
                    const float D = V[k + 1] - V[k];
                    int pol = 0;
                    if (D > cp) pol = 1;
                    else if (D < -cn) pol = -1;
                    if (!pol) continue;
                    const float phi = (float)(k + 1) / (float)S;
                    const int64_t t = t0 + (int64_t)floorf(phi * delta);
                    if (push_event(s, t, x, y, pol) != OR_OK) return OR_E_NOMEM;
                }
                continue;
            }
            /* threshold crossings against the reference level, sub-interval by sub-interval */
            float R = s->lref[p];
            for (int k = 0; k < S; ++k) {
                const float A = V[k], B = V[k + 1];
                const float D = B - A;
                for (;;) {
                    int pol;
                    float Rn;
                    if (B - R >= cp) { Rn = R + cp; pol = 1; }
                    else if (B - R <= -cn) { Rn = R - cn; pol = -1; }
                    else break;
                    float theta;
                    const int backlog = pol > 0 ? (A >= Rn) : (A <= Rn);
                    if (backlog) theta = 0.0f;
                    else {
                        theta = (D == 0.0f) ? 0.0f : (Rn - A) / D;
                        theta = fminf(fmaxf(theta, 0.0f), 1.0f);
                    }
                    const float phi = ((float)k + theta) / (float)S;
                    const int64_t t = t0 + (int64_t)floorf(phi * delta);
                    if (push_event(s, t, x, y, pol) != OR_OK) return OR_E_NOMEM;
                    R = Rn;
                }
            }
            s->lref[p] = R;
        }
    }
    qsort(s->ev, s->n_ev, sizeof(uint64_t), cmp_u64);
    memcpy(s->prev2, s->prev, n);
    memcpy(s->prev, frame, n);
    s->t_prev = t_us;
    s->n_int++;
    if (n_events) *n_events = s->n_ev;
    return OR_OK;
}

/* Copies up to cap sorted keys of the last interval. */
uint64_t oracle_events(const oracle_sim* s, uint64_t* keys, uint64_t cap) {
    uint64_t k = s->n_ev < cap ? s->n_ev : cap;
    if (k) memcpy(keys, s->ev, k * sizeof(uint64_t));
    return k;
}

uint64_t oracle_selected(const oracle_sim* s) { return s->n_selected; }
int64_t oracle_epoch(const oracle_sim* s) { return s->epoch; }

int oracle_lref(const oracle_sim* s, float* out) {
    memcpy(out, s->lref, (size_t)s->cfg.width * s->cfg.height * sizeof(float));
    return OR_OK;
}

/* The S + 1 interpolated samples of one pixel between two frames (diagnostics for tests). */
int oracle_pixel_samples(const oracle_sim* s, const uint8_t* f0, const uint8_t* f1,
                         const float* flow, int x, int y, float* out) {
    const int W = s->cfg.width, H = s->cfg.height, S = s->S;
    const size_t n = (size_t)W * H;
    float* L0 = (float*)malloc(n * sizeof(float));
    float* L1 = (float*)malloc(n * sizeof(float));
    if (!L0 || !L1) { free(L0); free(L1); return OR_E_NOMEM; }
    for (size_t i = 0; i < n; ++i) { L0[i] = s->lut[f0[i]]; L1[i] = s->lut[f1[i]]; }
    const size_t p = (size_t)y * W + x;
    out[0] = L0[p];
    out[S] = L1[p];
    for (int k = 1; k < S; ++k) {
        const float u = flow[2 * p], v = flow[2 * p + 1];
        const float tau = (float)k / (float)S;
        const float om = 1.0f - tau;
        const float a = bil(L0, W, H, (float)x - tau * u, (float)y - tau * v);
        const float b = bil(L1, W, H, (float)x + om * u, (float)y + om * v);
        out[k] = om * a + tau * b;
    }
    free(L0); free(L1);
    return OR_OK;
}

/* Frame of accumulated events (Fig. 1 caption): for every key whose time t = epoch + (key >> 25)
 * lies in [t_begin, t_end), adds one to counts[0][y][x] for a positive event or to
 * counts[1][y][x] for a negative one.  counts is uint32 [2][H][W]. */
void oracle_accumulate(const uint64_t* keys, uint64_t n, int64_t epoch, int64_t t_begin,
                       int64_t t_end, int W, int H, uint32_t* counts) {
    const size_t plane = (size_t)W * (size_t)H;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t k = keys[i];
        const int64_t t = epoch + (int64_t)(k >> 25);
        if (t < t_begin || t >= t_end) continue;
        const int y = (int)((k >> 13) & 0xFFF);
        const int x = (int)((k >> 1) & 0xFFF);
        const int pos = (int)(k & 1);
        counts[(pos ? 0 : 1) * plane + (size_t)y * W + x] += 1;
    }
}

/* Events per pixel and second over a window of `seconds` (the statistic of Sec. IV-C): with c the
 * per-pixel event count (both polarities) of every pixel of the sensor, the mean of c / seconds
 * and its population standard deviation over the pixels, from the exact integer sums
 * S1 = sum c and S2 = sum c^2:  m1 = S1 / npix,  m2 = S2 / npix,
 * mean = m1 / seconds,  std = sqrt(max(m2 - m1 * m1, 0)) / seconds  (double precision). */
void oracle_event_rate(const uint32_t* counts, int W, int H, double seconds, double* mean,
                       double* stddev, uint64_t* sums) {
    const size_t plane = (size_t)W * (size_t)H;
    uint64_t s1 = 0, s2 = 0;
    for (size_t p = 0; p < plane; ++p) {
        const uint64_t c = (uint64_t)counts[p] + (uint64_t)counts[plane + p];
        s1 += c;
        s2 += c * c;
    }
    const double m1 = (double)s1 / (double)plane;
    const double m2 = (double)s2 / (double)plane;
    const double var = m2 - m1 * m1;
    *mean = m1 / seconds;
    *stddev = sqrt(var > 0.0 ? var : 0.0) / seconds;
    if (sums) { sums[0] = s1; sums[1] = s2; }
}
