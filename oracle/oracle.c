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
 *   - Output: events <x, y, t, p> (Sec. III-A, Fig. 1 caption).
 *
 * Readings where the paper is silent:
 *   log transform ln(v/255 + eps) via a 256-entry table; interpolation of the transformed frames;
 *   S = N + 1 sub-intervals for N interpolated frames; gather-form bidirectional flow-guided blend
 *   with clamp-to-edge bilinear sampling; threshold crossing against a per-pixel reference level
 *   with ties counted (>= C_pos, <= -C_neg); crossing times linear within a sub-interval, floored
 *   to integer microseconds; backlog crossings stamped at the sub-interval start; sparse selection
 *   |L1 - L0| >= m; first frame initialises state only; canonical order by (t, y, x, p) per
 *   interval, intervals in push order.
 *
 * Parity is pinned (tests/test_oracle_*.py) by: the exhaustive table check against an exact
 * logarithm, zero-event invariants, the closed-form per-pixel count floor(|dL|/C) of the basic
 * method, endpoint exactness (dense with S = 1 equals basic), zero-flow and translating-edge
 * closed forms, time reversal, reference bookkeeping, hand-worked fixtures under tests/golden/ and
 * an independent float64 brute-force solver on 8x8 inputs.  The exact interpolation formula has
 * no anchor in the paper beyond those properties ("parity unpinned" against the paper itself for
 * that formula; pinned through endpoint exactness, the zero-flow and translating-edge closed forms
 * and the brute-force solver).
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

enum { OR_BASIC = 0, OR_DENSE = 1, OR_SPARSE = 2 };
enum { OR_LOG = 0, OR_LINEAR = 1 };

typedef struct {
    int32_t width, height;
    int32_t method, transform;
    float c_pos, c_neg;      /* magnitudes, > 0 */
    float log_eps;
    int32_t n_interp;        /* N interpolated frames; S = N + 1 (basic: S = 1) */
    float mask_threshold;    /* sparse: < 0 -> min(c_pos, c_neg) */
} oracle_cfg;

typedef struct {
    oracle_cfg cfg;
    int S;
    float m;                 /* sparse selection threshold */
    float lut[256];
    uint8_t* prev;           /* previous camera frame */
    float* lref;             /* per-pixel reference level */
    float* L0;               /* scratch: transformed previous frame */
    float* L1;               /* scratch: transformed current frame */
    float* V;                /* scratch: S + 1 samples of one pixel */
    int started;
    int64_t t_prev, epoch;
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

static void or_destroy(oracle_sim* s) {
    if (!s) return;
    free(s->prev); free(s->lref); free(s->L0); free(s->L1); free(s->V); free(s->ev);
    free(s);
}

void oracle_destroy(oracle_sim* s) { or_destroy(s); }

int oracle_create(const oracle_cfg* cfg, oracle_sim** out) {
    if (!cfg || !out) return OR_E_INVAL;
    *out = NULL;
    if (cfg->width < 1 || cfg->height < 1 || cfg->width > 4096 || cfg->height > 4096)
        return OR_E_INVAL;
    if (cfg->method < OR_BASIC || cfg->method > OR_SPARSE) return OR_E_INVAL;
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
    s->lref = (float*)malloc(n * sizeof(float));
    s->L0 = (float*)malloc(n * sizeof(float));
    s->L1 = (float*)malloc(n * sizeof(float));
    s->V = (float*)malloc((size_t)(s->S + 1) * sizeof(float));
    if (!s->prev || !s->lref || !s->L0 || !s->L1 || !s->V) { or_destroy(s); return OR_E_NOMEM; }
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
    if (s->cfg.method != OR_BASIC && !flow) return OR_E_INVAL;

    const int64_t t0 = s->t_prev;
    const float delta = (float)(t_us - t0);
    const float cp = s->cfg.c_pos, cn = s->cfg.c_neg;
    for (size_t i = 0; i < n; ++i) {
        s->L0[i] = s->lut[s->prev[i]];
        s->L1[i] = s->lut[frame[i]];
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
    memcpy(s->prev, frame, n);
    s->t_prev = t_us;
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
