"""Independent float64 pyramidal Lucas-Kanade (pins the oracle's flow estimator).

Written separately from oracle/oracle.c and sharing nothing with it: numpy, float64, the window
handled as arrays, the linear system solved with numpy.linalg.solve instead of Cramer's rule.  The
method is Lucas and Kanade's least-squares window fit, iterated, coarse to fine over a pyramid;
the conventions (binomial 1-2-1 pyramid, central-difference gradients, clamp-to-edge bilinear
sampling, window (2r+1)^2 centred on p / 2^l, guess doubled between levels, validity by texture
and conditioning of G) are those documented beside the oracle.
"""
from __future__ import annotations

import numpy as np


def _clamp_idx(i, n):
    return np.clip(i, 0, n - 1)


def pyramid(frame: np.ndarray, levels: int):
    out = [frame.astype(np.float64)]
    for _ in range(levels):
        a = out[-1]
        H, W = a.shape
        h, w = (H + 1) // 2, (W + 1) // 2
        ys = 2 * np.arange(h)[:, None]
        xs = 2 * np.arange(w)[None, :]

        def at(dy, dx):
            return a[_clamp_idx(ys + dy, H), _clamp_idx(xs + dx, W)]
        kernel = {(0, 0): 4, (0, -1): 2, (0, 1): 2, (-1, 0): 2, (1, 0): 2,
                  (-1, -1): 1, (-1, 1): 1, (1, -1): 1, (1, 1): 1}
        out.append(sum(wgt * at(dy, dx) for (dy, dx), wgt in kernel.items()) / 16.0)
    return out


def gradients(a: np.ndarray):
    H, W = a.shape
    xs = np.arange(W)
    ys = np.arange(H)
    gx = (a[:, _clamp_idx(xs + 1, W)] - a[:, _clamp_idx(xs - 1, W)]) / 2.0
    gy = (a[_clamp_idx(ys + 1, H), :] - a[_clamp_idx(ys - 1, H), :]) / 2.0
    return gx, gy


def bilinear(a: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    H, W = a.shape
    sx = np.clip(sx, 0.0, W - 1.0)
    sy = np.clip(sy, 0.0, H - 1.0)
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    fx, fy = sx - x0, sy - y0
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    return ((1 - fy) * ((1 - fx) * a[y0, x0] + fx * a[y0, x1])
            + fy * ((1 - fx) * a[y1, x0] + fx * a[y1, x1]))


def lk_point(I, J, px: int, py: int, levels: int = 3, radius: int = 7, iters: int = 10,
             eps: float = 1e-4, min_trace: float = 1.0, min_ratio: float = 1e-3):
    """Returns (flow (dx, dy), valid, margin) where margin is the smallest relative distance of
    a validity test from its threshold over the levels (small: the fp32 oracle may decide
    differently)."""
    g = np.zeros(2)
    off = np.arange(-radius, radius + 1, dtype=np.float64)
    dy, dx = np.meshgrid(off, off, indexing="ij")
    N = (2 * radius + 1) ** 2
    margin = np.inf
    for lvl in range(levels, -1, -1):
        u = np.array([px, py], dtype=np.float64) / 2.0 ** lvl
        x, y = u[0] + dx, u[1] + dy
        gxi, gyi = gradients(I[lvl])
        ix, iy = bilinear(gxi, x, y), bilinear(gyi, x, y)
        G = np.array([[np.sum(ix * ix), np.sum(ix * iy)], [np.sum(ix * iy), np.sum(iy * iy)]])
        trace, det = np.trace(G), np.linalg.det(G)
        t1 = (trace - min_trace * N) / max(trace, 1e-30)
        t2 = (det - min_ratio * trace * trace) / max(trace * trace, 1e-30)
        margin = min(margin, abs(t1), abs(t2))
        if not (trace >= min_trace * N and det >= min_ratio * trace * trace):
            return np.zeros(2), False, margin
        i0 = bilinear(I[lvl], x, y)
        v = np.zeros(2)
        for _ in range(iters):
            d = i0 - bilinear(J[lvl], x + g[0] + v[0], y + g[1] + v[1])
            step = np.linalg.solve(G, np.array([np.sum(d * ix), np.sum(d * iy)]))
            v += step
            if step @ step < eps:
                break
        if lvl > 0:
            g = 2.0 * (g + v)
        else:
            return g + v, True, margin
    raise AssertionError("unreachable")


def lk_flow(f0: np.ndarray, f1: np.ndarray, points, **params):
    levels = params.get("levels", 3)
    I, J = pyramid(f0, levels), pyramid(f1, levels)
    W = f0.shape[1]
    out = []
    for p in points:
        out.append(lk_point(I, J, int(p) % W, int(p) // W, **params))
    return out
