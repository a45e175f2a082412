"""Independent float64 brute-force event solver for tiny images (pins the oracle).

Written separately from oracle/oracle.c and sharing nothing with it.  It differs from the oracle in
how it computes, not in what it computes:

  * every quantity is float64 (the table, the samples, the reference level);
  * crossings of a sub-interval are solved in closed form: the n-th crossing level is R0 + n*C
    (not n repeated fp32 additions), the count is floor(|B - R0| / C);
  * each decision records its margin, so pixels where float64 and fp32 could legitimately
    disagree (a level within `tie_tol` of a sample) are reported as near-ties and excluded.

Model (paper Sec. I event pixel, Sec. III difference frames + interpolation, Sec. III-A
thresholds, Sec. III-B sparse selection), with the readings documented beside the oracle:
sub-interval samples at tau = k/S of a flow-guided bidirectional blend of the transformed frames;
a sub-interval [A, B] fires while B is at least C_pos above (or C_neg below) the reference level;
each crossing's time is linear in the sub-interval (0 if the level was already passed at A).
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np


def table64(transform: str, eps: float) -> np.ndarray:
    v = np.arange(256, dtype=np.float64)
    if transform == "log":
        return np.log(v / 255.0 + float(np.float32(eps)))
    return v


def _bilinear64(L: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    H, W = L.shape
    sx = np.clip(sx, 0.0, W - 1.0)
    sy = np.clip(sy, 0.0, H - 1.0)
    ix = np.floor(sx).astype(np.int64)
    iy = np.floor(sy).astype(np.int64)
    wx = sx - ix
    wy = sy - iy
    jx = np.minimum(ix + 1, W - 1)
    jy = np.minimum(iy + 1, H - 1)
    return ((1 - wy) * ((1 - wx) * L[iy, ix] + wx * L[iy, jx])
            + wy * ((1 - wx) * L[jy, ix] + wx * L[jy, jx]))


def samples64(L0: np.ndarray, L1: np.ndarray, flow: np.ndarray, S: int) -> np.ndarray:
    """[S+1, H, W] samples of every pixel's interpolated series."""
    H, W = L0.shape
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    out = np.empty((S + 1, H, W))
    out[0], out[S] = L0, L1
    if S > 1:
        u = flow[..., 0].astype(np.float64)
        v = flow[..., 1].astype(np.float64)
        for k in range(1, S):
            tau = k / S
            a = _bilinear64(L0, xs - tau * u, ys - tau * v)
            b = _bilinear64(L1, xs + (1 - tau) * u, ys + (1 - tau) * v)
            out[k] = (1 - tau) * a + tau * b
    return out


def solve_sequence(frames: np.ndarray, flows, t_us, method: str, transform: str = "log",
                   c_pos: float = 0.2, c_neg: float = 0.2, eps: float = 1e-3, n_interp: int = 10,
                   mask: float = -1.0, tie_tol: float = 3e-5, t_tol: float = 0.25):
    """Returns (events, near_tie) where events is a list (per interval) of dicts
    {(x, y): [(t, p, t_exact), ...]} and near_tie is a bool [H, W] mask of pixels to exclude.

    A pixel is a near-tie when some decision is within `tie_tol` (relative to the magnitude of
    the values compared) of flipping.  An event's time is flagged inexact (t_exact False) when
    its crossing time is ill-conditioned: the fp32 error of the level and samples, a few ulps per
    operation on the way, divided by the rise |B - A| of its sub-interval and scaled to
    microseconds, exceeds `t_tol`; counts and polarities are still compared for it."""
    T, H, W = frames.shape
    lut = table64(transform, eps)
    cp, cn = float(np.float32(c_pos)), float(np.float32(c_neg))
    m = min(cp, cn) if mask < 0 else float(np.float32(mask))
    S = 1 if method == "basic" else n_interp + 1
    R = lut[frames[0]].copy()
    near = np.zeros((H, W), dtype=bool)
    out: List[Dict[Tuple[int, int], List[Tuple[int, int]]]] = []
    for i in range(1, T):
        L0, L1 = lut[frames[i - 1]], lut[frames[i]]
        t0, t1 = int(t_us[i - 1]), int(t_us[i])
        delta = float(t1 - t0)
        V = samples64(L0, L1, flows[i - 1] if S > 1 else None, S) if S > 1 else np.stack([L0, L1])
        ev: Dict[Tuple[int, int], List[Tuple[int, int]]] = {}
        for y in range(H):
            for x in range(W):
                if method == "sparse":
                    d = abs(L1[y, x] - L0[y, x])
                    if abs(d - m) < tie_tol:
                        near[y, x] = True
                    if not d >= m:
                        continue
                r0 = R[y, x]
                lst = []
                nsteps = 0
                for k in range(S):
                    A, B = V[k, y, x], V[k + 1, y, x]
                    up = B - r0
                    if up >= cp:
                        n, pol, step = math.floor(up / cp), 1, cp
                    elif up <= -cn:
                        n, pol, step = math.floor(-up / cn), -1, -cn
                    else:
                        n, pol, step = 0, 0, 0.0
                    # near-tie: the end sample within tie_tol of a level (count could differ)
                    scale = max(1.0, abs(A), abs(B), abs(r0))
                    for c in (cp, cn):
                        q = abs(up) / c
                        if abs(q - round(q)) * c < tie_tol * scale and round(q) >= 1:
                            near[y, x] = True
                    for j in range(1, n + 1):
                        level = r0 + j * step
                        exact = True
                        if (pol > 0 and A >= level) or (pol < 0 and A <= level):
                            theta = 0.0
                            if abs(A - level) < tie_tol * scale:
                                near[y, x] = True
                        else:
                            D = B - A
                            ulp_err = (nsteps + j + 8) * scale * 2.0 ** -23
                            if D == 0 or delta / S * ulp_err / abs(D) > t_tol:
                                exact = False
                            theta = 0.0 if D == 0 else min(max((level - A) / D, 0.0), 1.0)
                        ph = (k + theta) / S * delta
                        lst.append((t0 + math.floor(ph), pol, exact))
                    r0 = r0 + n * step
                    nsteps += n
                R[y, x] = r0
                if lst:
                    ev[(x, y)] = lst
        out.append(ev)
    return out, near


def _time_on_grid(t0: int, j: int, S: int, delta: float, t_tol: float = 0.25):
    """t0 + floor(j/S * delta) exactly (rational arithmetic), and whether an fp32 evaluation of
    the product could land on the other side of an integer."""
    num = j * int(delta)
    q, r = divmod(num, S)
    frac = r / S
    exact = min(frac, 1.0 - frac) > max(delta, 1.0) * 2.0 ** -22
    return t0 + q, exact


def _difference_samples64(Dprev: np.ndarray, Dcur: np.ndarray, flow: np.ndarray,
                          S: int) -> np.ndarray:
    """[S+1, H, W]: the difference frames interpolated at tau = k/S, index 0 = Dprev, S = Dcur."""
    return samples64(Dprev, Dcur, flow, S)


def solve_memoryless_sequence(frames: np.ndarray, flows, t_us, method: str,
                              transform: str = "log", c_pos: float = 0.2, c_neg: float = 0.2,
                              eps: float = 1e-3, n_interp: int = 10, mask: float = -1.0,
                              tie_tol: float = 3e-5):
    """Memoryless thresholding (Sec. III-A equations taken literally) in float64: for the frame
    methods every difference of consecutive samples V_{k+1} - V_k, for the difference method
    (Sec. III-C) every interpolated difference frame D_k (k = 1..S), fires once if it is above
    C_pos (positive) or below -C_neg (negative), stamped at the later sample's time.  Returns
    (events, near_tie) like solve_sequence; a pixel is a near-tie when a compared value is within
    tie_tol (relative) of a threshold or, for the sparse method, of the selection threshold."""
    T, H, W = frames.shape
    lut = table64(transform, eps)
    cp, cn = float(np.float32(c_pos)), float(np.float32(c_neg))
    m = min(cp, cn) if mask < 0 else float(np.float32(mask))
    S = 1 if method == "basic" else n_interp + 1
    near = np.zeros((H, W), dtype=bool)
    out = []
    for i in range(1, T):
        L0, L1 = lut[frames[i - 1]], lut[frames[i]]
        t0, t1 = int(t_us[i - 1]), int(t_us[i])
        delta = float(t1 - t0)
        ev = {}
        if method == "difference":
            if i == 1:
                out.append(ev)
                continue
            Dprev = L0 - lut[frames[i - 2]]
            Dcur = L1 - L0
            V = _difference_samples64(Dprev, Dcur, flows[i - 1], S)
            values = V[1:]                                     # D_1 .. D_S
        else:
            V = samples64(L0, L1, flows[i - 1], S) if S > 1 else np.stack([L0, L1])
            values = V[1:] - V[:-1]                             # V_{k+1} - V_k, k = 0..S-1
        for y in range(H):
            for x in range(W):
                if method == "sparse":
                    d = abs(L1[y, x] - L0[y, x])
                    if abs(d - m) < tie_tol * max(1.0, abs(L0[y, x]), abs(L1[y, x])):
                        near[y, x] = True
                    if not d >= m:
                        continue
                lst = []
                for k in range(S):
                    D = values[k, y, x]
                    if method == "difference":
                        scale = max(1.0, float(np.max(np.abs(V[:, y, x]))),
                                    abs(L0[y, x]), abs(L1[y, x]))
                    else:
                        scale = max(1.0, abs(V[k, y, x]), abs(V[k + 1, y, x]))
                    if abs(D - cp) < tie_tol * scale or abs(D + cn) < tie_tol * scale:
                        near[y, x] = True
                    pol = 1 if D > cp else (-1 if D < -cn else 0)
                    if pol:
                        t, exact = _time_on_grid(t0, k + 1, S, delta)
                        lst.append((t, pol, exact))
                if lst:
                    ev[(x, y)] = lst
        out.append(ev)
    return out, near
