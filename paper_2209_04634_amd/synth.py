"""Seeded synthetic video for the event simulator: Gaussian-blob texture plus analytic flow.

The paper evaluates on a driving sequence (640x480, high event rate) and on a table-tennis
recording in front of a static background (1280x720, low event rate) (Sec. IV-A). Neither is
available here, so this module draws seeded stand-ins with the same resolutions, frame rates and
high- versus low-dynamics structure.

This module holds none of the simulator's arithmetic: it only produces uint8 frames, fp32 flow
fields and integer microsecond timestamps. Both the CPU oracle and the HIP library consume the very
same bytes.

Frame model (evaluated in float64, stored as uint8):

    I_k(x, y) = clip(rint(20 + sum_b A_b * exp(-|p - c_b - k v_b|^2 / (2 sigma_b^2))), 0, 255)

with sigma ~ U[4, 20] px, A ~ U[40, 200], centres uniform over the image. Each blob is evaluated
inside a square window of half-width ceil(5 sigma) around its centre; outside it, it contributes
nothing (its true value there is below 7.5e-4 intensity levels).

Flow for the interval from frame k to frame k+1, per pixel p: the blob velocities averaged with
weights w_b = A_b * exp(-|p - c_b(k + 1/2)|^2 / (2 sigma_b^2)) taken at the mid-interval blob
positions, over the same windows; 0 where no window covers p. Channel 0 is dx, channel 1 is dy,
both in pixels per camera interval.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

FLOOR = 20.0
WINDOW_SIGMAS = 5.0


@dataclasses.dataclass(frozen=True)
class BlobVideoSpec:
    width: int
    height: int
    n_frames: int
    fps: float
    n_blobs: int
    seed: int
    # "translate": every blob moves by `velocity` px/frame.
    # "random": every blob gets speed U[0, speed_max] px/frame at a uniform random angle.
    # "sparse": blobs get random velocities as in "random", but only a leading subset moves:
    #           blobs are switched to moving, in draw order, until the union of their 2-sigma
    #           discs covers at least `moving_cover` of the image; the rest are static.
    motion: str = "random"
    velocity: Tuple[float, float] = (3.0, 0.0)
    speed_max: float = 12.0
    moving_cover: float = 0.10


@dataclasses.dataclass
class BlobVideo:
    spec: BlobVideoSpec
    frames: np.ndarray      # uint8 [T, H, W]
    flows: np.ndarray       # float32 [T-1, H, W, 2]  (flow for interval k -> k+1)
    t_us: np.ndarray        # int64 [T]
    moving: np.ndarray      # bool [n_blobs]


def frame_times_us(n_frames: int, fps: float) -> np.ndarray:
    """t_k = round(k * 1e6 / fps) microseconds."""
    return np.array([int(round(k * 1e6 / fps)) for k in range(n_frames)], dtype=np.int64)


def _draw_blobs(spec: BlobVideoSpec):
    rng = np.random.default_rng(spec.seed)
    n = spec.n_blobs
    sigma = rng.uniform(4.0, 20.0, n)
    amp = rng.uniform(40.0, 200.0, n)
    cx = rng.uniform(0.0, spec.width, n)
    cy = rng.uniform(0.0, spec.height, n)
    if spec.motion == "translate":
        vx = np.full(n, float(spec.velocity[0]))
        vy = np.full(n, float(spec.velocity[1]))
        moving = np.ones(n, dtype=bool)
    elif spec.motion in ("random", "sparse"):
        speed = rng.uniform(0.0, spec.speed_max, n)
        angle = rng.uniform(0.0, 2.0 * math.pi, n)
        vx = speed * np.cos(angle)
        vy = speed * np.sin(angle)
        moving = np.ones(n, dtype=bool)
        if spec.motion == "sparse":
            moving[:] = False
            yy, xx = np.mgrid[0:spec.height, 0:spec.width]
            covered = np.zeros((spec.height, spec.width), dtype=bool)
            target = spec.moving_cover * spec.width * spec.height
            for b in range(n):
                moving[b] = True
                covered |= (xx - cx[b]) ** 2 + (yy - cy[b]) ** 2 <= (2.0 * sigma[b]) ** 2
                if covered.sum() >= target:
                    break
            vx = np.where(moving, vx, 0.0)
            vy = np.where(moving, vy, 0.0)
    else:
        raise ValueError(f"unknown motion {spec.motion!r}")
    return sigma, amp, cx, cy, vx, vy, moving


def _window(c: float, r: int, n: int):
    lo = max(int(math.floor(c)) - r, 0)
    hi = min(int(math.floor(c)) + r + 1, n)
    return lo, hi


def _splat(acc: np.ndarray, cx: float, cy: float, sigma: float, scale: float,
           acc_wv: Optional[Tuple[np.ndarray, np.ndarray, float, float]] = None) -> None:
    """Adds scale * gaussian(sigma) centred at (cx, cy) into acc over the blob's window."""
    h, w = acc.shape
    r = int(math.ceil(WINDOW_SIGMAS * sigma))
    x0, x1 = _window(cx, r, w)
    y0, y1 = _window(cy, r, h)
    if x0 >= x1 or y0 >= y1:
        return
    dx2 = (np.arange(x0, x1, dtype=np.float64) - cx) ** 2
    dy2 = (np.arange(y0, y1, dtype=np.float64) - cy) ** 2
    g = scale * np.exp(-(dy2[:, None] + dx2[None, :]) / (2.0 * sigma * sigma))
    acc[y0:y1, x0:x1] += g
    if acc_wv is not None:
        ax, ay, vx, vy = acc_wv
        if vx != 0.0:
            ax[y0:y1, x0:x1] += g * vx
        if vy != 0.0:
            ay[y0:y1, x0:x1] += g * vy


def blob_video(spec: BlobVideoSpec, with_flow: bool = True) -> BlobVideo:
    sigma, amp, cx, cy, vx, vy, moving = _draw_blobs(spec)
    h, w, T = spec.height, spec.width, spec.n_frames
    frames = np.empty((T, h, w), dtype=np.uint8)
    static = np.full((h, w), FLOOR, dtype=np.float64)
    for b in np.nonzero(~moving)[0]:
        _splat(static, cx[b], cy[b], sigma[b], amp[b])
    mov = np.nonzero(moving)[0]
    for k in range(T):
        acc = static.copy()
        for b in mov:
            _splat(acc, cx[b] + k * vx[b], cy[b] + k * vy[b], sigma[b], amp[b])
        frames[k] = np.clip(np.rint(acc), 0, 255).astype(np.uint8)
    flows = np.zeros((max(T - 1, 0), h, w, 2), dtype=np.float32)
    if with_flow and T > 1:
        wsum_static = np.zeros((h, w), dtype=np.float64)
        for b in np.nonzero(~moving)[0]:
            _splat(wsum_static, cx[b], cy[b], sigma[b], amp[b])
        for k in range(T - 1):
            wsum = wsum_static.copy()
            ax = np.zeros((h, w), dtype=np.float64)
            ay = np.zeros((h, w), dtype=np.float64)
            tm = k + 0.5
            for b in mov:
                _splat(wsum, cx[b] + tm * vx[b], cy[b] + tm * vy[b], sigma[b], amp[b],
                       (ax, ay, vx[b], vy[b]))
            nz = wsum > 0.0
            fx = np.zeros((h, w), dtype=np.float64)
            fy = np.zeros((h, w), dtype=np.float64)
            fx[nz] = ax[nz] / wsum[nz]
            fy[nz] = ay[nz] / wsum[nz]
            flows[k, :, :, 0] = fx
            flows[k, :, :, 1] = fy
    return BlobVideo(spec=spec, frames=frames, flows=flows,
                     t_us=frame_times_us(T, spec.fps), moving=moving)


# ---- the workloads: shapes, rates and thresholds of the paper's two runtime scenarios ----------

def basic_240x180(seed: int = 1) -> BlobVideoSpec:
    """240x180, 2 frames at 30 fps, 32 blobs translating +3 px/frame (basic method, C = 0.2)."""
    return BlobVideoSpec(240, 180, 2, 30.0, 32, seed, motion="translate", velocity=(3.0, 0.0))


def dense_346x260(seed: int = 2, n_frames: int = 60) -> BlobVideoSpec:
    """346x260, 60 frames at 30 fps, 32 blobs with speed U[0,12] px/frame (dense, C = 0.15)."""
    return BlobVideoSpec(346, 260, n_frames, 30.0, 32, seed, motion="random", speed_max=12.0)


def sparse_1280x720(seed: int = 3, n_frames: int = 120) -> BlobVideoSpec:
    """1280x720, 120 frames at 60 fps, 256 blobs, >= 10% of the image moving at U[0,24] px/frame
    over a static background (sparse, C = 0.2)."""
    return BlobVideoSpec(1280, 720, n_frames, 60.0, 256, seed, motion="sparse",
                         speed_max=24.0, moving_cover=0.10)


def scaled_blob_count(width: int, height: int) -> int:
    """32 blobs per 240x180 worth of area, capped at 512."""
    return int(min(512, max(1, round(32 * width * height / 43200.0))))


def mixed_stream(width: int, height: int, seed: int, n_frames: int = 30) -> BlobVideoSpec:
    """One stream of the mixed-resolution batch: the 346x260 recipe with area-scaled blob count."""
    return BlobVideoSpec(width, height, n_frames, 30.0, scaled_blob_count(width, height), seed,
                         motion="random", speed_max=12.0)


def serving_stream(width: int, height: int, seed: int, n_frames: int = 64) -> BlobVideoSpec:
    """A serving camera's pool: the sparse 1280x720 recipe (moving subset covering >= 10% of the
    image at U[0,24] px/frame over a static background) with the blob count scaled by area."""
    blobs = int(max(8, round(256 * width * height / 921600.0)))
    return BlobVideoSpec(width, height, n_frames, 60.0, blobs, seed, motion="sparse",
                         speed_max=24.0, moving_cover=0.10)


def random_frames(rng: np.random.Generator, n: int, h: int, w: int,
                  flow_scale: float = 2.0) -> Tuple[np.ndarray, np.ndarray]:
    """Unstructured uint8 frames and fp32 flows for brute-force and edge-case testing."""
    frames = rng.integers(0, 256, size=(n, h, w), dtype=np.uint8)
    flows = (rng.standard_normal((max(n - 1, 0), h, w, 2)) * flow_scale).astype(np.float32)
    return frames, flows
