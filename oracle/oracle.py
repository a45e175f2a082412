"""ctypes wrapper of oracle.c (TEST INFRASTRUCTURE ONLY: tests, smoke check, CPU baseline)."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

BASIC, DENSE, SPARSE, DIFFERENCE = 0, 1, 2, 3
LOG, LINEAR = 0, 1
REFERENCE, MEMORYLESS = 0, 1
FLOW_SUPPLIED, FLOW_LK = 0, 1
LK_DEFAULTS = dict(lk_levels=3, lk_radius=7, lk_iters=10, lk_eps=1e-4, lk_min_trace=1.0,
                   lk_min_ratio=1e-3)


def build(force: bool = True) -> str:
    """Compiles oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("method", ctypes.c_int32), ("transform", ctypes.c_int32),
                ("c_pos", ctypes.c_float), ("c_neg", ctypes.c_float),
                ("log_eps", ctypes.c_float), ("n_interp", ctypes.c_int32),
                ("mask_threshold", ctypes.c_float), ("thresh_mode", ctypes.c_int32),
                ("flow_source", ctypes.c_int32), ("lk_levels", ctypes.c_int32),
                ("lk_radius", ctypes.c_int32), ("lk_iters", ctypes.c_int32),
                ("lk_eps", ctypes.c_float), ("lk_min_trace", ctypes.c_float),
                ("lk_min_ratio", ctypes.c_float)]


class _Lk(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("eps", ctypes.c_float),
                ("min_trace", ctypes.c_float), ("min_ratio", ctypes.c_float)]


_lib = None


def _bind(lib):
    P = ctypes.c_void_p
    lib.oracle_lut.argtypes = [ctypes.c_int32, ctypes.c_float, P]
    lib.oracle_create.argtypes = [ctypes.POINTER(_Cfg), ctypes.POINTER(P)]
    lib.oracle_push.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_events.argtypes = [P, P, ctypes.c_uint64]
    lib.oracle_events.restype = ctypes.c_uint64
    lib.oracle_selected.argtypes = [P]
    lib.oracle_selected.restype = ctypes.c_uint64
    lib.oracle_epoch.argtypes = [P]
    lib.oracle_epoch.restype = ctypes.c_int64
    lib.oracle_lref.argtypes = [P, P]
    lib.oracle_pixel_samples.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, P]
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_accumulate.argtypes = [P, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int, ctypes.c_int, P]
    lib.oracle_accumulate.restype = None
    lib.oracle_event_rate.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), P]
    lib.oracle_event_rate.restype = None
    lib.oracle_lk_flow.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Lk), P,
                                   ctypes.c_uint64, P, P]
    return lib


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def load_variant(path: str):
    """Binds another build of oracle.c (used by the mutation test to plant mistakes)."""
    return _bind(ctypes.CDLL(path))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def lut(transform: int = LOG, log_eps: float = 1e-3) -> np.ndarray:
    out = np.zeros(256, dtype=np.float32)
    rc = _load().oracle_lut(transform, log_eps, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_lut failed ({rc})")
    return out


class OracleSim:
    def __init__(self, width: int, height: int, method: int = BASIC, transform: int = LOG,
                 c_pos: float = 0.2, c_neg: float = 0.2, log_eps: float = 1e-3,
                 n_interp: int = 10, mask_threshold: float = -1.0, thresh_mode: int = REFERENCE,
                 flow_source: int = FLOW_SUPPLIED, **lk):
        self.width, self.height = width, height
        lkp = dict(LK_DEFAULTS)
        for k, v in lk.items():
            if k not in lkp:
                raise TypeError(f"unknown argument {k}")
            lkp[k] = v
        cfg = _Cfg(width, height, method, transform, c_pos, c_neg, log_eps, n_interp,
                   mask_threshold, thresh_mode, flow_source, lkp["lk_levels"], lkp["lk_radius"],
                   lkp["lk_iters"], lkp["lk_eps"], lkp["lk_min_trace"], lkp["lk_min_ratio"])
        h = ctypes.c_void_p()
        self._lib = _load()
        rc = self._lib.oracle_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_create failed ({rc})")
        self._h = h

    def push(self, frame: np.ndarray, flow: Optional[np.ndarray], t_us: int) -> np.ndarray:
        """Returns the interval's events as sorted packed keys (uint64)."""
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        assert frame.shape == (self.height, self.width)
        if flow is not None:
            flow = np.ascontiguousarray(flow, dtype=np.float32)
            assert flow.shape == (self.height, self.width, 2)
        n = ctypes.c_uint64()
        rc = self._lib.oracle_push(self._h, _ptr(frame), _ptr(flow), int(t_us), ctypes.byref(n))
        if rc != 0:
            raise RuntimeError(f"oracle_push failed ({rc})")
        out = np.zeros(n.value, dtype=np.uint64)
        self._lib.oracle_events(self._h, _ptr(out), n.value)
        return out

    @property
    def selected(self) -> int:
        return int(self._lib.oracle_selected(self._h))

    @property
    def epoch(self) -> int:
        return int(self._lib.oracle_epoch(self._h))

    def lref(self) -> np.ndarray:
        out = np.zeros((self.height, self.width), dtype=np.float32)
        self._lib.oracle_lref(self._h, _ptr(out))
        return out

    def pixel_samples(self, f0, f1, flow, x: int, y: int, S: int) -> np.ndarray:
        f0 = np.ascontiguousarray(f0, dtype=np.uint8)
        f1 = np.ascontiguousarray(f1, dtype=np.uint8)
        flow = np.ascontiguousarray(flow, dtype=np.float32)
        out = np.zeros(S + 1, dtype=np.float32)
        self._lib.oracle_pixel_samples(self._h, _ptr(f0), _ptr(f1), _ptr(flow), x, y, _ptr(out))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.oracle_destroy(h)
            self._h = None


def run_sequence(frames: np.ndarray, flows: Optional[np.ndarray], t_us: Sequence[int],
                 **cfg) -> List[np.ndarray]:
    """Pushes every frame; returns the per-interval sorted key arrays (len = n_frames - 1)."""
    T, H, W = frames.shape
    sim = OracleSim(W, H, **cfg)
    out = []
    for k in range(T):
        fl = None if (flows is None or k == 0) else flows[k - 1]
        ev = sim.push(frames[k], fl, int(t_us[k]))
        if k > 0:
            out.append(ev)
    return out


def accumulate(keys: np.ndarray, epoch: int, t_begin: int, t_end: int, width: int,
               height: int, counts: Optional[np.ndarray] = None) -> np.ndarray:
    """Adds the events of `keys` with t in [t_begin, t_end) to uint32 counts [2][H][W]
    (plane 0 positive, plane 1 negative); returns the counts."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    if counts is None:
        counts = np.zeros((2, height, width), dtype=np.uint32)
    assert counts.dtype == np.uint32 and counts.shape == (2, height, width)
    assert counts.flags.c_contiguous
    _load().oracle_accumulate(_ptr(keys), keys.size, int(epoch), int(t_begin), int(t_end),
                              width, height, _ptr(counts))
    return counts


def event_rate(counts: np.ndarray, t_begin: int, t_end: int):
    """Events per pixel and second over [t_begin, t_end) from accumulated counts: returns
    (mean, std, (S1, S2))."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    _, H, W = counts.shape
    mean, std = ctypes.c_double(), ctypes.c_double()
    sums = np.zeros(2, dtype=np.uint64)
    _load().oracle_event_rate(_ptr(counts), W, H, (t_end - t_begin) * 1e-6, ctypes.byref(mean),
                              ctypes.byref(std), _ptr(sums))
    return mean.value, std.value, (int(sums[0]), int(sums[1]))


def lk_flow(f0: np.ndarray, f1: np.ndarray, points=None, levels: int = 3, radius: int = 7,
            iters: int = 10, eps: float = 1e-4, min_trace: float = 1.0,
            min_ratio: float = 1e-3):
    """Pyramidal Lucas-Kanade flow from f0 to f1 (uint8 [H, W]) at pixel indices `points`
    (y * W + x; default every pixel): returns (flow float32 [n, 2], valid bool [n])."""
    f0 = np.ascontiguousarray(f0, dtype=np.uint8)
    f1 = np.ascontiguousarray(f1, dtype=np.uint8)
    H, W = f0.shape
    assert f1.shape == (H, W)
    if points is None:
        points = np.arange(H * W, dtype=np.uint32)
    points = np.ascontiguousarray(points, dtype=np.uint32)
    flow = np.zeros((points.size, 2), dtype=np.float32)
    valid = np.zeros(points.size, dtype=np.uint8)
    P = _Lk(levels, radius, iters, eps, min_trace, min_ratio)
    rc = _load().oracle_lk_flow(_ptr(f0), _ptr(f1), W, H, ctypes.byref(P), _ptr(points),
                                points.size, _ptr(flow), _ptr(valid))
    if rc != 0:
        raise ValueError(f"oracle_lk_flow failed ({rc})")
    return flow, valid.astype(bool)


def decode(keys: np.ndarray, epoch: int = 0):
    """Unpacks keys into (t, x, y, p) arrays; p in {+1, -1}."""
    keys = np.asarray(keys, dtype=np.uint64)
    t = (keys >> np.uint64(25)).astype(np.int64) + epoch
    y = ((keys >> np.uint64(13)) & np.uint64(0xFFF)).astype(np.int64)
    x = ((keys >> np.uint64(1)) & np.uint64(0xFFF)).astype(np.int64)
    p = np.where((keys & np.uint64(1)) == 1, 1, -1).astype(np.int64)
    return t, x, y, p
