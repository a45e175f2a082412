"""ctypes binding of libevsim.so (include/sim.h): argument marshalling only.

Every step of the simulation runs in the HIP library.  numpy arrays are passed as host memory,
torch tensors on a GPU as device memory.  There is no fallback: if the library is missing the
import fails with an error that says how to build it.
"""
from __future__ import annotations

import collections
import ctypes
import os
from typing import Optional, Sequence, Union

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libevsim.so")

BASIC, DENSE, SPARSE, DIFFERENCE = 0, 1, 2, 3
LOG, LINEAR = 0, 1
REFERENCE, MEMORYLESS = 0, 1
FLOW_SUPPLIED, FLOW_LK = 0, 1
MEM_HOST, MEM_DEVICE, MEM_HOST_FRAME = 0, 1, 2
METHODS = {"basic": BASIC, "dense": DENSE, "sparse": SPARSE, "difference": DIFFERENCE}
TRANSFORMS = {"log": LOG, "linear": LINEAR}
THRESH_MODES = {"reference": REFERENCE, "memoryless": MEMORYLESS}
FLOW_SOURCES = {"supplied": FLOW_SUPPLIED, "lk": FLOW_LK}

OK, E_INVAL, E_ORDER, E_NOMEM, E_RANGE, E_HIP, E_POISONED, E_BUSY, E_EMPTY = 0, -1, -2, -3, -4, -5, -6, -7, -8
E_TOO_BIG = -9


class SimConfig(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("method", ctypes.c_int32), ("transform", ctypes.c_int32),
                ("c_pos", ctypes.c_float), ("c_neg", ctypes.c_float),
                ("log_eps", ctypes.c_float), ("n_interp", ctypes.c_int32),
                ("mask_threshold", ctypes.c_float), ("event_capacity", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p), ("thresh_mode", ctypes.c_int32),
                ("flow_source", ctypes.c_int32)]


class SimLkParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("eps", ctypes.c_float),
                ("min_trace", ctypes.c_float), ("min_ratio", ctypes.c_float)]


class SimEvent(ctypes.Structure):
    _fields_ = [("t_us", ctypes.c_int64), ("x", ctypes.c_uint16), ("y", ctypes.c_uint16),
                ("p", ctypes.c_int8), ("pad", ctypes.c_uint8 * 3)]


class SimStats(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_uint64), ("intervals", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("selected", ctypes.c_uint64),
                ("active", ctypes.c_uint64),
                ("retries", ctypes.c_uint64), ("event_capacity", ctypes.c_uint64),
                ("select_launches", ctypes.c_uint64), ("select_ms", ctypes.c_double),
                ("simulate_launches", ctypes.c_uint64), ("simulate_ms", ctypes.c_double),
                ("sort_launches", ctypes.c_uint64), ("sort_ms", ctypes.c_double)]


class SimFrames(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("mem_kind", ctypes.c_int32),
                ("frames", ctypes.c_void_p), ("flows", ctypes.c_void_p),
                ("t_us", ctypes.c_void_p), ("n_new_events", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "cameras", "admissions", "rejected_admissions", "submitted", "rejected_frames",
        "completed", "failed_frames", "steps", "events", "hbm_used", "hbm_budget")] + \
        [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "max_ms", "busy_ms",
                                         "lock_wait_ms")]


class SimBatchTiming(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_uint64)] + [(n, ctypes.c_double) for n in (
        "inputs_ms", "plan_ms", "launch_ms", "wait_ms", "finish_ms", "device_ms")]


EVENT_DTYPE = np.dtype([("t", "<i8"), ("x", "<u2"), ("y", "<u2"), ("p", "i1"), ("pad", "u1", 3)])
assert EVENT_DTYPE.itemsize == ctypes.sizeof(SimEvent) == 16

_lib = None


def load() -> ctypes.CDLL:
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2209_04634_amd.build` "
                          "(or __graft_entry__.build()) first")
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Loading torch
    # first makes the library bind to that runtime, so the process has one HIP runtime and
    # torch tensors, streams and this library share devices and memory.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    PU64 = ctypes.POINTER(ctypes.c_uint64)
    sigs = {
        "sim_config_init": (None, [ctypes.POINTER(SimConfig)]),
        "sim_create": (ctypes.c_int, [ctypes.POINTER(SimConfig), ctypes.POINTER(P)]),
        "sim_destroy": (ctypes.c_int, [P]),
        "sim_reset": (ctypes.c_int, [P]),
        "sim_push_frame": (ctypes.c_int, [P, P, P, I64, I32, PU64]),
        "sim_push_frames": (ctypes.c_int, [P, I32, P, P, P, I32, PU64]),
        "sim_pending_events": (ctypes.c_int, [P, PU64]),
        "sim_drain_events": (ctypes.c_int, [P, P, U64, PU64]),
        "sim_drain_keys": (ctypes.c_int, [P, P, U64, I32, PU64]),
        "sim_epoch": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64)]),
        "sim_get_reference": (ctypes.c_int, [P, P, I32]),
        "sim_sync": (ctypes.c_int, [P]),
        "sim_get_stats": (ctypes.c_int, [P, ctypes.POINTER(SimStats)]),
        "sim_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sim_set_kernel_timing": (ctypes.c_int, [P, I32]),
        "sim_clear_stats": (ctypes.c_int, [P]),
        "sim_last_error": (ctypes.c_char_p, [P]),
        "sim_push_batch": (ctypes.c_int, [ctypes.POINTER(P), ctypes.POINTER(SimFrames), I32]),
        "sim_batch_stats": (ctypes.c_int, [PU64, PU64, PU64]),
        "sim_batch_times": (ctypes.c_int, [P]),
        "sim_set_chain_variant": (ctypes.c_int, [P, I32]),
        "sim_get_chain_variant": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int32)]),
        "srv_footprint": (ctypes.c_int, [ctypes.POINTER(SimConfig), I32, PU64]),
        "srv_create": (ctypes.c_int, [U64, I32, I32, ctypes.POINTER(P)]),
        "srv_destroy": (ctypes.c_int, [P]),
        "srv_admit": (ctypes.c_int, [P, ctypes.POINTER(SimConfig), ctypes.POINTER(I32)]),
        "srv_release": (ctypes.c_int, [P, I32]),
        "srv_submit": (ctypes.c_int, [P, I32, P, P, I64, I32, I64]),
        "srv_step": (ctypes.c_int, [P, PU64]),
        "srv_start": (ctypes.c_int, [P]),
        "srv_stop": (ctypes.c_int, [P]),
        "srv_sync": (ctypes.c_int, [P]),
        "srv_pending": (ctypes.c_int, [P, I32, PU64]),
        "srv_drain": (ctypes.c_int, [P, I32, P, U64, I32, PU64]),
        "srv_stream": (ctypes.c_int, [P, I32, ctypes.POINTER(P)]),
        "srv_get_stats": (ctypes.c_int, [P, ctypes.POINTER(ServerStats)]),
        "srv_clear_stats": (ctypes.c_int, [P]),
        "srv_now_ns": (I64, []),
        "sim_lk_params_init": (None, [ctypes.POINTER(SimLkParams)]),
        "sim_set_lk_params": (ctypes.c_int, [P, ctypes.POINTER(SimLkParams)]),
        "sim_lk_flow": (ctypes.c_int, [P, P, I32, I32, P, U64, P, P,
                                       ctypes.POINTER(SimLkParams), I32, P]),
        "sim_lk_flow_noalloc": (ctypes.c_int, [P, P, I32, I32, P, U64, P, P,
                                               ctypes.POINTER(SimLkParams), P]),
        "sim_accumulate": (ctypes.c_int, [P, I64, I64, P, I32]),
        "sim_event_rate": (ctypes.c_int, [P, I64, I64, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), PU64]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SimError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().sim_strerror(status).decode()
        super().__init__(f"{where}: {msg} ({status})")


def _check(rc: int, where: str, handle=None) -> None:
    if rc != OK:
        if handle is not None and rc in (E_HIP, E_POISONED):
            detail = load().sim_last_error(handle).decode()
            if detail:
                where = f"{where} [{detail}]"
        raise SimError(rc, where)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _buffer(x, dtype, shape=None):
    """(pointer, mem_kind, keepalive) of a numpy array or a torch tensor."""
    if x is None:
        return None, None, None
    if _is_torch(x):
        import torch
        # uint32 buffers travel as int32 tensors (same bits)
        want = {np.uint8: torch.uint8, np.float32: torch.float32, np.int64: torch.int64,
                np.uint32: torch.int32}[dtype]
        if x.dtype != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if shape is not None and tuple(x.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(x.shape)}")
        kind = MEM_DEVICE if x.is_cuda else MEM_HOST
        return ctypes.c_void_p(x.data_ptr()), kind, x
    a = np.ascontiguousarray(x, dtype=dtype)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a.ctypes.data_as(ctypes.c_void_p), MEM_HOST, a


def _out_buffer(x, dtype, shape=None, also=()):
    """(pointer, mem_kind, keepalive) of a caller's output array or tensor, written in place: a
    numpy array must already have the dtype (or one of `also`), be C-contiguous and writeable,
    since a converted copy would receive the results instead."""
    if _is_torch(x):
        return _buffer(x, dtype, shape)
    ok = tuple(np.dtype(d) for d in (dtype,) + tuple(also))
    if not isinstance(x, np.ndarray) or x.dtype not in ok:
        raise TypeError(f"expected a numpy array of {' or '.join(str(d) for d in ok)}")
    if not x.flags.c_contiguous or not x.flags.writeable:
        raise TypeError("output array must be C-contiguous and writeable")
    if shape is not None and x.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {x.shape}")
    return x.ctypes.data_as(ctypes.c_void_p), MEM_HOST, x


def lk_params(levels: int = 3, radius: int = 7, iterations: int = 10, eps: float = 1e-4,
              min_trace: float = 1.0, min_ratio: float = 1e-3) -> SimLkParams:
    p = SimLkParams()
    load().sim_lk_params_init(ctypes.byref(p))
    p.levels, p.radius, p.iterations = int(levels), int(radius), int(iterations)
    p.eps, p.min_trace, p.min_ratio = float(eps), float(min_trace), float(min_ratio)
    return p


def batch_stats() -> dict:
    """sim_batch_stats: graphs recorded, graph launches and re-run windows of batched pushes."""
    lib = load()
    g, l, r = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.sim_batch_stats(ctypes.byref(g), ctypes.byref(l), ctypes.byref(r)),
           "sim_batch_stats")
    return {"graphs_recorded": g.value, "graph_launches": l.value, "rerun_windows": r.value}


def batch_times() -> dict:
    """sim_batch_times: accumulated host phases and device time of the batched pushes' chunks."""
    t = SimBatchTiming()
    _check(load().sim_batch_times(ctypes.byref(t)), "sim_batch_times")
    return {k: getattr(t, k) for k, _ in SimBatchTiming._fields_}


def lk_flow(f0, f1, points=None, hip_stream=None, **params):
    """Pyramidal Lucas-Kanade flow from f0 to f1 (uint8 [H, W], numpy or torch device tensors)
    at pixel indices `points` (y * W + x; default every pixel).  Returns (flow [n, 2] float32,
    valid [n] bool) as numpy arrays for host inputs, torch tensors for device inputs."""
    lib = load()
    H, W = int(f0.shape[0]), int(f0.shape[1])
    a, ka, keep_a = _buffer(f0, np.uint8, (H, W))
    b, kb, keep_b = _buffer(f1, np.uint8, (H, W))
    if ka != kb:
        raise ValueError("f0 and f1 must both be host or both be device memory")
    if ka == MEM_DEVICE:
        import torch
        if points is None:
            points = torch.arange(H * W, dtype=torch.int32, device=f0.device)
        n = int(points.numel())
        flow = torch.zeros((n, 2), dtype=torch.float32, device=f0.device)
        valid = torch.zeros(n, dtype=torch.uint8, device=f0.device)
        pp, pk, keep_p = _buffer(points, np.uint32, (n,))
        if pk != MEM_DEVICE:
            raise ValueError("points must be a device tensor when the frames are")
        fp = ctypes.c_void_p(flow.data_ptr())
        vp = ctypes.c_void_p(valid.data_ptr())
    else:
        if points is None:
            points = np.arange(H * W, dtype=np.uint32)
        pts = np.ascontiguousarray(points, dtype=np.uint32)
        n = pts.size
        flow = np.zeros((n, 2), dtype=np.float32)
        valid = np.zeros(n, dtype=np.uint8)
        pp, keep_p = pts.ctypes.data_as(ctypes.c_void_p), pts
        fp, vp = flow.ctypes.data_as(ctypes.c_void_p), valid.ctypes.data_as(ctypes.c_void_p)
    if hip_stream is not None and hasattr(hip_stream, "cuda_stream"):
        hip_stream = hip_stream.cuda_stream
    st = ctypes.c_void_p(int(hip_stream)) if hip_stream else None
    _check(lib.sim_lk_flow(a, b, W, H, pp, n, fp, vp, ctypes.byref(lk_params(**params)), ka, st),
           "sim_lk_flow")
    return flow, (valid != 0)


def lk_flow_noalloc(f0, f1, points, flow, valid=None, hip_stream=None, **params):
    """sim_lk_flow_noalloc: Lucas-Kanade flow into caller-allocated device tensors `flow`
    ([n, 2] float32) and `valid` ([n] uint8 or None), with no allocation in the library.  The
    work is queued on hip_stream (a torch stream, its handle, or None: the null stream) and not
    waited for."""
    lib = load()
    H, W = int(f0.shape[0]), int(f0.shape[1])
    a, ka, _ = _buffer(f0, np.uint8, (H, W))
    b, kb, _ = _buffer(f1, np.uint8, (H, W))
    n = int(points.numel())
    pp, pk, _ = _buffer(points, np.uint32, (n,))
    fp, fk, _ = _buffer(flow, np.float32, (n, 2))
    vp, vk, _ = _buffer(valid, np.uint8, (n,))
    if MEM_HOST in (ka, kb, pk, fk, vk) or not _is_torch(flow):
        raise ValueError("sim_lk_flow_noalloc takes device tensors only")
    if hip_stream is not None and hasattr(hip_stream, "cuda_stream"):
        hip_stream = hip_stream.cuda_stream
    st = ctypes.c_void_p(int(hip_stream)) if hip_stream else None
    _check(lib.sim_lk_flow_noalloc(a, b, W, H, pp, n, fp, vp,
                                   ctypes.byref(lk_params(**params)), st),
           "sim_lk_flow_noalloc")


def _check_flows(flows, needed: int, H: int, W: int) -> None:
    """The library reads `needed` flow fields of [H, W, 2] from `flows`: refuse anything smaller
    before it reaches the device."""
    if needed <= 0:
        return
    if flows is None:
        raise ValueError(f"{needed} flow field(s) [H, W, 2] required")
    shape = tuple(flows.shape)
    if len(shape) == 3:
        shape = (1,) + shape
    if len(shape) != 4 or shape[1:] != (H, W, 2) or shape[0] < needed:
        raise ValueError(f"flows must be [>= {needed}, {H}, {W}, 2], got {tuple(flows.shape)}")


def make_config(width: int, height: int, method: Union[str, int] = "basic",
                transform: Union[str, int] = "log", c_pos: float = 0.2, c_neg: float = 0.2,
                log_eps: float = 1e-3, n_interp: int = 10, mask_threshold: float = -1.0,
                event_capacity: int = 0, hip_stream=None,
                thresh_mode: Union[str, int] = "reference",
                flow_source: Union[str, int] = "supplied") -> SimConfig:
    lib = load()
    cfg = SimConfig()
    lib.sim_config_init(ctypes.byref(cfg))
    cfg.width, cfg.height = int(width), int(height)
    cfg.method = METHODS[method] if isinstance(method, str) else int(method)
    cfg.transform = TRANSFORMS[transform] if isinstance(transform, str) else int(transform)
    cfg.c_pos, cfg.c_neg, cfg.log_eps = float(c_pos), float(c_neg), float(log_eps)
    cfg.n_interp, cfg.mask_threshold = int(n_interp), float(mask_threshold)
    cfg.event_capacity = int(event_capacity)
    cfg.thresh_mode = (THRESH_MODES[thresh_mode] if isinstance(thresh_mode, str)
                       else int(thresh_mode))
    cfg.flow_source = (FLOW_SOURCES[flow_source] if isinstance(flow_source, str)
                       else int(flow_source))
    if hip_stream == "torch":
        import torch
        hip_stream = torch.cuda.current_stream().cuda_stream
    elif hip_stream is not None and hasattr(hip_stream, "cuda_stream"):
        hip_stream = hip_stream.cuda_stream
    cfg.hip_stream = ctypes.c_void_p(int(hip_stream)) if hip_stream else None
    return cfg


class Stream:
    """One simulated event camera (a sim_stream handle)."""

    def __init__(self, width: int, height: int, method: Union[str, int] = "basic",
                 transform: Union[str, int] = "log", c_pos: float = 0.2, c_neg: float = 0.2,
                 log_eps: float = 1e-3, n_interp: int = 10, mask_threshold: float = -1.0,
                 event_capacity: int = 0, hip_stream=None,
                 thresh_mode: Union[str, int] = "reference",
                 flow_source: Union[str, int] = "supplied", lk: Optional[dict] = None):
        lib = load()
        cfg = make_config(width, height, method, transform, c_pos, c_neg, log_eps, n_interp,
                          mask_threshold, event_capacity, hip_stream, thresh_mode, flow_source)
        h = ctypes.c_void_p()
        _check(lib.sim_create(ctypes.byref(cfg), ctypes.byref(h)), "sim_create")
        self._h = h
        self._lib = lib
        self.width, self.height = int(width), int(height)
        self.method = cfg.method
        self.n_interp = cfg.n_interp
        self.flow_source = cfg.flow_source
        if lk:
            _check(lib.sim_set_lk_params(self._h, ctypes.byref(lk_params(**lk))),
                   "sim_set_lk_params", self._h)

    def _flows_needed(self, n_frames: int) -> int:
        """Flow fields a push of n_frames reads: one per simulated interval for the
        interpolating methods with S > 1 (the first frame of a stream only initialises it)."""
        if self.method == BASIC or self.n_interp == 0 or self.flow_source == FLOW_LK:
            return 0
        e = ctypes.c_int64()
        started = self._lib.sim_epoch(self._h, ctypes.byref(e)) == OK
        return n_frames - (0 if started else 1)

    # -- frames ---------------------------------------------------------------------------
    def push(self, frame, flow=None, t_us: int = 0) -> int:
        """Pushes one frame (uint8 [H, W]) with its interval's flow (float32 [H, W, 2])."""
        H, W = self.height, self.width
        fp, fk, fa = _buffer(frame, np.uint8, (H, W))
        lp, lk, la = _buffer(flow, np.float32, (H, W, 2))
        if lk is not None and lk != fk:
            raise ValueError("frame and flow must both be host or both be device memory")
        n = ctypes.c_uint64()
        _check(self._lib.sim_push_frame(self._h, fp, lp, int(t_us), fk, ctypes.byref(n)),
               "sim_push_frame", self._h)
        return n.value

    def push_frames(self, frames, flows, t_us: Sequence[int]) -> int:
        """Pushes frames uint8 [n, H, W]; flows float32 [n_intervals, H, W, 2] (see sim.h)."""
        H, W = self.height, self.width
        n = int(frames.shape[0])
        fp, fk, fa = _buffer(frames, np.uint8, (n, H, W))
        _check_flows(flows, self._flows_needed(n), H, W)
        lp, lk, la = _buffer(flows, np.float32, None)
        if lk is not None and lk != fk:
            raise ValueError("frames and flows must both be host or both be device memory")
        t = np.ascontiguousarray(np.asarray(t_us, dtype=np.int64))
        if t.shape != (n,):
            raise ValueError("need one timestamp per frame")
        out = ctypes.c_uint64()
        _check(self._lib.sim_push_frames(self._h, n, fp, lp, t.ctypes.data_as(ctypes.c_void_p),
                                         fk, ctypes.byref(out)), "sim_push_frames", self._h)
        return out.value

    # -- events ---------------------------------------------------------------------------
    def pending(self) -> int:
        n = ctypes.c_uint64()
        _check(self._lib.sim_pending_events(self._h, ctypes.byref(n)), "sim_pending_events", self._h)
        return n.value

    def drain_events(self, max_events: Optional[int] = None) -> np.ndarray:
        """Oldest pending events as a structured array (t, x, y, p, pad)."""
        n = self.pending() if max_events is None else int(max_events)
        out = np.zeros(n, dtype=EVENT_DTYPE)
        got = ctypes.c_uint64()
        _check(self._lib.sim_drain_events(self._h, out.ctypes.data_as(ctypes.c_void_p), n,
                                          ctypes.byref(got)), "sim_drain_events", self._h)
        return out[:got.value]

    def drain_keys(self, max_events: Optional[int] = None, out=None):
        """Oldest pending events as packed uint64 keys: numpy (host) or, into `out` (a uint64 or
        int64 numpy array or an int64 torch tensor, at most its size), the number written."""
        if out is not None:
            ptr, kind, keep = _out_buffer(out, np.int64, None, also=(np.uint64,))
            cap = int(out.numel()) if _is_torch(out) else int(out.size)
            n = cap if max_events is None else int(max_events)
            if not 0 <= n <= cap:
                raise ValueError(f"max_events must be within 0..{cap} (the size of out)")
            got = ctypes.c_uint64()
            _check(self._lib.sim_drain_keys(self._h, ptr, n, kind, ctypes.byref(got)),
                   "sim_drain_keys", self._h)
            return got.value
        n = self.pending() if max_events is None else int(max_events)
        arr = np.zeros(n, dtype=np.uint64)
        got = ctypes.c_uint64()
        _check(self._lib.sim_drain_keys(self._h, arr.ctypes.data_as(ctypes.c_void_p), n,
                                        MEM_HOST, ctypes.byref(got)), "sim_drain_keys", self._h)
        return arr[:got.value]

    def accumulate(self, t_begin: int, t_end: int, counts=None):
        """Adds the pending events with t_begin <= t < t_end to a frame of accumulated events
        uint32 [2, H, W] (plane 0 positive, plane 1 negative): a new numpy array, a numpy array
        `counts`, or a torch int32 device tensor `counts` (stream-ordered).  Pending events stay
        pending."""
        shape = (2, self.height, self.width)
        if counts is None:
            counts = np.zeros(shape, dtype=np.uint32)
        ptr, kind, keep = _out_buffer(counts, np.uint32, shape)
        _check(self._lib.sim_accumulate(self._h, int(t_begin), int(t_end), ptr, kind),
               "sim_accumulate", self._h)
        return counts

    def event_rate(self, t_begin: int, t_end: int):
        """Events per pixel and second of the pending events in [t_begin, t_end): returns
        (mean, standard deviation over pixels, (sum c, sum c^2))."""
        mean, std = ctypes.c_double(), ctypes.c_double()
        sums = (ctypes.c_uint64 * 2)()
        _check(self._lib.sim_event_rate(self._h, int(t_begin), int(t_end), ctypes.byref(mean),
                                        ctypes.byref(std), sums), "sim_event_rate", self._h)
        return mean.value, std.value, (int(sums[0]), int(sums[1]))

    # -- state ----------------------------------------------------------------------------
    @property
    def epoch(self) -> int:
        e = ctypes.c_int64()
        _check(self._lib.sim_epoch(self._h, ctypes.byref(e)), "sim_epoch", self._h)
        return e.value

    def reference(self, out=None):
        """Per-pixel reference levels float32 [H, W] (numpy, or into a torch device tensor)."""
        if out is not None:
            ptr, kind, keep = _out_buffer(out, np.float32, (self.height, self.width))
            _check(self._lib.sim_get_reference(self._h, ptr, kind), "sim_get_reference", self._h)
            return out
        arr = np.zeros((self.height, self.width), dtype=np.float32)
        _check(self._lib.sim_get_reference(self._h, arr.ctypes.data_as(ctypes.c_void_p),
                                           MEM_HOST), "sim_get_reference", self._h)
        return arr

    def stats(self) -> dict:
        st = SimStats()
        _check(self._lib.sim_get_stats(self._h, ctypes.byref(st)), "sim_get_stats", self._h)
        return {k: getattr(st, k) for k, _ in SimStats._fields_}

    def clear_stats(self) -> None:
        _check(self._lib.sim_clear_stats(self._h), "sim_clear_stats", self._h)

    def set_kernel_timing(self, enable: bool = True) -> None:
        _check(self._lib.sim_set_kernel_timing(self._h, 1 if enable else 0),
               "sim_set_kernel_timing", self._h)

    def sync(self) -> None:
        _check(self._lib.sim_sync(self._h), "sim_sync", self._h)

    def set_chain_variant(self, variant: int = -1) -> None:
        """sim_set_chain_variant: -1 = autotuned, 0..2 = a fixed chain-pass variant."""
        _check(self._lib.sim_set_chain_variant(self._h, int(variant)), "sim_set_chain_variant",
               self._h)

    def chain_variant(self) -> int:
        """sim_get_chain_variant: the variant the last window's chain pass used (-1: none)."""
        v = ctypes.c_int32()
        _check(self._lib.sim_get_chain_variant(self._h, ctypes.byref(v)),
               "sim_get_chain_variant", self._h)
        return v.value

    def reset(self) -> None:
        _check(self._lib.sim_reset(self._h), "sim_reset", self._h)

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.sim_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def push_batch(entries) -> list:
    """Batched push: entries is a sequence of (stream, frames, flows, t_us).  Same result as one
    push_frames per stream; the streams' GPU work overlaps.  Returns the per-stream event counts
    and raises SimError (with the first failing stream's status) on error."""
    lib = load()
    n = len(entries)
    handles = (ctypes.c_void_p * n)()
    items = (SimFrames * n)()
    keep = []
    for i, (stream, frames, flows, t_us) in enumerate(entries):
        H, W = stream.height, stream.width
        nf = int(frames.shape[0])
        fp, fk, fa = _buffer(frames, np.uint8, (nf, H, W))
        _check_flows(flows, stream._flows_needed(nf), H, W)
        lp, lk, la = _buffer(flows, np.float32, None)
        if lk is not None and lk != fk:
            raise ValueError("frames and flows must both be host or both be device memory")
        t = np.ascontiguousarray(np.asarray(t_us, dtype=np.int64))
        if t.shape != (nf,):
            raise ValueError("need one timestamp per frame")
        keep += [fa, la, t]
        handles[i] = stream._h
        items[i].n_frames = nf
        items[i].mem_kind = fk
        items[i].frames = fp
        items[i].flows = lp
        items[i].t_us = t.ctypes.data_as(ctypes.c_void_p)
    rc = lib.sim_push_batch(handles, items, n)
    if rc != OK:
        bad = next((i for i in range(n) if items[i].status != OK), None)
        where = "sim_push_batch" if bad is None else f"sim_push_batch (stream {bad})"
        _check(rc, where, None if bad is None else entries[bad][0]._h)
    return [items[i].n_new_events for i in range(n)]


class Server:
    """Continuous-batching server of many virtual cameras (srv_* in include/sim.h)."""

    def __init__(self, hbm_budget_bytes: int, max_cameras: int = 256, queue_depth: int = 8):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.srv_create(int(hbm_budget_bytes), int(max_cameras), int(queue_depth),
                                    ctypes.byref(h)), "srv_create")
        self._h = h
        self.queue_depth = int(queue_depth)
        self._shape = {}
        # the inputs of each camera's recent submissions: the library reads them asynchronously,
        # and a ring slot is reused only after the step that read it
        self._keep = {}

    @staticmethod
    def footprint(queue_depth: int = 8, **cfg) -> int:
        c = make_config(**cfg)
        out = ctypes.c_uint64()
        _check(load().srv_footprint(ctypes.byref(c), int(queue_depth), ctypes.byref(out)),
               "srv_footprint")
        return out.value

    def admit(self, **cfg) -> int:
        """Admits a camera (keyword arguments as Stream); raises SimError(E_BUSY) when it does
        not fit the HBM budget or no slot is free."""
        c = make_config(**cfg)
        cam = ctypes.c_int32()
        _check(self._lib.srv_admit(self._h, ctypes.byref(c), ctypes.byref(cam)), "srv_admit")
        self._shape[cam.value] = (c.height, c.width)
        self._keep[cam.value] = collections.deque(maxlen=self.queue_depth + 1)
        return cam.value

    def release(self, cam: int) -> None:
        _check(self._lib.srv_release(self._h, int(cam)), "srv_release")
        self._shape.pop(int(cam), None)
        self._keep.pop(int(cam), None)

    def submit(self, cam: int, frame, flow=None, t_us: int = 0, arrival_ns: int = 0) -> None:
        H, W = self._shape[int(cam)]
        fp, fk, fa = _buffer(frame, np.uint8, (H, W))
        lp, lk, la = _buffer(flow, np.float32, (H, W, 2))
        kind = fk
        if lk is not None and lk != fk:
            if (fk, lk) != (MEM_HOST, MEM_DEVICE):
                raise ValueError("a device frame needs a device flow")
            kind = MEM_HOST_FRAME
        _check(self._lib.srv_submit(self._h, int(cam), fp, lp, int(t_us), kind, int(arrival_ns)),
               "srv_submit")
        self._keep[int(cam)].append((fa, la))

    def step(self) -> int:
        n = ctypes.c_uint64()
        _check(self._lib.srv_step(self._h, ctypes.byref(n)), "srv_step")
        return n.value

    def start(self) -> None:
        """srv_start: steps run on the server's worker thread while frames are queued."""
        _check(self._lib.srv_start(self._h), "srv_start")

    def stop(self) -> None:
        _check(self._lib.srv_stop(self._h), "srv_stop")

    def sync(self) -> None:
        """srv_sync: waits until every queued frame has completed."""
        _check(self._lib.srv_sync(self._h), "srv_sync")

    def pending(self, cam: int) -> int:
        n = ctypes.c_uint64()
        _check(self._lib.srv_pending(self._h, int(cam), ctypes.byref(n)), "srv_pending")
        return n.value

    def drain_keys(self, cam: int, max_events: Optional[int] = None, out=None):
        """Drains a camera's ordered events: into a new numpy array, or into `out` (an int64
        device tensor, returning the number written)."""
        if out is not None:
            p, kind, _ = _out_buffer(out, np.int64, None, also=(np.uint64,))
            n = out.numel() if max_events is None else min(int(max_events), out.numel())
            got = ctypes.c_uint64()
            _check(self._lib.srv_drain(self._h, int(cam), p, n, kind, ctypes.byref(got)),
                   "srv_drain")
            return got.value
        pend = ctypes.c_uint64()
        _check(self._lib.srv_pending(self._h, int(cam), ctypes.byref(pend)), "srv_pending")
        n = pend.value if max_events is None else int(max_events)
        arr = np.zeros(n, dtype=np.uint64)
        got = ctypes.c_uint64()
        _check(self._lib.srv_drain(self._h, int(cam), arr.ctypes.data_as(ctypes.c_void_p), n,
                                   MEM_HOST, ctypes.byref(got)), "srv_drain")
        return arr[:got.value]

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.srv_get_stats(self._h, ctypes.byref(st)), "srv_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def clear_stats(self) -> None:
        _check(self._lib.srv_clear_stats(self._h), "srv_clear_stats")

    def now_ns(self) -> int:
        return int(self._lib.srv_now_ns())

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.srv_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_keys(keys: np.ndarray, epoch: int = 0):
    """Unpacks packed keys into (t, x, y, p) int64 arrays."""
    keys = np.asarray(keys).view(np.uint64) if np.asarray(keys).dtype == np.int64 else np.asarray(keys, dtype=np.uint64)
    t = (keys >> np.uint64(25)).astype(np.int64) + epoch
    y = ((keys >> np.uint64(13)) & np.uint64(0xFFF)).astype(np.int64)
    x = ((keys >> np.uint64(1)) & np.uint64(0xFFF)).astype(np.int64)
    p = np.where((keys & np.uint64(1)) == 1, 1, -1).astype(np.int64)
    return t, x, y, p
