#!/usr/bin/env python3
"""Throughput benchmark of the MI355X event simulator.

One step = the whole hot path over one synthetic sequence with inputs already resident in HBM:
reset the stream, push every frame (transform, interpolation, threshold crossing, emission and
time ordering, all in the HIP library), then drain the ordered events into a device buffer.

Default workload: 1280x720 sparse-flow interpolation, 120 frames at 60 fps (119 intervals),
256 blobs with >= 10% of the image moving at up to 24 px/frame over a static background, C = 0.2,
10 interpolated frames per interval (the paper's low-dynamics scenario, Sec. IV-A).

Prints one JSON line (rank 0, N = 1).  Extra fields report the events/s rate, the per-frame
latency of plain one-frame pushes (p50 / p99) next to the batched window push, and the dominant
kernel against the HBM roofline.  After the main measurement (and the CPU baseline), a child
process times the extra legs and the line carries them under "extra_legs" (or an "error" entry if
the child fails or exceeds --legs-timeout; the main figures are unaffected): the memoryless,
difference-frame and estimated-flow workloads, 64 mixed-resolution streams pushed as one batch
per frame step against one push per stream (methods round-robin, then each method alone), and a
60 s serving run with 256 cameras (Poisson arrivals, the server's worker stepping continuously).
--no-legs skips them; --workload, --batched STREAMS and --serve SECONDS run single legs in
process.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "sparse_1280x720": dict(spec="sparse_1280x720", method="sparse", c=0.2, n_interp=10),
    "dense_346x260": dict(spec="dense_346x260", method="dense", c=0.15, n_interp=10),
    "basic_240x180": dict(spec="basic_240x180", method="basic", c=0.2, n_interp=0),
    # the paper-literal thresholding, the difference-frame method and estimated flow
    "memoryless_dense_346x260": dict(spec="dense_346x260", method="dense", c=0.03, n_interp=10,
                                     thresh="memoryless"),
    "difference_346x260": dict(spec="dense_346x260", method="difference", c=0.3, n_interp=10),
    "lk_sparse_1280x720": dict(spec="sparse_1280x720", method="sparse", c=0.2, n_interp=10,
                               flow="lk"),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sparse_1280x720", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-frame-push latency leg")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--batched", type=int, default=0, metavar="STREAMS",
                    help="also time STREAMS mixed-resolution streams (240x180, 346x260, "
                         "640x480, 1920x1080; all three methods) pushed as one batch per frame "
                         "step against one push per stream and step")
    ap.add_argument("--serve", type=float, default=0.0, metavar="SECONDS",
                    help="also run the serving loop for SECONDS: sparse cameras of 346x260, "
                         "640x480 and 1280x720 with Poisson frame arrivals at 30-240 fps")
    ap.add_argument("--cameras", type=int, default=32, help="cameras of the serving leg")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the extra legs (memoryless, difference, estimated flow, 64 batched "
                         "streams, 256-camera serving) that run in a child process after the "
                         "main measurement")
    ap.add_argument("--legs-timeout", type=float, default=420.0)
    ap.add_argument("--legs-child", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


def chain_bytes(npix: int, K: int, active: int, selected: int, events: int, method: str,
                memoryless: bool = False) -> int:
    """Minimum HBM bytes of one chain-kernel launch (the dominant kernel) over a window of K
    intervals.  Per chain (an active pixel for sparse, every pixel otherwise): its list slot and
    selected-interval bitmask (sparse: 4 + 16 B), its reference level read and written (8 B; none
    for the memoryless and difference thresholding).  Per interpolated pixel-interval: the
    endpoint bytes (2; the difference method reads 3 frames) and the flow vector (8 B; basic
    reads none).  Per event: one 8-byte key written."""
    ref = 0 if (memoryless or method == "difference") else 8
    if method == "sparse":
        per_chain = 4 + 16 + ref
        chains = active
    else:
        per_chain, chains = ref, npix
        selected = npix * K
    per_sel = (3 if method == "difference" else 2) + (0 if method == "basic" else 8)
    return chains * per_chain + selected * per_sel + 8 * events


def step_bytes(npix: int, K: int, selected: int, events: int, method: str,
               memoryless: bool = False) -> int:
    """Algorithmic HBM bytes of a whole step (every phase of the path, sort passes excluded),
    per pixel-interval with the state in HBM between intervals: both frame endpoints (1 + 1 B;
    the difference method reads 3), per interpolated pixel-interval (every one for the dense and
    difference methods, the selected ones for sparse) the flow (8 B) and the reference level
    read and written (8 B; none for memoryless and difference thresholding), and 8 B per event."""
    ends = 3 if method == "difference" else 2
    ref = 0 if (memoryless or method == "difference") else 8
    if method == "basic":
        return npix * K * (ends + ref) + 8 * events
    interp = selected if method == "sparse" else npix * K
    return npix * K * ends + interp * (8 + ref) + 8 * events


def kernel_source_hash() -> str:
    """SHA-256 of the sources the simulation kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2209_04634_amd",
                        "csrc")
    for name in ("evsim_kernels.hip", "evsim_internal.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(workload: str, kernel: str = "k_chain", variant=None, folder=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary of this
    workload (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the counter reads for a
    copy of known size), or None when there is none, the kernels changed since it was taken, or
    it was taken on another chain variant than the one this run uses."""
    import glob
    import re
    folder = folder or os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
    src = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(folder, "*counters*.md"))):
        with open(path) as f:
            text = f.read()
        for block in re.findall(r"```json\n(.*?)```", text, flags=re.S):
            try:
                d = json.loads(block)
            except ValueError:
                continue
            if d.get("workload") != workload or d.get("kernel") != kernel:
                continue
            if d.get("source_sha256") != src:
                return None
            if variant is not None and d.get("variant") not in (None, variant):
                return None
            return (d["fetch_kib_per_dispatch"] * d["fetch_scale"] +
                    d["write_kib_per_dispatch"] * d["write_scale"]) * 1024.0
    return None


BATCH_SHAPES = [(240, 180), (346, 260), (640, 480), (1920, 1080)]
SERVE_SHAPES = [(346, 260), (640, 480), (1280, 720)]


def batched_leg(args, sim, synth, torch, dev, shapes=BATCH_SHAPES, n_frames=30,
                methods=("dense", "sparse", "basic")):
    """Streams of mixed resolution (the batched configuration's recipe, scaled to `args.batched`
    streams), methods round-robin over `methods`: per frame step, one sim_push_batch of every
    stream's frame against one push per stream.  Inputs resident in HBM; events drained into
    device buffers.  Also reports the timed batched run's per-frame-step host phases and device
    time (sim_batch_times)."""
    methods = list(methods)
    videos = {}
    for W, H in shapes:              # one device-resident video per resolution, shared
        v = synth.blob_video(synth.mixed_stream(W, H, seed=W + H, n_frames=n_frames))
        videos[(W, H)] = (torch.from_numpy(v.frames).to(dev), torch.from_numpy(v.flows).to(dev),
                          v.t_us)
    streams, data = [], []
    for i in range(args.batched):
        W, H = shapes[i % len(shapes)]
        method = methods[(i // len(shapes)) % len(methods)]
        c = [0.12, 0.15, 0.2, 0.25][(i // 12) % 4]
        fr, fl, t = videos[(W, H)]
        data.append((fr, None if method == "basic" else fl, t, W * H))
        streams.append(sim.Stream(W, H, method=method, c_pos=c, c_neg=c))
    torch.cuda.synchronize()
    px_per_step = sum(d[3] for d in data)

    def run(batched):
        for st in streams:
            st.reset()
        for k in range(n_frames):
            if batched:
                sim.push_batch([(st, fr[k:k + 1], None if (fl is None or k == 0)
                                 else fl[k - 1:k], t[k:k + 1])
                                for st, (fr, fl, t, _) in zip(streams, data)])
            else:
                for st, (fr, fl, t, _) in zip(streams, data):
                    st.push(fr[k], None if (fl is None or k == 0) else fl[k - 1], int(t[k]))
        ev = 0
        for st in streams:
            ev += st.pending()
            out = torch.empty(max(1, st.pending()), dtype=torch.int64, device=dev)
            st.drain_keys(out=out)
        torch.cuda.synchronize()
        return ev

    res, secs = {}, {}
    g0 = sim.batch_stats()
    for name, batched in (("batched", True), ("plain", False)):
        run(batched)                                   # warm-up: buffers reach their sizes
        b0 = sim.batch_times()
        t0 = time.perf_counter()
        ev = run(batched)
        dt = time.perf_counter() - t0
        if batched:
            b1 = sim.batch_times()
            steps = max(1, n_frames - 1)
            res["batched_per_step_ms"] = {k: round((b1[k] - b0[k]) / steps, 3) for k in
                                          ("inputs_ms", "plan_ms", "launch_ms", "wait_ms",
                                           "finish_ms", "device_ms")}
        secs[name] = dt
        res[name] = {"mpix_frames_per_s": round(px_per_step * (n_frames - 1) / dt / 1e6, 1),
                     "ms_per_frame_step": round(1e3 * dt / (n_frames - 1), 3),
                     "events_per_s": round(ev / dt, 1)}
    for st in streams:
        st.close()
    res["streams"] = args.batched
    res["methods"] = methods
    res["speedup"] = round(secs["plain"] / secs["batched"], 3)
    g1 = sim.batch_stats()
    res["graphs"] = {k: g1[k] - g0[k] for k in g1}   # recorded, launched, re-run windows
    return res


def host_cpu() -> dict:
    """The host's logical CPUs (those this process may run on) and CPU model."""
    import subprocess
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "model": model}


def _oracle_worker(job):
    """One process of the all-cores baseline: the oracle over the memory-mapped sequence, from
    a common start time, repeated until `seconds` have passed; returns (px-intervals, events,
    elapsed seconds)."""
    folder, W, H, cfg, start_at, seconds, supplied = job
    import numpy as np
    from oracle.oracle import OracleSim
    frames = np.load(os.path.join(folder, "frames.npy"), mmap_mode="r")
    flows = np.load(os.path.join(folder, "flows.npy"), mmap_mode="r") if supplied else None
    t_us = np.load(os.path.join(folder, "t_us.npy"))
    K = len(t_us) - 1
    while time.time() < start_at:
        time.sleep(0.001)
    a = time.perf_counter()
    done = ev = 0
    while time.perf_counter() - a < seconds:
        o = OracleSim(W, H, **cfg)
        o.push(np.asarray(frames[0]), None, int(t_us[0]))
        for k in range(K):
            e = o.push(np.asarray(frames[k + 1]), np.asarray(flows[k]) if supplied else None,
                       int(t_us[k + 1]))
            ev += len(e)
            done += 1
            if time.perf_counter() - a >= seconds:
                break
    return W * H * done, ev, time.perf_counter() - a


def cpu_all_cores(video, W, H, cfg, supplied, seconds):
    """The oracle on every logical CPU this process may use (at most 16): one process per CPU,
    each simulating the same sequence from a shared memory-mapped copy, all starting together.
    Returns the aggregate rate in Mpixel-frames/s and events/s, and the processes used."""
    import multiprocessing as mp
    import shutil
    import tempfile
    import numpy as np
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    base = "/dev/shm" if os.path.isdir("/dev/shm") else None
    folder = tempfile.mkdtemp(prefix="evsim_oracle_", dir=base)
    try:
        np.save(os.path.join(folder, "frames.npy"), video.frames)
        if supplied:
            np.save(os.path.join(folder, "flows.npy"), video.flows)
        np.save(os.path.join(folder, "t_us.npy"), np.asarray(video.t_us))
        start_at = time.time() + 8.0       # after every process has started and loaded
        jobs = [(folder, W, H, cfg, start_at, seconds, supplied)] * procs
        with mp.get_context("spawn").Pool(procs) as pool:
            res = pool.map(_oracle_worker, jobs)
    finally:
        shutil.rmtree(folder, ignore_errors=True)
    wall = max(r[2] for r in res)
    return (sum(r[0] for r in res) / wall / 1e6, sum(r[1] for r in res) / wall, procs, wall)


def serve_leg(args, sim, synth, torch, dev, res_opts=SERVE_SHAPES):
    """Serving loop (continuous batching): cameras of the serving configuration's resolutions,
    sparse method, frames arriving as Poisson processes (rate U[30, 240] fps per camera) and
    handed to the server as they arrive (frames copied from pinned host memory, flows from a
    device-resident pool), while the server's worker runs one batched step after another over
    whatever is queued; events are drained into a device buffer every 20 ms.  Reports per-frame latency (arrival to ordered events), throughput and
    the frames refused because a camera's staging ring was full."""
    import ctypes
    import numpy as np
    rng = np.random.default_rng(7)
    pools = {}
    P = 64
    for W, H in res_opts:
        v = synth.blob_video(synth.serving_stream(W, H, seed=W, n_frames=P))
        fr = torch.from_numpy(v.frames).pin_memory()
        fl = torch.from_numpy(v.flows).to(dev)
        pools[(W, H)] = (fr, fl, [fr[j].data_ptr() for j in range(P)],
                         [fl[j].data_ptr() for j in range(P - 1)])
    torch.cuda.synchronize()
    srv = sim.Server(hbm_budget_bytes=160 << 30, max_cameras=args.cameras, queue_depth=8)
    cams = []
    for c in range(args.cameras):
        W, H = res_opts[int(rng.integers(3))]
        try:
            cid = srv.admit(width=W, height=H, method="sparse", c_pos=0.2, c_neg=0.2)
        except sim.SimError:
            continue
        cams.append(dict(id=cid, W=W, H=H, rate=float(rng.uniform(30, 240)),
                         k=int(rng.integers(P)), next=0.0, t=0))
    lib, h = sim.load(), srv._h
    drain = torch.empty(1 << 24, dtype=torch.int64, device=dev)

    def submit(c, arrival):
        """Frame k of the camera's pass over the pool (the flow of the interval ending there)."""
        fr, fl, fp, lp = pools[(c["W"], c["H"])]
        j = c["k"] % P
        c["t"] += 1 + int(1e6 / c["rate"])
        rc = lib.srv_submit(h, c["id"], ctypes.c_void_p(fp[j]),
                            ctypes.c_void_p(lp[(j - 1) % (P - 1)]), c["t"], sim.MEM_HOST_FRAME,
                            arrival)
        c["k"] += 1                          # a refused frame (ring full) is dropped
        return rc

    for c in cams:       # warm-up, two frames per camera: buffers, tuning, recorded graphs
        submit(c, 0)
        submit(c, 0)
    srv.sync()
    for c in cams:
        srv.drain_keys(c["id"], out=drain)
    srv.clear_stats()
    t0 = sim.batch_times()
    srv.start()
    start = time.perf_counter()
    for c in cams:
        c["next"] = start + float(rng.exponential(1.0 / c["rate"]))
    offered = 0
    last_drain = start
    while time.perf_counter() - start < args.serve:
        now = time.perf_counter()
        base_ns = srv.now_ns()
        for c in cams:
            while c["next"] <= now:
                submit(c, int(base_ns - (now - c["next"]) * 1e9))
                offered += 1
                c["next"] += float(rng.exponential(1.0 / c["rate"]))
        if now - last_drain > 0.02:
            for c in cams:
                srv.drain_keys(c["id"], out=drain)
            last_drain = now
    srv.sync()
    wall = time.perf_counter() - start
    srv.stop()
    st = srv.stats()
    t1 = sim.batch_times()
    srv.close()
    steps = max(1, st["steps"])
    phases = {k: round((t1[k] - t0[k]) / steps, 3) for k in
              ("inputs_ms", "plan_ms", "launch_ms", "wait_ms", "finish_ms", "device_ms")}
    return {"cameras": len(cams), "seconds": round(wall, 2), "offered_frames": offered,
            "frames": st["completed"], "frames_per_s": round(st["completed"] / wall, 1),
            "events_per_s": round(st["events"] / wall, 1),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "max_ms": round(st["max_ms"], 3), "rejected_frames": st["rejected_frames"],
            "rejected_admissions": st["rejected_admissions"], "steps": st["steps"],
            "frames_per_step": round(st["completed"] / steps, 1),
            "step_ms": round(st["busy_ms"] / steps, 3),
            "worker_busy_frac": round(st["busy_ms"] / 1e3 / wall, 3),
            "lock_wait_ms_per_step": round(st["lock_wait_ms"] / steps, 3),
            "per_step_ms": phases}


def measure(wl_name, steps, warmup, sim, synth, torch, dev, plain=True):
    """Times `steps` whole-sequence steps of a workload (after `warmup`); returns the figures of
    the bench line and the objects the CPU-baseline leg needs."""
    import numpy as np
    wl = WORKLOADS[wl_name]
    spec = getattr(synth, wl["spec"])()
    supplied = wl["method"] != "basic" and wl.get("flow", "supplied") == "supplied"
    video = synth.blob_video(spec, with_flow=wl["method"] != "basic")
    T, H, W = video.frames.shape
    npix = H * W
    K = T - 1
    frames = torch.from_numpy(video.frames).to(dev)
    flows = torch.from_numpy(video.flows).to(dev) if supplied else None
    t_us = video.t_us
    torch.cuda.synchronize()

    s = sim.Stream(W, H, method=wl["method"], c_pos=wl["c"], c_neg=wl["c"],
                   n_interp=wl["n_interp"], hip_stream="torch",
                   thresh_mode=wl.get("thresh", "reference"), flow_source=wl.get("flow", "supplied"))
    s.set_kernel_timing(True)
    # the drain buffer grows to the sequence's event count during the warm-up steps (every step
    # pushes the same sequence, so the timed steps never grow it)
    out_box = [torch.empty(max(1, npix * K // 10), dtype=torch.int64, device=dev)]

    def step():
        s.reset()
        n = s.push_frames(frames, flows, t_us)
        if n > out_box[0].numel():
            out_box[0] = torch.empty(n + n // 8 + 1, dtype=torch.int64, device=dev)
        got = s.drain_keys(out=out_box[0], max_events=n)
        assert got == n
        return n

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s.clear_stats()
    events = 0
    marks = []
    t0 = time.perf_counter()
    for _ in range(steps):
        events += step()                 # each step ends with a synchronising drain
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_step = np.diff(np.array([t0] + marks)) * 1e3
    st = s.stats()
    chain_variant = s.chain_variant()
    selected = st["selected"]
    sim_ms, sim_launches = st["simulate_ms"], st["simulate_launches"]
    sel_ms = st["select_ms"]
    sort_ms = st["sort_ms"]
    ev_per_step = events // steps
    sel_per_step = (selected // steps) if wl["method"] == "sparse" else npix * K

    # dominant kernel: the per-pixel chain launch (one per step: the window holds every interval)
    launch_ms = sim_ms / max(1, sim_launches)
    launches_per_step = sim_launches / steps
    act_per_step = st["active"] // steps
    alg = chain_bytes(npix, K, act_per_step, sel_per_step, ev_per_step, wl["method"],
                      memoryless=wl.get("thresh") == "memoryless")
    alg_per_launch = alg / launches_per_step
    achieved = alg_per_launch / (launch_ms * 1e-3) / 1e9
    traffic = counter_traffic(wl_name, variant=chain_variant)
    # the whole step (every phase, sort passes excluded) against the same roof
    sb = step_bytes(npix, K, sel_per_step, ev_per_step, wl["method"],
                    memoryless=wl.get("thresh") == "memoryless")
    step_gbs = sb / (elapsed / steps) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "kernel": "k_chain", "launch_ms": round(launch_ms, 4),
                "algorithmic_bytes_per_launch": int(alg_per_launch),
                "traffic_gbs": None if traffic is None else
                round(traffic / (launch_ms * 1e-3) / 1e9, 1),
                "step_algorithmic_bytes": int(sb), "step_achieved": round(step_gbs, 1),
                "step_frac": round(step_gbs / HBM_PEAK_GBS, 4)}

    # plain path: one push per frame, latency of each push until its events are ordered
    plain_res = None
    if plain:
        s.reset()
        s.push(frames[0], None, int(t_us[0]))
        lat = []
        for k in range(1, T):
            a = time.perf_counter()
            s.push(frames[k], None if flows is None else flows[k - 1], int(t_us[k]))
            lat.append(time.perf_counter() - a)
        out = out_box[0]
        if s.pending() > out.numel():
            out = torch.empty(s.pending(), dtype=torch.int64, device=dev)
        s.drain_keys(out=out)
        lat_ms = np.array(lat) * 1e3
        plain_res = {"p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
                     "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
                     "mpix_frames_per_s": round(npix * K / lat_ms.sum() * 1e3 / 1e6, 1)}
    s.close()
    return {
        "value": round(npix * K * steps / elapsed / 1e6, 1),
        "ms_per_step": round(1e3 * elapsed / steps, 4),
        "ms_per_step_std": round(float(per_step.std()), 4),
        "events_per_s": round(ev_per_step * steps / elapsed, 1),
        "events_per_step": ev_per_step,
        "selected_fraction": round(sel_per_step / (npix * K), 5),
        "active_pixels_per_step": act_per_step,
        "select_ms_per_step": round(sel_ms / steps, 4),
        "simulate_ms_per_step": round(sim_ms / steps, 4),
        "sort_ms_per_step": round(sort_ms / steps, 4),
        "chain_variant": chain_variant,
        "plain_one_frame_pushes": plain_res,
        "roofline": roofline,
        "_video": video, "_spec": spec, "_wl": wl, "_shape": (T, H, W),
    }


LEG_WORKLOADS = ["memoryless_dense_346x260", "difference_346x260", "lk_sparse_1280x720"]


def legs_child(args):
    """The optional legs, run in a child process of the default bench so that the main line is
    measured and printed whatever happens here: the memoryless, difference-frame and
    estimated-flow workloads; 64 mixed-resolution streams batched against plain pushes; the
    serving loop with 256 cameras.  Each leg prints its own JSON line when it ends (an error
    inside a leg is recorded and the next leg runs), so finished legs survive a later failure."""
    import torch
    from paper_2209_04634_amd import sim, synth
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    def leg(name, fn):
        t0 = time.perf_counter()
        try:
            out = fn()
        except Exception as e:   # recorded in the bench line; the remaining legs still run
            out = {"error": repr(e)[:400]}
        if isinstance(out, dict):
            out.setdefault("wall_s", round(time.perf_counter() - t0, 1))
        print(json.dumps({name: out}), flush=True)
        print(f"leg {name} done", file=sys.stderr, flush=True)

    def workload(name):
        m = measure(name, 5, 2, sim, synth, torch, dev, plain=False)
        wl = m["_wl"]
        r = {k: v for k, v in m.items() if not k.startswith("_") and v is not None}
        r["config"] = {"method": wl["method"], "c": wl["c"], "n_interp": wl["n_interp"],
                       "thresh_mode": wl.get("thresh", "reference"),
                       "flow_source": wl.get("flow", "supplied"),
                       "width": m["_shape"][2], "height": m["_shape"][1],
                       "frames": m["_shape"][0]}
        return r

    for name in LEG_WORKLOADS:
        leg(name, lambda name=name: workload(name))
    args.batched = args.batched or 64
    leg("batched_vs_plain_streams", lambda: batched_leg(args, sim, synth, torch, dev))
    for method in ("dense", "sparse", "basic"):
        leg(f"batched_vs_plain_{method}",
            lambda method=method: batched_leg(args, sim, synth, torch, dev, methods=(method,)))
    args.cameras = 256
    args.serve = args.serve or 60.0
    leg("serving", lambda: serve_leg(args, sim, synth, torch, dev))


def merge_leg_lines(text):
    """The legs' JSON lines (one object per finished leg) merged into one object."""
    res = {}
    for line in (text or "").splitlines():
        line = line.strip()
        if not line.startswith("{"):
            continue
        try:
            obj = json.loads(line)
        except ValueError:
            continue
        if isinstance(obj, dict):
            res.update(obj)
    return res


def run_legs(timeout_s):
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--legs-child"]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired as e:
        out = e.stdout.decode() if isinstance(e.stdout, bytes) else e.stdout
        res = merge_leg_lines(out)
        res["error"] = f"legs did not finish within {timeout_s} s"
        return res
    sys.stderr.write(r.stderr[-2000:])
    res = merge_leg_lines(r.stdout)
    if r.returncode != 0:
        res["error"] = f"legs exited with status {r.returncode}"
        res["stderr_tail"] = r.stderr[-600:]
    elif not res:
        res["error"] = "legs printed no result"
    return res


def main():
    args = parse()
    if args.legs_child:
        legs_child(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this simulator runs on one GPU; sharding across GPUs is "
                          "designed but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2209_04634_amd import sim, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    m = measure(args.workload, args.steps, args.warmup, sim, synth, torch, dev,
                plain=not args.no_plain)
    wl, spec, video = m["_wl"], m["_spec"], m["_video"]
    T, H, W = m["_shape"]
    npix, K, t_us = H * W, T - 1, video.t_us

    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle.oracle import OracleSim
        oracle.build(force=False)
        o = OracleSim(W, H, method=sim.METHODS[wl["method"]], c_pos=wl["c"], c_neg=wl["c"],
                      n_interp=wl["n_interp"],
                      thresh_mode=sim.THRESH_MODES[wl.get("thresh", "reference")],
                      flow_source=sim.FLOW_SOURCES[wl.get("flow", "supplied")])
        supplied = wl["method"] != "basic" and wl.get("flow", "supplied") == "supplied"
        o.push(video.frames[0], None, int(t_us[0]))
        a = time.perf_counter()
        done, oev = 0, 0
        while done < K and (time.perf_counter() - a) < args.cpu_seconds:
            e = o.push(video.frames[done + 1], video.flows[done] if supplied else None,
                       int(t_us[done + 1]))
            oev += len(e)
            done += 1
        ct = time.perf_counter() - a
        single = round(npix * done / ct / 1e6, 3)
        ocfg = dict(method=sim.METHODS[wl["method"]], c_pos=wl["c"], c_neg=wl["c"],
                    n_interp=wl["n_interp"],
                    thresh_mode=sim.THRESH_MODES[wl.get("thresh", "reference")],
                    flow_source=sim.FLOW_SOURCES[wl.get("flow", "supplied")])
        rate, ev_rate, procs, wall = cpu_all_cores(video, W, H, ocfg, supplied,
                                                   args.cpu_seconds)
        cpu = {"value": round(rate, 3), "unit": "Mpixel-frames/s", "cores": procs,
               "kind": "oracle",
               "sample": f"the same {W}x{H} sequence ({K} intervals) simulated by {procs} "
                         f"concurrent single-threaded C-oracle processes for {wall:.1f} s "
                         f"({ev_rate:.3g} events/s in total); one process alone: {single} "
                         f"Mpixel-frames/s over the first {done} intervals ({ct:.1f} s, "
                         f"{oev} events)",
               "single_core_value": single, "host": host_cpu()}

    batched = batched_leg(args, sim, synth, torch, dev) if args.batched else None
    served = serve_leg(args, sim, synth, torch, dev) if args.serve > 0 else None
    legs = None
    if not args.no_legs and not args.batched and args.serve <= 0:
        legs = run_legs(args.legs_timeout)

    line = {
        "metric": "Mpixel-frames/s + events/s vs HBM roofline; p50/p99 frame latency, batched vs plain",
        "value": m["value"],
        "unit": "Mpixel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "ms_per_step_std": m["ms_per_step_std"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "width": W, "height": H, "frames": T,
                   "fps": spec.fps, "method": wl["method"], "c_pos": wl["c"],
                   "c_neg": wl["c"], "n_interp": wl["n_interp"], "blobs": spec.n_blobs,
                   "seed": spec.seed, "mode": "window push (one launch per sequence)"},
    }
    for k in ("events_per_s", "events_per_step", "selected_fraction", "active_pixels_per_step",
              "select_ms_per_step", "simulate_ms_per_step", "sort_ms_per_step", "chain_variant",
              "plain_one_frame_pushes", "roofline"):
        line[k] = m[k]
    line["cpu_baseline"] = cpu
    if wl.get("thresh"):
        line["config"]["thresh_mode"] = wl["thresh"]
    if wl.get("flow"):
        line["config"]["flow_source"] = wl["flow"]
        line["flow_estimation_note"] = "flow estimation runs inside select_ms_per_step"
    if batched is not None:
        line["batched_vs_plain_streams"] = batched
    if served is not None:
        line["serving"] = served
    if legs is not None:
        line["extra_legs"] = legs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
