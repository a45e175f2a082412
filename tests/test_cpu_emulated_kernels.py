"""The exact HIP kernel and runtime sources, executed on the CPU (tests/cpu_emu), against the oracle.

These tests do not replace the GPU parity tests (test_parity_gpu.py, marked gpu): they run the
same source files compiled for the host through a HIP emulation layer (one fiber per GPU thread,
lockstep wave64 intrinsics, block barriers), so index arithmetic, overflow re-runs, window splits
and every intrinsic use can be checked without a GPU -- and, in the AddressSanitizer build, every
memory access is bounds-checked.  The product never loads these builds.
"""
import ctypes
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import golden_io
from oracle.oracle import OracleSim
from paper_2209_04634_amd import sim, synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "cpu_emu"))
import build as emu_build  # noqa: E402


@pytest.fixture(scope="module")
def emu_sim(monkeypatch_module):
    path = emu_build.build()
    monkeypatch_module.setattr(sim, "LIB_PATH", path)
    monkeypatch_module.setattr(sim, "_lib", None)
    yield sim
    sim._lib = None


@pytest.fixture(scope="module")
def monkeypatch_module():
    mp = pytest.MonkeyPatch()
    yield mp
    mp.undo()


def oracle_run(frames, flows, t, **cfg):
    T, H, W = frames.shape
    o = OracleSim(W, H, **cfg)
    out = []
    for k in range(T):
        ev = o.push(frames[k], None if (flows is None or k == 0) else flows[k - 1], int(t[k]))
        if k:
            out.append(ev)
    return (np.concatenate(out) if out else np.zeros(0, np.uint64)), o.lref()


def emu_run(s_mod, frames, flows, t, mode="window", **cfg):
    T, H, W = frames.shape
    s = s_mod.Stream(W, H, **cfg)
    if mode == "window":
        s.push_frames(frames, flows, t)
    else:
        for k in range(T):
            s.push(frames[k], None if (flows is None or k == 0) else flows[k - 1], int(t[k]))
    keys, ref, st = s.drain_keys(), s.reference(), s.stats()
    s.close()
    return keys, ref, st


def check(s_mod, frames, flows, t, modes=("window",), **cfg):
    ok, oref = oracle_run(frames, flows, t, **cfg)
    for mode in modes:
        keys, ref, st = emu_run(s_mod, frames, flows, t, mode=mode, **cfg)
        np.testing.assert_array_equal(keys, ok, err_msg=mode)
        np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32), err_msg=mode)
    return len(ok)


@pytest.mark.parametrize("path", golden_io.all_fixtures(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_emulated_hand_worked_fixtures(emu_sim, path):
    g = golden_io.load(path)
    for mode in ("window", "single"):
        keys, ref, _ = emu_run(emu_sim, g.frames, g.flows, g.t_us, mode=mode, **g.cfg)
        t, x, y, p = emu_sim.decode_keys(keys, g.t_us[0])
        assert list(zip(t.tolist(), x.tolist(), y.tolist(), p.tolist())) == \
            [e for iv in g.events for e in iv]
        np.testing.assert_array_equal(ref, g.lref)


@pytest.mark.parametrize("S", [1, 2, 11, 33])
@pytest.mark.parametrize("method", [sim.BASIC, sim.DENSE, sim.SPARSE])
def test_emulated_ragged_image(emu_sim, method, S):
    if method == sim.BASIC and S != 1:
        pytest.skip("basic has one sub-interval")
    rng = np.random.default_rng(100 * S + method)
    frames, flows = synth.random_frames(rng, 4, 23, 37, flow_scale=3.0)
    t = np.array([0, 33333, 50000, 83333])
    check(emu_sim, frames, flows, t, modes=("window", "single"), method=method, c_pos=0.2,
          c_neg=0.25, n_interp=S - 1)


def test_emulated_blob_video_dense_and_sparse(emu_sim):
    spec = synth.BlobVideoSpec(96, 64, 8, 30.0, 10, seed=5, motion="random", speed_max=8.0)
    v = synth.blob_video(spec)
    n1 = check(emu_sim, v.frames, v.flows, v.t_us, modes=("window", "single"),
               method=sim.DENSE, c_pos=0.15, c_neg=0.15)
    n2 = check(emu_sim, v.frames, v.flows, v.t_us, method=sim.SPARSE, c_pos=0.15, c_neg=0.15)
    assert n1 > n2 > 0


def test_emulated_overflow_reruns(emu_sim):
    spec = synth.BlobVideoSpec(64, 48, 6, 30.0, 8, seed=9, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, method=sim.DENSE, c_pos=0.15, c_neg=0.15)
    for cap in (1, 300, 5000):
        keys, ref, st = emu_run(emu_sim, v.frames, v.flows, v.t_us, method=sim.DENSE,
                                c_pos=0.15, c_neg=0.15, event_capacity=cap)
        np.testing.assert_array_equal(keys, ok)
        np.testing.assert_array_equal(ref, oref)
        assert st["retries"] > 0


def test_emulated_long_sparse_sequence_spans_windows(emu_sim):
    """140 frames: two windows (128 + 11 intervals) and all four selection mask words."""
    spec = synth.BlobVideoSpec(24, 16, 140, 60.0, 3, seed=4, motion="random", speed_max=2.0)
    v = synth.blob_video(spec)
    check(emu_sim, v.frames, v.flows, v.t_us, method=sim.SPARSE, c_pos=0.1, c_neg=0.1,
          n_interp=3)


@pytest.mark.parametrize("method", [sim.DENSE, sim.DIFFERENCE])
def test_emulated_host_push_stages_one_window_at_a_time(emu_sim, method):
    """A 300-frame push from host memory (three windows) copies one window of frames and flows
    to the device at a time: the staging buffers hold 128 frames and 128 flow fields, never the
    whole push, and the events equal the oracle's."""
    W, H = 32, 16
    spec = synth.BlobVideoSpec(W, H, 300, 60.0, 3, seed=8, motion="random", speed_max=4.0)
    v = synth.blob_video(spec)
    lib = emu_sim.load()
    lib.emu_alloc_log.restype = ctypes.c_size_t
    lib.emu_alloc_log.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.c_size_t]
    lib.emu_reset_alloc_log()
    cfg = dict(method=method, c_pos=0.05, c_neg=0.05, n_interp=3)
    s = emu_sim.Stream(W, H, **cfg)
    s.push_frames(v.frames, v.flows, v.t_us)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    assert len(ok) > 1000
    np.testing.assert_array_equal(s.drain_keys(), ok)
    np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
    s.close()
    buf = (ctypes.c_size_t * 4096)()
    sizes = set(buf[:min(lib.emu_alloc_log(buf, 4096), 4096)])
    assert {128 * W * H, 128 * W * H * 2 * 4} <= sizes, sorted(sizes)
    assert not {300 * W * H, 299 * W * H, 299 * W * H * 2 * 4} & sizes, sorted(sizes)


@pytest.mark.parametrize("shape", [(1, 1), (1, 70), (70, 1), (9, 2), (3, 129)])
def test_emulated_degenerate_shapes(emu_sim, shape):
    """One- and two-pixel-wide images: every bilinear footprint is clamped at a border."""
    H, W = shape
    rng = np.random.default_rng(H * 7 + W)
    frames, flows = synth.random_frames(rng, 3, H, W)
    for method in (sim.BASIC, sim.DENSE, sim.SPARSE, sim.DIFFERENCE):
        check(emu_sim, frames, flows, np.array([0, 900, 2100]), method=method, n_interp=4)


@pytest.mark.parametrize("shape", [(300, 1), (40, 2), (2, 129)])
def test_emulated_degenerate_shapes_gpu_cases(emu_sim, shape):
    """The GPU suite's degenerate cases with the same seeds, flows and times."""
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    frames, flows = synth.random_frames(rng, 3, H, W, flow_scale=2.0)
    for method in (sim.BASIC, sim.DENSE, sim.SPARSE, sim.DIFFERENCE):
        check(emu_sim, frames, flows, np.array([5, 1005, 3000]), method=method, n_interp=4)


def test_emulated_batched_push_equals_streams_alone(emu_sim):
    """A batch mixing resolutions and methods gives each stream exactly its solo result, and
    pushing the batch twice continues every stream's state."""
    specs = [((48, 32), emu_sim.DENSE, 1), ((40, 24), emu_sim.SPARSE, 2), ((33, 17), emu_sim.BASIC, 3),
             ((64, 40), emu_sim.SPARSE, 4)]
    vids, solo = [], []
    for (W, H), method, seed in specs:
        v = synth.blob_video(synth.BlobVideoSpec(W, H, 7, 30.0, 6, seed=seed, motion="random",
                                                 speed_max=5.0))
        vids.append(v)
        flows = None if method == emu_sim.BASIC else v.flows
        solo.append(oracle_run(v.frames, flows, v.t_us, method=method, c_pos=0.15, c_neg=0.15,
                               n_interp=5))
    streams = [emu_sim.Stream(W, H, method=m, c_pos=0.15, c_neg=0.15, n_interp=5,
                              event_capacity=64)
               for (W, H), m, _ in specs]
    # first half of every sequence, then the second half, each as one batch
    for a, b in ((0, 4), (4, 7)):
        entries = []
        for st, v, ((W, H), m, _) in zip(streams, vids, specs):
            fl = None
            if m != emu_sim.BASIC:
                fl = v.flows[max(a - 1, 0):b - 1]
            entries.append((st, v.frames[a:b], fl, v.t_us[a:b]))
        emu_sim.push_batch(entries)
    for st, (ok, oref) in zip(streams, solo):
        np.testing.assert_array_equal(st.drain_keys(), ok)
        np.testing.assert_array_equal(st.reference(), oref)
        st.close()


def test_emulated_batch_validation_is_all_or_nothing(emu_sim):
    v = synth.blob_video(synth.BlobVideoSpec(20, 12, 3, 30.0, 2, seed=1))
    a = emu_sim.Stream(20, 12, method="dense")
    b = emu_sim.Stream(20, 12, method="dense")
    with pytest.raises(emu_sim.SimError) as e:
        emu_sim.push_batch([(a, v.frames, v.flows, v.t_us), (b, v.frames, v.flows, v.t_us[::-1])])
    assert e.value.status == emu_sim.E_ORDER
    assert a.pending() == 0 and b.pending() == 0
    with pytest.raises(emu_sim.SimError):
        emu_sim.push_batch([(a, v.frames, v.flows, v.t_us), (a, v.frames, v.flows, v.t_us)])
    emu_sim.push_batch([(a, v.frames, v.flows, v.t_us), (b, v.frames, v.flows, v.t_us)])
    np.testing.assert_array_equal(a.drain_keys(), b.drain_keys())


def _camera_videos(emu):
    cams = [((40, 24), "dense", 11), ((33, 21), "sparse", 12), ((28, 16), "basic", 13),
            ((48, 30), "sparse", 14)]
    out = []
    for (W, H), method, seed in cams:
        v = synth.blob_video(synth.BlobVideoSpec(W, H, 9, 30.0, 5, seed=seed, motion="random",
                                                 speed_max=5.0))
        m = emu.METHODS[method]
        flows = None if method == "basic" else v.flows
        ok, oref = oracle_run(v.frames, flows, v.t_us, method=m, c_pos=0.15, c_neg=0.15,
                              n_interp=4)
        out.append(dict(W=W, H=H, method=method, v=v, ok=ok, oref=oref))
    return out


def test_emulated_server_results_match_cameras_alone(emu_sim):
    """Frames of four cameras (mixed resolution and method) arrive interleaved; steps run at
    irregular points, so batches mix cameras at different positions of their sequences.  Every
    camera's events equal the oracle's for that camera alone."""
    cams = _camera_videos(emu_sim)
    srv = emu_sim.Server(hbm_budget_bytes=1 << 34, max_cameras=8, queue_depth=4)
    ids = [srv.admit(width=c["W"], height=c["H"], method=c["method"], c_pos=0.15, c_neg=0.15,
                     n_interp=4, event_capacity=16) for c in cams]
    rng = np.random.default_rng(0)
    pos = [0] * len(cams)
    while any(p < 9 for p in pos):
        i = int(rng.integers(len(cams)))
        if pos[i] >= 9:
            continue
        c, k = cams[i], pos[i]
        flow = None if (c["method"] == "basic" or k == 0) else c["v"].flows[k - 1]
        try:
            srv.submit(ids[i], c["v"].frames[k], flow, int(c["v"].t_us[k]))
            pos[i] += 1
        except emu_sim.SimError as e:
            assert e.status == emu_sim.E_BUSY       # queue full: step, then retry
            srv.step()
        if rng.random() < 0.3:
            srv.step()
    srv.step()
    for cid, c in zip(ids, cams):
        np.testing.assert_array_equal(srv.drain_keys(cid), c["ok"])
    st = srv.stats()
    assert st["completed"] == 9 * len(cams) and st["failed_frames"] == 0
    assert 0 <= st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    srv.close()


@pytest.mark.parametrize("pinned", [False, True], ids=["copied-at-submit", "pulled-by-step"])
def test_emulated_server_worker_continuous_batching(emu_sim, pinned):
    """The same cameras with the server's worker running: frames are submitted from this thread
    while the worker steps on its own (a full ring is retried after a short wait), then
    srv_sync.  Host inputs are either pageable (copied into the ring at submission) or pinned
    (pulled into the ring by the step's copy kernel).  Every camera's events equal the oracle's
    for that camera alone, every frame is completed, and manual steps are refused while the
    worker runs."""
    emu_sim.load().emu_host_memory_pinned(1 if pinned else 0)
    try:
        _server_worker_run(emu_sim)
    finally:
        emu_sim.load().emu_host_memory_pinned(0)


def _server_worker_run(emu_sim):
    import time
    cams = _camera_videos(emu_sim)
    srv = emu_sim.Server(hbm_budget_bytes=1 << 34, max_cameras=8, queue_depth=3)
    ids = [srv.admit(width=c["W"], height=c["H"], method=c["method"], c_pos=0.15, c_neg=0.15,
                     n_interp=4, event_capacity=16) for c in cams]
    srv.start()
    with pytest.raises(emu_sim.SimError) as e:
        srv.step()
    assert e.value.status == emu_sim.E_BUSY
    rng = np.random.default_rng(1)
    pos = [0] * len(cams)
    while any(p < 9 for p in pos):
        i = int(rng.integers(len(cams)))
        if pos[i] >= 9:
            continue
        c, k = cams[i], pos[i]
        flow = None if (c["method"] == "basic" or k == 0) else c["v"].flows[k - 1]
        try:
            srv.submit(ids[i], c["v"].frames[k], flow, int(c["v"].t_us[k]))
            pos[i] += 1
        except emu_sim.SimError as e:
            assert e.status == emu_sim.E_BUSY       # ring full: the worker frees it
            time.sleep(0.001)
    srv.sync()
    st = srv.stats()
    assert st["completed"] == 9 * len(cams) and st["failed_frames"] == 0 and st["steps"] >= 1
    for cid, c in zip(ids, cams):
        np.testing.assert_array_equal(srv.drain_keys(cid), c["ok"])
    srv.stop()
    srv.close()


def test_emulated_server_admission_by_footprint(emu_sim):
    fp = emu_sim.Server.footprint(queue_depth=2, width=64, height=48, method="sparse")
    srv = emu_sim.Server(hbm_budget_bytes=2 * fp + fp // 2, max_cameras=8, queue_depth=2)
    a = srv.admit(width=64, height=48, method="sparse")
    b = srv.admit(width=64, height=48, method="sparse")
    with pytest.raises(emu_sim.SimError) as e:
        srv.admit(width=64, height=48, method="sparse")
    assert e.value.status == emu_sim.E_BUSY
    st = srv.stats()
    assert st["cameras"] == 2 and st["rejected_admissions"] == 1 and st["hbm_used"] == 2 * fp
    srv.release(a)
    c = srv.admit(width=64, height=48, method="sparse")          # memory freed: admitted
    assert c == a
    # queue depth 2: a third frame before a step is refused, and timestamps must increase
    f = np.zeros((48, 64), np.uint8)
    fl = np.zeros((48, 64, 2), np.float32)
    srv.submit(b, f, None, 0)
    srv.submit(b, f, fl, 10)
    with pytest.raises(emu_sim.SimError) as e:
        srv.submit(b, f, fl, 20)
    assert e.value.status == emu_sim.E_BUSY
    assert srv.step() == 2
    with pytest.raises(emu_sim.SimError) as e:
        srv.submit(b, f, fl, 10)
    assert e.value.status == emu_sim.E_ORDER
    assert srv.stats()["rejected_frames"] == 1
    srv.close()


ASAN_SCRIPT = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim, synth
    sim.LIB_PATH = {lib!r}; sim._lib = None
    from test_cpu_emulated_kernels import oracle_run, emu_run
    cases = []
    spec = synth.BlobVideoSpec(64, 48, 6, 30.0, 8, seed=9, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    for method in (0, 1, 2):
        for cap in (1, 0):
            cases.append((v.frames, v.flows, v.t_us, dict(method=method, c_pos=0.15,
                          c_neg=0.15, event_capacity=cap)))
    spec = synth.BlobVideoSpec(20, 12, 140, 60.0, 3, seed=4, motion="random", speed_max=2.0)
    w = synth.blob_video(spec)
    cases.append((w.frames, w.flows, w.t_us, dict(method=2, c_pos=0.1, c_neg=0.1, n_interp=3,
                  event_capacity=1)))
    rng = np.random.default_rng(1)
    f, fl = synth.random_frames(rng, 3, 5, 7)
    cases.append((f, fl, np.array([0, 10, 20]), dict(method=1, n_interp=40, event_capacity=1)))
    from test_cpu_emulated_kernels import _camera_videos
    import time
    cams = _camera_videos(sim)[:2]     # two cameras of different shape and method suffice here
    for pinned in (0, 1):              # host inputs copied at submission / pulled by the worker
        sim.load().emu_host_memory_pinned(pinned)
        srv = sim.Server(hbm_budget_bytes=1 << 34, max_cameras=4, queue_depth=3)
        ids = [srv.admit(width=c["W"], height=c["H"], method=c["method"], c_pos=0.15,
                         c_neg=0.15, n_interp=4, event_capacity=8) for c in cams]
        if pinned:
            srv.start()
        for k in range(9):
            for cid, c in zip(ids, cams):
                fl = None if (c["method"] == "basic" or k == 0) else c["v"].flows[k - 1]
                while True:
                    try:
                        srv.submit(cid, c["v"].frames[k], fl, int(c["v"].t_us[k]))
                        break
                    except sim.SimError:
                        time.sleep(0.002)
            if k % 3 == 2 and not pinned:
                srv.step()
        srv.sync()
        for cid, c in zip(ids, cams):
            assert np.array_equal(srv.drain_keys(cid), c["ok"])
        srv.close()
    sim.load().emu_host_memory_pinned(0)
    for frames, flows, t, cfg in cases:
        ocfg = dict((k, v) for k, v in cfg.items() if k != "event_capacity")
        ok, oref = oracle_run(frames, flows, t, **ocfg)
        keys, ref, st = emu_run(sim, frames, flows, t, **cfg)
        assert np.array_equal(keys, ok) and np.array_equal(ref, oref), cfg
    print("asan-clean", len(cases))
""")


@pytest.mark.long
def test_emulated_kernels_are_memory_safe_under_asan(tmp_path):
    """Every device-memory access of the runtime and kernels, bounds-checked by AddressSanitizer
    (device buffers are host allocations in this build), on overflow re-runs, window splits and
    the recompute path beyond the LDS stash."""
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_case.py"
    script.write_text(ASAN_SCRIPT.format(root=os.path.dirname(HERE), tests=HERE, lib=lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]
