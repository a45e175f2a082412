"""Failure handling on the CPU emulation: every device allocation a call makes is made to fail in
turn, and the call must end in one of the two documented ways -- SIM_E_NOMEM with the stream
untouched (a later push gives the oracle's result), or SIM_E_NOMEM with the stream poisoned
(every later call SIM_E_POISONED, destroy still fine) when part of the image had already
advanced.  No crash, no wrong result.  The same for batched pushes, server admission and the flow
estimator.  These run on the host only; nothing here faults a GPU."""
import ctypes
import os
import subprocess
import sys
import textwrap
import time

import numpy as np
import pytest

from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import (emu_build, emu_sim, monkeypatch_module,  # noqa: F401
                                       oracle_run, HERE)


def _video():
    return synth.blob_video(synth.BlobVideoSpec(40, 24, 5, 30.0, 5, seed=3, motion="random",
                                                speed_max=5.0))


def _arm(emu, k):
    """The emulated library's device allocation after k more successful ones fails."""
    lib = emu.load()
    lib.emu_fail_alloc_after.argtypes = [ctypes.c_long]
    lib.emu_fail_alloc_after(k)


def _disarm(emu):
    _arm(emu, -1)


def _outcome(emu, s):
    try:
        s.pending()
        return "untouched"
    except emu.SimError as e:
        assert e.status == emu.E_POISONED
        return "poisoned"


@pytest.mark.parametrize("method", ["dense", "sparse", "difference"])
def test_every_allocation_failure_of_a_push(emu_sim, method):
    v = _video()
    cfg = dict(method=method, c_pos=0.12, c_neg=0.12, n_interp=4)
    ocfg = dict(cfg, method=emu_sim.METHODS[method])
    ok, _ = oracle_run(v.frames, v.flows, v.t_us, **ocfg)
    seen = set()
    for k in range(40):
        s = emu_sim.Stream(40, 24, event_capacity=1, **cfg)     # forces buffer growth mid-push
        _arm(emu_sim, k)
        try:
            s.push_frames(v.frames, v.flows, v.t_us)
            _disarm(emu_sim)
            np.testing.assert_array_equal(s.drain_keys(), ok)
            seen.add("completed")
        except emu_sim.SimError as e:
            _disarm(emu_sim)
            assert e.status == emu_sim.E_NOMEM, e
            out = _outcome(emu_sim, s)
            seen.add(out)
            if out == "untouched":
                assert s.pending() == 0
                s.push_frames(v.frames, v.flows, v.t_us)
                np.testing.assert_array_equal(s.drain_keys(), ok)
            else:
                with pytest.raises(emu_sim.SimError):
                    s.push_frames(v.frames, v.flows, v.t_us)
        s.close()
    assert {"untouched", "poisoned", "completed"} <= seen, seen


def test_every_allocation_failure_of_create(emu_sim):
    outcomes = set()
    for k in range(30):
        _arm(emu_sim, k)
        try:
            s = emu_sim.Stream(32, 16, method="sparse")
            outcomes.add("ok")
            s.close()
        except emu_sim.SimError as e:
            assert e.status == emu_sim.E_NOMEM
            outcomes.add("nomem")
        _disarm(emu_sim)
    assert outcomes == {"ok", "nomem"}
    emu_sim.Stream(32, 16, method="sparse").close()


@pytest.mark.long
def test_every_allocation_failure_of_a_batch(emu_sim):
    """Per entry: completed (the oracle's events), untouched (failed while staging or
    reserving: nothing pending, a later push works) or poisoned (failed inside the fused
    launches, like every stream of that window)."""
    v = _video()
    cfgs = [dict(method="dense", c_pos=0.12, c_neg=0.12, n_interp=4, event_capacity=1),
            dict(method="sparse", c_pos=0.12, c_neg=0.12, n_interp=4, event_capacity=1),
            dict(method="basic", c_pos=0.12, c_neg=0.12)]
    oks = []
    for c in cfgs:
        oc = {k: x for k, x in c.items() if k != "event_capacity"}
        oc["method"] = emu_sim.METHODS[c["method"]]
        oks.append(oracle_run(v.frames, None if c["method"] == "basic" else v.flows, v.t_us,
                              **oc)[0])
    seen = set()
    for k in range(45):
        streams = [emu_sim.Stream(40, 24, **c) for c in cfgs]
        entries = [(s, v.frames, None if c["method"] == "basic" else v.flows, v.t_us)
                   for s, c in zip(streams, cfgs)]
        _arm(emu_sim, k)
        try:
            emu_sim.push_batch(entries)
        except emu_sim.SimError as e:
            assert e.status == emu_sim.E_NOMEM, e
        _disarm(emu_sim)
        for s, c, ok in zip(streams, cfgs, oks):
            out = _outcome(emu_sim, s)
            if out == "untouched" and s.pending() == len(ok) and len(ok):
                np.testing.assert_array_equal(s.drain_keys(), ok)
                out = "completed"
            elif out == "untouched":
                assert s.pending() == 0
                s.push_frames(v.frames, None if c["method"] == "basic" else v.flows, v.t_us)
                np.testing.assert_array_equal(s.drain_keys(), ok)
            seen.add(out)
            s.close()
    assert {"completed", "untouched", "poisoned"} <= seen, seen


def test_server_admission_allocation_failure(emu_sim):
    srv = emu_sim.Server(hbm_budget_bytes=1 << 32, max_cameras=2, queue_depth=2)
    failures = 0
    for k in range(25):
        _arm(emu_sim, k)
        try:
            cid = srv.admit(width=24, height=16, method="dense")
            _disarm(emu_sim)
            srv.release(cid)
        except emu_sim.SimError as e:
            _disarm(emu_sim)
            assert e.status == emu_sim.E_NOMEM
            failures += 1
        st = srv.stats()
        assert st["cameras"] == 0 and st["hbm_used"] == 0
    assert failures > 0
    v = _video()
    cid = srv.admit(width=40, height=24, method="dense", c_pos=0.12, c_neg=0.12, n_interp=4)
    for k in range(5):
        srv.submit(cid, v.frames[k], None if k == 0 else v.flows[k - 1], int(v.t_us[k]))
        srv.step()
    ok, _ = oracle_run(v.frames, v.flows, v.t_us, method=sim.DENSE, c_pos=0.12, c_neg=0.12,
                       n_interp=4)
    np.testing.assert_array_equal(srv.drain_keys(cid), ok)
    srv.close()


def test_flow_estimator_allocation_failure(emu_sim):
    v = _video()
    pts = np.arange(40 * 24, dtype=np.uint32)
    ref, _ = emu_sim.lk_flow(v.frames[0], v.frames[1], pts, levels=1, radius=2)
    failures = 0
    for k in range(8):
        _arm(emu_sim, k)
        try:
            got, _ = emu_sim.lk_flow(v.frames[0], v.frames[1], pts, levels=1, radius=2)
            np.testing.assert_array_equal(got, ref)
        except emu_sim.SimError as e:
            assert e.status == emu_sim.E_NOMEM
            failures += 1
        _disarm(emu_sim)
    assert failures > 0



def alternating_wave(c, pixels=range(320, 384)):
    """A 640x1 image whose given pixels (inside 255 .. 383) see a period-2 pattern move 256 px in
    one interval: with n_interp = 255 and the linear table all 256 samples alternate between 0 and
    255, the most crossings a pixel can make.  With C a power of two every level step is exact,
    so each such pixel fires exactly 256 * 255 / C events."""
    pixels = list(pixels)
    assert 255 <= min(pixels) and max(pixels) <= 383
    W = 640
    f0 = np.where(np.arange(W) % 2 == 1, 255, 0).astype(np.uint8)
    flow = np.zeros((1, 1, W, 2), np.float32)
    flow[0, 0, pixels, 0] = 256.0
    cfg = dict(method="dense", transform="linear", c_pos=c, c_neg=c, n_interp=255)
    return np.stack([f0, f0]).reshape(2, 1, W), flow, np.array([0, 1000], np.int64), cfg


# (stream options, accepted): with a reference level S * (2 (max T - min T) / C + 3) <= 2^24
BOUND_CASES = [
    (dict(transform="linear", c=2.0 ** -12, n_interp=255), False),
    (dict(transform="linear", c=0.0077, n_interp=255), False),
    (dict(transform="linear", c=2.0 ** -7, n_interp=255), True),      # 16,712,448 <= 2^24
    (dict(transform="log", c=2.0e-4, n_interp=255), False),
    (dict(transform="log", c=2.2e-4, n_interp=255), True),
    (dict(transform="linear", c=2.0 ** -12, n_interp=10), False),
    (dict(transform="linear", c=2.0 ** -12, method="basic"), True),   # S = 1
    (dict(transform="linear", c=2.0 ** -12, n_interp=255, thresh_mode="memoryless"), True),
    (dict(transform="linear", c=2.0 ** -12, n_interp=255, method="difference"), True),
]


@pytest.mark.parametrize("opts,accepted", BOUND_CASES)
def test_events_per_pixel_and_interval_bound(emu_sim, opts, accepted):
    """Configurations in which one pixel could fire more than 2^24 events in one interval with a
    reference level are refused (the chain kernel sums 64 pixels' counts in 32 bits); memoryless
    thresholding fires at most S per interval and is not limited."""
    o = dict(opts)
    c = o.pop("c")
    o.setdefault("method", "dense")
    if accepted:
        emu_sim.Stream(64, 4, c_pos=c, c_neg=c, **o).close()
        emu_sim.Stream(64, 4, c_pos=c, c_neg=4 * c, **o).close()
    else:
        with pytest.raises(emu_sim.SimError) as e:
            emu_sim.Stream(64, 4, c_pos=c, c_neg=c, **o)
        assert e.value.status == emu_sim.E_INVAL
        with pytest.raises(emu_sim.SimError):
            emu_sim.Stream(64, 4, c_pos=4 * c, c_neg=c, **o)


def run_heaviest_wave(s_mod, arm):
    """The heaviest wave an accepted configuration allows: 64 pixels of 256 * 255 * 128 =
    8,355,840 events each in one interval (5.3e8 in all; no sub-arena can hold that).  The k-th
    device allocation of the push fails, k = 0, 1, ...: early failures leave the stream untouched;
    the first that lands on the growth of the event arena, after the chain kernel counted, must
    poison it.  Returns the seconds that push took."""
    frames, flows, t, cfg = alternating_wave(2.0 ** -7)
    for k in range(8):
        s = s_mod.Stream(640, 1, **cfg)
        arm(k)
        t0 = time.time()
        try:
            s.push_frames(frames, flows, t)
            raise AssertionError("5.3e8 events of one wave cannot fit a sub-arena")
        except s_mod.SimError as e:
            assert e.status == s_mod.E_NOMEM, e
        finally:
            arm(-1)
        dt = time.time() - t0
        try:
            assert s.pending() == 0
        except s_mod.SimError as e:
            assert e.status == s_mod.E_POISONED
            s.close()
            return dt
        s.close()
    raise AssertionError("no allocation of the push failed after the chain kernel")


@pytest.mark.long
def test_heaviest_wave_fails_cleanly(emu_sim):
    dt = run_heaviest_wave(emu_sim, lambda k: _arm(emu_sim, k))
    assert dt < 120, dt


def test_alternating_pixel_count_on_the_oracle():
    """The count the heaviest wave relies on: one alternating pixel at C = 2^-7 fires exactly
    256 * 255 * 128 events in the oracle."""
    frames, flows, t, _ = alternating_wave(2.0 ** -7, [340])
    ok, _ = oracle_run(frames, flows, t, method=sim.DENSE, transform=sim.LINEAR,
                       c_pos=2.0 ** -7, c_neg=2.0 ** -7, n_interp=255)
    assert len(ok) == 256 * 255 * 128


def test_alternating_pixels_equal_the_oracle(emu_sim):
    """The same construction at a size that fits: one pixel in each of two waves."""
    frames, flows, t, cfg = alternating_wave(1.0, [300, 330])
    s = emu_sim.Stream(640, 1, event_capacity=256 * 65536, **cfg)
    s.push_frames(frames, flows, t)
    ok, oref = oracle_run(frames, flows, t, method=sim.DENSE, transform=sim.LINEAR,
                          c_pos=1.0, c_neg=1.0, n_interp=255)
    assert len(ok) == 2 * 256 * 255
    np.testing.assert_array_equal(s.drain_keys(), ok)
    np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
    s.close()


ASAN_SCRIPT = textwrap.dedent("""
    import ctypes, sys
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim
    sim.LIB_PATH = {lib!r}; sim._lib = None
    import test_cpu_emulated_failures as t
    lib = sim.load()
    lib.emu_fail_alloc_after.argtypes = [ctypes.c_long]
    t.run_heaviest_wave(sim, lib.emu_fail_alloc_after)
    print("asan-clean")
""")


@pytest.mark.long
def test_heaviest_wave_is_memory_safe_under_asan(tmp_path):
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_wave.py"
    script.write_text(ASAN_SCRIPT.format(root=os.path.dirname(HERE), tests=HERE, lib=lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]
