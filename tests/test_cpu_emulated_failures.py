"""Failure handling on the CPU emulation: every device allocation a call makes is made to fail in
turn, and the call must end in one of the two documented ways -- SIM_E_NOMEM with the stream
untouched (a later push gives the oracle's result), or SIM_E_NOMEM with the stream poisoned
(every later call SIM_E_POISONED, destroy still fine) when part of the image had already
advanced.  No crash, no wrong result.  The same for batched pushes, server admission and the flow
estimator.  These run on the host only; nothing here faults a GPU."""
import ctypes

import numpy as np
import pytest

from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import emu_sim, monkeypatch_module, oracle_run  # noqa: F401


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
