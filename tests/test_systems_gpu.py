"""GPU: batched pushes over streams of mixed resolution and method, and the continuous-batching
server, give every stream / camera exactly the oracle's result for it alone."""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2209_04634_amd import sim, synth

pytestmark = pytest.mark.gpu

SHAPES = [(240, 180), (346, 260), (640, 480), (1920, 1080)]   # the mixed-resolution batch


def oracle_keys(frames, flows, t, **cfg):
    T, H, W = frames.shape
    o = OracleSim(W, H, **cfg)
    out = []
    for k in range(T):
        ev = o.push(frames[k], None if (flows is None or k == 0) else flows[k - 1], int(t[k]))
        if k:
            out.append(ev)
    return np.concatenate(out), o.lref()


def _videos(n_frames):
    vids = []
    for i, (W, H) in enumerate(SHAPES * 2):
        method = [sim.DENSE, sim.SPARSE, sim.BASIC][i % 3]
        v = synth.blob_video(synth.mixed_stream(W, H, seed=40 + i, n_frames=n_frames))
        flows = None if method == sim.BASIC else v.flows
        vids.append(dict(v=v, method=method, W=W, H=H, flows=flows))
    return vids


def test_batched_push_mixed_resolutions_equals_streams_alone():
    import torch
    vids = _videos(5)
    streams = [sim.Stream(d["W"], d["H"], method=d["method"], c_pos=0.15, c_neg=0.15)
               for d in vids]
    torch.cuda.synchronize()
    dev = [(torch.from_numpy(d["v"].frames).cuda(),
            None if d["flows"] is None else torch.from_numpy(d["flows"]).cuda()) for d in vids]
    torch.cuda.synchronize()
    # two batches: frames 0..2, then 3..4 (continuing every stream)
    for a, b in ((0, 3), (3, 5)):
        entries = []
        for st, d, (fr, fl) in zip(streams, vids, dev):
            fls = None if fl is None else fl[max(a - 1, 0):b - 1].contiguous()
            entries.append((st, fr[a:b].contiguous(), fls, d["v"].t_us[a:b]))
        sim.push_batch(entries)
    for st, d in zip(streams, vids):
        ok, oref = oracle_keys(d["v"].frames, d["flows"], d["v"].t_us, method=d["method"],
                               c_pos=0.15, c_neg=0.15)
        np.testing.assert_array_equal(st.drain_keys(), ok)
        np.testing.assert_array_equal(st.reference(), oref)
        st.close()


def test_server_interleaved_cameras_equal_cameras_alone():
    import torch
    vids = _videos(6)[:6]
    srv = sim.Server(hbm_budget_bytes=64 << 30, max_cameras=16, queue_depth=4)
    ids = [srv.admit(width=d["W"], height=d["H"], method=d["method"], c_pos=0.15, c_neg=0.15)
           for d in vids]
    torch.cuda.synchronize()
    dev = [(torch.from_numpy(d["v"].frames).cuda(),
            None if d["flows"] is None else torch.from_numpy(d["flows"]).cuda()) for d in vids]
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    pos = [0] * len(vids)
    while any(p < 6 for p in pos):
        i = int(rng.integers(len(vids)))
        if pos[i] >= 6:
            continue
        k = pos[i]
        fr, fl = dev[i]
        flow = None if (fl is None or k == 0) else fl[k - 1]
        try:
            srv.submit(ids[i], fr[k], flow, int(vids[i]["v"].t_us[k]))
            pos[i] += 1
        except sim.SimError as e:
            assert e.status == sim.E_BUSY
            srv.step()
        if rng.random() < 0.25:
            srv.step()
    srv.step()
    for cid, d in zip(ids, vids):
        ok, _ = oracle_keys(d["v"].frames, d["flows"], d["v"].t_us, method=d["method"],
                            c_pos=0.15, c_neg=0.15)
        np.testing.assert_array_equal(srv.drain_keys(cid), ok)
    st = srv.stats()
    assert st["completed"] == 36 and st["failed_frames"] == 0
    assert 0 <= st["p50_ms"] <= st["p99_ms"]
    srv.close()


def test_c4_batched_64_streams_full_size():
    """The batched configuration at full size: 64 streams, 16 each of 240x180, 346x260, 640x480
    and 1920x1080, all three methods, 30 frames, pushed as one batch per frame step (the launch
    configuration of bench.py --batched).  Every stream equals the same stream pushed alone on
    the GPU; sampled streams covering every resolution and method equal the oracle."""
    import torch
    vids = {}
    for W, H in SHAPES:
        v = synth.blob_video(synth.mixed_stream(W, H, seed=W + H, n_frames=30))
        vids[(W, H)] = (v, torch.from_numpy(v.frames).cuda(), torch.from_numpy(v.flows).cuda())
    torch.cuda.synchronize()
    cfgs = []
    for i in range(64):
        W, H = SHAPES[i % 4]
        method = [sim.DENSE, sim.SPARSE, sim.BASIC][(i // 4) % 3]
        c = [0.12, 0.15, 0.2, 0.25][(i // 12) % 4]
        cfgs.append(dict(W=W, H=H, method=method, c=c))
    streams = [sim.Stream(d["W"], d["H"], method=d["method"], c_pos=d["c"], c_neg=d["c"])
               for d in cfgs]
    before = sim.batch_stats()
    for k in range(30):
        entries = []
        for st, d in zip(streams, cfgs):
            v, fr, fl = vids[(d["W"], d["H"])]
            flow = None if (d["method"] == sim.BASIC or k == 0) else fl[k - 1:k]
            entries.append((st, fr[k:k + 1], flow, v.t_us[k:k + 1]))
        sim.push_batch(entries)
    after = sim.batch_stats()
    launches = after["graph_launches"] - before["graph_launches"]
    recorded = after["graphs_recorded"] - before["graphs_recorded"]
    assert launches == 29 and recorded < launches, (launches, recorded)   # steps replay graphs
    batched = [st.drain_keys() for st in streams]
    for st in streams:
        st.close()
    for i, d in enumerate(cfgs):
        v, fr, fl = vids[(d["W"], d["H"])]
        s = sim.Stream(d["W"], d["H"], method=d["method"], c_pos=d["c"], c_neg=d["c"])
        s.push_frames(fr, None if d["method"] == sim.BASIC else fl, v.t_us)
        np.testing.assert_array_equal(batched[i], s.drain_keys(), err_msg=str(d))
        s.close()
    # sampled against the oracle: every resolution and every method
    sampled = [0, 5, 10, 3, 7]
    assert {(cfgs[i]["W"], cfgs[i]["method"]) for i in sampled} == {
        (SHAPES[0][0], sim.DENSE), (SHAPES[1][0], sim.SPARSE), (SHAPES[2][0], sim.BASIC),
        (SHAPES[3][0], sim.DENSE), (SHAPES[3][0], sim.SPARSE)}
    for i in sampled:
        d = cfgs[i]
        v = vids[(d["W"], d["H"])][0]
        ok, _ = oracle_keys(v.frames, None if d["method"] == sim.BASIC else v.flows, v.t_us,
                            method=d["method"], c_pos=d["c"], c_neg=d["c"])
        np.testing.assert_array_equal(batched[i], ok, err_msg=str(d))


@pytest.mark.parametrize("worker", [False, True], ids=["manual-steps", "worker"])
def test_c5_serving_256_cameras(worker):
    """The serving configuration's camera population: 256 sparse cameras (C = 0.2) with
    resolutions drawn from 346x260, 640x480 and 1280x720 (the sparse recipe with blob count
    scaled by area), admitted by footprint, frames from
    device-resident pools at per-camera phases and rates U[30, 240] fps, submitted in random
    interleaving, with steps at random points or by the server's worker thread while frames keep
    arriving (continuous batching; half the cameras then send host frames with device flows).
    Every camera equals the same frames pushed alone on the GPU;
    sampled cameras equal the oracle; latency percentiles are reported."""
    import time
    import torch
    rng = np.random.default_rng(11)
    res = [(346, 260), (640, 480), (1280, 720)]
    pools = {}
    for W, H in res:
        v = synth.blob_video(synth.serving_stream(W, H, seed=3 * W, n_frames=16))
        pools[(W, H)] = (v, torch.from_numpy(v.frames).cuda(), torch.from_numpy(v.flows).cuda(),
                         torch.from_numpy(v.frames).pin_memory())
    torch.cuda.synchronize()
    srv = sim.Server(hbm_budget_bytes=200 << 30, max_cameras=256, queue_depth=4)
    cams = []
    for c in range(256):
        W, H = res[int(rng.integers(3))]
        cid = srv.admit(width=W, height=H, method="sparse", c_pos=0.2, c_neg=0.2)
        rate = float(rng.uniform(30, 240))
        cams.append(dict(id=cid, W=W, H=H, phase=int(rng.integers(8)), step=int(1e6 / rate),
                         k=0))
    n_frames = 6
    order = [c for c in range(256) for _ in range(n_frames)]
    rng.shuffle(order)
    if worker:
        srv.start()
    for c in order:
        cam = cams[c]
        v, fr, fl, hfr = pools[(cam["W"], cam["H"])]
        j = cam["phase"] + cam["k"]
        flow = None if cam["k"] == 0 else fl[j - 1]
        t = 1000 + cam["k"] * cam["step"]
        while True:
            try:
                # with the worker, odd cameras send frames from pinned host memory
                srv.submit(cam["id"], hfr[j] if worker and c % 2 else fr[j], flow, t)
                break
            except sim.SimError as e:
                assert e.status == sim.E_BUSY
                if worker:
                    time.sleep(0.0005)        # the worker frees the ring
                else:
                    srv.step()
        cam["k"] += 1
        if not worker and rng.random() < 0.02:
            srv.step()
    srv.sync()
    if worker:
        srv.stop()
    st = srv.stats()
    assert st["cameras"] == 256 and st["completed"] == 256 * n_frames
    assert st["failed_frames"] == 0 and 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    for idx, cam in enumerate(cams):
        v, fr, fl, _ = pools[(cam["W"], cam["H"])]
        a, b = cam["phase"], cam["phase"] + n_frames
        t = [1000 + k * cam["step"] for k in range(n_frames)]
        got = srv.drain_keys(cam["id"])
        s = sim.Stream(cam["W"], cam["H"], method="sparse", c_pos=0.2, c_neg=0.2)
        s.push_frames(fr[a:b].contiguous(), fl[a:b - 1].contiguous(), t)
        np.testing.assert_array_equal(got, s.drain_keys(), err_msg=str(cam))
        s.close()
        if idx < 6:
            ok, _ = oracle_keys(v.frames[a:b], v.flows[a:b - 1], t, method=sim.SPARSE,
                                c_pos=0.2, c_neg=0.2)
            np.testing.assert_array_equal(got, ok, err_msg=str(cam))
    srv.close()


MODES_MIX = [
    # (W, H, stream options, oracle options, flows supplied)
    (346, 260, dict(method="dense", thresh_mode="memoryless", c_pos=0.03, c_neg=0.03),
     dict(method=sim.DENSE, thresh_mode=sim.MEMORYLESS, c_pos=0.03, c_neg=0.03), True),
    (640, 480, dict(method="sparse", thresh_mode="memoryless", c_pos=0.03, c_neg=0.03),
     dict(method=sim.SPARSE, thresh_mode=sim.MEMORYLESS, c_pos=0.03, c_neg=0.03), True),
    (346, 260, dict(method="difference", c_pos=0.2, c_neg=0.2),
     dict(method=sim.DIFFERENCE, c_pos=0.2, c_neg=0.2), True),
    (640, 480, dict(method="sparse", flow_source="lk", c_pos=0.15, c_neg=0.15),
     dict(method=sim.SPARSE, flow_source=1, c_pos=0.15, c_neg=0.15), False),
    (240, 180, dict(method="dense", c_pos=0.15, c_neg=0.15, event_capacity=64),
     dict(method=sim.DENSE, c_pos=0.15, c_neg=0.15), True),
]


def test_batched_push_every_mode_equals_streams_alone():
    """One fused batch holding every thresholding mode, the difference method and estimated flow
    (host inputs, two batches, one stream forced through overflow re-runs): each stream equals
    the oracle for it alone."""
    vids = [synth.blob_video(synth.mixed_stream(W, H, seed=70 + i, n_frames=6))
            for i, (W, H, _, _, _) in enumerate(MODES_MIX)]
    streams = [sim.Stream(W, H, **opts) for (W, H, opts, _, _) in MODES_MIX]
    for a, b in ((0, 3), (3, 6)):
        entries = []
        for st, v, (_, _, _, _, supplied) in zip(streams, vids, MODES_MIX):
            fl = v.flows[max(a - 1, 0):b - 1] if supplied else None
            entries.append((st, v.frames[a:b], fl if fl is None or len(fl) else None,
                            v.t_us[a:b]))
        sim.push_batch(entries)
    for st, v, (_, _, opts, ocfg, supplied) in zip(streams, vids, MODES_MIX):
        ok, oref = oracle_keys(v.frames, v.flows if supplied else None, v.t_us, **ocfg)
        assert len(ok) > 0, opts
        np.testing.assert_array_equal(st.drain_keys(), ok, err_msg=str(opts))
        np.testing.assert_array_equal(st.reference().view(np.uint32), oref.view(np.uint32),
                                      err_msg=str(opts))
        st.close()
