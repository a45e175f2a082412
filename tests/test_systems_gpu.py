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
