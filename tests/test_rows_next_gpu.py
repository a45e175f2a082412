"""GPU parity of the memoryless thresholding (the paper's Sec. III-A equations taken literally),
the difference-frame method (Sec. III-C), the accumulated event frame (Fig. 1 caption) and the
events/(pixel s) statistic (Sec. IV-C): through the C ABI, bit for bit against the CPU oracle.

Collected after the parity tests of the reference-level path, so a failure here cannot hide them.
"""
import numpy as np
import pytest

import golden_io
from oracle.oracle import accumulate as oracle_accumulate, event_rate as oracle_event_rate
from paper_2209_04634_amd import sim, synth
from test_parity_gpu import assert_parity, oracle_keys

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("path", golden_io.next_fixtures(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_next_hand_worked_fixtures(path):
    g = golden_io.load(path)
    for mode in ("window", "single"):
        s = sim.Stream(g.frames.shape[2], g.frames.shape[1], **g.cfg)
        if mode == "window":
            s.push_frames(g.frames, g.flows, g.t_us)
        else:
            for k in range(len(g.t_us)):
                s.push(g.frames[k], None if k == 0 else g.flows[k - 1], g.t_us[k])
        t, x, y, p = sim.decode_keys(s.drain_keys(), g.t_us[0])
        assert list(zip(t.tolist(), x.tolist(), y.tolist(), p.tolist())) == \
            [e for iv in g.events for e in iv], mode
        np.testing.assert_array_equal(s.reference(), g.lref)
        s.close()


@pytest.mark.parametrize("S", [1, 2, 11, 33])
@pytest.mark.parametrize("method", [sim.BASIC, sim.DENSE, sim.SPARSE, sim.DIFFERENCE])
def test_memoryless_ragged_image(method, S):
    """A 61x97 image (ragged against every tile), four intervals; S = 33 exceeds the LDS stash
    so interior samples are recomputed."""
    if method == sim.BASIC and S != 1:
        pytest.skip("basic has one sub-interval")
    rng = np.random.default_rng(900 + 100 * S + method)
    frames, flows = synth.random_frames(rng, 5, 61, 97, flow_scale=3.0)
    t = np.array([0, 33333, 50000, 83333, 90001])
    C = 0.3 if method == sim.BASIC else 0.05
    assert_parity(frames, flows, t, modes=("window", "single"), method=method, c_pos=C,
                  c_neg=C * 1.2, n_interp=S - 1, thresh_mode=sim.MEMORYLESS)


@pytest.mark.parametrize("cfg", [dict(method=sim.DIFFERENCE),
                                 dict(method=sim.DENSE, thresh_mode=sim.MEMORYLESS),
                                 dict(method=sim.SPARSE, thresh_mode=sim.MEMORYLESS)],
                         ids=["difference", "dense-memoryless", "sparse-memoryless"])
def test_non_finite_flow_in_the_new_samplers(cfg):
    """NaN and infinite flow components clamp sample positions to the border in the difference
    sampler and the memoryless mode, as in the oracle."""
    rng = np.random.default_rng(77)
    frames, flows = synth.random_frames(rng, 4, 19, 41, flow_scale=4.0)
    flows[0, 3, 5] = [np.nan, 1.0]
    flows[1, 7, 8] = [np.inf, -np.inf]
    flows[2, 2, 2] = [-np.inf, np.nan]
    flows[2, 0, 40] = [np.nan, np.nan]
    assert_parity(frames, flows, np.array([0, 100, 200, 300]), modes=("window", "single"),
                  c_pos=0.05, c_neg=0.05, n_interp=5, **cfg)


def test_difference_346x260_full_sequence():
    """The dense workload's 346x260 60-frame blob video through the difference method (Table I:
    10 interpolated difference frames), one window, chunks and device inputs."""
    v = synth.blob_video(synth.dense_346x260())
    n = assert_parity(v.frames, v.flows, v.t_us, modes=("window", "chunks", "device"),
                      method=sim.DIFFERENCE, c_pos=0.3, c_neg=0.3, n_interp=10,
                      event_capacity=1 << 23)
    assert n > 10000


def test_memoryless_dense_346x260_full_sequence():
    v = synth.blob_video(synth.dense_346x260())
    n = assert_parity(v.frames, v.flows, v.t_us, modes=("window", "chunks"), method=sim.DENSE,
                      c_pos=0.03, c_neg=0.03, n_interp=10, thresh_mode=sim.MEMORYLESS,
                      event_capacity=1 << 23)
    assert n > 10000


def test_memoryless_sparse_1280x720_full_sequence():
    v = synth.blob_video(synth.sparse_1280x720())
    n = assert_parity(v.frames, v.flows, v.t_us, method=sim.SPARSE, c_pos=0.03, c_neg=0.03,
                      n_interp=10, thresh_mode=sim.MEMORYLESS, event_capacity=1 << 24)
    assert n > 10000


def test_difference_spans_windows():
    """140 frames in one push: two windows; the second takes its older frames from the state."""
    spec = synth.BlobVideoSpec(64, 48, 140, 60.0, 6, seed=4, motion="random", speed_max=3.0)
    v = synth.blob_video(spec)
    assert_parity(v.frames, v.flows, v.t_us, modes=("window", "chunks"), method=sim.DIFFERENCE,
                  c_pos=0.05, c_neg=0.05, n_interp=3)


def test_accumulated_frame_and_event_rate():
    """Accumulated frames (host numpy and device int32 tensor) and the events/(pixel s)
    statistic of the sparse 1280x720 sequence over 1/fps windows and the whole sequence."""
    import torch
    v = synth.blob_video(synth.sparse_1280x720())
    cfg = dict(method=sim.SPARSE, c_pos=0.2, c_neg=0.2, n_interp=10)
    ok, _ = oracle_keys(v.frames, v.flows, v.t_us, **cfg)
    s = sim.Stream(1280, 720, **cfg)
    s.push_frames(v.frames, v.flows, v.t_us)
    epoch = int(v.t_us[0])
    t = [int(x) for x in v.t_us]
    windows = [(t[10], t[11]), (t[0], t[-1] + 1), (t[50] + 7, t[90] - 3), (t[-1] + 1, t[-1] + 9)]
    for a, b in windows:
        ref = oracle_accumulate(ok, epoch, a, b, 1280, 720)
        np.testing.assert_array_equal(s.accumulate(a, b), ref)
        dev = torch.zeros((2, 720, 1280), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()            # the zero fill runs on torch's stream
        s.accumulate(a, b, counts=dev)
        s.sync()
        np.testing.assert_array_equal(dev.cpu().numpy().view(np.uint32), ref)
        m, sd, sums = s.event_rate(a, b)
        rm, rsd, rsums = oracle_event_rate(ref, a, b)
        assert sums == rsums and m == rm and sd == rsd
    assert s.pending() == len(ok)
    s.close()


# ------------------------------------------------------------------------------------------
# Pyramidal Lucas-Kanade flow estimation (NEXT-4)
# ------------------------------------------------------------------------------------------

def _lk_frames(H, W, seed, motion):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    c = [(rng.uniform(0, W), rng.uniform(0, H), rng.uniform(3, 10), rng.uniform(60, 180))
         for _ in range(40)]

    def img(dx, dy):
        v = np.full((H, W), 25.0)
        for cx, cy, s, a in c:
            v += a * np.exp(-((x - cx - dx) ** 2 + (y - cy - dy) ** 2) / (2 * s * s))
        return np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return img(0, 0), img(*motion)


@pytest.mark.parametrize("levels,radius", [(0, 3), (3, 7), (4, 10)])
def test_lk_flow_equals_oracle(levels, radius):
    """Host and device inputs, every 9th pixel of a 320x240 pair plus corners and indices
    outside the image, bit for bit."""
    import torch
    from oracle.oracle import lk_flow as oracle_lk_flow
    H, W = 240, 320
    f0, f1 = _lk_frames(H, W, levels + radius, (4.5, -2.25))
    pts = np.concatenate([np.arange(0, H * W, 9, dtype=np.uint32),
                          np.array([W - 1, (H - 1) * W, H * W - 1, H * W, 1 << 30], np.uint32)])
    ref, rvalid = oracle_lk_flow(f0, f1, pts, levels=levels, radius=radius)
    flow, valid = sim.lk_flow(f0, f1, pts, levels=levels, radius=radius)
    np.testing.assert_array_equal(valid, rvalid)
    np.testing.assert_array_equal(flow.view(np.uint32), ref.view(np.uint32))
    assert rvalid.sum() > 1000
    torch.cuda.synchronize()
    d0, d1 = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda()
    dp = torch.from_numpy(pts.view(np.int32)).cuda()
    torch.cuda.synchronize()
    dflow, dvalid = sim.lk_flow(d0, d1, dp, levels=levels, radius=radius)
    np.testing.assert_array_equal(dflow.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    np.testing.assert_array_equal(dvalid.cpu().numpy(), rvalid)


@pytest.mark.parametrize("method,shape,frames", [(sim.SPARSE, (240, 320), 6),
                                                 (sim.DENSE, (64, 96), 5)])
def test_estimated_flow_simulation(method, shape, frames):
    """Sparse and dense simulation with flow estimated on the device: one window, single
    pushes; events and reference levels bit for bit."""
    from oracle.oracle import FLOW_LK
    H, W = shape
    spec = synth.BlobVideoSpec(W, H, frames, 30.0, 24, seed=5, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    ok, oref = oracle_keys(v.frames, None, v.t_us, method=method, c_pos=0.15, c_neg=0.15,
                           n_interp=10, flow_source=FLOW_LK)
    assert len(ok) > 100
    for mode in ("window", "single"):
        s = sim.Stream(W, H, method=method, c_pos=0.15, c_neg=0.15, n_interp=10,
                       flow_source="lk")
        if mode == "window":
            s.push_frames(v.frames, None, v.t_us)
        else:
            for k in range(frames):
                s.push(v.frames[k], None, int(v.t_us[k]))
        np.testing.assert_array_equal(s.drain_keys(), ok, err_msg=mode)
        np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
        s.close()


@pytest.mark.parametrize("radius", [11, 15])
def test_estimated_flow_large_windows(radius):
    """Lucas-Kanade windows of 23x23 and 31x31 positions (8 and 16 per lane of the window pass)
    in a sparse simulation, bit for bit."""
    from oracle.oracle import FLOW_LK
    spec = synth.BlobVideoSpec(160, 120, 4, 30.0, 12, seed=radius, motion="random",
                               speed_max=5.0)
    v = synth.blob_video(spec)
    ok, oref = oracle_keys(v.frames, None, v.t_us, method=sim.SPARSE, c_pos=0.15, c_neg=0.15,
                           n_interp=10, flow_source=FLOW_LK, lk_levels=2, lk_radius=radius)
    assert len(ok) > 100
    s = sim.Stream(160, 120, method="sparse", c_pos=0.15, c_neg=0.15, n_interp=10,
                   flow_source="lk", lk=dict(levels=2, radius=radius))
    s.push_frames(v.frames, None, v.t_us)
    np.testing.assert_array_equal(s.drain_keys(), ok)
    np.testing.assert_array_equal(s.reference().view(np.uint32), oref.view(np.uint32))
    s.close()


def test_selection_statistics():
    """The device statistics of the sparse 1280x720 sequence: selected pixel-intervals equal the
    oracle's per-interval counts summed, active pixels those selected at least once."""
    from oracle.oracle import OracleSim, lut
    v = synth.blob_video(synth.sparse_1280x720())
    o = OracleSim(1280, 720, method=sim.SPARSE, c_pos=0.2, c_neg=0.2)
    o.push(v.frames[0], None, int(v.t_us[0]))
    sel = 0
    for k in range(1, len(v.t_us)):
        o.push(v.frames[k], v.flows[k - 1], int(v.t_us[k]))
        sel += o.selected
    L = lut()[v.frames].astype(np.float32)
    active = int((np.abs(L[1:] - L[:-1]) >= np.float32(0.2)).any(axis=0).sum())
    s = sim.Stream(1280, 720, method="sparse", c_pos=0.2, c_neg=0.2)
    s.push_frames(v.frames, v.flows, v.t_us)
    st = s.stats()
    assert st["selected"] == sel > 0 and st["active"] == active > 0
    s.close()
