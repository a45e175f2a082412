"""The non-allocating Lucas-Kanade call (sim_lk_flow_noalloc, pyramids in the library's fixed
device scratch) equals the allocating sim_lk_flow bit for bit: two calls in a row through the C
ABI, the second on a smaller image, so the second reuses scratch the first left behind."""
import numpy as np
import pytest

from paper_2209_04634_amd import sim

pytestmark = pytest.mark.gpu


def _frames(H, W, seed, motion):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    blobs = [(rng.uniform(0, W), rng.uniform(0, H), rng.uniform(3, 10), rng.uniform(60, 180))
             for _ in range(40)]

    def img(dx, dy):
        v = np.full((H, W), 25.0)
        for cx, cy, s, a in blobs:
            v += a * np.exp(-((x - cx - dx) ** 2 + (y - cy - dy) ** 2) / (2 * s * s))
        return np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return img(0, 0), img(*motion)


CASES = [((240, 320), (4.5, -2.25), 3, 7, 11), ((96, 128), (-1.5, 2.0), 2, 5, 12)]


def test_noalloc_equals_allocating_call_on_two_calls_the_second_smaller():
    import torch
    print("noalloc: two calls, 320x240 then 128x96", flush=True)
    for (H, W), motion, levels, radius, seed in CASES:
        f0, f1 = _frames(H, W, seed, motion)
        pts = np.concatenate([np.arange(0, H * W, 7, dtype=np.uint32),
                              np.array([W - 1, (H - 1) * W, H * W - 1, H * W, 1 << 30],
                                       np.uint32)])
        n = len(pts)
        d0, d1 = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda()
        dp = torch.from_numpy(pts.view(np.int32)).cuda()
        torch.cuda.synchronize()
        ref_flow, ref_valid = sim.lk_flow(d0, d1, dp, levels=levels, radius=radius)
        flow = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda")
        valid = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()            # the fills run on torch's stream
        sim.lk_flow_noalloc(d0, d1, dp, flow, valid, hip_stream=torch.cuda.current_stream(),
                            levels=levels, radius=radius)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(flow.cpu().numpy().view(np.uint32),
                                      ref_flow.cpu().numpy().view(np.uint32))
        np.testing.assert_array_equal(valid.cpu().numpy(), ref_valid.cpu().numpy().astype(np.uint8))
        assert int(ref_valid.sum()) > 100


def test_noalloc_rejects_what_does_not_fit_and_host_memory():
    import torch
    big = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    pts = torch.zeros(4, dtype=torch.int32, device="cuda")
    flow = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(sim.SimError) as e:
        sim.lk_flow_noalloc(big, big, pts, flow)
    assert e.value.status == sim.E_TOO_BIG
    with pytest.raises(ValueError):
        sim.lk_flow_noalloc(np.zeros((8, 8), np.uint8), np.zeros((8, 8), np.uint8),
                            pts, flow)
