"""Pins of the oracle's pyramidal Lucas-Kanade flow estimator (the flow of the sparse method,
Sec. III-B) against facts fixed by the method and by mathematics: recovery of known translations
of smooth textures (sub-pixel and beyond one window, which needs the pyramid), rejection of
textureless and one-dimensional windows (aperture problem), antisymmetry, the independent float64
implementation in tests/lk64.py, and the integration of estimated flow into the sparse and dense
methods.  The estimator's quality against real scenes is "parity unpinned": the paper's data and
the library it used are not available."""
import numpy as np
import pytest

import lk64
from oracle.oracle import OracleSim, lk_flow, DENSE, SPARSE, FLOW_LK, MEMORYLESS
from paper_2209_04634_amd import synth


def _blobs(H, W, centres, sigma=5.0, amp=160.0, shift=(0.0, 0.0)):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((H, W), 30.0)
    for cx, cy in centres:
        img += amp * np.exp(-((x - cx - shift[0]) ** 2 + (y - cy - shift[1]) ** 2)
                            / (2 * sigma * sigma))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("motion", [(0.25, 0.0), (-1.5, 0.75), (3.0, -2.0), (6.5, 4.25)])
def test_recovers_subpixel_and_pixel_translations(oracle_mod, motion):
    H, W = 64, 80
    c = [(40, 32)]
    f0 = _blobs(H, W, c)
    f1 = _blobs(H, W, c, shift=motion)
    pts = np.array([32 * W + 40, 30 * W + 37, 35 * W + 43], np.uint32)
    flow, valid = lk_flow(f0, f1, pts)
    assert valid.all()
    np.testing.assert_allclose(flow, np.tile(motion, (3, 1)), atol=0.06)


def test_large_motion_needs_the_pyramid(oracle_mod):
    """A small blob (sigma 2.5 px) moved 11 px: one level cannot see it move (the window at full
    resolution hardly overlaps the displaced blob), three levels recover it."""
    H, W = 64, 96
    f0 = _blobs(H, W, [(40, 32)], sigma=2.5)
    f1 = _blobs(H, W, [(40, 32)], sigma=2.5, shift=(11.0, -3.0))
    pts = np.array([32 * W + 40], np.uint32)
    flat, _ = lk_flow(f0, f1, pts, levels=0)
    deep, ok = lk_flow(f0, f1, pts, levels=3)
    assert ok[0]
    assert np.abs(flat[0] - (11.0, -3.0)).max() > 2.0
    np.testing.assert_allclose(deep[0], (11.0, -3.0), atol=0.1)


def test_static_scene_has_zero_flow(oracle_mod):
    f = _blobs(48, 48, [(20, 22), (30, 30)])
    flow, valid = lk_flow(f, f, np.arange(48 * 48, dtype=np.uint32))
    assert valid.sum() > 500
    assert (flow[valid] == 0).all()


def test_textureless_and_edge_windows_are_rejected(oracle_mod):
    H, W = 40, 40
    flat = np.full((H, W), 90, np.uint8)
    flow, valid = lk_flow(flat, flat, np.array([20 * W + 20], np.uint32))
    assert not valid[0] and (flow == 0).all()
    x = np.arange(W)[None, :].repeat(H, 0)
    edge0 = np.where(x < 20, 40, 200).astype(np.uint8)          # vertical edge: 1-D structure
    edge1 = np.where(x < 23, 40, 200).astype(np.uint8)
    flow, valid = lk_flow(edge0, edge1, np.array([20 * W + 20], np.uint32))
    assert not valid[0] and (flow == 0).all()
    # a corner has 2-D structure and is accepted
    y = np.arange(H)[:, None].repeat(W, 1)
    c0 = np.where((x < 20) & (y < 20), 200, 40).astype(np.uint8)
    c1 = np.where((x < 21) & (y < 19), 200, 40).astype(np.uint8)
    flow, valid = lk_flow(c0, c1, np.array([20 * W + 20], np.uint32), levels=0)
    assert valid[0]


OUTSIDE = [1, 2, 1000, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 5, 2 ** 32 - 1]   # offsets past W * H - 1


@pytest.mark.parametrize("shape", [(37, 1), (1, 53), (9, 7)])
def test_indices_outside_the_image_are_invalid(oracle_mod, shape):
    """An index at or beyond W * H names no pixel: invalid, flow (0, 0), even with both
    rejection tests off, and also where p / W exceeds an int (a one-pixel-wide image)."""
    H, W = shape
    rng = np.random.default_rng(H * 100 + W)
    f0 = rng.integers(0, 256, (H, W), dtype=np.uint8)
    f1 = rng.integers(0, 256, (H, W), dtype=np.uint8)
    last = W * H - 1
    pts = np.array([last] + [min(last + d, 2 ** 32 - 1) for d in OUTSIDE], np.uint32)
    pts[-4:] = np.array(OUTSIDE[-4:], np.uint32)
    flow, valid = lk_flow(f0, f1, pts, levels=0, radius=1, min_trace=0.0, min_ratio=0.0)
    assert not valid[1:].any()
    assert (flow[1:] == 0).all()


def test_antisymmetry(oracle_mod):
    H, W = 64, 64
    f0 = _blobs(H, W, [(30, 30), (40, 36)], sigma=6.0)
    f1 = _blobs(H, W, [(30, 30), (40, 36)], sigma=6.0, shift=(2.25, -1.5))
    pts = np.array([31 * W + 31], np.uint32)
    fwd, _ = lk_flow(f0, f1, pts)
    bwd, _ = lk_flow(f1, f0, pts)
    np.testing.assert_allclose(fwd[0], (2.25, -1.5), atol=0.06)    # the windows sit at the
    np.testing.assert_allclose(bwd[0], (-2.25, 1.5), atol=0.06)    # same pixel of each frame


@pytest.mark.parametrize("levels,radius", [(0, 3), (2, 4), (3, 7)])
def test_matches_independent_float64_implementation(oracle_mod, levels, radius):
    rng = np.random.default_rng(levels * 10 + radius)
    H, W = 36, 44
    compared = 0
    for trial in range(3):
        centres = [(rng.uniform(5, W - 5), rng.uniform(5, H - 5)) for _ in range(6)]
        motion = tuple(rng.uniform(-2.5, 2.5, 2))
        f0 = _blobs(H, W, centres, sigma=4.0, amp=120.0)
        f1 = _blobs(H, W, centres, sigma=4.0, amp=120.0, shift=motion)
        pts = rng.choice(H * W, 60, replace=False).astype(np.uint32)
        flow, valid = lk_flow(f0, f1, pts, levels=levels, radius=radius)
        ref = lk64.lk_flow(f0, f1, pts, levels=levels, radius=radius)
        for j, (rf, rv, margin) in enumerate(ref):
            if margin < 1e-3:
                continue                      # a validity test too close to its threshold
            assert bool(valid[j]) == rv, (j, rf, flow[j])
            if rv:
                np.testing.assert_allclose(flow[j], rf, atol=2e-3)
                compared += 1
    assert compared > 60


@pytest.mark.parametrize("method", [SPARSE, DENSE])
def test_estimated_flow_drives_the_interpolation(oracle_mod, method):
    """A simulation with flow_source = Lucas-Kanade emits exactly the events of the same
    simulation given, as supplied flow, the Lucas-Kanade flow of each frame pair at the pixels
    that are interpolated."""
    spec = synth.BlobVideoSpec(48, 40, 4, 30.0, 5, seed=2, motion="random", speed_max=5.0)
    v = synth.blob_video(spec)
    cfg = dict(method=method, c_pos=0.15, c_neg=0.15, n_interp=4)
    est = OracleSim(48, 40, flow_source=FLOW_LK, **cfg)
    sup = OracleSim(48, 40, **cfg)
    est.push(v.frames[0], None, int(v.t_us[0]))
    sup.push(v.frames[0], None, int(v.t_us[0]))
    total = 0
    for k in range(1, 4):
        flow, _ = lk_flow(v.frames[k - 1], v.frames[k])
        a = est.push(v.frames[k], None, int(v.t_us[k]))
        b = sup.push(v.frames[k], flow.reshape(40, 48, 2), int(v.t_us[k]))
        np.testing.assert_array_equal(a, b)
        total += len(a)
    assert total > 50
    np.testing.assert_array_equal(est.lref(), sup.lref())


def test_estimated_flow_with_memoryless_thresholding(oracle_mod):
    spec = synth.BlobVideoSpec(40, 32, 3, 30.0, 4, seed=8, motion="random", speed_max=4.0)
    v = synth.blob_video(spec)
    cfg = dict(method=SPARSE, c_pos=0.02, c_neg=0.02, n_interp=4, thresh_mode=MEMORYLESS)
    est = OracleSim(40, 32, flow_source=FLOW_LK, **cfg)
    sup = OracleSim(40, 32, **cfg)
    est.push(v.frames[0], None, 0)
    sup.push(v.frames[0], None, 0)
    flow, _ = lk_flow(v.frames[0], v.frames[1])
    np.testing.assert_array_equal(est.push(v.frames[1], None, 1000),
                                  sup.push(v.frames[1], flow.reshape(32, 40, 2), 1000))


def test_invalid_configurations(oracle_mod):
    with pytest.raises(ValueError):
        OracleSim(8, 8, method=0, flow_source=FLOW_LK)             # basic has no flow
    with pytest.raises(ValueError):
        OracleSim(8, 8, method=SPARSE, flow_source=FLOW_LK, lk_levels=5)
    with pytest.raises(ValueError):
        OracleSim(8, 8, method=SPARSE, flow_source=FLOW_LK, lk_radius=0)
