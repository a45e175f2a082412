"""The HIP Lucas-Kanade kernels and their runtime integration, executed on the CPU (tests/cpu_emu),
against the oracle bit for bit.  Complements (never replaces) the GPU parity tests."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from oracle.oracle import lk_flow as oracle_lk_flow, FLOW_LK
from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import (emu_build, emu_run, emu_sim, monkeypatch_module,  # noqa: F401
                                       oracle_run, HERE)


def _blob_pair(H, W, seed, motion):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    c = [(rng.uniform(0, W), rng.uniform(0, H), rng.uniform(3, 8), rng.uniform(60, 180))
         for _ in range(8)]

    def img(dx, dy):
        v = np.full((H, W), 25.0)
        for cx, cy, s, a in c:
            v += a * np.exp(-((x - cx - dx) ** 2 + (y - cy - dy) ** 2) / (2 * s * s))
        return np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return img(0, 0), img(*motion)


@pytest.mark.parametrize("levels,radius", [(0, 2), (2, 4), (3, 7), (4, 3)])
def test_emulated_lk_flow_equals_oracle(emu_sim, levels, radius):
    f0, f1 = _blob_pair(37, 53, levels * 7 + radius, (2.5, -1.25))
    pts = np.arange(37 * 53, dtype=np.uint32)[::3].copy()
    pts = np.concatenate([pts, np.array([0, 52, 36 * 53, 37 * 53 - 1, 37 * 53, 10 ** 6],
                                        np.uint32)])                    # corners, out of range
    params = dict(levels=levels, radius=radius)
    flow, valid = emu_sim.lk_flow(f0, f1, pts, **params)
    ref, rvalid = oracle_lk_flow(f0, f1, pts, levels=levels, radius=radius)
    np.testing.assert_array_equal(valid, rvalid)
    np.testing.assert_array_equal(flow.view(np.uint32), ref.view(np.uint32))
    assert valid.sum() > 50 and not valid[-1] and not valid[-2]


@pytest.mark.parametrize("shape", [(37, 1), (9, 7)])
def test_emulated_lk_indices_outside_the_image(emu_sim, shape):
    """Indices at or beyond W * H (up to 2^32 - 1, where p / W exceeds an int for a one-pixel-
    wide image) are invalid with flow (0, 0), as in the oracle, with both rejection tests off."""
    H, W = shape
    rng = np.random.default_rng(H * 100 + W)
    f0 = rng.integers(0, 256, (H, W), dtype=np.uint8)
    f1 = rng.integers(0, 256, (H, W), dtype=np.uint8)
    pts = np.array([0, W * H - 1, W * H, W * H + 7, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 5,
                    2 ** 32 - 1], np.uint32)
    params = dict(levels=0, radius=1, min_trace=0.0, min_ratio=0.0)
    flow, valid = emu_sim.lk_flow(f0, f1, pts, **params)
    ref, rvalid = oracle_lk_flow(f0, f1, pts, **params)
    np.testing.assert_array_equal(valid, rvalid)
    np.testing.assert_array_equal(flow.view(np.uint32), ref.view(np.uint32))
    assert not valid[2:].any() and (flow[2:] == 0).all()


@pytest.mark.parametrize("method", [sim.SPARSE, sim.DENSE])
def test_emulated_estimated_flow_simulation(emu_sim, method):
    """Windows of several intervals (pyramids of every frame of a window), with and without
    overflow re-runs, and single pushes, against the oracle estimating the same flow."""
    spec = synth.BlobVideoSpec(40, 32, 6, 30.0, 6, seed=3, motion="random", speed_max=5.0)
    v = synth.blob_video(spec)
    cfg = dict(method=method, c_pos=0.12, c_neg=0.12, n_interp=4, flow_source=FLOW_LK,
               lk_levels=2, lk_radius=4)
    ok, oref = oracle_run(v.frames, None, v.t_us, **cfg)
    assert len(ok) > 100
    scfg = dict(method=method, c_pos=0.12, c_neg=0.12, n_interp=4, flow_source="lk",
                lk=dict(levels=2, radius=4))
    for mode, cap in (("window", 0), ("window", 16), ("single", 0)):
        keys, ref, st = emu_run(emu_sim, v.frames, None, v.t_us, mode=mode,
                                event_capacity=cap, **scfg)
        np.testing.assert_array_equal(keys, ok, err_msg=f"{mode} {cap}")
        np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32))


@pytest.mark.parametrize("radius", [8, 11, 12, 15])
def test_emulated_estimated_flow_large_windows(emu_sim, radius):
    """Window radii whose (2r + 1)^2 positions need 8 (r = 8 .. 11) and 16 (r = 12 .. 15)
    positions per lane of the one-wave-per-point window pass, against the oracle."""
    spec = synth.BlobVideoSpec(36, 30, 4, 30.0, 5, seed=40 + radius, motion="random",
                               speed_max=4.0)
    v = synth.blob_video(spec)
    ok, oref = oracle_run(v.frames, None, v.t_us, method=sim.SPARSE, c_pos=0.1, c_neg=0.1,
                          n_interp=3, flow_source=FLOW_LK, lk_levels=1, lk_radius=radius)
    assert len(ok) > 20
    keys, ref, _ = emu_run(emu_sim, v.frames, None, v.t_us, method=sim.SPARSE, c_pos=0.1,
                           c_neg=0.1, n_interp=3, flow_source="lk",
                           lk=dict(levels=1, radius=radius))
    np.testing.assert_array_equal(keys, ok)
    np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32))


def test_emulated_estimated_flow_in_a_batch_and_a_server(emu_sim):
    spec = synth.BlobVideoSpec(40, 32, 5, 30.0, 5, seed=6, motion="random", speed_max=4.0)
    v = synth.blob_video(spec)
    ok, _ = oracle_run(v.frames, None, v.t_us, method=sim.SPARSE, c_pos=0.1, c_neg=0.1,
                       n_interp=3, flow_source=FLOW_LK)
    a = emu_sim.Stream(40, 32, method="sparse", c_pos=0.1, c_neg=0.1, n_interp=3,
                       flow_source="lk")
    b = emu_sim.Stream(40, 32, method="dense", c_pos=0.1, c_neg=0.1, n_interp=3)
    emu_sim.push_batch([(a, v.frames, None, v.t_us), (b, v.frames, v.flows, v.t_us)])
    np.testing.assert_array_equal(a.drain_keys(), ok)
    a.close()
    b.close()
    srv = emu_sim.Server(hbm_budget_bytes=1 << 33, max_cameras=2, queue_depth=2)
    cam = srv.admit(width=40, height=32, method="sparse", c_pos=0.1, c_neg=0.1, n_interp=3,
                    flow_source="lk")
    for k in range(5):
        try:
            srv.submit(cam, v.frames[k], None, int(v.t_us[k]))
        except emu_sim.SimError:
            srv.step()
            srv.submit(cam, v.frames[k], None, int(v.t_us[k]))
    srv.step()
    np.testing.assert_array_equal(srv.drain_keys(cam), ok)
    srv.close()


def test_emulated_lk_configuration_errors(emu_sim):
    for method in ("basic", "difference"):
        with pytest.raises(emu_sim.SimError):
            emu_sim.Stream(8, 8, method=method, flow_source="lk")
    with pytest.raises(emu_sim.SimError):
        emu_sim.Stream(8, 8, method="sparse", flow_source="lk", lk=dict(levels=5))
    with pytest.raises(emu_sim.SimError):
        emu_sim.Stream(8, 8, method="sparse", flow_source="lk", lk=dict(radius=16))
    f = np.zeros((8, 8), np.uint8)
    with pytest.raises(emu_sim.SimError):
        emu_sim.lk_flow(f, f, np.array([0], np.uint32), iterations=0)
    flow, valid = emu_sim.lk_flow(f, f, np.zeros(0, np.uint32))
    assert flow.shape == (0, 2)


ASAN_SCRIPT = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim, synth
    sim.LIB_PATH = {lib!r}; sim._lib = None
    from test_cpu_emulated_kernels import oracle_run, emu_run
    from oracle.oracle import lk_flow as olk, FLOW_LK
    rng = np.random.default_rng(2)
    f0 = rng.integers(0, 256, (21, 17), dtype=np.uint8)
    f1 = np.roll(f0, 2, axis=1)
    pts = np.arange(21 * 17 + 3, dtype=np.uint32)
    for levels in (0, 4):
        a, va = sim.lk_flow(f0, f1, pts, levels=levels, radius=15)
        b, vb = olk(f0, f1, pts, levels=levels, radius=15)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)) and np.array_equal(va, vb)
    spec = synth.BlobVideoSpec(33, 19, 7, 30.0, 5, seed=5, motion="random", speed_max=5.0)
    v = synth.blob_video(spec)
    for method in (1, 2):
        ok, _ = oracle_run(v.frames, None, v.t_us, method=method, c_pos=0.1, c_neg=0.1,
                           n_interp=3, flow_source=FLOW_LK, lk_levels=4, lk_radius=6)
        keys, _, _ = emu_run(sim, v.frames, None, v.t_us, method=method, c_pos=0.1, c_neg=0.1,
                             n_interp=3, flow_source="lk", lk=dict(levels=4, radius=6),
                             event_capacity=1)
        assert np.array_equal(keys, ok)
    print("asan-clean")
""")


@pytest.mark.long
def test_emulated_lk_is_memory_safe_under_asan(tmp_path):
    """Pyramids down to 2x2 texels, windows larger than the image, indices out of range and
    overflow re-runs of estimated-flow windows under AddressSanitizer."""
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_lk.py"
    script.write_text(ASAN_SCRIPT.format(root=os.path.dirname(HERE), tests=HERE, lib=lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]


def test_emulated_estimated_flow_beyond_one_mask_word(emu_sim):
    """Sparse with estimated flow over a 40-frame window: the flow kernel reads the selection
    bitmask words of intervals 32 and later; window and single pushes equal the oracle."""
    spec = synth.BlobVideoSpec(28, 20, 40, 60.0, 4, seed=12, motion="random", speed_max=3.0)
    v = synth.blob_video(spec)
    cfg = dict(method=sim.SPARSE, c_pos=0.08, c_neg=0.08, n_interp=3, flow_source=FLOW_LK,
               lk_levels=1, lk_radius=3)
    ok, oref = oracle_run(v.frames, None, v.t_us, **cfg)
    assert len(ok) > 100
    scfg = dict(method=sim.SPARSE, c_pos=0.08, c_neg=0.08, n_interp=3, flow_source="lk",
                lk=dict(levels=1, radius=3))
    for mode in ("window", "single"):
        keys, ref, _ = emu_run(emu_sim, v.frames, None, v.t_us, mode=mode, event_capacity=32,
                               **scfg)
        np.testing.assert_array_equal(keys, ok, err_msg=mode)
        np.testing.assert_array_equal(ref.view(np.uint32), oref.view(np.uint32))
