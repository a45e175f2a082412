"""The HIP kernel and runtime sources, executed on the CPU (tests/cpu_emu), against the oracle for
the memoryless thresholding, the difference-frame method, the accumulated event frame and the
events/(pixel s) statistic.  Like test_cpu_emulated_kernels.py, these complement (never replace)
the GPU parity tests; the product never loads these builds."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import golden_io
from oracle.oracle import accumulate as oracle_accumulate, event_rate as oracle_event_rate
from paper_2209_04634_amd import sim, synth
from test_cpu_emulated_kernels import (emu_build, emu_run, emu_sim, monkeypatch_module,  # noqa: F401
                                       oracle_run, check, HERE)


@pytest.mark.parametrize("path", golden_io.next_fixtures(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_emulated_next_fixtures(emu_sim, path):
    g = golden_io.load(path)
    for mode in ("window", "single"):
        keys, ref, _ = emu_run(emu_sim, g.frames, g.flows, g.t_us, mode=mode, **g.cfg)
        t, x, y, p = emu_sim.decode_keys(keys, g.t_us[0])
        assert list(zip(t.tolist(), x.tolist(), y.tolist(), p.tolist())) == \
            [e for iv in g.events for e in iv]
        np.testing.assert_array_equal(ref, g.lref)


@pytest.mark.parametrize("S", [1, 2, 11, 33])
@pytest.mark.parametrize("method", [sim.BASIC, sim.DENSE, sim.SPARSE, sim.DIFFERENCE])
def test_emulated_memoryless_ragged_image(emu_sim, method, S):
    """Every method in memoryless mode on a ragged 23x37 image; S = 33 exceeds the LDS stash,
    so interior samples are recomputed."""
    if method == sim.BASIC and S != 1:
        pytest.skip("basic has one sub-interval")
    rng = np.random.default_rng(500 + 100 * S + method)
    frames, flows = synth.random_frames(rng, 5, 23, 37, flow_scale=3.0)
    t = np.array([0, 33333, 50000, 83333, 90001])
    C = 0.3 if method == sim.BASIC else 0.05
    check(emu_sim, frames, flows, t, modes=("window", "single"), method=method, c_pos=C,
          c_neg=C * 1.2, n_interp=S - 1, thresh_mode=sim.MEMORYLESS)


@pytest.mark.parametrize("cfg", [dict(method=sim.DIFFERENCE),
                                 dict(method=sim.DENSE, thresh_mode=sim.MEMORYLESS),
                                 dict(method=sim.SPARSE, thresh_mode=sim.MEMORYLESS)],
                         ids=["difference", "dense-memoryless", "sparse-memoryless"])
def test_emulated_non_finite_flow_clamps_like_the_oracle(emu_sim, cfg):
    """NaN and infinite flow components clamp the sample position to the border (fmin/fmax return
    the other operand for NaN) in the difference-frame sampler too, as in the oracle."""
    rng = np.random.default_rng(77)
    frames, flows = synth.random_frames(rng, 4, 19, 41, flow_scale=4.0)
    flows[0, 3, 5] = [np.nan, 1.0]
    flows[1, 7, 8] = [np.inf, -np.inf]
    flows[2, 2, 2] = [-np.inf, np.nan]
    flows[2, 0, 40] = [np.nan, np.nan]
    n = check(emu_sim, frames, flows, [0, 100, 200, 300], modes=("window", "single"),
              c_pos=0.05, c_neg=0.05, n_interp=5, **cfg)
    assert n > 0


def test_emulated_difference_blob_video_and_chunked_pushes(emu_sim):
    """A blob video through the difference method: one window, single frames, and chunks of
    1, 2, 3 frames (the frame before the previous one comes from the window or the saved state)."""
    spec = synth.BlobVideoSpec(96, 64, 12, 30.0, 8, seed=6, motion="random", speed_max=8.0)
    v = synth.blob_video(spec)
    cfg = dict(method=sim.DIFFERENCE, c_pos=0.4, c_neg=0.4, n_interp=10)
    n = check(emu_sim, v.frames, v.flows, v.t_us, modes=("window", "single"), **cfg)
    assert n > 100
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    s = emu_sim.Stream(96, 64, **cfg)
    j = 0
    for size in (1, 2, 1, 3, 2, 3):
        fl = v.flows[max(j - 1, 0):j + size - 1] if j + size > 1 else None
        if j == 0 and size > 1:
            fl = v.flows[0:size - 1]
        s.push_frames(v.frames[j:j + size], fl, v.t_us[j:j + size])
        j += size
    assert j == 12
    np.testing.assert_array_equal(s.drain_keys(), ok)
    s.close()


@pytest.mark.parametrize("method", [sim.DENSE, sim.SPARSE])
def test_emulated_memoryless_blob_video(emu_sim, method):
    spec = synth.BlobVideoSpec(96, 64, 10, 30.0, 8, seed=5, motion="random", speed_max=8.0)
    v = synth.blob_video(spec)
    n = check(emu_sim, v.frames, v.flows, v.t_us, modes=("window", "single"), method=method,
              c_pos=0.01, c_neg=0.01, thresh_mode=sim.MEMORYLESS)
    assert n > 100


@pytest.mark.parametrize("method", [sim.SPARSE, sim.DENSE])
def test_emulated_memoryless_window_of_70_intervals(emu_sim, method):
    """Memoryless thresholding over a 71-frame window (three selection mask words for sparse),
    with a small event capacity so that chains re-run."""
    spec = synth.BlobVideoSpec(30, 18, 71, 60.0, 4, seed=14, motion="random", speed_max=3.0)
    v = synth.blob_video(spec)
    cfg = dict(method=method, c_pos=0.02, c_neg=0.02, n_interp=3, thresh_mode=sim.MEMORYLESS)
    ok, _ = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    assert len(ok) > 500
    keys, _, st = emu_run(emu_sim, v.frames, v.flows, v.t_us, event_capacity=64, **cfg)
    np.testing.assert_array_equal(keys, ok)
    assert st["retries"] > 0


@pytest.mark.parametrize("method,thresh", [(sim.DIFFERENCE, sim.MEMORYLESS),
                                           (sim.DENSE, sim.MEMORYLESS),
                                           (sim.SPARSE, sim.MEMORYLESS)])
def test_emulated_next_overflow_reruns(emu_sim, method, thresh):
    spec = synth.BlobVideoSpec(64, 48, 8, 30.0, 8, seed=9, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    C = 0.05 if method == sim.DIFFERENCE else 0.01
    cfg = dict(method=method, c_pos=C, c_neg=C, thresh_mode=thresh)
    ok, oref = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    assert len(ok) > 1000
    for cap in (1, 700):
        keys, ref, st = emu_run(emu_sim, v.frames, v.flows, v.t_us, event_capacity=cap, **cfg)
        np.testing.assert_array_equal(keys, ok)
        np.testing.assert_array_equal(ref, oref)
        assert st["retries"] > 0


def test_emulated_difference_spans_windows(emu_sim):
    """140 frames in one push: two windows (128 + 11 intervals); the second window's first
    intervals take their older frames from the saved state."""
    spec = synth.BlobVideoSpec(24, 16, 140, 60.0, 3, seed=4, motion="random", speed_max=2.0)
    v = synth.blob_video(spec)
    check(emu_sim, v.frames, v.flows, v.t_us, method=sim.DIFFERENCE, c_pos=0.05, c_neg=0.05,
          n_interp=3)


def _keys_of(emu, v, **cfg):
    s = emu.Stream(v.frames.shape[2], v.frames.shape[1], **cfg)
    s.push_frames(v.frames, v.flows, v.t_us)
    return s


@pytest.mark.parametrize("method", [sim.DENSE, sim.SPARSE, sim.DIFFERENCE])
def test_emulated_accumulate_and_event_rate(emu_sim, method):
    """Accumulated frames over several windows (inclusive start, exclusive end, before the
    epoch, beyond the last event), host counts added to; the statistic equals the oracle's bit
    for bit (exact integer sums, the same double formula)."""
    spec = synth.BlobVideoSpec(40, 30, 9, 30.0, 6, seed=2, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    cfg = dict(method=method, c_pos=0.1, c_neg=0.1)
    ok, _ = oracle_run(v.frames, v.flows, v.t_us, **cfg)
    s = _keys_of(emu_sim, v, **cfg)
    epoch = int(v.t_us[0])
    t = v.t_us
    windows = [(t[1], t[3]), (t[0] - 5000, t[2] + 1), (t[4], t[4]), (t[7], t[8] + 1),
               (t[8] + 1, t[8] + 10 ** 6), (t[0], t[8] + 1)]
    for a, b in windows:
        got = s.accumulate(int(a), int(b))
        ref = oracle_accumulate(ok, epoch, int(a), int(b), 40, 30)
        np.testing.assert_array_equal(got, ref)
        if b > a:
            m, sd, sums = s.event_rate(int(a), int(b))
            rm, rsd, rsums = oracle_event_rate(ref, int(a), int(b))
            assert sums == rsums and m == rm and sd == rsd
    base = np.arange(2 * 30 * 40, dtype=np.uint32).reshape(2, 30, 40)
    got = s.accumulate(int(t[2]), int(t[6]), counts=base.copy())
    np.testing.assert_array_equal(got, oracle_accumulate(ok, epoch, int(t[2]), int(t[6]), 40, 30,
                                                         counts=base.copy()))
    assert s.pending() == len(ok)          # accumulation does not consume events
    np.testing.assert_array_equal(s.drain_keys(), ok)
    m, sd, sums = s.event_rate(int(t[0]), int(t[8]) + 1)    # nothing pending any more
    assert sums == (0, 0) and m == 0.0 and sd == 0.0
    s.close()


def test_emulated_accumulate_argument_errors(emu_sim):
    s = emu_sim.Stream(8, 6, method="basic")
    with pytest.raises(emu_sim.SimError):
        s.accumulate(10, 5)
    with pytest.raises(emu_sim.SimError):
        s.event_rate(10, 10)
    # before any frame: nothing pending, zero statistic
    assert s.accumulate(0, 100).sum() == 0
    assert s.event_rate(0, 100)[2] == (0, 0)
    with pytest.raises(emu_sim.SimError) as e:
        emu_sim.Stream(8, 6, method=4)
    assert e.value.status == emu_sim.E_INVAL
    with pytest.raises(emu_sim.SimError):
        emu_sim.Stream(8, 6, method="dense", thresh_mode=2)
    s.close()


def test_emulated_batch_and_server_with_new_modes(emu_sim):
    """A batch mixing the difference method and memoryless streams with reference-level ones
    equals every stream alone."""
    specs = [((40, 24), dict(method=sim.DIFFERENCE, c_pos=0.2, c_neg=0.2, n_interp=4)),
             ((33, 17), dict(method=sim.DENSE, c_pos=0.05, c_neg=0.05, n_interp=4,
                             thresh_mode=sim.MEMORYLESS)),
             ((36, 20), dict(method=sim.SPARSE, c_pos=0.15, c_neg=0.15, n_interp=4))]
    vids, solo, streams = [], [], []
    for i, ((W, H), cfg) in enumerate(specs):
        v = synth.blob_video(synth.BlobVideoSpec(W, H, 7, 30.0, 6, seed=20 + i,
                                                 motion="random", speed_max=5.0))
        vids.append(v)
        solo.append(oracle_run(v.frames, v.flows, v.t_us, **cfg)[0])
        streams.append(emu_sim.Stream(W, H, event_capacity=32, **cfg))
    for a, b in ((0, 3), (3, 7)):
        emu_sim.push_batch([(st, v.frames[a:b], v.flows[max(a - 1, 0):b - 1], v.t_us[a:b])
                            for st, v in zip(streams, vids)])
    for st, ok in zip(streams, solo):
        np.testing.assert_array_equal(st.drain_keys(), ok)
        st.close()


ASAN_SCRIPT = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    from paper_2209_04634_amd import sim, synth
    sim.LIB_PATH = {lib!r}; sim._lib = None
    from test_cpu_emulated_kernels import oracle_run, emu_run
    from oracle.oracle import accumulate as oacc
    spec = synth.BlobVideoSpec(48, 40, 7, 30.0, 8, seed=9, motion="random", speed_max=6.0)
    v = synth.blob_video(spec)
    cases = []
    for cap in (1, 0):
        cases.append(dict(method=3, c_pos=0.05, c_neg=0.05, event_capacity=cap))
        cases.append(dict(method=1, c_pos=0.01, c_neg=0.01, thresh_mode=1, event_capacity=cap))
        cases.append(dict(method=2, c_pos=0.01, c_neg=0.01, thresh_mode=1, event_capacity=cap))
    cases.append(dict(method=3, c_pos=0.05, c_neg=0.05, n_interp=40, event_capacity=1))
    for cfg in cases:
        ocfg = dict((k, x) for k, x in cfg.items() if k != "event_capacity")
        ok, oref = oracle_run(v.frames, v.flows, v.t_us, **ocfg)
        s = sim.Stream(48, 40, **cfg)
        s.push_frames(v.frames, v.flows, v.t_us)
        for a, b in ((v.t_us[1], v.t_us[4]), (0, 10 ** 9)):
            got = s.accumulate(int(a), int(b))
            assert np.array_equal(got, oacc(ok, int(v.t_us[0]), int(a), int(b), 48, 40)), cfg
            s.event_rate(int(a), int(b))
        assert np.array_equal(s.drain_keys(), ok) and np.array_equal(s.reference(), oref), cfg
        s.close()
    spec = synth.BlobVideoSpec(20, 12, 140, 60.0, 3, seed=4, motion="random", speed_max=2.0)
    w = synth.blob_video(spec)
    ok, _ = oracle_run(w.frames, w.flows, w.t_us, method=3, c_pos=0.05, c_neg=0.05, n_interp=3)
    keys, _, _ = emu_run(sim, w.frames, w.flows, w.t_us, method=3, c_pos=0.05, c_neg=0.05,
                         n_interp=3, event_capacity=1)
    assert np.array_equal(keys, ok)
    print("asan-clean", len(cases) + 1)
""")


@pytest.mark.long
def test_emulated_next_paths_are_memory_safe_under_asan(tmp_path):
    """The difference method (window splits, overflow re-runs, the recompute path beyond the LDS
    stash), memoryless thresholding and the accumulation kernels under AddressSanitizer."""
    lib = emu_build.build(asan=True)
    asan_rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.exists(asan_rt):
        pytest.skip("libasan not available")
    script = tmp_path / "asan_next.py"
    script.write_text(ASAN_SCRIPT.format(root=os.path.dirname(HERE), tests=HERE, lib=lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    res = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                         timeout=900)
    assert res.returncode == 0 and "asan-clean" in res.stdout, res.stderr[-4000:]


def test_binding_refuses_short_flow_arrays(emu_sim):
    """The binding checks that a push hands over every flow field the library will read, so a
    short array never reaches the device."""
    rng = np.random.default_rng(0)
    frames, flows = synth.random_frames(rng, 4, 6, 9)
    for method in ("dense", "sparse", "difference"):
        s = emu_sim.Stream(9, 6, method=method, n_interp=2)
        with pytest.raises(ValueError):
            s.push_frames(frames, flows[:2], [0, 1, 2, 3])       # needs 3
        with pytest.raises(ValueError):
            s.push_frames(frames, flows[:, :5], [0, 1, 2, 3])    # wrong image shape
        s.push_frames(frames[:1], None, [0])                     # first frame: no flow
        with pytest.raises(ValueError):
            s.push_frames(frames[1:], flows[:2], [1, 2, 3])      # started: needs 3
        with pytest.raises(ValueError):
            emu_sim.push_batch([(s, frames[1:], None, [1, 2, 3])])
        s.push_frames(frames[1:], flows, [1, 2, 3])
        s.close()
    s = emu_sim.Stream(9, 6, method="basic")
    s.push_frames(frames, None, [0, 1, 2, 3])                    # basic reads no flow
    s.close()


def test_emulated_selection_statistics(emu_sim):
    """sim_get_stats of a sparse stream: selected pixel-intervals equal the oracle's per-interval
    selection counts summed; active pixels are the pixels selected at least once in the window."""
    from oracle.oracle import OracleSim, lut
    spec = synth.BlobVideoSpec(64, 48, 9, 30.0, 6, seed=11, motion="random", speed_max=5.0)
    v = synth.blob_video(spec)
    o = OracleSim(64, 48, method=sim.SPARSE, c_pos=0.2, c_neg=0.2)
    o.push(v.frames[0], None, int(v.t_us[0]))
    sel = 0
    for k in range(1, 9):
        o.push(v.frames[k], v.flows[k - 1], int(v.t_us[k]))
        sel += o.selected
    L = lut()[v.frames].astype(np.float32)
    active = int((np.abs(L[1:] - L[:-1]) >= np.float32(0.2)).any(axis=0).sum())
    s = emu_sim.Stream(64, 48, method="sparse", c_pos=0.2, c_neg=0.2)
    s.push_frames(v.frames, v.flows, v.t_us)
    st = s.stats()
    assert st["selected"] == sel > 0 and st["active"] == active > 0
    s.clear_stats()
    assert s.stats()["selected"] == 0
    s.close()
